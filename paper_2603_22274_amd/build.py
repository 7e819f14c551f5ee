"""Compile libfelis.so (HIP kernels + C ABI) for gfx950, in-tree.

Every translation unit is built with hipcc for gfx950 with packed FP32
instructions disabled; the neighbour-list unit additionally disables FMA
contraction so its FP64 inclusion test is an exact, documented sequence of
rounded operations.  Objects go to ``_build/`` beside this file and the
shared library to ``libfelis.so`` in the package directory.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
BUILD = os.path.join(HERE, '_build')
LIB = os.path.join(HERE, 'libfelis.so')
ARCH = 'gfx950'
HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')

COMMON = ['-O3', '-fPIC', '-std=c++17', f'--offload-arch={ARCH}',
          '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
          '-Wno-unused-result', '-I', os.path.join(HERE, '..', 'include')]
UNITS = {
    'nlist.hip': ['-ffp-contract=off'],
    'nonbonded.hip': [],
    'pme.hip': [],
    'integrate.hip': [],
    'ukn.hip': [],
    'mbar.hip': [],
    'hrex.hip': [],
    'barostat.hip': [],
    'felis.cpp': [],
}


def _compile(src, extra):
    obj = os.path.join(BUILD, src + '.o')
    cmd = [HIPCC, '-c', os.path.join(CSRC, src), '-o', obj] + COMMON + extra
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    warn = [l for l in r.stderr.splitlines() if 'packed-fp32-ops' not in l and l.strip()]
    return obj, warn


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        futs = {ex.submit(_compile, s, e): s for s, e in UNITS.items()}
        objs = []
        for f in cf.as_completed(futs):
            obj, warn = f.result()
            objs.append(obj)
            if verbose and warn:
                print(f"[{futs[f]}]\n" + "\n".join(warn), file=sys.stderr)
    tmp = LIB + '.tmp'
    cmd = [HIPCC, '-shared', '-o', tmp, f'--offload-arch={ARCH}'] + sorted(objs)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    print(build(verbose=True))
