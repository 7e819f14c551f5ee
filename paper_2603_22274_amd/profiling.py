"""Summaries of rocprofv3 output databases (kernel traces and PMC counters).

    python -m paper_2603_22274_amd.profiling stats <trace_dir> [n]
    python -m paper_2603_22274_amd.profiling traffic <fetch_dir> <write_dir> <kernel-substring>
    python -m paper_2603_22274_amd.profiling counters <pmc_dir> <kernel-substring> ...
    python -m paper_2603_22274_amd.profiling profiles <run_dir> <profiles_dir> [workload]

    python -m paper_2603_22274_amd.profiling steps <trace_dir> [min_pair_us]
    python -m paper_2603_22274_amd.profiling timeline <trace_dir> [after_gap_ms]

``stats`` prints per-kernel call counts, average and total durations.
``steps`` splits a kernel trace at the pair kernel's launches (one per MD
step) into device time per kernel, busy and idle time per step; ``timeline``
measures the idle device time of a whole run (queue packets between launches
and host time between calls) per MD step.
``profiles`` writes the committed summaries of the pair kernel's HBM traffic
(JSON with the digest of the kernel's sources, read by bench.py) and of the
VALU counters of the main kernels from the four counter passes
(pmc_<workload>_A, _B, _FETCH_SIZE, _WRITE_SIZE under <run_dir>).
``traffic`` scales the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch)
of one kernel by what the same counters read for the largest plain device
copy in the run (bytes actually moved / bytes counted), and prints the
per-launch HBM traffic as JSON.
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
import sqlite3
import sys


def _db(d):
    hits = glob.glob(d.rstrip('/') + '/*results.db')
    if not hits:
        raise FileNotFoundError(f"no rocprofv3 database under {d}")
    return sqlite3.connect(hits[0])


def short(name):
    n = name.replace('felis::(anonymous namespace)::', '')
    return n.split('(felis::')[0].split('(double const')[0].split('(long long')[0].strip()


def kernel_stats(trace_dir, top=25):
    con = _db(trace_dir)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    out = [f"{'kernel':44s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for name, n, tot, avg, pct in rows[:top]:      # the view reports microseconds
        out.append(f"{short(name)[:44]:44s} {n:7d} {avg:10.2f} {tot / 1e3:10.3f} {pct:6.1f}")
    return "\n".join(out)


def _kernel_rows(trace_dir):
    con = _db(trace_dir)
    return con.execute("select name, start, end from kernels order by start").fetchall()


def _union(iv):
    """Total length covered by the intervals ``iv`` [(start, end)]."""
    tot, cur_s, cur_e = 0, None, None
    for a, b in sorted(iv):
        if cur_e is None or a > cur_e:
            if cur_e is not None:
                tot += cur_e - cur_s
            cur_s, cur_e = a, b
        else:
            cur_e = max(cur_e, b)
    if cur_e is not None:
        tot += cur_e - cur_s
    return tot


def step_breakdown(trace_dir, min_pair_us=0.0, max_step_us=20000.0):
    """Device time per MD step between consecutive launches of the pair kernel
    (one per MD step): per kernel, the sum over kernels, the wall time, the
    time at least one kernel ran (busy) and the rest (idle queue).  Pair
    launches shorter than ``min_pair_us`` (other legs or passes) do not
    delimit steps; intervals longer than ``max_step_us`` (host work between
    calls) are skipped."""
    import collections
    import re
    rows = _kernel_rows(trace_dir)

    def nm(n):
        m = re.search(r'(k_\w+(<[^>(]*>)?)', n)
        return m.group(1) if m else short(n)[:40]
    p = [i for i, r in enumerate(rows) if 'k_pairs' in r[0] and (r[2] - r[1]) >= min_pair_us * 1e3]
    acc, cnt = collections.defaultdict(float), collections.Counter()
    steps, wall, busy = 0, 0.0, 0.0
    for a, b in zip(p, p[1:]):
        t0, t1 = rows[a][1], rows[b][1]
        if t1 - t0 > max_step_us * 1e3:
            continue
        steps += 1
        wall += t1 - t0
        iv = []
        for r in rows[max(0, a - 64):b]:
            s0, s1 = max(r[1], t0), min(r[2], t1)
            if s1 > s0:
                iv.append((s0, s1))
        busy += _union(iv)
        for r in rows[a:b]:
            acc[nm(r[0])] += r[2] - r[1]
            cnt[nm(r[0])] += 1
    if not steps:
        return {"steps": 0}
    per = {k: {"us_per_step": v / steps / 1e3, "launches_per_step": cnt[k] / steps}
           for k, v in sorted(acc.items(), key=lambda kv: -kv[1])}
    return {"steps": steps, "wall_us_per_step": wall / steps / 1e3, "busy_us_per_step": busy / steps / 1e3,
            "idle_us_per_step": (wall - busy) / steps / 1e3,
            "kernel_sum_us_per_step": sum(v for v in acc.values()) / steps / 1e3, "kernels": per}


def timeline(trace_dir, host_gap_us=100.0, after_gap_ms=0.0):
    """Idle device time over a whole run, from the first to the last pair
    launch: gaps between kernels shorter than ``host_gap_us`` (queue packets
    between launches inside a call) and longer ones (the host between calls),
    per MD step (pair launches).  ``after_gap_ms`` > 0: only the part after
    the first idle gap of at least that length (a pause the program makes
    between its preparation and the measured phase)."""
    rows = _kernel_rows(trace_dir)
    if after_gap_ms > 0:
        end = None
        for i, r in enumerate(rows):
            if end is not None and r[1] - end >= after_gap_ms * 1e6:
                rows = rows[i:]
                break
            end = r[2] if end is None else max(end, r[2])
    p = [i for i, r in enumerate(rows) if 'k_pairs' in r[0]]
    if len(p) < 2:
        return {"md_steps": len(p)}
    t0, t1 = rows[p[0]][1], rows[p[-1]][2]
    iv = sorted((max(r[1], t0), min(r[2], t1)) for r in rows if r[2] > t0 and r[1] < t1)
    busy = _union(iv)
    short_gap = long_gap = 0
    n_long = 0
    cur_e = None
    for a, b in iv:
        if cur_e is not None and a > cur_e:
            g = a - cur_e
            if g < host_gap_us * 1e3:
                short_gap += g
            else:
                long_gap += g
                n_long += 1
        cur_e = b if cur_e is None else max(cur_e, b)
    n = len(p)
    return {"md_steps": n, "span_ms": (t1 - t0) / 1e6, "busy_ms": busy / 1e6,
            "idle_fraction": 1.0 - busy / (t1 - t0),
            "queue_gaps_us_per_md_step": short_gap / n / 1e3,
            "host_gaps_us_per_md_step": long_gap / n / 1e3, "host_gaps": n_long,
            "busy_us_per_md_step": busy / n / 1e3}


def _counter(con, kernel_sub):
    """Mean per dispatch over the kernel's largest launches (the workload's
    own: a run also launches the kernel for smaller preparation legs)."""
    rows = [(g, v) for (n, g, v) in con.execute("select kernel_name, grid_size, value from counters_collection")
            if kernel_sub in n]
    if not rows:
        return None, 0
    gmax = max(g for g, _ in rows)
    vals = [v for g, v in rows if g == gmax]
    return sum(vals) / len(vals), len(vals)


def _copy_reference(con):
    r = con.execute("select grid_size, value from counters_collection where kernel_name like '%copyBuffer%' "
                    "order by value desc limit 1").fetchone()
    return r


def traffic(fetch_dir, write_dir, kernel_sub, copy_bytes=256 << 20):
    cf, cw = _db(fetch_dir), _db(write_dir)
    f_kib, nf = _counter(cf, kernel_sub)
    w_kib, nw = _counter(cw, kernel_sub)
    f_copy = _copy_reference(cf)[1]
    w_copy = _copy_reference(cw)[1]
    f_scale = copy_bytes / (f_copy * 1024.0)
    w_scale = copy_bytes / (w_copy * 1024.0)
    fetch = f_kib * 1024.0 * f_scale
    write = w_kib * 1024.0 * w_scale
    return {"kernel": kernel_sub, "dispatches": [nf, nw],
            "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
            "copy_reference": {"bytes": copy_bytes, "fetch_kib": f_copy, "write_kib": w_copy,
                               "fetch_scale": f_scale, "write_scale": w_scale},
            "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
            "bytes_per_launch": fetch + write}


def counters(pmc_dir, kernels):
    """Per-dispatch averages of every counter collected in ``pmc_dir`` for the
    kernels whose names contain one of ``kernels``."""
    con = _db(pmc_dir)
    rows = con.execute("select kernel_name, grid_size, counter_name, value from counters_collection").fetchall()
    gmax = {}
    for name, g, cname, v in rows:
        for k in kernels:
            if k in name:
                gmax[k] = max(gmax.get(k, 0), g)
    out = {}
    for name, g, cname, v in rows:
        for k in kernels:
            if k in name and g == gmax[k]:       # the workload's own launches
                out.setdefault(k, {}).setdefault(cname, []).append(v)
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in out.items()}


_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'csrc')
PAIR_SOURCES = ('nonbonded.hip', 'erfc_coeffs.h', 'felis_internal.h')
WORKLOADS = {
    'complex42': ("42-window complex leg (70527 atoms, 96^3 grid)",
                  "python -u <repo>/bench.py --workload complex42 --steps 2 --warmup 0 --md 10 --equil 20 "
                  "--no-cpu-baseline --no-per-window --serve-legs 0 --ukn-frames 0 --ddg-segment '' "
                  "--copy-calibration", 'k_pairs<0>', 42 * 70527 * 3 * 8),
    'solvent20': ("20-window solvent leg (7540 atoms, 48^3 grid)",
                  "python -u <repo>/bench.py --workload solvent20 --steps 2 --warmup 0 --md 10 --equil 20 "
                  "--no-cpu-baseline --no-per-window --serve-legs 0 --ukn-frames 0 --ddg-segment '' "
                  "--copy-calibration", 'k_pairs<0>', 20 * 7540 * 3 * 8),
}
WORKLOADS_SIZE = {'complex42': (42, 70527, 96 ** 3), 'solvent20': (20, 7540, 48 ** 3)}
_PASSES = {
    'A': 'SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU '
         'SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VMEM',
    'B': 'SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VALU_FLOPS_FP32 '
         'SQ_INSTS_VALU_TRANS_F32 SQ_THREAD_CYCLES_VALU GRBM_GUI_ACTIVE',
    'FETCH_SIZE': 'FETCH_SIZE', 'WRITE_SIZE': 'WRITE_SIZE'}


def src_digest():
    """Digest of the pair kernel's sources (a stored traffic figure is valid
    only for these)."""
    h = hashlib.sha256()
    for f in PAIR_SOURCES:
        with open(os.path.join(_CSRC, f), 'rb') as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _cmd(name, workload):
    return (f"cd /tmp && TMPDIR=/tmp timeout -s KILL 120 rocprofv3 --pmc {_PASSES[name]} "
            f"-d <run_dir>/pmc_{workload}_{name} -o run -- {WORKLOADS[workload][1]}")


def write_profiles(out_dir, prof_dir, workload='complex42'):
    """Committed summaries from the four counter passes of ``workload``
    (pmc_<workload>_{A,B,FETCH_SIZE,WRITE_SIZE} under ``out_dir``)."""
    desc, _, kernel, force_bytes = WORKLOADS[workload]
    pre = os.path.join(out_dir, f'pmc_{workload}_')
    t = traffic(pre + 'FETCH_SIZE', pre + 'WRITE_SIZE', kernel)
    t['kernel_digest'] = src_digest()
    t['commands'] = [_cmd('FETCH_SIZE', workload), _cmd('WRITE_SIZE', workload),
                     f"python -m paper_2603_22274_amd.profiling profiles <run_dir> profiles {workload}"]
    with open(os.path.join(prof_dir, f'pairs_traffic_{workload}.json'), 'w') as fh:
        json.dump(t, fh, indent=1)
    f, w, c = t['fetch_bytes_per_launch'] / 1e6, t['write_bytes_per_launch'] / 1e6, t['copy_reference']
    txt = [f"HBM traffic of the real-space pair kernel {kernel}, {desc}, MI355X.",
           "Two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE) of bench.py with a 256 MiB device copy at start.",
           f"Copy reference: FETCH_SIZE {c['fetch_kib']:.0f} KiB and WRITE_SIZE {c['write_kib']:.0f} KiB for 262144 KiB "
           f"read + 262144 KiB written -> scale {c['fetch_scale']:.3f} (fetch), {c['write_scale']:.3f} (write).",
           f"{kernel}: FETCH_SIZE {t['fetch_kib_per_dispatch']:.1f} KiB/dispatch, WRITE_SIZE "
           f"{t['write_kib_per_dispatch']:.1f} KiB/dispatch",
           f"  -> {f:.1f} MB read + {w:.1f} MB written = {f + w:.1f} MB per launch ({t['dispatches'][0]} dispatches)",
           f"  (forces of every atom-window, {force_bytes / 1e6:.1f} MB, are written once; the half-cluster lists",
           "   are read once; the rest is partner coordinates and parameters re-read through L2)",
           f"kernel source digest: {t['kernel_digest']}", "Commands:"] + t['commands']
    # every main kernel of the step: HBM bytes per launch against its
    # algorithmic bytes (read once / written once; none for the list build,
    # whose work depends on the windows due)
    W, N, K3 = WORKLOADS_SIZE[workload]
    npair = (W + 1) // 2
    alg = {kernel: 48 * W * N,
           'k_spread': W * (32 * N + 4 * K3),                 # stencils + charges in, own grid component out
           'k_fft_xy<false>': npair * K3 * 16, 'k_fft<0, 0, 32>': npair * K3 * 16, 'k_fft<1, 0, 32>': npair * K3 * 16,
           'k_fft<2, 3, 32>': npair * K3 * 16, 'k_fft<1, 1, 32>': npair * K3 * 16, 'k_fft<0, 1, 32>': npair * K3 * 16,
           'k_fft_xy<true>': npair * K3 * 16,
           'k_gather<false, true>': W * (4 * K3 + 56 * N),    # own grid component, stencils + charges, forces
           'k_integrate': W * N * 76, 'k_pack<true>': W * N * 48, 'k_build': None}
    txt += ["", "Every main kernel of the MD step (same two passes, same scaling; MB per launch):",
            f"{'kernel':24s} {'launches':>8s} {'read':>9s} {'written':>9s} {'algorithmic':>11s} {'ratio':>7s}"]
    cf, cw = _db(pre + 'FETCH_SIZE'), _db(pre + 'WRITE_SIZE')
    fs, ws = c['fetch_scale'], c['write_scale']
    for k, a in alg.items():
        fk, nk = _counter(cf, k)
        wk, _ = _counter(cw, k)
        if fk is None:
            continue
        rd, wr = fk * 1024 * fs / 1e6, wk * 1024 * ws / 1e6
        txt.append(f"{k:24s} {nk:8d} {rd:9.1f} {wr:9.1f} " +
                   (f"{a / 1e6:11.1f} {(rd + wr) / (a / 1e6):7.2f}" if a else f"{'-':>11s} {'-':>7s}"))
    txt += ["algorithmic: pairs 48 B per atom-window; spreading 32 B per atom-window + 4 B per grid point per",
            "window; an FFT pass 16 B per complex point of each pair grid; gather 4 B per grid point + 56 B per",
            "atom-window; integrator 76 B and pack 48 B per atom-window."]
    with open(os.path.join(prof_dir, f'pairs_traffic_{workload}.txt'), 'w') as fh:
        fh.write("\n".join(txt) + "\n")
    # per-axis FFT passes of the step: 32 lines per workgroup (the u_kn passes,
    # with 16 lines and a larger grid, are other launches)
    ks = [kernel, 'k_build', 'k_spread', 'k_gather<false, true>', 'k_fft_xy<false>', 'k_fft<0, 0, 32>',
          'k_fft<1, 0, 32>', 'k_fft<2, 3, 32>', 'k_fft<1, 1, 32>', 'k_fft<0, 1, 32>', 'k_fft_xy<true>', 'k_integrate',
          'k_pack<true>']
    A = counters(pre + 'A', ks)
    B = counters(pre + 'B', ks)
    lines = [f"VALU counters per dispatch, bench.py workload ({desc}), MI355X.",
             "issue_util = SQ_INSTS_VALU / (1024 SIMDs x GRBM_GUI_ACTIVE/8 cycles / 4 cycles per wave64 instruction):",
             "a relative VALU issue rate (1.0 = one wave64 instruction per SIMD every 4 cycles);",
             "FP32 flops = SQ_INSTS_VALU_FLOPS_FP32 x 64 lanes; duration = GRBM_GUI_ACTIVE/8 cycles at a nominal 2.4 GHz "
             "(under counter collection, kernels serialised; HIP events time the pair kernel alone at ~6 % longer, "
             "i.e. the clock runs below 2.4 GHz under this load).", "",
             f"{'kernel':22s} {'us':>8s} {'VALU instr':>11s} {'issue_util':>10s} {'FP32 Gflop':>10s} {'TFLOP/s':>8s} "
             f"{'LDS instr':>10s} {'VMEM rd':>9s} {'wait/wave-cyc':>13s}"]
    for k in ks:
        a, b = A.get(k, {}), B.get(k, {})
        if not b:
            continue
        cyc = b['GRBM_GUI_ACTIVE'] / 8
        us = cyc / 2400
        fl = b['SQ_INSTS_VALU_FLOPS_FP32'] * 64
        lines.append(f"{k:22s} {us:8.1f} {b['SQ_INSTS_VALU']:11.3g} {b['SQ_INSTS_VALU'] / (1024 * cyc / 4):10.2f} "
                     f"{fl / 1e9:10.2f} {fl / us / 1e6:8.1f} {b['SQ_INSTS_LDS']:10.3g} {b['SQ_INSTS_VMEM_RD']:9.3g} "
                     f"{a.get('SQ_WAIT_ANY', 0) / max(a.get('SQ_WAVE_CYCLES', 1), 1):13.2f}")
    lines += ["", "Commands (one pass each):", _cmd('A', workload), _cmd('B', workload),
              f"python -m paper_2603_22274_amd.profiling profiles <run_dir> profiles {workload}"]
    with open(os.path.join(prof_dir, f'valu_counters_{workload}.txt'), 'w') as fh:
        fh.write("\n".join(lines) + "\n")
    return t


if __name__ == '__main__':
    if sys.argv[1] == 'stats':
        print(kernel_stats(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25))
    elif sys.argv[1] == 'steps':
        print(json.dumps(step_breakdown(sys.argv[2], float(sys.argv[3]) if len(sys.argv) > 3 else 0.0), indent=1))
    elif sys.argv[1] == 'timeline':
        print(json.dumps(timeline(sys.argv[2], after_gap_ms=float(sys.argv[3]) if len(sys.argv) > 3 else 0.0),
                         indent=1))
    elif sys.argv[1] == 'profiles':
        print(json.dumps(write_profiles(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else 'complex42'),
                         indent=1))
    elif sys.argv[1] == 'counters':
        print(json.dumps(counters(sys.argv[2], sys.argv[3:]), indent=1))
    elif sys.argv[1] == 'traffic':
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4]), indent=1))
