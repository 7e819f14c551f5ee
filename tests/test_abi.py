"""Host-side checks of the C ABI (no GPU needed).

* libfelis.so loads and exports every function include/felis.h declares.
* The ctypes mirror of felis_leg has the C layout (size and offsets).
* Work-size validation rejects unsupported configurations without a device.
* The SETTLE constraint solve (csrc/settle.h, compiled for the host) equals
  the oracle's converged SHAKE on perturbed rigid waters.
"""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'felis.h')


def _lib():
    from paper_2603_22274_amd import build, felis
    if not os.path.exists(felis.LIB_PATH):
        build.build()
    return felis.lib()


def test_exports_every_declared_symbol():
    names = set(re.findall(r'\b(felis_[a-z_0-9]+)\s*\(', open(HEADER).read()))
    assert len(names) >= 14
    L = _lib()
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def test_leg_struct_layout_matches_header():
    from paper_2603_22274_amd.felis import FelisLeg
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "felis.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(felis_leg), offsetof(felis_leg, charge),
         offsetof(felis_leg, restraint_k), offsetof(felis_leg, lambdas), offsetof(felis_leg, seed),
         offsetof(felis_leg, work_bytes));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, 'l.c')
        open(c, 'w').write(src)
        exe = os.path.join(d, 'l')
        subprocess.run(['gcc', '-I', os.path.join(ROOT, 'include'), c, '-o', exe], check=True)
        out = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    py = [C.sizeof(FelisLeg)] + [getattr(FelisLeg, f).offset for f in
                                 ('charge', 'restraint_k', 'lambdas', 'seed', 'work_bytes')]
    assert out == py


def test_work_size_validation():
    from paper_2603_22274_amd import felis, gen
    L = _lib()
    s = gen.config0()
    leg = felis.FelisLeg()
    leg.n_atoms = s.n_atoms
    leg.box = (C.c_double * 3)(*s.box)
    leg.r_cut, leg.skin, leg.ewald_alpha, leg.sc_alpha, leg.sc_p = 9.0, 0.25, s.ewald_alpha, 0.5, 1
    leg.grid = (C.c_int32 * 3)(20, 20, 20)
    leg.spline_order = 4
    dummy = C.c_void_p(16)
    for f in ('charge', 'sigma', 'epsilon', 'mass', 'is_ligand', 'x', 'y', 'z', 'vx', 'vy', 'vz', 'fx', 'fy',
              'fz', 'energy', 'lambdas', 'excl_ptr'):
        setattr(leg, f, dummy)
    leg.n_windows = 12
    n = C.c_size_t(0)
    assert L.felis_leg_work_size(C.byref(leg), C.byref(n)) == 0 and n.value > 0
    leg.skin = 0.4          # 9.4 > 18.6 / 2
    assert L.felis_leg_work_size(C.byref(leg), C.byref(n)) == felis.E_BOX
    leg.skin = 0.25
    leg.spline_order = 6
    assert L.felis_leg_work_size(C.byref(leg), C.byref(n)) == felis.E_UNSUPPORTED
    leg.spline_order = 4
    leg.grid = (C.c_int32 * 3)(20, 21 * 7, 20)
    assert L.felis_leg_work_size(C.byref(leg), C.byref(n)) == felis.E_UNSUPPORTED
    leg.grid = (C.c_int32 * 3)(20, 20, 20)
    leg.ewald_alpha = 3.6 / 9.0             # the real-space erfc fit covers alpha r_c <= 3.5
    assert L.felis_leg_work_size(C.byref(leg), C.byref(n)) == felis.E_UNSUPPORTED


def test_leg_footprint_without_allocation():
    from paper_2603_22274_amd import felis, gen
    s0, s1 = gen.config0(), gen.config1()
    a = felis.leg_footprint(s0)
    b = felis.leg_footprint(s0, n_windows=2 * s0.n_windows)
    c = felis.leg_footprint(s1)
    # state, lists and grids scale with the windows; a larger system costs more
    assert 0 < a < b < 2.2 * a
    assert c > 5 * a
    assert felis.leg_footprint(s1, list_cap=4096) > c


def test_settle_matches_oracle_shake():
    from oracle.integrate import shake_waters
    from paper_2603_22274_amd import gen
    shim = r'''
#include "settle.h"
extern "C" void settle_many(int n, const float* old, float* nw, float mO, float mH, float doh, float dhh) {
  for (int i = 0; i < n; ++i) {
    const float* o = old + 9 * i; float* p = nw + 9 * i;
    felis::v3 b0 = felis::mk(o[3] - o[0], o[4] - o[1], o[5] - o[2]);
    felis::v3 c0 = felis::mk(o[6] - o[0], o[7] - o[1], o[8] - o[2]);
    felis::v3 a1 = felis::mk(p[0] - o[0], p[1] - o[1], p[2] - o[2]);
    felis::v3 b1 = felis::mk(p[3] - o[0], p[4] - o[1], p[5] - o[2]);
    felis::v3 c1 = felis::mk(p[6] - o[0], p[7] - o[1], p[8] - o[2]);
    felis::settle(b0, c0, a1, b1, c1, mO, mH, doh, dhh);
    p[0] = a1.x + o[0]; p[1] = a1.y + o[1]; p[2] = a1.z + o[2];
    p[3] = b1.x + o[0]; p[4] = b1.y + o[1]; p[5] = b1.z + o[2];
    p[6] = c1.x + o[0]; p[7] = c1.y + o[1]; p[8] = c1.z + o[2];
  }
}
'''
    s = gen.config0()
    rng = np.random.default_rng(0)
    W = s.waters[:64]
    old = s.pos[W].astype(np.float64)                        # (64, 3, 3) rigid
    new = old + rng.normal(0, 0.02, old.shape)               # unconstrained step
    with tempfile.TemporaryDirectory() as d:
        cpp = os.path.join(d, 's.cpp')
        open(cpp, 'w').write(shim)
        so = os.path.join(d, 's.so')
        subprocess.run(['g++', '-O2', '-shared', '-fPIC', '-I',
                        os.path.join(ROOT, 'paper_2603_22274_amd', 'csrc'), cpp, '-o', so], check=True)
        lib = C.CDLL(so)
        o32 = np.ascontiguousarray(old, np.float32)
        n32 = np.ascontiguousarray(new, np.float32)
        lib.settle_many(len(W), o32.ctypes.data_as(C.c_void_p), n32.ctypes.data_as(C.c_void_p),
                        C.c_float(s.mass[W[0, 0]]), C.c_float(s.mass[W[0, 1]]), C.c_float(s.d_oh),
                        C.c_float(s.d_hh))
    # oracle: SHAKE over the same waters (indices relabelled 0..191)
    x_old = old.reshape(-1, 3)
    x_new = np.asarray(o32, np.float64).reshape(-1, 3) * 0 + new.reshape(-1, 3)
    wat = np.arange(3 * len(W)).reshape(-1, 3)
    mass = np.tile(s.mass[W[0]], len(W))
    ref = shake_waters(np.asarray(o32, np.float64).reshape(-1, 3), np.asarray(new.astype(np.float32), np.float64).reshape(-1, 3),
                       wat, mass, s.d_oh, s.d_hh, np.array([1e4] * 3))
    got = n32.reshape(-1, 3).astype(np.float64)
    assert np.max(np.abs(got - ref)) < 2e-5
    # constraints met in FP32
    r = np.linalg.norm(got[0::3] - got[1::3], axis=1)
    assert np.max(np.abs(r - s.d_oh)) < 1e-5


def test_rigid_velocity_matches_oracle_constraint():
    """The integrator's velocity constraint of a rigid water (rigid-body
    projection, FP32, compiled for the host) against the oracle's RATTLE
    multipliers solved in FP64."""
    from oracle.integrate import constrain_velocities
    from paper_2603_22274_amd import gen
    shim = r'''
#include "settle.h"
extern "C" void project_many(int n, const float* x, float* v, float mO, float mH) {
  for (int i = 0; i < n; ++i) {
    const float* o = x + 9 * i; float* p = v + 9 * i;
    felis::v3 b0 = felis::mk(o[3] - o[0], o[4] - o[1], o[5] - o[2]);
    felis::v3 c0 = felis::mk(o[6] - o[0], o[7] - o[1], o[8] - o[2]);
    felis::v3 a = felis::mk(p[0], p[1], p[2]), b = felis::mk(p[3], p[4], p[5]), c = felis::mk(p[6], p[7], p[8]);
    felis::rigid_velocity(b0, c0, mO, mH, a, b, c);
    p[0] = a.x; p[1] = a.y; p[2] = a.z; p[3] = b.x; p[4] = b.y; p[5] = b.z; p[6] = c.x; p[7] = c.y; p[8] = c.z;
  }
}
'''
    s = gen.config0()
    rng = np.random.default_rng(1)
    W = s.waters[:64]
    x = np.ascontiguousarray(s.pos[W], np.float32)              # (64, 3, 3)
    v = np.ascontiguousarray(rng.normal(0, 8.0, x.shape), np.float32)
    with tempfile.TemporaryDirectory() as d:
        cpp = os.path.join(d, 'p.cpp')
        open(cpp, 'w').write(shim)
        so = os.path.join(d, 'p.so')
        subprocess.run(['g++', '-O2', '-shared', '-fPIC', '-I',
                        os.path.join(ROOT, 'paper_2603_22274_amd', 'csrc'), cpp, '-o', so], check=True)
        lib = C.CDLL(so)
        got = v.copy()
        lib.project_many(len(W), x.ctypes.data_as(C.c_void_p), got.ctypes.data_as(C.c_void_p),
                         C.c_float(s.mass[W[0, 0]]), C.c_float(s.mass[W[0, 1]]))
    wat = np.arange(3 * len(W)).reshape(-1, 3)
    mass = np.tile(s.mass[W[0]], len(W))
    ref = constrain_velocities(x.reshape(-1, 3).astype(np.float64), v.reshape(-1, 3).astype(np.float64), wat,
                               mass, np.array([1e4] * 3))
    err = np.abs(got.reshape(-1, 3) - ref).max() / np.abs(ref).max()
    assert err < 2e-6, err


def test_free_energy_assembly_on_the_host():
    """felis_delta_g, felis_segment_bounds and felis_binding_dg (host
    arithmetic, no device) against the oracle's estimator."""
    import math
    from oracle import estimator as oest
    from paper_2603_22274_amd import felis
    rng = np.random.default_rng(9)
    f = rng.normal(0, 20, 11)
    assert math.isclose(felis.delta_g(f, 310.0), oest.KB * 310.0 * (f[-1] - f[0]), rel_tol=1e-15)
    for W, n in ((42, 3), (73, 8), (12, 1), (80, 79)):
        b = felis.segment_bounds(W, n)
        segs = [list(range(int(b[s]), int(b[s + 1]) + 1)) for s in range(n)]
        assert segs == oest.segments(W, n)
    g0, k = np.array([6.0, 1.4, 1.7, 0.3, -1.0, 2.0]), np.array([10.0, 100, 100, 100, 100, 100])
    sol, cpx = [1.5, -2.25, 0.5], [3.0, 4.5]
    got = felis.binding_dg(sol, cpx, g0, k, 300.0)
    ref = oest.binding_dg(sum(sol), sum(cpx), oest.boresch_restraint_dg(g0, k, 300.0))
    assert math.isclose(got, ref, rel_tol=1e-13)
    for bad in (lambda: felis.delta_g([1.0], 300.0), lambda: felis.segment_bounds(3, 3),
                lambda: felis.binding_dg([], cpx, g0, k), lambda: felis.delta_g([0.0, np.nan], 300.0)):
        with pytest.raises(felis.FelisError):
            bad()


def test_restraint_term_matches_oracle_on_the_host():
    """felis_restraint_dg is host arithmetic: it runs without a device."""
    import math
    from oracle import estimator as oest
    from paper_2603_22274_amd import felis
    rng = np.random.default_rng(8)
    for _ in range(20):
        g0 = np.array([rng.uniform(3, 9), rng.uniform(0.3, 2.8), rng.uniform(0.3, 2.8),
                       rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-3, 3)])
        k = rng.uniform(1.0, 200.0, 6)
        T = rng.uniform(250.0, 350.0)
        assert math.isclose(felis.restraint_dg(g0, k, T), oest.boresch_restraint_dg(g0, k, T), rel_tol=1e-13)
    good_g, good_k = np.array([5.0, 1.5, 1.5, 0, 0, 0]), np.full(6, 10.0)
    for g, k, T in ((good_g, -good_k, 300.0), (np.array([0.0, 1.5, 1.5, 0, 0, 0]), good_k, 300.0),
                    (np.array([5.0, 3.2, 1.5, 0, 0, 0]), good_k, 300.0), (good_g, good_k, 0.0)):
        with pytest.raises(felis.FelisError):
            felis.restraint_dg(g, k, T)
