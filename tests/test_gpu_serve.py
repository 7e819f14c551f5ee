"""Served form on the GPU.  A leg's trajectory, u_kn and Delta G are bitwise
the same alone and in any mixed batch (other legs ahead, behind, joining
mid-run, in any order); a leg that latches a list-capacity error is named in
the error, retried with a larger list or evicted, and the legs beside it are
unaffected.  The capacity failure is forced from the host with a tiny list
capacity: the list builder clamps at capacity, so every kernel exits normally.
"""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2603_22274_amd import gen

pytestmark = pytest.mark.gpu

KB = 0.0019872043
BETA = 1.0 / (KB * 300.0)


@pytest.fixture(scope='module')
def F():
    if not torch.cuda.is_available():
        pytest.skip('no HIP device')
    from paper_2603_22274_amd import felis
    ctx = felis.Context(0)
    yield felis, ctx
    torch.cuda.synchronize()
    ctx.close()


@pytest.fixture(scope='module')
def legs():
    a = gen.sized_leg(2400, 12, 5)
    # closely spaced electrostatic windows so that MBAR converges on short runs
    lam = np.zeros((6, 3))
    lam[:, 0] = np.linspace(1.0, 0.95, 6)
    lam[:, 1] = 1.0
    lam[:, 2] = 1.0
    a = dataclasses.replace(a, lambdas=lam)
    return a, gen.sized_leg(3300, 20, 6), gen.sized_leg(4000, 42, 7)


def test_step_repeatable_from_scratch(F, legs):
    """A leg stepped from its initial state gives the same bits whatever ran
    on the device before (clusters with padding slots included: 3298 atoms)."""
    felis, ctx = F
    _, B, C = legs

    def run(sysd, steps):
        leg = felis.Leg(ctx, sysd, seed=22)
        felis.step(ctx, [leg], steps)
        ctx.device_check()
        return _state(leg)

    first = run(B, 3)
    run(C, 5)                                   # other kernels leave other LDS and cache contents
    run(gen.config1(), 2)
    again = run(B, 3)
    assert all(torch.equal(p, q) for p, q in zip(first, again))


def _state(leg):
    return [t.clone() for t in (leg.x, leg.y, leg.z, leg.vx, leg.vy, leg.vz, leg.fx, leg.fy, leg.fz)]


def test_trajectory_alone_equals_mixed(F, legs):
    felis, ctx = F
    A, B, C = legs

    def run(mix):
        la = felis.Leg(ctx, A, seed=11)
        if not mix:
            felis.step(ctx, [la], 20)
        else:
            lb = felis.Leg(ctx, B, seed=12)
            felis.step(ctx, [lb], 6)                 # another leg already in flight
            felis.step(ctx, [la, lb], 10)
            lc = felis.Leg(ctx, C, seed=13)          # a third joins, order changes
            felis.step(ctx, [lc, lb, la], 10)
        ctx.device_check()
        u = felis.ukn(ctx, la, la.lambdas, la.x, la.y, la.z, BETA)
        ctx.device_check()
        return _state(la), u.clone(), la.s.step

    sa, ua, na = run(False)
    sb, ub, nb = run(True)
    assert na == nb == 20
    for x, y in zip(sa, sb):
        assert torch.equal(x, y)
    assert torch.equal(ua, ub)


def test_capacity_error_names_the_leg(F, legs):
    felis, ctx = F
    A, B, _ = legs
    la = felis.Leg(ctx, A, seed=11)
    lb = felis.Leg(ctx, B, seed=12, list_cap=8)
    felis.step(ctx, [la, lb], 1)
    with pytest.raises(felis.FelisError) as ei:
        ctx.device_check()
    e = ei.value
    assert e.code == felis.E_CAPACITY and e.leg == 1 and 0 <= e.window < B.n_windows
    assert e.needed_cap > 8
    ctx.device_check()                               # the error word was cleared


def _serve(ctx, reqs, **kw):
    from paper_2603_22274_amd.serve import FelisEngine, Server
    eng = FelisEngine(ctx, mbar_max_iter=20000)
    srv = Server(eng, hbm_budget=16 << 30, epoch_steps=10, **kw)
    return srv.serve(reqs)


def _req(rid, sysd, t, seed, cap=0, exchange_every=0, pressure_bar=0.0):
    from paper_2603_22274_amd.serve import Request
    return Request(rid, t, sysd, n_steps=40, sample_every=10, seed=seed, list_cap=cap, exchange_every=exchange_every,
                   pressure_bar=pressure_bar, barostat_every=10)


def test_served_dg_alone_equals_mixed(F, legs):
    felis, ctx = F
    A, B, C = legs
    alone, _ = _serve(ctx, [_req(0, A, 0.0, 21)])
    mixed, stats = _serve(ctx, [_req(1, B, 0.0, 22), _req(0, A, 0.0, 21), _req(2, C, 0.02, 23)])
    a = alone[0]
    m = next(r for r in mixed if r.rid == 0)
    assert a.status == 'ok' and m.status == 'ok'
    assert a.dG is not None and np.isfinite(a.dG)
    assert a.dG == m.dG and a.mbar_iters == m.mbar_iters
    assert stats['completed'] == 3
    assert 0 < stats['latency_p50_s'] <= stats['latency_p99_s']


def test_served_replica_exchange_alone_equals_mixed(F, legs):
    """Replica exchange every two samples: the leg's swaps, and so its dG,
    depend only on its own u_kn and seed, whatever runs beside it."""
    felis, ctx = F
    A, B, C = legs
    alone, _ = _serve(ctx, [_req(0, A, 0.0, 21, exchange_every=20)])
    mixed, _ = _serve(ctx, [_req(1, B, 0.0, 22, exchange_every=20), _req(0, A, 0.0, 21, exchange_every=20),
                            _req(2, C, 0.02, 23)])
    a = alone[0]
    m = next(r for r in mixed if r.rid == 0)
    assert a.status == 'ok' and m.status == 'ok' and a.dG is not None
    assert a.dG == m.dG and a.mbar_iters == m.mbar_iters


def test_served_npt_leg_alone_equals_mixed(F, legs):
    """A leg with a barostat (a volume move of every window every 10 steps, u_kn
    of each sample in its windows' boxes) gives the same dG alone and served
    beside fixed-box legs."""
    felis, ctx = F
    A, B, C = legs
    alone, _ = _serve(ctx, [_req(0, A, 0.0, 21, pressure_bar=1.01325)])
    mixed, _ = _serve(ctx, [_req(1, B, 0.0, 22), _req(0, A, 0.0, 21, pressure_bar=1.01325), _req(2, C, 0.02, 23)])
    a = alone[0]
    m = next(r for r in mixed if r.rid == 0)
    assert a.status == 'ok' and m.status == 'ok' and a.dG is not None and np.isfinite(a.dG)
    assert a.dG == m.dG and a.mbar_iters == m.mbar_iters


def test_capacity_retry_and_eviction_isolated(F, legs):
    felis, ctx = F
    A, B, _ = legs
    ref_a, _ = _serve(ctx, [_req(0, A, 0.0, 21)])
    ref_b, _ = _serve(ctx, [_req(1, B, 0.0, 22)])
    # retried with the capacity it asked for: same result as a large list from the start
    out, stats = _serve(ctx, [_req(0, A, 0.0, 21), _req(1, B, 0.0, 22, cap=8)])
    assert out[1].retries == 1 and out[1].status == ref_b[0].status
    assert out[1].dG == ref_b[0].dG
    assert out[0].dG == ref_a[0].dG
    # no retries left: evicted, the other leg untouched
    out, stats = _serve(ctx, [_req(0, A, 0.0, 21), _req(1, B, 0.0, 22, cap=8)], max_retries=0)
    assert out[1].status.startswith('evicted') and 'capacity' in out[1].status
    assert out[0].status == 'ok' and out[0].dG == ref_a[0].dG


def test_served_dg_matches_oracle_on_its_frames(F, legs):
    """A served leg's Delta G (GPU u_kn at sample time + GPU MBAR at the end,
    inside the serving loop, beside another leg) against the oracle's u_kn and
    MBAR evaluated on the frames that leg produced."""
    felis, ctx = F
    from oracle import mbar as ombar, ukn as oukn
    from paper_2603_22274_amd import serve
    A, B, _ = legs
    reqs = [serve.Request(0, 0.0, A, 300, 50, seed=31), serve.Request(1, 0.0, B, 300, 50, seed=32)]
    eng = serve.FelisEngine(ctx, keep_frames=True, mbar_tol=1e-12)
    out, _ = serve.Server(eng, hbm_budget=16 << 30, epoch_steps=50).serve(reqs)
    res = out[0]
    assert res.status == 'ok', res.status
    W = A.n_windows
    frames = torch.cat(eng.frames[0], 0).cpu().numpy().astype(np.float64)     # sample-major, replica order
    n_samples = len(eng.frames[0])
    assert frames.shape == (n_samples * W, A.n_atoms, 3)
    ref_u = oukn.ukn(A, frames, A.lambdas, BETA)
    f_ref, _ = ombar.mbar(ref_u, np.full(W, n_samples), tol=1e-12, max_iter=2000000)
    dg_ref = (f_ref[-1] - f_ref[0]) / BETA
    print('served dG', res.dG, 'oracle', dg_ref)
    assert abs(res.dG - dg_ref) <= 0.01, (res.dG, dg_ref)
