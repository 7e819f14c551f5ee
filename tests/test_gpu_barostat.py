"""NPT on the GPU (section "Simulation protocol": Monte Carlo barostat at
1.01325 bar) against the oracle: one volume move of every window (energies
before and after, the proposal, the rigid molecule move, the decision, the
restore of rejected windows); forces and energies of windows that each sit in
their own box; u_kn of frames in their own boxes, with the P V term; a leg
with a barostat alone and batched with a fixed-box leg."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import barostat as ob, energy as oenergy, pairs as opairs, ukn as oukn
from oracle.ewald import PME
from paper_2603_22274_amd import gen

pytestmark = pytest.mark.gpu

T = 300.0
P_BAR = 1.01325
KB = 0.0019872043
BETA = 1.0 / (KB * T)


@pytest.fixture(scope='module')
def F():
    if not torch.cuda.is_available():
        pytest.skip('no HIP device')
    from paper_2603_22274_amd import felis
    ctx = felis.Context(0)
    yield felis, ctx
    torch.cuda.synchronize()
    ctx.close()


def _sys(windows):
    s = gen.config0()
    return dataclasses.replace(s, lambdas=s.lambdas[windows])


def _rel_rms(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def _energy(sysd, x, box, lam):
    """oracle total and the sum of |components| (the scale of its FP32 error)"""
    e = oenergy.window_energy(dataclasses.replace(sysd, box=np.asarray(box, np.float64)), x, lam)[0]
    return e['total'], sum(abs(v) for k, v in e.items() if k != 'total')


@pytest.mark.parametrize('name', ['config0', 'small_complex'])
def test_volume_move_matches_oracle(F, name):
    """One move of every window; the complex leg has a chain 'protein' as one
    molecule, ions, and the Boresch restraint across two molecules."""
    felis, ctx = F
    base = getattr(gen, name)()
    pick = [0, 3, 6, 11] if name == 'config0' else [0, 12, 25, 41]
    s = dataclasses.replace(base, lambdas=base.lambdas[pick])
    seed = 9
    leg = felis.Leg(ctx, s, seed=seed, pressure_bar=P_BAR, barostat_every=1000)
    felis.step(ctx, [leg], 20, 0.002, T, 5.0)
    x0 = leg.positions().cpu().numpy().astype(np.float64)
    b0 = felis.leg_boxes(ctx, leg)
    felis.barostat(ctx, leg, T, attempt=3)
    st = felis.barostat_stats(ctx, leg)
    b1 = felis.leg_boxes(ctx, leg)
    x1 = leg.positions().cpu().numpy().astype(np.float64)
    ctx.device_check()
    kT = KB * T
    decided = 0
    for w in range(leg.n_windows):
        u1, u2 = ob.draws(seed, w, 3)
        dv = 0.01 * float(np.prod(s.box))
        r = ob.attempt(s, x0[w], b0[w], s.lambdas[w], dv, u1, u2, P_BAR, T)
        U0, U1, work, v_old, v_new, scale, acc = st[w, :7]
        e0, m0 = _energy(s, x0[w], b0[w], s.lambdas[w])
        # U after the move at the trial positions as the GPU holds them (FP32)
        e1, m1 = _energy(s, r['x_trial'].astype(np.float32).astype(np.float64), r['box_trial'], s.lambdas[w])
        assert abs(U0 - e0) <= 1e-6 * m0, (w, U0, e0, m0)
        assert abs(U1 - e1) <= 1e-6 * m1, (w, U1, e1, m1)
        assert abs(v_old - np.prod(b0[w])) <= 1e-9 * v_old
        assert abs(scale - r['s']) <= 1e-12 and st[w, 8] == 1
        w_ref = float(ob.work(e1 - e0, v_old, v_new, r['n_mol'], P_BAR, T))
        assert abs(work - w_ref) <= 1e-6 * (m0 + m1), (w, work, w_ref)
        assert abs(w_ref - r['w']) <= 1e-6 * (m0 + m1) + 0.01, (w, w_ref, r['w'])
        # the decision is unique unless w lies within the energy error of the threshold
        if abs(r['w'] + kT * np.log(u2)) > 0.02 + 1e-6 * (m0 + m1):
            assert bool(acc) == r['accepted'], (w, work, r['w'], u2)
            decided += 1
        if acc:
            assert np.abs(b1[w] - r['box_trial']).max() <= 1e-9
            assert np.abs(x1[w] - r['x_trial']).max() <= 1e-4
        else:
            assert np.array_equal(b1[w], b0[w]) and np.array_equal(x1[w], x0[w])
    assert decided >= 2


def test_npt_run_moves_each_window_on_its_own(F):
    felis, ctx = F
    s = gen.config0()
    leg = felis.Leg(ctx, s, seed=4, pressure_bar=P_BAR, barostat_every=5)
    felis.step(ctx, [leg], 300, 0.002, T, 5.0)
    st = felis.barostat_stats(ctx, leg)
    boxes = felis.leg_boxes(ctx, leg)
    ctx.device_check()
    v0 = float(np.prod(s.box))
    vol = np.prod(boxes, axis=1)
    assert np.all(st[:, 8] == 300 // 5 - 1)                       # steps 5, 10, ..., 295
    rate = st[:, 9].sum() / st[:, 8].sum()
    assert 0.05 < rate < 0.95, rate
    # the lattice start is far from equilibrium (its configurational pressure
    # is ~3e5 bar: overlapping randomly oriented waters), so the windows
    # expand on average, each by a bounded amount in 59 moves
    assert np.all(vol / v0 > 0.8) and np.all(vol / v0 < 1.5) and np.mean(vol / v0) > 1.0, vol / v0
    assert len(np.unique(np.round(vol, 6))) > leg.n_windows // 2   # independent moves
    assert np.allclose(boxes[:, 0], boxes[:, 1]) and np.allclose(boxes[:, 0], boxes[:, 2])   # isotropic
    e = leg.energy.cpu().numpy()
    assert np.all(np.isfinite(e))


def test_forces_and_energies_in_each_windows_box(F):
    felis, ctx = F
    s = _sys([0, 5, 9, 11])
    leg = felis.Leg(ctx, s, seed=12, pressure_bar=P_BAR, barostat_every=1000)
    felis.step(ctx, [leg], 10, 0.002, T, 5.0)
    # three large forced moves so that the windows sit in visibly different boxes
    for t in range(3):
        felis.barostat(ctx, leg, T, attempt=100 + t)
    boxes = felis.leg_boxes(ctx, leg)
    felis.nonbonded(ctx, [leg])
    f_real = leg.forces().cpu().numpy()
    felis.pme(ctx, [leg])
    f_all = leg.forces().cpu().numpy()
    E = leg.energy.cpu().numpy()
    x = leg.positions().cpu().numpy().astype(np.float64)
    ctx.device_check()
    for w in range(leg.n_windows):
        sw = dataclasses.replace(s, box=boxes[w])
        lam = s.lambdas[w]
        ec, elj, fr = opairs.real_space(x[w], sw, lam)
        ex, fx = opairs.exclusion_correction(x[w], sw, lam)
        es = opairs.self_and_background(sw, lam)
        er, frec = PME(sw.box, sw.grid, sw.ewald_alpha).energy_forces(x[w], opairs.scaled_charges(sw, lam[0]))
        assert abs(E[w, 2] - ex) <= 1e-6 * abs(ex), (w, E[w, 2], ex)
        assert abs(E[w, 3] - es) <= 1e-6 * abs(es), (w, E[w, 3], es)
        assert abs(E[w, 4] - er) <= 1e-6 * abs(er) + 1e-4, (w, E[w, 4], er)
        assert _rel_rms(f_real[w], fr + fx) <= 1e-5, w
        assert _rel_rms(f_all[w], fr + fx + frec) <= 1e-5, w


def test_ukn_of_frames_in_their_own_boxes(F):
    felis, ctx = F
    s = gen.config0()
    leg = felis.Leg(ctx, s, seed=21, pressure_bar=P_BAR, barostat_every=5)
    felis.step(ctx, [leg], 100, 0.002, T, 5.0)
    boxes = felis.leg_boxes(ctx, leg)
    frames = leg.positions().cpu().numpy()[[0, 4, 8, 11]]
    fb = boxes[[0, 4, 8, 11]]
    xt, yt, zt = (torch.as_tensor(np.ascontiguousarray(frames[..., d])).cuda() for d in range(3))
    u = felis.ukn(ctx, leg, s.lambdas, xt, yt, zt, BETA, boxes=torch.as_tensor(fb).cuda()).cpu().numpy()
    ctx.device_check()
    for f in range(len(frames)):
        ref = oukn.ukn(dataclasses.replace(s, box=fb[f]), frames[f:f + 1].astype(np.float64), s.lambdas, BETA)[:, 0]
        du = (u[:, f] - u[0, f]) - (ref - ref[0])
        assert np.max(np.abs(du)) <= 1e-6 * np.abs(ref - ref[0]).max() + 2e-4, (f, np.abs(du).max())
    # the P V term: the same frames and boxes through a fixed-box leg differ by beta P V only
    nvt = felis.Leg(ctx, s, seed=21)
    u0 = felis.ukn(ctx, nvt, s.lambdas, xt, yt, zt, BETA, boxes=torch.as_tensor(fb).cuda()).cpu().numpy()
    pv = BETA * P_BAR * ob.BAR * np.prod(fb, axis=1)
    assert np.abs((u - u0) - pv[None, :]).max() <= 1e-9 * np.abs(u).max() + 1e-9


def test_barostat_leg_alone_equals_batched_with_fixed_box_leg(F):
    felis, ctx = F
    s = _sys([0, 4, 8, 11])
    c = dataclasses.replace(gen.config0(seed=77), lambdas=gen.config0().lambdas[[2, 7]])

    def run(batch):
        legs = []
        if 'npt' in batch:
            legs.append(felis.Leg(ctx, s, seed=31, pressure_bar=P_BAR, barostat_every=10))
        if 'nvt' in batch:
            legs.append(felis.Leg(ctx, c, seed=32))
        felis.step(ctx, legs, 60, 0.002, T, 5.0)
        ctx.device_check()
        return legs

    a = run(['npt'])[0]
    b = run(['nvt'])[0]
    mixed = run(['npt', 'nvt'])
    assert torch.equal(a.positions(), mixed[0].positions())
    assert np.array_equal(felis.leg_boxes(ctx, a), felis.leg_boxes(ctx, mixed[0]))
    assert np.array_equal(felis.barostat_stats(ctx, a), felis.barostat_stats(ctx, mixed[0]))
    assert torch.equal(b.positions(), mixed[1].positions())
