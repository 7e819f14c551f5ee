"""The paper's production schedules (appendix B: 29 charge, 45 vdW and 8
restraint factors -> 73 solvent and 80 complex windows) through the same
kernels: per-window energies and forces of sampled windows, u_kn at every
state, MD steps and a replica-exchange attempt, against the oracle."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import pairs as opairs, ukn as oukn
from oracle.ewald import PME
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


def _rel_rms(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def _sum_abs_coulomb(s, pos, lam):
    """sum over pairs within r_c of |E_coul|: the normaliser of a cancelling sum"""
    x = np.asarray(pos, np.float64)
    p = opairs.neighbor_pairs(pos, s.box, s, s.r_cut)
    _, _, ec, _, _ = opairs._pair_block(x, s.box, s, lam, p[:, 0], p[:, 1])
    return np.abs(ec).sum()


def test_solvent_73_windows(F):
    felis, ctx = F
    s = dataclasses.replace(gen.config0(), lambdas=gen.schedule('paper_solvent'))
    assert s.n_windows == 73
    leg = felis.Leg(ctx, s, seed=5)
    felis.build_nlist(ctx, [leg], force=True)
    felis.nonbonded(ctx, [leg])
    f_real = leg.forces().cpu().numpy()
    felis.pme(ctx, [leg])
    f_all = leg.forces().cpu().numpy()
    E = leg.energy.cpu().numpy()
    ctx.device_check()
    pme = PME(s.box, s.grid, s.ewald_alpha)
    x = s.pos.astype(np.float64)
    for w in (0, 14, 28, 29, 50, 72):
        lam = s.lambdas[w]
        ec, elj, fr = opairs.real_space(x, s, lam)
        ex, fx = opairs.exclusion_correction(x, s, lam)
        er, frec = pme.energy_forces(x, opairs.scaled_charges(s, lam[0]))
        assert abs(E[w, 0] - ec) <= 1e-6 * max(abs(ec), _sum_abs_coulomb(s, s.pos, lam)), (w, E[w, 0], ec)
        assert abs(E[w, 2] - ex) <= 1e-6 * abs(ex), (w, E[w, 2], ex)
        assert abs(E[w, 4] - er) <= 1e-6 * abs(er) + 1e-4, (w, E[w, 4], er)
        assert _rel_rms(f_real[w], fr + fx) <= 1e-5 and _rel_rms(f_all[w], fr + fx + frec) <= 1e-5, w
    # u_kn of four frames at all 73 states
    rng = np.random.default_rng(2)
    frames = (s.pos[None].astype(np.float64) + rng.normal(0, 0.05, (4, s.n_atoms, 3))).astype(np.float32)
    xt, yt, zt = (torch.as_tensor(frames[..., d]).cuda() for d in range(3))
    u = felis.ukn(ctx, leg, s.lambdas, xt, yt, zt, BETA).cpu().numpy()
    ref = oukn.ukn(s, frames.astype(np.float64), s.lambdas, BETA)
    du = (u - u[0]) - (ref - ref[0])
    assert np.max(np.abs(du)) <= 1e-6 * np.abs(ref - ref[0]).max() + 2e-4


def test_complex_80_windows(F):
    felis, ctx = F
    s = dataclasses.replace(gen.small_complex(), lambdas=gen.schedule('paper_complex'))
    assert s.n_windows == 80
    leg = felis.Leg(ctx, s, seed=6)
    rng = np.random.default_rng(3)
    frames = (s.pos[None].astype(np.float64) + rng.normal(0, 0.04, (2, s.n_atoms, 3))).astype(np.float32)
    xt, yt, zt = (torch.as_tensor(frames[..., d]).cuda() for d in range(3))
    u = felis.ukn(ctx, leg, s.lambdas, xt, yt, zt, BETA).cpu().numpy()
    ctx.device_check()
    ref = oukn.ukn(s, frames.astype(np.float64), s.lambdas, BETA)
    du = (u - u[0]) - (ref - ref[0])
    assert np.max(np.abs(du)) <= 1e-6 * np.abs(ref - ref[0]).max() + 2e-4
    # the whole path at 80 windows: steps, sample, one exchange attempt
    felis.step(ctx, [leg], 10, 0.002, 300.0, 5.0)
    uu = felis.ukn(ctx, leg, s.lambdas, leg.x, leg.y, leg.z, BETA)
    n = felis.hrex(ctx, leg, uu, 0, seed=11)
    ctx.device_check()
    st = felis.leg_states(ctx, leg)
    assert sorted(st.tolist()) == list(range(80)) and 0 <= n <= 40
