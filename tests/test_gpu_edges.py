"""Edge cases of the GPU path against the oracle: a ragged leg (67 atoms: not
a multiple of the 8-atom cluster or the 64-atom gather block; a 15^3 grid:
not a multiple of the spreading bricks or the FFT line groups) in every
window and over 10 MD steps; u_kn at a single state, over zero frames, and a
zero-step felis_step; the largest PME grid the library takes (128^3) and
the grids it rejects."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import energy as oenergy, integrate as ointeg, ukn as oukn
from oracle.ewald import PME
from oracle import pairs as opairs
from paper_2603_22274_amd import gen

pytestmark = pytest.mark.gpu
KB = 0.0019872043


@pytest.fixture(scope='module')
def F():
    if not torch.cuda.is_available():
        pytest.skip('no HIP device')
    from paper_2603_22274_amd import felis
    ctx = felis.Context(0)
    yield felis, ctx
    torch.cuda.synchronize()
    ctx.close()


def rel_rms(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def _ragged():
    return gen.solvent_leg(config=77, n_waters=21, lattice_n=4, box_edge=13.5, n_lig=4, r_cut=6.0,
                           grid=(15, 15, 15), skin=0.25, sched='cfg0')


def test_ragged_leg_every_window(F):
    felis, ctx = F
    s = _ragged()
    assert s.n_atoms == 67 and s.n_atoms % 8 and s.grid[0] % 16
    leg = felis.Leg(ctx, s, seed=3)
    felis.forces_and_energy(ctx, [leg])
    ctx.device_check()
    f = leg.forces().cpu().numpy()
    E = leg.energy.cpu().numpy()
    pme = PME(s.box, s.grid, s.ewald_alpha)
    for w in range(s.n_windows):
        e, fo = oenergy.window_energy(s, s.pos.astype(np.float64), s.lambdas[w], pme=pme)
        assert rel_rms(f[w], fo) <= 1e-5, (w, rel_rms(f[w], fo))
        # every component within 1e-6 of its own magnitude; this 67-atom leg's
        # total (about -10 kcal/mol) is a near-cancellation of components two
        # orders of magnitude larger, so it is held to 1e-6 of the largest one
        comp = {c: (E[w, i], e[c]) for i, c in enumerate(oenergy.COMPONENTS[:-1])}
        print(w, {c: float(a - b) for c, (a, b) in comp.items()}, 'total', e['total'])
        for c, (a, b) in comp.items():
            assert abs(a - b) <= 1e-6 * max(abs(b), 1e-3), (w, c, a, b)
        big = max(abs(b) for _, b in comp.values())
        assert abs(E[w, 7] - e['total']) <= 1e-6 * big, (w, E[w, 7], e['total'], big)


def test_ragged_leg_steps(F):
    felis, ctx = F
    s = _ragged()
    w = 6
    leg = felis.Leg(ctx, s, windows=[w], seed=9)
    felis.build_nlist(ctx, [leg], force=True)
    rng = np.random.default_rng(2)
    v0 = rng.normal(0, 2.0, (1, s.n_atoms, 3)).astype(np.float32)
    leg.vx.copy_(torch.as_tensor(v0[..., 0])); leg.vy.copy_(torch.as_tensor(v0[..., 1]))
    leg.vz.copy_(torch.as_tensor(v0[..., 2]))
    felis.step(ctx, [leg], 10, 0.002, 300.0, 0.5)
    ctx.device_check()
    got = leg.positions().cpu().numpy()[0]
    pme = PME(s.box, s.grid, s.ewald_alpha)
    x, v = s.pos.astype(np.float64), v0[0].astype(np.float64)
    force = lambda y: oenergy.window_energy(s, y, s.lambdas[w], pme=pme)[1]
    for st in range(10):
        x, v = ointeg.langevin_middle_step(s, x, v, force, 0.002, 300.0, 0.5, 9, 0, st)
    assert np.max(np.abs(got - x)) < 1e-4 and np.sqrt(np.mean((got - x) ** 2)) < 2e-5


def test_single_state_empty_frames_zero_steps(F):
    felis, ctx = F
    s = _ragged()
    leg = felis.Leg(ctx, s, windows=[0, 5], seed=4)
    felis.build_nlist(ctx, [leg], force=True)
    beta = 1.0 / (KB * 300.0)
    rng = np.random.default_rng(5)
    frames = (s.pos[None].astype(np.float64) + rng.normal(0, 0.05, (3, s.n_atoms, 3))).astype(np.float32)
    xt, yt, zt = (torch.as_tensor(np.ascontiguousarray(frames[..., d])).cuda() for d in range(3))
    lam1 = s.lambdas[[7]]
    u = felis.ukn(ctx, leg, lam1, xt, yt, zt, beta).cpu().numpy()
    ref = oukn.ukn(s, frames.astype(np.float64), lam1, beta)
    assert u.shape == (1, 3)
    assert np.max(np.abs(u - ref)) <= 1e-6 * np.abs(ref).max() + 2e-4
    empty = torch.empty((0, s.n_atoms), dtype=torch.float32, device='cuda')
    u0 = felis.ukn(ctx, leg, s.lambdas, empty, empty, empty, beta)
    assert tuple(u0.shape) == (s.n_windows, 0)
    before = leg.positions().clone()
    felis.step(ctx, [leg], 0, 0.002, 300.0, 0.5)
    ctx.device_check()
    assert torch.equal(before, leg.positions())


def test_largest_grid_and_rejected_grids(F):
    felis, ctx = F
    s = dataclasses.replace(gen.config0(), grid=(128, 128, 128))
    leg = felis.Leg(ctx, s, windows=[0, 3], seed=1)
    felis.build_nlist(ctx, [leg], force=True)
    leg.fx.zero_(); leg.fy.zero_(); leg.fz.zero_()
    felis.pme(ctx, [leg])
    ctx.device_check()
    f = leg.forces().cpu().numpy()
    E = leg.energy.cpu().numpy()
    pme = PME(s.box, s.grid, s.ewald_alpha)
    for k, w in enumerate((0, 3)):
        er, fr = pme.energy_forces(s.pos.astype(np.float64), opairs.scaled_charges(s, s.lambdas[w][0]))
        assert rel_rms(f[k], fr) <= 1e-5, (w, rel_rms(f[k], fr))
        assert abs(E[k, 4] - er) <= 1e-6 * abs(er), (w, E[k, 4], er)
    for bad in ((130, 130, 130), (135, 135, 135), (14, 20, 20)):
        with pytest.raises(felis.FelisError) as e:
            felis.Leg(ctx, dataclasses.replace(gen.config0(), grid=bad), windows=[0], seed=1)
        assert e.value.code == felis.E_UNSUPPORTED, bad
