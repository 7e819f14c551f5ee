"""The plain form (FP32 pair and reciprocal forces summed with FP64 atomics,
one window per leg) against the oracle and against the default fixed-point
form: the comparator of the batched mixed-precision path must itself be a
correct integrator of the same dynamics."""
import numpy as np
import pytest
import torch

from oracle import energy as oenergy, integrate as ointeg
from oracle.ewald import PME
from paper_2603_22274_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def F():
    if not torch.cuda.is_available():
        pytest.skip('no HIP device')
    from paper_2603_22274_amd import felis
    ctx = felis.Context(0)
    yield felis, ctx
    torch.cuda.synchronize()
    ctx.close()


def _set_v(leg, v0):
    leg.vx.copy_(torch.as_tensor(v0[..., 0]))
    leg.vy.copy_(torch.as_tensor(v0[..., 1]))
    leg.vz.copy_(torch.as_tensor(v0[..., 2]))


@pytest.mark.parametrize('name,w', [('config0', 7), ('small_complex', 30)])
def test_plain_step_matches_oracle(F, name, w):
    """One-window plain leg, 10 steps with the oracle's noise stream."""
    felis, ctx = F
    s = getattr(gen, name)()
    leg = felis.Leg(ctx, s, windows=[w], seed=11, plain_fp64=True)
    felis.build_nlist(ctx, [leg], force=True)
    rng = np.random.default_rng(5)
    v0 = rng.normal(0, 2.0, (1, s.n_atoms, 3)).astype(np.float32)
    _set_v(leg, v0)
    nsteps = 10
    felis.step(ctx, [leg], nsteps, dt=0.002, temperature=300.0, gamma=0.5)
    ctx.device_check()
    got = leg.positions().cpu().numpy()[0]
    pme = PME(s.box, s.grid, s.ewald_alpha)
    x, v = s.pos.astype(np.float64), v0[0].astype(np.float64)
    force = lambda y: oenergy.window_energy(s, y, s.lambdas[w], pme=pme)[1]
    for st in range(nsteps):
        x, v = ointeg.langevin_middle_step(s, x, v, force, 0.002, 300.0, 0.5, 11, 0, st)
    err = np.max(np.abs(got - x))
    rms = float(np.sqrt(np.mean((got - x) ** 2)))
    print(name, 'window', w, 'max |dx|', err, 'rms', rms)
    assert err < 1e-4 and rms < 2e-5, (err, rms)


def test_plain_and_fixed_point_forms_agree(F):
    """Same one-window leg, same noise: the two accumulations differ only by
    rounding after 10 steps; the fixed-point force stored by the kick equals
    the FP64 sum to one fixed-point unit per term."""
    felis, ctx = F
    s = gen.small_complex()
    w = 16
    rng = np.random.default_rng(6)
    v0 = rng.normal(0, 2.0, (1, s.n_atoms, 3)).astype(np.float32)
    out = []
    for plain in (True, False):
        leg = felis.Leg(ctx, s, windows=[w], seed=13, plain_fp64=plain)
        felis.build_nlist(ctx, [leg], force=True)
        _set_v(leg, v0)
        felis.step(ctx, [leg], 10, dt=0.002, temperature=300.0, gamma=0.5)
        ctx.device_check()
        out.append((leg.positions().cpu().numpy()[0], leg.forces().cpu().numpy()[0]))
    (xp, fp), (xf, ff) = out
    assert np.max(np.abs(xp - xf)) < 5e-5, np.max(np.abs(xp - xf))
    rr = float(np.sqrt(((fp - ff) ** 2).sum() / (ff ** 2).sum()))
    assert rr < 1e-5, rr


def test_plain_form_rejects_pressure(F):
    felis, ctx = F
    s = gen.config0()
    with pytest.raises(felis.FelisError) as e:
        leg = felis.Leg(ctx, s, windows=[0], seed=1, plain_fp64=True, pressure_bar=1.01325)
        felis.step(ctx, [leg], 1, dt=0.002, temperature=300.0, gamma=0.5)
    assert e.value.code == felis.E_UNSUPPORTED
