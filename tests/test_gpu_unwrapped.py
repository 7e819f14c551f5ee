"""Positions far outside the periodic box: the solvent leg (7,540 atoms,
42 A box, r_c 10 A, so some of its clusters lie r_c inside every face and
take no periodic image in the pair kernel) with every atom moved by whole box
lengths (+3 L, -2 L, +5 L; the shifted FP32 coordinates are what both sides
read).  Real-space, reciprocal and total forces match the oracle to 1e-5
relative RMS and every energy component (FP64 form, from the raw unwrapped
coordinates) to 1e-6 of its magnitude, in two windows."""
import numpy as np
import pytest
import torch

from oracle import pairs as opairs
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


def _rel_rms(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def test_positions_whole_boxes_away(F):
    felis, ctx = F
    s = gen.config1()
    windows = [0, 19]
    W = len(windows)
    base = np.repeat(s.pos[None].astype(np.float32), W, axis=0)
    moved = (base.astype(np.float64) + s.box * np.array([3.0, -2.0, 5.0])).astype(np.float32)
    out = {}
    for tag, pos in (('base', base), ('moved', moved)):
        leg = felis.Leg(ctx, s, windows=windows, positions=pos, seed=7)
        felis.build_nlist(ctx, [leg], force=True)
        felis.nonbonded(ctx, [leg])
        f_real = leg.forces().cpu().numpy()
        felis.pme(ctx, [leg])
        f_all = leg.forces().cpu().numpy()
        ctx.device_check()
        out[tag] = (f_real, f_all, leg.energy.cpu().numpy().copy())
    f_real, f_all, E = out['moved']
    pme = PME(s.box, s.grid, s.ewald_alpha)
    x = moved[0].astype(np.float64)
    for k, w in enumerate(windows):
        lam = s.lambdas[w]
        ec, elj, fr = opairs.real_space(x, s, lam)
        ex, fx = opairs.exclusion_correction(x, s, lam)
        es = opairs.self_and_background(s, lam)
        er, frec = pme.energy_forces(x, opairs.scaled_charges(s, lam[0]))
        for name, got, ref in (('coul', E[k, 0], ec), ('lj', E[k, 1], elj), ('excl', E[k, 2], ex),
                               ('self', E[k, 3], es), ('recip', E[k, 4], er)):
            assert abs(got - ref) <= 1e-6 * abs(ref), (w, name, got, ref)
        assert _rel_rms(f_real[k], fr + fx) <= 1e-5, (w, 'real', _rel_rms(f_real[k], fr + fx))
        assert _rel_rms(f_all[k] - f_real[k], frec) <= 1e-5, (w, 'recip', _rel_rms(f_all[k] - f_real[k], frec))
        assert _rel_rms(f_all[k], fr + fx + frec) <= 1e-5, (w, 'total')
        # for information: the unshifted coordinates differ from the shifted
        # ones by the FP32 rounding of the shift (up to half an ulp of 5 L =
        # 210 A, 7.6e-6 A), which moves the forces by ~1e-5 of their RMS
        print('window', w, 'moved vs unshifted forces rel-RMS', _rel_rms(f_all[k], out['base'][1][k]))
