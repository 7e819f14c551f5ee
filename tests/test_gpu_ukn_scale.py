"""u_kn of the ~70k-atom complex leg at all 42 states over a seeded subset of
210 frames (30 from each of the 7 electrostatic windows 16..22), element by
element against the oracle, and the segment's Delta G from GPU MBAR over the
GPU u_kn against oracle MBAR over the oracle u_kn (section "Simulation
protocol": MBAR per segment of neighbouring windows)."""
import multiprocessing as mp
import os

import numpy as np
import pytest
import torch

from oracle import mbar as ombar
from paper_2603_22274_amd import gen

pytestmark = pytest.mark.gpu

KB = 0.0019872043
_W = {}


def _init(sysd):
    from threadpoolctl import threadpool_limits

    from oracle.ewald import PME
    _W['limit'] = threadpool_limits(limits=1)
    _W['s'] = sysd
    _W['pme'] = PME(sysd.box, sysd.grid, sysd.ewald_alpha)


def _frame(args):
    from oracle import ukn as oukn
    pos, beta = args
    return oukn.ukn_frame(_W['s'], pos.astype(np.float64), _W['s'].lambdas, beta, _W['pme'])


@pytest.fixture(scope='module')
def F():
    if not torch.cuda.is_available():
        pytest.skip('no HIP device')
    from paper_2603_22274_amd import felis
    ctx = felis.Context(0)
    yield felis, ctx
    torch.cuda.synchronize()
    ctx.close()


def test_ukn_subset_and_segment_ddg(F):
    felis, ctx = F
    s = gen.config2()
    seg = list(range(16, 23))
    per = 30
    rng = np.random.default_rng(2603)
    frames = (s.pos[None].astype(np.float64) + rng.normal(0, 0.05, (len(seg) * per, s.n_atoms, 3))).astype(np.float32)
    states = np.repeat(np.array(seg), per)
    beta = 1.0 / (KB * 300.0)
    leg = felis.Leg(ctx, s, seed=3)
    felis.build_nlist(ctx, [leg], force=True)
    xt, yt, zt = (torch.as_tensor(np.ascontiguousarray(frames[..., d])).cuda() for d in range(3))
    u = felis.ukn(ctx, leg, s.lambdas, xt, yt, zt, beta)
    ctx.device_check()
    ug = u.cpu().numpy()
    nproc = max(1, min(16, (os.cpu_count() or 1) - 1))
    with mp.get_context('spawn').Pool(nproc, initializer=_init, initargs=(s,)) as p:
        ref = np.stack(p.map(_frame, [(f, beta) for f in frames], chunksize=1), 1)
    assert ref.shape == ug.shape == (42, len(frames))
    du = (ug - ug[0]) - (ref - ref[0])
    scale = np.abs(ref - ref[0]).max()
    print('max |du|', np.abs(du).max(), 'scale', scale, 'max |u - ref|', np.abs(ug - ref).max())
    assert np.max(np.abs(du)) <= 1e-6 * scale + 2e-4
    assert np.max(np.abs(ug - ref)) <= 1e-6 * np.abs(ref).max() + 2e-4
    N_k = np.full(len(seg), per)
    f_g, _ = felis.mbar(ctx, torch.as_tensor(np.ascontiguousarray(ug[seg])).cuda(), N_k, tol=1e-12, max_iter=20000)
    f_o, _ = ombar.mbar(ref[seg], N_k, tol=1e-12, max_iter=2000000)
    dg_g = felis.delta_g(f_g, 300.0)
    dg_o = float((f_o[-1] - f_o[0]) / beta)
    print('segment dG gpu', dg_g, 'oracle', dg_o)
    assert abs(dg_g - dg_o) <= 0.01
