"""Replica exchange on the GPU against the oracle.

* The same reduced-potential matrix fed to both sides gives the same swaps
  (integer decisions: bit-exact) over many attempts of both parities, for a
  12-window and an 80-window leg.
* After swaps every kernel uses the lambda row of the state a replica holds:
  energies, forces and a short trajectory are bitwise those of a leg built
  directly with the permuted lambda rows.
* Exchanges driven by the GPU's own u_kn of the replicas' current frames
  agree with the oracle's decisions on that u.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import hrex as ohrex
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


def _many_windows(s, K):
    lam = np.zeros((K, 3))
    lam[:, 0] = np.linspace(1.0, 0.0, K)
    lam[:, 1] = np.linspace(1.0, 0.3, K)
    return dataclasses.replace(s, lambdas=lam)


@pytest.mark.parametrize('K', [12, 80])
def test_swaps_match_oracle_on_given_u(F, K):
    felis, ctx = F
    s = gen.config0() if K == 12 else _many_windows(gen.config0(), K)
    leg = felis.Leg(ctx, s, seed=3)
    assert felis.leg_states(ctx, leg).tolist() == list(range(K))
    rng = np.random.default_rng(21 + K)
    st = np.arange(K)
    total = 0
    for t in range(40):
        u = rng.normal(0.0, 1.5, (K, K + 3))            # row stride larger than K
        n = felis.hrex(ctx, leg, torch.as_tensor(u, device='cuda'), t, seed=777)
        st, acc = ohrex.attempt(u[:, :K], st, t, 777)
        got = felis.leg_states(ctx, leg)
        assert got.tolist() == st.tolist(), (t, got, st)
        assert n == len(acc), (t, n, acc)
        total += n
    pairs = sum(len(range(t & 1, K - 1, 2)) for t in range(40))
    assert 0 < total < pairs
    ctx.device_check()


def test_kernels_use_the_held_state(F):
    felis, ctx = F
    s = gen.config0()
    K = len(s.lambdas)
    rng = np.random.default_rng(4)
    pos = (s.pos[None].astype(np.float64) + rng.normal(0, 0.05, (K, s.n_atoms, 3))).astype(np.float32)
    a = felis.Leg(ctx, s, positions=pos, seed=5)
    # u independent of the state: every swap is taken
    zero = torch.zeros((K, K), dtype=torch.float64, device='cuda')
    for t in range(3):
        felis.hrex(ctx, a, zero, t, seed=1)
    st = felis.leg_states(ctx, a)
    assert sorted(st.tolist()) == list(range(K)) and st.tolist() != list(range(K))
    b = felis.Leg(ctx, s, windows=st.tolist(), positions=pos, seed=5)   # window r built at state st[r]
    for leg in (a, b):
        felis.build_nlist(ctx, [leg], force=True)
        felis.nonbonded(ctx, [leg], energy=True)
        felis.pme(ctx, [leg], energy=True)
        felis.bonded(ctx, [leg], energy=True)
    ctx.device_check()
    assert torch.equal(a.energy, b.energy)
    assert torch.equal(a.fx, b.fx) and torch.equal(a.fy, b.fy) and torch.equal(a.fz, b.fz)
    felis.step(ctx, [a], 10)
    felis.step(ctx, [b], 10)
    ctx.device_check()
    for t1, t2 in ((a.x, b.x), (a.vx, b.vx), (a.fz, b.fz)):
        assert torch.equal(t1, t2)


def test_exchange_from_gpu_ukn(F):
    felis, ctx = F
    s = gen.config0()
    K = len(s.lambdas)
    leg = felis.Leg(ctx, s, seed=9)
    felis.step(ctx, [leg], 20)
    st = np.arange(K)
    for t in range(6):
        u = felis.ukn(ctx, leg, s.lambdas, leg.x, leg.y, leg.z, BETA)      # [state][replica]
        n = felis.hrex(ctx, leg, u, t, seed=99)
        st, acc = ohrex.attempt(u.cpu().numpy(), st, t, 99)
        assert felis.leg_states(ctx, leg).tolist() == st.tolist() and n == len(acc)
        felis.step(ctx, [leg], 10)
    ctx.device_check()
