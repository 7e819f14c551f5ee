"""Pins of the replica-exchange oracle against what the mathematics fixes:
the stationary distribution of the state permutation (exact enumeration for
three replicas), the Metropolis acceptance rate at a known energy change,
and the always / never accepting limits."""
import itertools
import math

import numpy as np

from oracle import hrex


def _stationary(u):
    """Exact invariant distribution over permutations: pi(p) ~ exp(-sum_r u[p[r]][r])."""
    K = u.shape[0]
    perms = list(itertools.permutations(range(K)))
    w = np.array([math.exp(-sum(u[p[r], r] for r in range(K))) for p in perms])
    return perms, w / w.sum()


def test_chain_samples_the_joint_distribution():
    rng = np.random.default_rng(7)
    u = rng.normal(0.0, 1.0, (3, 3))
    perms, pi = _stationary(u)
    index = {p: k for k, p in enumerate(perms)}
    counts = np.zeros(len(perms))
    st = np.arange(3)
    n = 60000
    for t in range(n):
        st, _ = hrex.attempt(u, st, t, seed=12345)
        counts[index[tuple(int(v) for v in st)]] += 1
    freq = counts / n
    assert np.max(np.abs(freq - pi)) < 0.015, (freq, pi)


def test_acceptance_rate_matches_metropolis():
    # two states: the swap raises the reduced potential by ln 2 -> accepted half the time
    d = math.log(2.0)
    u = np.array([[0.0, d], [0.0, 0.0]])
    n, acc = 20000, 0
    for k in range(n):
        st, a = hrex.attempt(u, [0, 1], 2 * k, seed=99)     # even attempts try the pair (0, 1)
        acc += len(a)
        assert sorted(st.tolist()) == [0, 1]
    rate = acc / n
    assert abs(rate - 0.5) < 4 * math.sqrt(0.25 / n), rate


def test_equal_hamiltonians_always_swap():
    # u independent of the state: every swap leaves the total unchanged and is taken
    K = 5
    u = np.tile(np.linspace(-3.0, 2.0, K), (K, 1))
    st, a = hrex.attempt(u, np.arange(K), 0, seed=1)
    assert st.tolist() == [1, 0, 3, 2, 4] and a == [0, 2]
    st, a = hrex.attempt(u, st, 1, seed=1)
    assert st.tolist() == [2, 0, 4, 1, 3] and a == [1, 3]


def test_prohibitive_swaps_never_taken():
    K = 6
    k = np.arange(K)
    u = 1.0e6 * np.abs(k[:, None] - k[None, :]).astype(np.float64)
    st = np.arange(K)
    for t in range(50):
        st, a = hrex.attempt(u, st, t, seed=3)
        assert a == [] and st.tolist() == list(range(K))


def test_uniforms_are_distinct_and_in_range():
    u0 = hrex.uniforms(5, 0, np.arange(40))
    u1 = hrex.uniforms(5, 1, np.arange(40))
    u2 = hrex.uniforms(6, 0, np.arange(40))
    for v in (u0, u1, u2):
        assert np.all(v >= 0.0) and np.all(v < 1.0)
    assert len(set(np.concatenate([u0, u1, u2]).tolist())) == 120
    big = hrex.uniforms(11, 3, np.arange(20000))
    assert abs(big.mean() - 0.5) < 0.01 and abs(big.var() - 1.0 / 12.0) < 0.005
