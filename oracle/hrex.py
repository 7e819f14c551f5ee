"""Hamiltonian replica exchange among the windows of one leg (FP64) -- test
infrastructure: only the tests and the CPU baseline use this module.

The paper attempts exchanges among the windows hosted on one GPU every 5 ps
(simulation details; openmmtools replica exchange) and does not print the
swap scheme.  Reading used here: Metropolis swaps of neighbouring states,
pairs (0,1), (2,3), ... on even attempts and (1,2), (3,4), ... on odd ones.
With u[k][r] the reduced potential of replica r's configuration in state k,
the swap of states s and s+1, held by replicas i and j, changes the total
reduced potential by

    D = u[s][j] + u[s+1][i] - u[s][i] - u[s+1][j]

and is accepted when D <= 0 or U < exp(-D) (Metropolis).  Every such move
leaves the joint distribution exp(-sum_r u[state(r)][r]) invariant.

The uniform U of the pair (s, s+1) at attempt t comes from Philox4x32-10
(Salmon et al. 2011) with counter (s, 0x48524558, t_lo, t_hi) and key
(seed_lo, seed_hi): U = ((w0 >> 5) 2^26 + (w1 >> 6)) 2^-53 in [0, 1).
"""
from __future__ import annotations

import math

import numpy as np

from .integrate import philox4x32_10

_TAG = 0x48524558                 # counter word that separates these draws from the MD noise


def uniforms(seed, attempt, states):
    """U for the pairs starting at the given states (float64 array)."""
    s = np.asarray(states, np.uint64)
    z = np.zeros_like(s)
    ctr = (s, z + np.uint64(_TAG), z + np.uint64(attempt & 0xFFFFFFFF), z + np.uint64((attempt >> 32) & 0xFFFFFFFF))
    key = (np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    w = philox4x32_10(ctr, key)
    hi = (w[0] >> np.uint64(5)).astype(np.float64)
    lo = (w[1] >> np.uint64(6)).astype(np.float64)
    return (hi * 67108864.0 + lo) * 2.0 ** -53


def attempt(u, state_of_replica, t, seed):
    """One exchange attempt.  ``u``: (K, K) reduced potentials u[state][replica];
    ``state_of_replica``: the current permutation.  Returns the new
    permutation and the list of accepted pairs (lower state of each)."""
    u = np.asarray(u, np.float64)
    st = np.array(state_of_replica, dtype=np.int64)
    K = len(st)
    rep = np.empty(K, np.int64)
    rep[st] = np.arange(K)
    pairs = list(range(t & 1, K - 1, 2))
    U = uniforms(seed, t, pairs) if pairs else np.zeros(0)
    accepted = []
    for s, us in zip(pairs, U):
        i, j = int(rep[s]), int(rep[s + 1])
        d = u[s, j] + u[s + 1, i] - u[s, i] - u[s + 1, j]
        if d <= 0.0 or us < math.exp(-d):
            st[i], st[j] = s + 1, s
            rep[s], rep[s + 1] = j, i
            accepted.append(s)
    return st, accepted
