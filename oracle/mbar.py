"""MBAR (Shirts & Chodera 2008), FP64, plus BAR and EXP for reductions.

Section "Simulation protocol": the free energy between the terminal windows
of a segment is estimated with MBAR.  The self-consistent equations
  f_i = -ln sum_n exp(-u_i(x_n)) / sum_k N_k exp(f_k - u_k(x_n))
are iterated as a plain fixed point in log-sum-exp form, gauge f_0 = 0, until
max_i |f_i^{t+1} - f_i^t| <= tol * max(1, max_i |f_i|).
"""
from __future__ import annotations

import numpy as np
from scipy.special import logsumexp
from scipy.optimize import brentq


def mbar(u, N_k, tol=1e-10, max_iter=200000, f0=None):
    """Dimensionless free energies f (K,) and the iteration count."""
    u = np.asarray(u, np.float64)
    N_k = np.asarray(N_k, np.float64)
    K = u.shape[0]
    f = np.zeros(K) if f0 is None else np.asarray(f0, np.float64).copy()
    logN = np.where(N_k > 0, np.log(np.maximum(N_k, 1e-300)), -np.inf)
    for it in range(1, max_iter + 1):
        logden = logsumexp(logN[:, None] + f[:, None] - u, axis=0)
        fn = -logsumexp(-u - logden[None, :], axis=1)
        fn -= fn[0]
        delta = np.max(np.abs(fn - f))
        f = fn
        if delta <= tol * max(1.0, np.max(np.abs(f))):
            return f, it
    raise RuntimeError("MBAR did not converge")


def weights(u, N_k, f):
    """W_nk = exp(f_k - u_kn) / sum_j N_j exp(f_j - u_jn)  (K, N)."""
    N_k = np.asarray(N_k, np.float64)
    logN = np.where(N_k > 0, np.log(np.maximum(N_k, 1e-300)), -np.inf)
    logden = logsumexp(logN[:, None] + f[:, None] - u, axis=0)
    return np.exp(f[:, None] - u - logden[None, :])


def bar(w_f, w_r):
    """Bennett (1976) acceptance ratio: dimensionless df solving
    sum_F 1/(1 + (nF/nR) exp(wF - df)) = sum_R 1/(1 + (nR/nF) exp(wR + df))."""
    w_f = np.asarray(w_f, np.float64)
    w_r = np.asarray(w_r, np.float64)
    M = np.log(len(w_f) / len(w_r))

    def g(df):
        return (np.sum(1.0 / (1.0 + np.exp(M + w_f - df)))
                - np.sum(1.0 / (1.0 + np.exp(-M + w_r + df))))
    lo, hi = -100.0, 100.0
    return brentq(g, lo, hi, xtol=1e-14)


def exp_estimator(w):
    """Zwanzig: df = -ln < exp(-w) >."""
    w = np.asarray(w, np.float64)
    return -(logsumexp(-w) - np.log(len(w)))
