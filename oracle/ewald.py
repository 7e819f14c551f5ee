"""Reciprocal-space electrostatics in FP64: direct Ewald and smooth PME.

The paper (appendix B, and the PME tuning remarks in the discussion) names PME
with a 1.0 nm real-space cutoff but prints no PME formulas; both routines
below follow the published methods: the Ewald reciprocal sum, and the smooth
particle-mesh Ewald of Essmann et al. (1995) with cardinal B-splines of order
n, their Euler exponential-spline moduli, and forces from analytic
differentiation of the interpolated energy.

Conventions: m runs over reciprocal vectors m = (n1/L1, n2/L2, n3/L3),
S(m) = sum_j q_j exp(2 pi i m.r_j),
E_rec = KE / (2 pi V) sum_{m != 0} exp(-pi^2 |m|^2 / alpha^2) / |m|^2 |S(m)|^2.
"""
from __future__ import annotations

import math

import numpy as np

from .pairs import KE


def _mvectors(box, alpha, rel=1e-16):
    box = np.asarray(box, np.float64)
    # exp(-pi^2 |m|^2 / alpha^2) / |m|^2 < rel * (largest term) beyond this radius
    kmax2 = -math.log(rel) * alpha * alpha / (math.pi ** 2)
    nmax = [int(math.ceil(math.sqrt(kmax2) * L)) + 1 for L in box]
    g = [np.arange(-k, k + 1) for k in nmax]
    n = np.stack(np.meshgrid(*g, indexing='ij'), -1).reshape(-1, 3)
    n = n[np.any(n != 0, 1)]
    m = n / box
    m2 = (m * m).sum(1)
    keep = m2 <= kmax2 * 1.0000001
    return m[keep], m2[keep]


def direct_ewald(pos, q, box, alpha, rel=1e-16, chunk=4096):
    """Reciprocal energy and forces by the explicit Ewald sum."""
    x = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    V = float(np.prod(box))
    m, m2 = _mvectors(box, alpha, rel)
    e = 0.0
    f = np.zeros_like(x)
    pref = KE / (2.0 * math.pi * V)
    for c0 in range(0, len(m), chunk):
        mc, m2c = m[c0:c0 + chunk], m2[c0:c0 + chunk]
        w = np.exp(-math.pi ** 2 * m2c / alpha ** 2) / m2c
        th = 2.0 * math.pi * (x @ mc.T)                 # (N, M)
        c, s = np.cos(th), np.sin(th)
        Sr = q @ c
        Si = q @ s
        e += pref * np.sum(w * (Sr * Sr + Si * Si))
        # dE/dr_i = pref * w * 2 * Re(dS/dr_i * conj(S)); dS/dr_i = 2 pi i m q_i e^{i th_i}
        # => F_i = pref * sum_m w * 4 pi q_i m * (s_i Sr - c_i Si)
        g = (s * Sr[None, :] - c * Si[None, :]) * w[None, :]   # (N, M)
        f += (4.0 * math.pi * pref) * q[:, None] * (g @ mc)
    return e, f


def bspline(u, n):
    """Cardinal B-spline M_n(u) by the recursion
    M_n(u) = [u M_{n-1}(u) + (n - u) M_{n-1}(u - 1)] / (n - 1), M_2(u) = 1 - |u - 1|."""
    u = np.asarray(u, np.float64)
    if n == 2:
        return np.where((u >= 0) & (u <= 2), 1.0 - np.abs(u - 1.0), 0.0)
    return (u * bspline(u, n - 1) + (n - u) * bspline(u - 1.0, n - 1)) / (n - 1)


def bspline_deriv(u, n):
    """dM_n/du = M_{n-1}(u) - M_{n-1}(u - 1)."""
    return bspline(u, n - 1) - bspline(u - 1.0, n - 1)


def bspline_moduli(K, n):
    """|b(m)|^2 with b(m) = exp(2 pi i (n-1) m / K) / sum_{k=0}^{n-2} M_n(k+1) exp(2 pi i m k / K)."""
    m = np.arange(K)
    den = np.zeros(K, np.complex128)
    for k in range(n - 1):
        den += bspline(k + 1.0, n) * np.exp(2j * math.pi * m * k / K)
    return 1.0 / np.abs(den) ** 2


class PME:
    """FP64 smooth PME for a fixed box, grid, order and alpha."""

    def __init__(self, box, grid, alpha, order=4):
        self.box = np.asarray(box, np.float64)
        self.K = tuple(int(k) for k in grid)
        self.alpha = float(alpha)
        self.n = int(order)
        V = float(np.prod(self.box))
        freqs = []
        for K, L in zip(self.K, self.box):
            mi = np.fft.fftfreq(K, 1.0 / K)            # signed integers
            freqs.append(mi / L)
        mx, my, mz = np.meshgrid(*freqs, indexing='ij')
        m2 = mx * mx + my * my + mz * mz
        m2[0, 0, 0] = 1.0
        C = np.exp(-math.pi ** 2 * m2 / self.alpha ** 2) / m2
        C[0, 0, 0] = 0.0
        b = [bspline_moduli(K, self.n) for K in self.K]
        B = b[0][:, None, None] * b[1][None, :, None] * b[2][None, None, :]
        self.BC = B * C
        self.A = KE / (2.0 * math.pi * V)

    def _weights(self, pos):
        x = np.asarray(pos, np.float64)
        frac = x / self.box
        frac = frac - np.floor(frac)
        u = frac * np.array(self.K)
        base = np.floor(u).astype(np.int64)
        n = self.n
        idx, w, dw = [], [], []
        for ax in range(3):
            j = np.arange(n)
            k = base[:, ax, None] - j[None, :]           # grid points base, base-1, ...
            t = u[:, ax, None] - k                       # in (0, n)
            idx.append(np.mod(k, self.K[ax]))
            w.append(bspline(t, n))
            dw.append(bspline_deriv(t, n) * self.K[ax] / self.box[ax])
        return idx, w, dw

    def spread(self, pos, q):
        idx, w, _ = self._weights(pos)
        Q = np.zeros(self.K)
        n = self.n
        q = np.asarray(q, np.float64)
        for a in range(n):
            for b in range(n):
                for c in range(n):
                    np.add.at(Q, (idx[0][:, a], idx[1][:, b], idx[2][:, c]),
                              q * w[0][:, a] * w[1][:, b] * w[2][:, c])
        return Q

    def energy_of_grids(self, Qa, Qb=None):
        """A sum_m BC Re(F(Qa) conj F(Qb)) (Qb = Qa gives the PME energy)."""
        Fa = np.fft.fftn(Qa)
        Fb = Fa if Qb is None else np.fft.fftn(Qb)
        return self.A * float(np.sum(self.BC * (Fa * np.conj(Fb)).real))

    def potential(self, Q):
        """phi(k) = dE/dQ(k) = 2 A K^3 Re(ifftn(BC * fftn(Q)))."""
        Ktot = float(np.prod(self.K))
        return 2.0 * self.A * Ktot * np.fft.ifftn(self.BC * np.fft.fftn(Q)).real

    def gather(self, pos, q, phi):
        """Forces -q_i sum_k grad(w) phi(k), and phi interpolated at each atom."""
        idx, w, dw = self._weights(pos)
        n = self.n
        q = np.asarray(q, np.float64)
        f = np.zeros((len(q), 3))
        pot = np.zeros(len(q))
        for a in range(n):
            for b in range(n):
                for c in range(n):
                    p = phi[idx[0][:, a], idx[1][:, b], idx[2][:, c]]
                    pot += w[0][:, a] * w[1][:, b] * w[2][:, c] * p
                    f[:, 0] -= q * dw[0][:, a] * w[1][:, b] * w[2][:, c] * p
                    f[:, 1] -= q * w[0][:, a] * dw[1][:, b] * w[2][:, c] * p
                    f[:, 2] -= q * w[0][:, a] * w[1][:, b] * dw[2][:, c] * p
        return f, pot

    def energy_forces(self, pos, q):
        Q = self.spread(pos, q)
        e = self.energy_of_grids(Q)
        f, _ = self.gather(pos, q, self.potential(Q))
        return e, f
