"""Langevin-middle step with rigid-water constraints (FP64).

Section "Simulation protocol": LangevinMiddleIntegrator (Zhang et al. 2019),
2 fs step, friction 0.5/ps, rigid TIP3P water.  One step, in order:
  v <- v + dt F(x)/m                    (kick)
  v <- v + M^-1 G^T mu, G v = 0         (velocity constraint of rigid waters)
  x' <- x + dt/2 v                      (half drift)
  v <- a v + sqrt((1 - a^2) kT / m) xi  (Ornstein-Uhlenbeck, a = exp(-gamma dt))
  x' <- x' + dt/2 v                     (half drift)
  x'' <- constrain(x, x')               (rigid water; iterative SHAKE to 1e-12)
  v <- v + (x'' - x') / dt              (constraint correction of velocity)
Noise xi comes from Philox4x32-10 (Salmon et al. 2011) with counter
(atom, window, step_lo, step_hi) and key (seed_lo, seed_hi); each draw gives
four 32-bit words w0..w3 -> uniforms u = ((w >> 8) + 0.5) 2^-24 -> Box-Muller
normals (sqrt(-2 ln u0) cos 2 pi u1, ... sin ..., sqrt(-2 ln u2) cos 2 pi u3)
for the x, y, z components.
"""
from __future__ import annotations

import math

import numpy as np

KB = 0.0019872043        # kcal / (mol K)
ACCEL = 418.4            # (kcal/mol/A/amu) -> A/ps^2

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on uint64 arrays holding 32-bit words.
    ``ctr``: (4, M), ``key``: (2, M) or (2,) -- returns (4, M) words."""
    c = [np.asarray(ctr[i], np.uint64) & _MASK for i in range(4)]
    k0 = np.asarray(key[0], np.uint64) & _MASK
    k1 = np.asarray(key[1], np.uint64) & _MASK
    for r in range(10):
        p0 = np.uint64(_M0) * c[0]
        p1 = np.uint64(_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        if r < 9:
            k0 = (k0 + np.uint64(_W0)) & np.uint64(_MASK)
            k1 = (k1 + np.uint64(_W1)) & np.uint64(_MASK)
    return np.stack(c)


def normals(seed, window, step, n_atoms):
    """(n_atoms, 3) standard normals for one window at one step."""
    a = np.arange(n_atoms, dtype=np.uint64)
    z = np.zeros_like(a)
    ctr = (a, z + np.uint64(window), z + np.uint64(step & _MASK), z + np.uint64((step >> 32) & _MASK))
    key = (np.uint64(seed & _MASK), np.uint64((seed >> 32) & _MASK))
    w = philox4x32_10(ctr, key)
    u = ((w >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24
    r1 = np.sqrt(-2.0 * np.log(u[0]))
    r2 = np.sqrt(-2.0 * np.log(u[2]))
    return np.stack([r1 * np.cos(2 * np.pi * u[1]), r1 * np.sin(2 * np.pi * u[1]),
                     r2 * np.cos(2 * np.pi * u[3])], 1)


def shake_waters(x_old, x_new, waters, mass, d_oh, d_hh, box, tol=1e-12, max_iter=1000):
    """Iterative SHAKE for rigid waters: displacements along the old bond
    vectors weighted by inverse masses until every bond length is within
    ``tol`` (relative) of its target."""
    from .pairs import min_image
    x = x_new.copy()
    if len(waters) == 0:
        return x
    o, h1, h2 = waters[:, 0], waters[:, 1], waters[:, 2]
    cons = [(o, h1, d_oh), (o, h2, d_oh), (h1, h2, d_hh)]
    invm = 1.0 / mass.astype(np.float64)
    for it in range(max_iter):
        worst = 0.0
        for a, b, d in cons:
            rab = min_image(x[a] - x[b], box)
            r0 = min_image(x_old[a] - x_old[b], box)
            diff = (rab * rab).sum(1) - d * d
            worst = max(worst, float(np.max(np.abs(diff)) / (d * d)))
            g = diff / (2.0 * (invm[a] + invm[b]) * (rab * r0).sum(1))
            x[a] -= (g * invm[a])[:, None] * r0
            x[b] += (g * invm[b])[:, None] * r0
        if worst < tol:
            return x
    raise RuntimeError("SHAKE did not converge")


def constrain_velocities(x, v, waters, mass, box):
    """Velocity part of the rigid-water constraints (the RATTLE condition
    d/dt |r_a - r_b|^2 = 0 for the three distances of every water): each
    constraint k = (a, b) moves v_a by mu_k r_ab / m_a and v_b by
    -mu_k r_ab / m_b along its bond vector r_ab = x_a - x_b, with the three
    multipliers of a water solved exactly from the 3x3 linear system
    r_k . (v'_a - v'_b) = 0.  The result is the mass-weighted projection of v
    onto the velocities the rigid molecules allow."""
    from .pairs import min_image
    v = np.array(v, np.float64, copy=True)
    if len(waters) == 0:
        return v
    invm = 1.0 / np.asarray(mass, np.float64)
    cons = [(waters[:, 0], waters[:, 1]), (waters[:, 0], waters[:, 2]), (waters[:, 1], waters[:, 2])]
    r = [min_image(x[a] - x[b], box) for a, b in cons]                 # (nw, 3) each
    c = np.stack([(r[k] * (v[a] - v[b])).sum(1) for k, (a, b) in enumerate(cons)], 1)
    A = np.empty((len(waters), 3, 3))
    for k, (ak, bk) in enumerate(cons):
        for l, (al, bl) in enumerate(cons):
            # rate of constraint k per unit mu_l: r_k . (dv_ak - dv_bk)
            wa = np.where(ak == al, invm[ak], 0.0) - np.where(ak == bl, invm[ak], 0.0)
            wb = np.where(bk == al, invm[bk], 0.0) - np.where(bk == bl, invm[bk], 0.0)
            A[:, k, l] = (r[k] * r[l]).sum(1) * (wa - wb)
    mu = np.linalg.solve(A, -c[:, :, None])[:, :, 0]
    for k, (a, b) in enumerate(cons):
        v[a] += (mu[:, k] * invm[a])[:, None] * r[k]
        v[b] -= (mu[:, k] * invm[b])[:, None] * r[k]
    return v


def langevin_middle_step(sysd, x, v, force_fn, dt, temperature, gamma, seed, window, step):
    """One step; ``force_fn(x)`` returns (N,3) forces in kcal/mol/A."""
    m = sysd.mass.astype(np.float64)[:, None]
    F = force_fn(x)
    v = v + dt * F * ACCEL / m
    v = constrain_velocities(x, v, sysd.waters, sysd.mass, sysd.box)
    x1 = x + 0.5 * dt * v
    a = math.exp(-gamma * dt)
    sd = np.sqrt((1.0 - a * a) * KB * temperature * ACCEL / m)
    v = a * v + sd * normals(seed, window, step, len(x))
    x2 = x1 + 0.5 * dt * v
    x3 = shake_waters(x, x2, sysd.waters, sysd.mass, sysd.d_oh, sysd.d_hh, sysd.box)
    v = v + (x3 - x2) / dt
    return x3, v
