"""Bonded and Boresch restraint terms (FP64).

Section "Restraints": anchors P1, P2, P3 (protein) and L1, L2, L3 (ligand);
one distance P1-L1, two angles P1-L1-L2 and L1-P1-P2, three dihedrals
P2-P1-L1-L2, P1-L1-L2-L3 and L1-P1-P2-P3.  Distance and angle terms use
(k/2)(g - g0)^2, dihedrals k[1 - cos(g - g0)].  The whole restraint is scaled
by lambda_restraint (appendix B schedules).

Harmonic chain bonds use (k/2)(r - r0)^2 (the same harmonic convention).
Rotatable ligand torsions (section "Double annihilation protocol": periodic
torsions of rotatable bonds scaled linearly by the alchemical parameter, here
lambda_vdw) use lambda_vdw k [1 + cos(n phi - delta)].
Dihedral: phi(a,b,c,d) = atan2(|b2| b1.(b2 x b3), (b1 x b2).(b2 x b3)) with
b1 = b - a, b2 = c - b, b3 = d - c.  All vectors use the minimum image.
"""
from __future__ import annotations

import numpy as np

from .pairs import min_image


def bonds(pos, sysd):
    x = np.asarray(pos, dtype=np.float64)
    n = len(x)
    f = np.zeros((n, 3))
    if len(sysd.bonds) == 0:
        return 0.0, f
    i, j = sysd.bonds[:, 0].astype(np.int64), sysd.bonds[:, 1].astype(np.int64)
    k = sysd.bond_k.astype(np.float64)
    r0 = sysd.bond_r0.astype(np.float64)
    d = min_image(x[i] - x[j], sysd.box)
    r = np.sqrt((d * d).sum(1))
    e = 0.5 * k * (r - r0) ** 2
    fv = -(k * (r - r0) / r)[:, None] * d
    for ax in range(3):
        f[:, ax] += np.bincount(i, fv[:, ax], n) - np.bincount(j, fv[:, ax], n)
    return e.sum(), f


def _angle_grad(a, b, c, box):
    """theta at b and its gradients with respect to a, b, c."""
    u = min_image(a - b, box)
    v = min_image(c - b, box)
    nu, nv = np.linalg.norm(u), np.linalg.norm(v)
    cr = np.cross(u, v)
    th = np.arctan2(np.linalg.norm(cr), u @ v)
    uh, vh = u / nu, v / nv
    cs, sn = np.cos(th), np.sin(th)
    ga = (cs * uh - vh) / (nu * sn)
    gc = (cs * vh - uh) / (nv * sn)
    return th, ga, -(ga + gc), gc


def _dihedral_grad(a, b, c, d, box):
    """phi and its gradients with respect to a, b, c, d."""
    b1 = min_image(b - a, box)
    b2 = min_image(c - b, box)
    b3 = min_image(d - c, box)
    n1 = np.cross(b1, b2)
    n2 = np.cross(b2, b3)
    nb2 = np.linalg.norm(b2)
    phi = np.arctan2(nb2 * (b1 @ n2), n1 @ n2)
    ga = -nb2 / (n1 @ n1) * n1
    gd = nb2 / (n2 @ n2) * n2
    p = -(b1 @ b2) / (nb2 * nb2)
    s = -(b3 @ b2) / (nb2 * nb2)
    gb = (p - 1.0) * ga - s * gd
    gc = (s - 1.0) * gd - p * ga
    return phi, ga, gb, gc, gd


def boresch(pos, sysd, lam_rest):
    """lambda_r * [k_r/2 (r-r0)^2 + k_t/2 (tA-tA0)^2 + k_t/2 (tB-tB0)^2
    + sum_3 k_p (1 - cos(phi - phi0))] and its forces."""
    x = np.asarray(pos, dtype=np.float64)
    f = np.zeros_like(x)
    if sysd.restraint_atoms is None or lam_rest == 0.0:
        return 0.0, f
    p1, p2, p3, l1, l2, l3 = [int(a) for a in sysd.restraint_atoms]
    g0 = sysd.restraint_g0
    k = sysd.restraint_k
    box = sysd.box
    e = 0.0
    d = min_image(x[p1] - x[l1], box)
    r = np.linalg.norm(d)
    e += 0.5 * k[0] * (r - g0[0]) ** 2
    g = k[0] * (r - g0[0]) * d / r
    f[p1] -= g; f[l1] += g
    for t, (ia, ib, ic) in enumerate(((p1, l1, l2), (l1, p1, p2))):
        th, ga, gb, gc = _angle_grad(x[ia], x[ib], x[ic], box)
        e += 0.5 * k[1 + t] * (th - g0[1 + t]) ** 2
        dE = k[1 + t] * (th - g0[1 + t])
        f[ia] -= dE * ga; f[ib] -= dE * gb; f[ic] -= dE * gc
    for t, quad in enumerate(((p2, p1, l1, l2), (p1, l1, l2, l3), (l1, p1, p2, p3))):
        phi, ga, gb, gc, gd = _dihedral_grad(*(x[i] for i in quad), box)
        e += k[3 + t] * (1.0 - np.cos(phi - g0[3 + t]))
        dE = k[3 + t] * np.sin(phi - g0[3 + t])
        for i, gg in zip(quad, (ga, gb, gc, gd)):
            f[i] -= dE * gg
    return lam_rest * e, lam_rest * f


def torsions(pos, sysd, lam_vdw):
    """lambda_vdw * sum_t k_t [1 + cos(n_t phi_t - delta_t)] over the leg's
    rotatable torsions, and its forces (zero when the leg has none)."""
    x = np.asarray(pos, dtype=np.float64)
    f = np.zeros_like(x)
    if sysd.torsions is None or len(sysd.torsions) == 0 or lam_vdw == 0.0:
        return 0.0, f
    e = 0.0
    for t, quad in enumerate(sysd.torsions):
        quad = [int(a) for a in quad]
        k = float(sysd.torsion_k[t])
        n = float(sysd.torsion_n[t])
        dl = float(sysd.torsion_phase[t])
        phi, ga, gb, gc, gd = _dihedral_grad(*(x[i] for i in quad), sysd.box)
        e += k * (1.0 + np.cos(n * phi - dl))
        dE = -k * n * np.sin(n * phi - dl)
        for i, gg in zip(quad, (ga, gb, gc, gd)):
            f[i] -= dE * gg
    return lam_vdw * e, lam_vdw * f
