"""Brute-force real-space terms (FP64).

Section "Double annihilation protocol": the Beutler softcore 12-6 form
U = lambda_ij 4 eps_ij (sigma_ij^12 / r_eff^12 - sigma_ij^6 / r_eff^6) with
r_eff^6 = alpha (1 - lambda_ij)^p sigma_ij^6 + r^6, Lorentz-Berthelot mixing,
lambda_ij = min(lambda_i, lambda_j) with environment atoms fully coupled
(lambda_i = 1), alpha = 0.5, p = 1; ligand partial charges scaled linearly by
lambda_elec.  Appendix B: real-space electrostatics and vdW both cut at r_c.
The real-space Coulomb kernel is the Ewald direct-space term erfc(a r)/r.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

KE = 332.06371            # kcal A / (mol e^2)
SQRT_PI = math.sqrt(math.pi)


def min_image(d, box):
    """Minimum-image displacement, computed as d - L * rint(d * (1/L)) with
    separate multiply and subtract (no fused operations), in FP64."""
    box = np.asarray(box, np.float64)
    inv = 1.0 / box
    k = np.rint(d * inv)
    return d - box * k


def scaled_charges(sysd, lam_elec):
    """Charges of a window: ligand charges times lambda_elec (section "Double
    annihilation protocol"); the oxygens of the alchemical waters take up
    (1 - lambda_elec) of their offset, which keeps the net charge of every
    window that of the coupled state (same section)."""
    q = sysd.charge.astype(np.float64)
    q = np.where(sysd.is_ligand.astype(bool), q * lam_elec, q)
    off = getattr(sysd, 'alch_offset', None)
    if off is not None:
        q = q + (1.0 - lam_elec) * off.astype(np.float64)
    return q


def _excl_keys(sysd):
    n = sysd.n_atoms
    e = sysd.excl.astype(np.int64)
    return np.sort(e[:, 0] * n + e[:, 1])


def neighbor_pairs(pos, box, sysd, r):
    """Canonical list: {(i, j) : i < j, not excluded, |d_ij|^2 < r^2} with the
    min-image distance in FP64 from the float32 coordinates; sorted."""
    x = np.asarray(pos, dtype=np.float64)
    n = len(x)
    keys = _excl_keys(sysd)
    out = []
    r2 = r * r
    blk = 512
    for i0 in range(0, n, blk):
        i1 = min(n, i0 + blk)
        d = x[None, :, :] - x[i0:i1, None, :]
        d = min_image(d, box)
        d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        ii, jj = np.nonzero(d2 < r2)
        ii = ii + i0
        m = jj > ii
        ii, jj = ii[m], jj[m]
        k = ii.astype(np.int64) * n + jj
        keep = ~np.isin(k, keys)
        out.append(np.stack([ii[keep], jj[keep]], 1))
    p = np.concatenate(out) if out else np.zeros((0, 2), np.int64)
    order = np.lexsort((p[:, 1], p[:, 0]))
    return p[order].astype(np.int64)


def neighbor_pairs_tree(pos, box, sysd, r, margin=1e-3):
    """The canonical list of ``neighbor_pairs`` for large systems: candidate
    pairs within r + margin from a periodic k-d tree (a library search over
    the coordinates wrapped into the box), then exactly the same FP64
    inclusion test, exclusion filter and ordering as the brute force."""
    from scipy.spatial import cKDTree
    x = np.asarray(pos, dtype=np.float64)
    n = len(x)
    box = np.asarray(box, np.float64)
    wrapped = np.mod(x, box)
    wrapped[wrapped >= box] = 0.0
    cand = cKDTree(wrapped, boxsize=box).query_pairs(r + margin, output_type='ndarray').astype(np.int64)
    ii = np.minimum(cand[:, 0], cand[:, 1])
    jj = np.maximum(cand[:, 0], cand[:, 1])
    d = min_image(x[jj] - x[ii], box)
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    m = d2 < r * r
    ii, jj = ii[m], jj[m]
    keep = ~np.isin(ii * n + jj, _excl_keys(sysd))
    p = np.stack([ii[keep], jj[keep]], 1)
    order = np.lexsort((p[:, 1], p[:, 0]))
    return p[order].astype(np.int64)


def softcore_lj(r, sig, eps, lam, sc_alpha):
    """Energy and dE/dr of the softcore form with p = 1."""
    s6 = sig ** 6
    s = sc_alpha * (1.0 - lam) * s6 + r ** 6
    e = lam * 4.0 * eps * (s6 * s6 / (s * s) - s6 / s)
    de = 24.0 * lam * eps * r ** 5 * (s6 / (s * s) - 2.0 * s6 * s6 / (s ** 3))
    return e, de


def coulomb_real(r, qq, alpha):
    """Energy and dE/dr of KE qq erfc(alpha r) / r."""
    e = KE * qq * erfc(alpha * r) / r
    de = -KE * qq * (erfc(alpha * r) / (r * r) + 2.0 * alpha / SQRT_PI * np.exp(-(alpha * r) ** 2) / r)
    return e, de


def _pair_block(x, box, sysd, lam, i_idx, j_idx):
    """Pair energies and force contributions for explicit index arrays."""
    lam_e, lam_v = lam[0], lam[1]
    q = scaled_charges(sysd, lam_e)
    lig = sysd.is_ligand.astype(bool)
    sig = sysd.sigma.astype(np.float64)
    eps = sysd.epsilon.astype(np.float64)
    d = min_image(x[i_idx] - x[j_idx], box)          # r_i - r_j
    r = np.sqrt((d * d).sum(1))
    m = r < sysd.r_cut
    i_idx, j_idx, d, r = i_idx[m], j_idx[m], d[m], r[m]
    ec, dec = coulomb_real(r, q[i_idx] * q[j_idx], sysd.ewald_alpha)
    lij = np.where(lig[i_idx] | lig[j_idx], lam_v, 1.0)
    e_lj, de_lj = softcore_lj(r, 0.5 * (sig[i_idx] + sig[j_idx]), np.sqrt(eps[i_idx] * eps[j_idx]),
                              lij, sysd.sc_alpha)
    fvec = -((dec + de_lj) / r)[:, None] * d          # force on i
    return i_idx, j_idx, ec, e_lj, fvec


def real_space(pos, sysd, lam, blk=384):
    """All non-excluded pairs i < j within r_c (brute force).  Returns
    (E_coul_real, E_lj, forces[N,3])."""
    x = np.asarray(pos, dtype=np.float64)
    n = len(x)
    keys = _excl_keys(sysd)
    f = np.zeros((n, 3))
    ec_tot = 0.0
    elj_tot = 0.0
    for i0 in range(0, n, blk):
        i1 = min(n, i0 + blk)
        ii, jj = np.meshgrid(np.arange(i0, i1), np.arange(n), indexing='ij')
        ii, jj = ii.ravel(), jj.ravel()
        m = jj > ii
        ii, jj = ii[m], jj[m]
        keep = ~np.isin(ii.astype(np.int64) * n + jj, keys)
        ii, jj = ii[keep], jj[keep]
        ii, jj, ec, elj, fv = _pair_block(x, sysd.box, sysd, lam, ii, jj)
        ec_tot += ec.sum()
        elj_tot += elj.sum()
        for ax in range(3):
            f[:, ax] += np.bincount(ii, fv[:, ax], n) - np.bincount(jj, fv[:, ax], n)
    return ec_tot, elj_tot, f


def real_space_atoms(pos, sysd, lam, atoms):
    """Per-atom real-space force and per-atom pair energy (each pair's energy
    split half/half) for the sampled ``atoms``, by brute force over all j."""
    x = np.asarray(pos, dtype=np.float64)
    n = len(x)
    keys = set((_excl_keys(sysd)).tolist())
    fo = np.zeros((len(atoms), 3))
    eo = np.zeros(len(atoms))
    for k, a in enumerate(atoms):
        j = np.arange(n)
        j = j[j != a]
        lo, hi = np.minimum(a, j), np.maximum(a, j)
        keep = np.array([int(p) not in keys for p in (lo.astype(np.int64) * n + hi)])
        j = j[keep]
        ii = np.full(len(j), a)
        ii, jj, ec, elj, fv = _pair_block(x, sysd.box, sysd, lam, ii, j)
        fo[k] = fv.sum(0)
        eo[k] = 0.5 * (ec.sum() + elj.sum())
    return fo, eo


def exclusion_correction(pos, sysd, lam):
    """Remove the reciprocal-space interaction of excluded pairs:
    E = -KE q_i q_j erf(alpha r)/r per excluded pair (series near r = 0)."""
    x = np.asarray(pos, dtype=np.float64)
    n = len(x)
    q = scaled_charges(sysd, lam[0])
    a = sysd.ewald_alpha
    i, j = sysd.excl[:, 0].astype(np.int64), sysd.excl[:, 1].astype(np.int64)
    d = min_image(x[i] - x[j], sysd.box)
    r = np.sqrt((d * d).sum(1))
    qq = q[i] * q[j]
    small = r < 1e-6
    rs = np.where(small, 1.0, r)
    e = np.where(small, -KE * qq * 2 * a / SQRT_PI, -KE * qq * erf(a * rs) / rs)
    de = np.where(small, 0.0, -KE * qq * (2 * a / SQRT_PI * np.exp(-(a * rs) ** 2) / rs - erf(a * rs) / (rs * rs)))
    fv = -(de / rs)[:, None] * d
    f = np.zeros((n, 3))
    for ax in range(3):
        f[:, ax] += np.bincount(i, fv[:, ax], n) - np.bincount(j, fv[:, ax], n)
    return e.sum(), f


def self_and_background(sysd, lam):
    """Ewald self term -KE alpha/sqrt(pi) sum q^2 and the uniform neutralising
    background -KE pi Q^2 / (2 V alpha^2) for a net charge Q."""
    q = scaled_charges(sysd, lam[0])
    a = sysd.ewald_alpha
    V = float(np.prod(sysd.box))
    return -KE * a / SQRT_PI * (q * q).sum() - KE * math.pi * q.sum() ** 2 / (2.0 * V * a * a)
