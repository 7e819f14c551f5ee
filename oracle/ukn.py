"""Cross-lambda reduced potentials u_k(x_n) (FP64).

Section "Simulation protocol" estimates each segment's free energy with MBAR,
which needs every stored sample's reduced potential at every window.  With
ligand charges scaled by lambda_e (section "Double annihilation protocol"),
the potential of window k splits exactly into
  U_k(x) = U_env(x) + lam_e E_LE(x) + lam_e^2 E_LL(x) + E_sc(x; lam_v) + lam_r U_B(x),
where U_env (environment-only terms and all bonded terms) does not depend on
lambda and is dropped (MBAR is invariant under u_kn += c_n):
  E_LE: ligand-environment real-space Coulomb + reciprocal cross term + the
        cross term of the neutralising background (with alchemical waters:
        the cross term 2 E[a, b] of the bilinear form, see frame_terms);
  E_LL: ligand intramolecular real-space Coulomb + ligand reciprocal term +
        ligand self term + excluded-pair corrections + ligand background
        (with alchemical waters: E[b, b]);
  E_sc: softcore LJ of all ligand-environment and non-excluded ligand-ligand
        pairs at lambda_ij = lam_v;
  U_B:  Boresch energy (unscaled);
  U_T:  rotatable ligand torsions (unscaled), which scale with lam_v.
u_kn = beta U_k(x_n), U_k = ... + lam_v U_T.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

from .ewald import PME
from .pairs import KE, SQRT_PI, min_image, softcore_lj
from .bonded import boresch, torsions


def frame_terms(sysd, pos, pme=None):
    """(E_LE, E_LL, pair data for E_sc, U_B, U_T) for one frame.

    A window's charges are q(lam_e) = a + lam_e b with a = the environment
    charges plus the alchemical-water offsets (zero on ligand atoms) and
    b = the ligand charges minus those offsets (zero elsewhere), so its
    electrostatic energy is E[a, a] + 2 lam_e E[a, b] + lam_e^2 E[b, b] for
    the symmetric bilinear Ewald form E (real space over non-excluded pairs
    within r_c, minus the excluded pairs' erf terms, reciprocal, self and
    background).  E_LE = 2 E[a, b], E_LL = E[b, b]; without alchemical
    waters these are the ligand-environment and ligand-ligand terms."""
    x = np.asarray(pos, dtype=np.float64)
    lig = sysd.is_ligand.astype(bool)
    L = np.where(lig)[0]
    E = np.where(~lig)[0]
    q = sysd.charge.astype(np.float64)
    off = getattr(sysd, 'alch_offset', None)
    c = np.zeros_like(q) if off is None else off.astype(np.float64)
    ca = np.where(lig, 0.0, q + c)
    cb = np.where(lig, q, -c)
    Bset = np.where(lig | (c != 0.0))[0]
    sig = sysd.sigma.astype(np.float64)
    eps = sysd.epsilon.astype(np.float64)
    a = sysd.ewald_alpha
    rc = sysd.r_cut
    box = sysd.box
    V = float(np.prod(box))
    excl = {(int(i), int(j)) for i, j in sysd.excl}
    is_ex = lambda i, j: (min(i, j), max(i, j)) in excl
    partners = {}
    for i, j in excl:
        partners.setdefault(i, []).append(j)
        partners.setdefault(j, []).append(i)
    # 2 E[a, b], real space: ordered pairs (i in B, j != i)
    e_le = 0.0
    for i in Bset:
        d = min_image(x[i][None, :] - x, box)
        r = np.sqrt((d * d).sum(-1))
        ex = np.zeros(len(x), bool)
        ex[partners.get(int(i), [])] = True
        use = (ca != 0.0) & (np.arange(len(x)) != i)
        m = use & ~ex & (r < rc)
        e_le += float(np.sum(KE * cb[i] * ca[m] * erfc(a * r[m]) / r[m]))
        m = use & ex
        e_le -= float(np.sum(KE * cb[i] * ca[m] * erf(a * r[m]) / r[m]))
    # E[b, b], real space: unordered pairs within B
    e_ll = 0.0
    for n1, i in enumerate(Bset):
        for j in Bset[n1 + 1:]:
            d = min_image(x[i] - x[j], box)
            r = float(np.sqrt((d * d).sum()))
            if is_ex(i, j):
                e_ll -= KE * cb[i] * cb[j] * erf(a * r) / r
            elif r < rc:
                e_ll += KE * cb[i] * cb[j] * erfc(a * r) / r
    # softcore LJ: ligand-environment pairs and non-excluded ligand-ligand pairs
    d = min_image(x[L][:, None, :] - x[E][None, :, :], box)
    r = np.sqrt((d * d).sum(-1))
    li, ej = np.nonzero(r < rc)
    gi, gj = L[li], E[ej]
    sc = [(r[li, ej], 0.5 * (sig[gi] + sig[gj]), np.sqrt(eps[gi] * eps[gj]))]
    if len(L) > 1:
        ii, jj = np.triu_indices(len(L), 1)
        gi, gj = L[ii], L[jj]
        dl = min_image(x[gi] - x[gj], box)
        rl = np.sqrt((dl * dl).sum(1))
        m = np.array([not is_ex(p, t) for p, t in zip(gi, gj)]) & (rl < rc)
        sc.append((rl[m], 0.5 * (sig[gi[m]] + sig[gj[m]]), np.sqrt(eps[gi[m]] * eps[gj[m]])))
    # self terms
    e_le -= 2.0 * KE * a / SQRT_PI * float(np.sum(ca * cb))
    e_ll -= KE * a / SQRT_PI * float(np.sum(cb * cb))
    # reciprocal: E(lam) = E[a,a] + lam 2 E[a,b] + lam^2 E[b,b]
    pme = pme or PME(box, sysd.grid, a, sysd.spline_order)
    QA = pme.spread(x, ca)
    QB = pme.spread(x, cb)
    e_le += 2.0 * pme.energy_of_grids(QA, QB)
    e_ll += pme.energy_of_grids(QB)
    # background -KE pi (Q_a + lam Q_b)^2 / (2 V a^2)
    bg = KE * math.pi / (2.0 * V * a * a)
    e_le -= bg * 2.0 * ca.sum() * cb.sum()
    e_ll -= bg * cb.sum() ** 2
    ub, _ = boresch(x, sysd, 1.0)
    ut, _ = torsions(x, sysd, 1.0)
    r_all = np.concatenate([s[0] for s in sc])
    s_all = np.concatenate([s[1] for s in sc])
    e_all = np.concatenate([s[2] for s in sc])
    return e_le, e_ll, (r_all, s_all, e_all), ub, ut


def ukn_frame(sysd, pos, lambdas, beta, pme=None):
    """u_k(x) for every row of ``lambdas`` (K,3)."""
    e_le, e_ll, (r, s, e), ub, ut = frame_terms(sysd, pos, pme)
    out = np.empty(len(lambdas))
    for k, (le, lv, lr) in enumerate(lambdas):
        esc, _ = softcore_lj(r, s, e, np.full_like(r, lv), sysd.sc_alpha)
        out[k] = beta * (le * e_le + le * le * e_ll + esc.sum() + lr * ub + lv * ut)
    return out


def ukn(sysd, frames, lambdas, beta):
    """u [K, n_frames] for frames (n, N, 3)."""
    pme = PME(sysd.box, sysd.grid, sysd.ewald_alpha, sysd.spline_order)
    return np.stack([ukn_frame(sysd, f, lambdas, beta, pme) for f in frames], 1)
