"""Cross-lambda reduced potentials u_k(x_n) (FP64).

Section "Simulation protocol" estimates each segment's free energy with MBAR,
which needs every stored sample's reduced potential at every window.  With
ligand charges scaled by lambda_e (section "Double annihilation protocol"),
the potential of window k splits exactly into
  U_k(x) = U_env(x) + lam_e E_LE(x) + lam_e^2 E_LL(x) + E_sc(x; lam_v) + lam_r U_B(x),
where U_env (environment-only terms and all bonded terms) does not depend on
lambda and is dropped (MBAR is invariant under u_kn += c_n):
  E_LE: ligand-environment real-space Coulomb + reciprocal cross term + the
        cross term of the neutralising background;
  E_LL: ligand intramolecular real-space Coulomb + ligand reciprocal term +
        ligand self term + excluded-pair corrections + ligand background;
  E_sc: softcore LJ of all ligand-environment and non-excluded ligand-ligand
        pairs at lambda_ij = lam_v;
  U_B:  Boresch energy (unscaled).
u_kn = beta U_k(x_n).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

from .ewald import PME
from .pairs import KE, SQRT_PI, min_image, softcore_lj
from .bonded import boresch


def frame_terms(sysd, pos, pme=None):
    """(E_LE, E_LL, pair data for E_sc, U_B) for one frame."""
    x = np.asarray(pos, dtype=np.float64)
    lig = sysd.is_ligand.astype(bool)
    L = np.where(lig)[0]
    E = np.where(~lig)[0]
    q = sysd.charge.astype(np.float64)
    sig = sysd.sigma.astype(np.float64)
    eps = sysd.epsilon.astype(np.float64)
    a = sysd.ewald_alpha
    rc = sysd.r_cut
    box = sysd.box
    V = float(np.prod(box))
    # ligand-environment pairs
    d = min_image(x[L][:, None, :] - x[E][None, :, :], box)
    r = np.sqrt((d * d).sum(-1))
    li, ej = np.nonzero(r < rc)
    rr = r[li, ej]
    gi, gj = L[li], E[ej]
    e_le = float(np.sum(KE * q[gi] * q[gj] * erfc(a * rr) / rr))
    sc = [(rr, 0.5 * (sig[gi] + sig[gj]), np.sqrt(eps[gi] * eps[gj]))]
    # ligand-ligand pairs (non-excluded, i < j) and excluded corrections
    ex = {(int(i), int(j)) for i, j in sysd.excl if lig[i] and lig[j]}
    e_ll = 0.0
    if len(L) > 1:
        ii, jj = np.triu_indices(len(L), 1)
        gi, gj = L[ii], L[jj]
        dl = min_image(x[gi] - x[gj], box)
        rl = np.sqrt((dl * dl).sum(1))
        isx = np.array([(int(p), int(s)) in ex for p, s in zip(gi, gj)])
        m = (~isx) & (rl < rc)
        e_ll += float(np.sum(KE * q[gi[m]] * q[gj[m]] * erfc(a * rl[m]) / rl[m]))
        sc.append((rl[m], 0.5 * (sig[gi[m]] + sig[gj[m]]), np.sqrt(eps[gi[m]] * eps[gj[m]])))
        e_ll -= float(np.sum(KE * q[gi[isx]] * q[gj[isx]] * erf(a * rl[isx]) / rl[isx]))
    e_ll -= KE * a / SQRT_PI * float(np.sum(q[L] ** 2))
    # reciprocal: E(lam) = E_EE + lam E_LE_rec + lam^2 E_LL_rec
    pme = pme or PME(box, sysd.grid, a, sysd.spline_order)
    qe = np.where(lig, 0.0, q)
    ql = np.where(lig, q, 0.0)
    QE = pme.spread(x, qe)
    QL = pme.spread(x, ql)
    e_le += 2.0 * pme.energy_of_grids(QE, QL)
    e_ll += pme.energy_of_grids(QL)
    # background -KE pi (Q_E + lam Q_L)^2 / (2 V a^2)
    bg = KE * math.pi / (2.0 * V * a * a)
    e_le -= bg * 2.0 * qe.sum() * ql.sum()
    e_ll -= bg * ql.sum() ** 2
    ub, _ = boresch(x, sysd, 1.0)
    r_all = np.concatenate([s[0] for s in sc])
    s_all = np.concatenate([s[1] for s in sc])
    e_all = np.concatenate([s[2] for s in sc])
    return e_le, e_ll, (r_all, s_all, e_all), ub


def ukn_frame(sysd, pos, lambdas, beta, pme=None):
    """u_k(x) for every row of ``lambdas`` (K,3)."""
    e_le, e_ll, (r, s, e), ub = frame_terms(sysd, pos, pme)
    out = np.empty(len(lambdas))
    for k, (le, lv, lr) in enumerate(lambdas):
        esc, _ = softcore_lj(r, s, e, np.full_like(r, lv), sysd.sc_alpha)
        out[k] = beta * (le * e_le + le * le * e_ll + esc.sum() + lr * ub)
    return out


def ukn(sysd, frames, lambdas, beta):
    """u [K, n_frames] for frames (n, N, 3)."""
    pme = PME(sysd.box, sysd.grid, sysd.ewald_alpha, sysd.spline_order)
    return np.stack([ukn_frame(sysd, f, lambdas, beta, pme) for f in frames], 1)
