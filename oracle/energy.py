"""Total potential of one lambda window (FP64): the sum the MD step needs.

U(window) = real-space Coulomb (erfc) + softcore/plain LJ + excluded-pair
correction + self and background + reciprocal (PME or direct Ewald) + bonds
+ lambda_restraint * Boresch.  Component names match the HIP path's energy
vector so tests can compare them one by one.
"""
from __future__ import annotations

import numpy as np

from . import bonded, pairs
from .ewald import PME, direct_ewald

COMPONENTS = ('coul_real', 'lj', 'excl', 'self', 'recip', 'bond', 'restraint', 'total')


def window_energy(sysd, pos, lam, recip='pme', pme=None):
    """Energies (dict) and forces (N,3) for coordinates ``pos`` at the lambda
    triple ``lam`` = (elec, vdw, restraint)."""
    lam = np.asarray(lam, np.float64)
    x = np.asarray(pos, dtype=np.float64)
    e = {}
    ec, elj, f = pairs.real_space(x, sysd, lam)
    e['coul_real'], e['lj'] = ec, elj
    ex, fx = pairs.exclusion_correction(x, sysd, lam)
    e['excl'] = ex
    f = f + fx
    e['self'] = pairs.self_and_background(sysd, lam)
    q = pairs.scaled_charges(sysd, lam[0])
    if recip == 'pme':
        pme = pme or PME(sysd.box, sysd.grid, sysd.ewald_alpha, sysd.spline_order)
        er, fr = pme.energy_forces(x, q)
    elif recip == 'ewald':
        er, fr = direct_ewald(x, q, sysd.box, sysd.ewald_alpha)
    else:
        er, fr = 0.0, np.zeros_like(x)
    e['recip'] = er
    f = f + fr
    eb, fb = bonded.bonds(x, sysd)
    et, ft = bonded.torsions(x, sysd, lam[1])
    e['bond'] = eb + et                  # bonded: harmonic bonds + lambda-scaled rotatable torsions
    f = f + fb + ft
    erest, frest = bonded.boresch(x, sysd, lam[2])
    e['restraint'] = erest
    f = f + frest
    e['total'] = sum(e[k] for k in COMPONENTS[:-1])
    return e, f
