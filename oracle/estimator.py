"""Free-energy assembly (FP64) -- test infrastructure: only the tests and the
CPU baseline use this module.

Section "Simulation protocol" partitions each leg's window path into
overlapping segments (the boundary window of two neighbouring segments is
duplicated), estimates each segment with MBAR, and sums the segment
differences; the binding free energy then adds the analytic restraint term
(figure 1 / section "Restraints"):

    dG_bind = dG_solvent - dG_complex + dG_restrain

for legs whose windows run from the coupled to the decoupled (and, in the
complex, restrained) state, each leg's dG = kT (f_last - f_first).

dG_restrain is the free energy of imposing the Boresch restraints on the
decoupled ligand from the standard state.  The paper uses the closed form of
Chen et al. 2023, which it does not print; this oracle uses Boresch et al.
2003 (harmonic limit) as a labelled stand-in:

    dG_restrain = kT ln[ 8 pi^2 V0 sqrt(K_r K_thA K_thB K_phA K_phB K_phC)
                         / (r0^2 sin thA0 sin thB0 (2 pi kT)^3) ]

with U = (K/2)(g - g0)^2 for the distance and angles and the cosine dihedral
k[1 - cos(g - g0)] taken at its second-order (harmonic) limit K = k, and
V0 = 1661 A^3 (1 mol/L).
"""
from __future__ import annotations

import math

import numpy as np

from . import mbar as ombar

KB = 0.0019872043           # kcal / (mol K)
V0 = 1660.5390              # A^3 per molecule at 1 mol/L


def boresch_restraint_dg(g0, k, temperature=300.0, v0=V0):
    """dG of restraining the decoupled ligand (kcal/mol): g0 = (r0, thA0, thB0,
    phA0, phB0, phC0) in A and rad, k = the six force constants."""
    kT = KB * temperature
    r0, ta, tb = g0[0], g0[1], g0[2]
    prodk = float(np.prod(np.asarray(k, np.float64)))
    num = 8.0 * math.pi ** 2 * v0 * math.sqrt(prodk)
    den = r0 ** 2 * math.sin(ta) * math.sin(tb) * (2.0 * math.pi * kT) ** 3
    return kT * math.log(num / den)


def segments(n_windows, n_segments):
    """Window index lists of n_segments overlapping segments covering
    0..n_windows-1; neighbouring segments share their boundary window, the
    s-th boundary being window floor(s (n_windows - 1) / n_segments)."""
    if n_segments < 1 or n_windows < n_segments + 1:
        raise ValueError('need at least two windows per segment')
    cuts = [s * (n_windows - 1) // n_segments for s in range(n_segments + 1)]
    return [list(range(cuts[s], cuts[s + 1] + 1)) for s in range(n_segments)]


def segmented_dg(u_segments, n_k_segments, temperature=300.0, tol=1e-12, max_iter=200000):
    """Sum over segments of kT (f_last - f_first) from each segment's own
    reduced potentials u[k][n] (states and frames of that segment only)."""
    kT = KB * temperature
    total = 0.0
    for u, nk in zip(u_segments, n_k_segments):
        f, _ = ombar.mbar(np.asarray(u, np.float64), np.asarray(nk), tol=tol, max_iter=max_iter)
        total += kT * (f[-1] - f[0])
    return total


def binding_dg(dg_solvent, dg_complex, dg_restrain):
    return dg_solvent - dg_complex + dg_restrain
