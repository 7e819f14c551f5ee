"""Free-energy assembly over the C ABI (section "Simulation protocol",
figure 1 / section "Restraints").

A leg's window path is cut into overlapping segments -- neighbouring segments
share (duplicate) their boundary window, so a segment never needs another's
coordinates or energies -- each segment is simulated as its own leg, its
u_kn is estimated with MBAR on the device (``felis_mbar``), and the leg's
free energy is the sum of the segment differences kT (f_last - f_first).
The binding free energy of legs run from the coupled to the decoupled state
adds the analytic restraint term (``felis_restraint_dg``):

    dG_bind = dG_solvent - dG_complex + dG_restrain
"""
from __future__ import annotations

import numpy as np

from . import felis

KB = 0.0019872043           # kcal / (mol K)


def segments(n_windows: int, n_segments: int) -> list[list[int]]:
    """Window indices of each segment: n_segments contiguous ranges over
    0..n_windows-1 with boundaries at windows floor(s (n_windows - 1) /
    n_segments), each sharing its last window with the next one's first."""
    if n_segments < 1 or n_windows < n_segments + 1:
        raise ValueError('every segment needs at least two windows')
    edges = [(s * (n_windows - 1)) // n_segments for s in range(n_segments + 1)]
    return [list(range(edges[s], edges[s + 1] + 1)) for s in range(n_segments)]


def segment_dg(ctx, u, n_k, temperature=300.0, tol=1e-10, max_iter=20000):
    """kT (f_last - f_first) of one segment from its own reduced potentials
    u[k][n] (device float64; the segment's states and frames only)."""
    f, _ = felis.mbar(ctx, u, n_k, tol=tol, max_iter=max_iter)
    return KB * temperature * float(f[-1] - f[0])


def segmented_dg(ctx, u_segments, n_k_segments, temperature=300.0, tol=1e-10, max_iter=20000):
    """A leg's free energy as the sum of its segments' MBAR differences."""
    return sum(segment_dg(ctx, u, nk, temperature, tol, max_iter) for u, nk in zip(u_segments, n_k_segments))


def binding_dg(dg_solvent, dg_complex, restraint_g0, restraint_k, temperature=300.0):
    """dG_bind from the two legs' free energies (coupled -> decoupled) and the
    restraint geometry and force constants of the complex leg."""
    return dg_solvent - dg_complex + felis.restraint_dg(restraint_g0, restraint_k, temperature)
