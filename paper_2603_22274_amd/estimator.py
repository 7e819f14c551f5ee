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

from . import felis


def segments(n_windows: int, n_segments: int) -> list[list[int]]:
    """Window indices of each segment (boundaries from ``felis_segment_bounds``),
    each sharing its last window with the next one's first."""
    b = felis.segment_bounds(n_windows, n_segments)
    return [list(range(int(b[s]), int(b[s + 1]) + 1)) for s in range(n_segments)]


def segment_dg(ctx, u, n_k, temperature=300.0, tol=1e-10, max_iter=20000):
    """kT (f_last - f_first) of one segment from its own reduced potentials
    u[k][n] (device float64; the segment's states and frames only)."""
    f, _ = felis.mbar(ctx, u, n_k, tol=tol, max_iter=max_iter)
    return felis.delta_g(f, temperature)


def segment_dgs(ctx, u_segments, n_k_segments, temperature=300.0, tol=1e-10, max_iter=20000):
    """Each segment's MBAR difference, in segment order."""
    return [segment_dg(ctx, u, nk, temperature, tol, max_iter) for u, nk in zip(u_segments, n_k_segments)]


def binding_dg(dg_solvent_segments, dg_complex_segments, restraint_g0, restraint_k, temperature=300.0):
    """dG_bind from the two legs' segment free energies (coupled -> decoupled)
    and the restraint geometry and force constants of the complex leg."""
    return felis.binding_dg(dg_solvent_segments, dg_complex_segments, restraint_g0, restraint_k, temperature)
