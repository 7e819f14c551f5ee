"""Monte Carlo barostat (FP64) -- test infrastructure: only the tests and the
CPU baseline use this module.

Section "Simulation protocol" samples NPT at 1.01325 bar with a Monte Carlo
barostat attempted every 25 MD steps (OpenMM) and prints nothing more about
the move.  Reading used here: the isotropic volume move of OpenMM's Monte
Carlo barostat (Chow & Ferguson 1995; Aqvist et al. 2004), applied to every
window (replica) on its own:

  proposal    V' = V + dV_max (2 u1 - 1),  s = (V'/V)^(1/3),  box L' = s L
  move        every molecule is translated rigidly so that its centre, the
              mean of its atoms' positions, goes from c to s c
  criterion   w = U(x', L') - U(x, L) + P (V' - V) - N_mol kT ln(V'/V);
              accepted when w <= 0 or u2 < exp(-w / kT); a rejected move
              restores x and L (velocities are never scaled)
  adaptation  after every 10 attempts of a window, dV_max is divided by 1.1
              when fewer than a quarter were accepted and multiplied by 1.1
              (at most 0.3 V) when more than three quarters were

Molecules are the connected components of the bond graph in which each rigid
water's three atoms are joined.  The pressure term makes a window's reduced
potential u = beta (U + P V).

u1 and u2 are inputs.  ``draws`` gives the ones the HIP path uses: Philox4x32-10
(Salmon et al. 2011) with counter (window, 0x4241524F, attempt_lo, attempt_hi)
and the leg's seed as key; u1 = ((w0 >> 5) 2^26 + (w1 >> 6)) 2^-53 and u2 the
same from (w2, w3).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import energy as oenergy
from .integrate import philox4x32_10

KB = 0.0019872043                    # kcal / (mol K)
AVOGADRO = 6.02214076e23
BAR = 1.0e5 * 1.0e-30 * AVOGADRO / 4184.0   # 1 bar in kcal / (mol A^3)
_TAG = 0x4241524F


def molecules(sysd):
    """(mol_id per atom, number of molecules): connected components of the
    bonds plus the O-H1 and O-H2 links of every rigid water."""
    n = len(sysd.charge)
    parent = np.arange(n)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    edges = [tuple(b) for b in np.asarray(sysd.bonds).reshape(-1, 2)]
    for o, h1, h2 in np.asarray(sysd.waters).reshape(-1, 3):
        edges += [(o, h1), (o, h2)]
    for a, b in edges:
        ra, rb = find(int(a)), find(int(b))
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(a) for a in range(n)])
    _, mol = np.unique(roots, return_inverse=True)   # numbered by their lowest atom
    return mol.astype(np.int64), int(mol.max()) + 1


def centres(x, mol, n_mol):
    """(n_mol, 3) mean position of each molecule's atoms."""
    x = np.asarray(x, np.float64)
    c = np.zeros((n_mol, 3))
    np.add.at(c, mol, x)
    return c / np.bincount(mol, minlength=n_mol)[:, None]


def scale_molecules(x, mol, n_mol, s):
    """Rigid translation of every molecule: centre c -> s c."""
    x = np.asarray(x, np.float64)
    return x + (s - 1.0) * centres(x, mol, n_mol)[mol]


def propose(volume, dv_max, u1):
    """(V', s) for the uniform u1 in [0, 1); works on arrays."""
    v_new = volume + dv_max * (2.0 * np.asarray(u1, np.float64) - 1.0)
    return v_new, np.cbrt(v_new / volume)


def work(du, volume, v_new, n_mol, pressure_bar, temperature):
    """w = dU + P dV - N_mol kT ln(V'/V) (kcal/mol); works on arrays."""
    kT = KB * temperature
    return du + pressure_bar * BAR * (v_new - volume) - n_mol * kT * np.log(v_new / volume)


def accepted(w, u2, temperature):
    """Metropolis test of the work w with the uniform u2; works on arrays."""
    w = np.asarray(w, np.float64)
    with np.errstate(over='ignore'):
        return (w <= 0.0) | (np.asarray(u2) < np.exp(-w / (KB * temperature)))


def adapt(dv_max, n_accepted, n_attempted, volume):
    """dV_max after a block of 10 attempts (unchanged before that)."""
    if n_attempted < 10:
        return dv_max
    rate = n_accepted / n_attempted
    if rate < 0.25:
        return dv_max / 1.1
    if rate > 0.75:
        return min(dv_max * 1.1, 0.3 * volume)
    return dv_max


def draws(seed, window, attempt):
    """(u1, u2) of one window's attempt from the leg's Philox stream."""
    ctr = (np.uint64(window), np.uint64(_TAG), np.uint64(attempt & 0xFFFFFFFF),
           np.uint64((attempt >> 32) & 0xFFFFFFFF))
    key = (np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    w = [int(v) for v in philox4x32_10(ctr, key).reshape(4)]
    u1 = ((w[0] >> 5) * 2.0 ** 26 + (w[1] >> 6)) * 2.0 ** -53
    u2 = ((w[2] >> 5) * 2.0 ** 26 + (w[3] >> 6)) * 2.0 ** -53
    return u1, u2


def total_energy(sysd, x, box, lam):
    """U of one window in the box ``box`` (PME at the system's grid)."""
    s = dataclasses.replace(sysd, box=np.asarray(box, np.float64))
    return oenergy.window_energy(s, x, lam)[0]['total']


def attempt(sysd, x, box, lam, dv_max, u1, u2, pressure_bar=1.01325, temperature=300.0, energy_fn=None):
    """One volume move of one window.  Returns a dict with the new positions
    and box (the old ones if rejected), U0, U1, w, s and the decision."""
    energy_fn = energy_fn or total_energy
    box = np.asarray(box, np.float64)
    x = np.asarray(x, np.float64)
    mol, n_mol = molecules(sysd)
    volume = float(np.prod(box))
    v_new, s = propose(volume, dv_max, u1)
    v_new, s = float(v_new), float(s)
    x_new = scale_molecules(x, mol, n_mol, s)
    box_new = s * box
    u0 = energy_fn(sysd, x, box, lam)
    u1e = energy_fn(sysd, x_new, box_new, lam)
    w = float(work(u1e - u0, volume, v_new, n_mol, pressure_bar, temperature))
    ok = bool(accepted(w, u2, temperature))
    return {'x': x_new if ok else x, 'box': box_new if ok else box, 'accepted': ok, 'U0': u0, 'U1': u1e,
            'w': w, 's': s, 'x_trial': x_new, 'box_trial': box_new, 'n_mol': n_mol}
