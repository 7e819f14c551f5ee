"""Pins of the oracle's integrator, noise stream and constraints.

* Philox4x32-10 known-answer vectors (golden file, cited there).
* Free particles: <m v^2> = kT per degree of freedom (exact for the
  Ornstein-Uhlenbeck part of the step).
* Harmonic oscillators: <x^2> = kT / k (the middle scheme samples the exact
  configurational distribution of a harmonic potential).
* Rigid water: SHAKE meets every bond length to 1e-10 A; gamma = 0 gives a
  bounded total-energy drift.
"""
import copy
import math
import os

import numpy as np

from oracle import energy
from oracle.ewald import PME
from oracle.integrate import ACCEL, KB, langevin_middle_step, normals, philox4x32_10
from paper_2603_22274_amd import gen

from ._systems import point_charges

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden')


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, 'philox4x32_10_kat.txt')) if l.strip() and not l.startswith('#')]
    for r in rows:
        v = [int(t, 16) for t in r]
        out = philox4x32_10([np.array([c], np.uint64) for c in v[0:4]], [np.uint64(v[4]), np.uint64(v[5])])
        assert [int(o[0]) for o in out] == v[6:10]


def test_normals_moments():
    z = np.concatenate([normals(7, w, s, 5000) for w in range(3) for s in range(4)])
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1) < 0.01
    assert abs(np.mean(z ** 4) - 3) < 0.05


def _free_system(n, mass):
    s = point_charges(np.zeros((n, 3)), np.zeros(n), [1e3] * 3, 1.0, 0.1)
    s.mass = np.full(n, mass, np.float32)
    return s


def test_free_particle_kinetic_energy():
    n, m, T = 2000, 12.0, 300.0
    s = _free_system(n, m)
    x = np.zeros((n, 3)); v = np.zeros((n, 3))
    acc = []
    for step in range(400):
        x, v = langevin_middle_step(s, x, v, lambda y: np.zeros_like(y), 0.002, T, 50.0, 11, 0, step)
        if step >= 100:
            acc.append((v * v).mean())
    assert abs(np.mean(acc) / (KB * T * ACCEL / m) - 1) < 0.02


def test_harmonic_oscillator_position_variance():
    n, m, T, k = 2000, 12.0, 300.0, 10.0
    s = _free_system(n, m)
    x = np.zeros((n, 3)); v = np.zeros((n, 3))
    acc = []
    for step in range(700):
        x, v = langevin_middle_step(s, x, v, lambda y: -k * y, 0.005, T, 20.0, 5, 1, step)
        if step >= 100 and step % 5 == 0:
            acc.append((x * x).mean())
    assert abs(np.mean(acc) / (KB * T / k) - 1) < 0.02


def _water_box():
    s = gen.solvent_leg(config=9, n_waters=64, lattice_n=4, box_edge=12.4, n_lig=4, r_cut=6.0,
                        grid=(16, 16, 16), skin=0.0, sched='cfg0', keep_all_sites=True)
    return s


def test_shake_and_nve_drift():
    s = _water_box()
    pme = PME(s.box, s.grid, s.ewald_alpha)
    lam = (1.0, 1.0, 0.0)
    x = s.pos.astype(np.float64)
    v = np.zeros_like(x)
    m = s.mass.astype(np.float64)[:, None]
    # thermalise briefly with friction, then run gamma = 0
    force = lambda y: energy.window_energy(s, y, lam, pme=pme)[1]
    for step in range(20):
        x, v = langevin_middle_step(s, x, v, force, 0.001, 300.0, 20.0, 3, 0, step)
    o, h1, h2 = s.waters[:, 0], s.waters[:, 1], s.waters[:, 2]
    for a, b, d in ((o, h1, s.d_oh), (o, h2, s.d_oh), (h1, h2, s.d_hh)):
        assert np.max(np.abs(np.linalg.norm(x[a] - x[b], axis=1) - d)) < 1e-10
    tot = []
    ke_prev = 0.5 * (m * v * v).sum() / ACCEL
    for step in range(150):
        e, _ = energy.window_energy(s, x, lam, pme=pme)
        x, v = langevin_middle_step(s, x, v, force, 0.001, 300.0, 0.0, 3, 0, 100 + step)
        ke = 0.5 * (m * v * v).sum() / ACCEL
        tot.append(e['total'] + 0.5 * (ke + ke_prev))
        ke_prev = ke
    tot = np.array(tot)
    dof = 6 * len(s.waters) + 3 * 4 - 3
    slope = np.polyfit(np.arange(len(tot)) * 0.001, tot, 1)[0]      # kcal/mol/ps
    kin = 0.5 * dof * KB * 300
    assert abs(slope) / dof < 0.05                  # kcal/mol/ps per DOF
    assert np.std(tot) < 0.05 * kin
