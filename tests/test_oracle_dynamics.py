"""Pins of the oracle's integrator, noise stream and constraints.

* Philox4x32-10 known-answer vectors (golden file, cited there).
* Free particles: <m v^2> = kT per degree of freedom (exact for the
  Ornstein-Uhlenbeck part of the step).
* Harmonic oscillators: <x^2> = kT / k (the middle scheme samples the exact
  configurational distribution of a harmonic potential).
* Rigid water: SHAKE meets every bond length to 1e-10 A; gamma = 0 gives a
  bounded total-energy drift.
* Velocity constraint after the kick: the three rates d|r_ab|^2/dt vanish,
  each water keeps its momentum and angular momentum, and the result equals
  the rigid-body projection V + omega x r written out independently below.
* Kinetic temperature of rigid waters under strong friction: the velocities
  a step leaves behind, projected on the 6 rigid-body degrees of freedom of
  each water, carry 3 kT per water (the reading "v = total constrained
  displacement / dt" gives about half of that).
* Smooth potential, gamma = 0: total energy conserved to 1e-4 kcal/mol/ps
  per degree of freedom; the step is time-reversible to 1e-9 A.
* At gamma = 0 positions do not depend on the velocity constraint after the
  kick (SHAKE moves atoms along the old bond vectors only, which absorbs any
  velocity component along them); with friction the stored velocity keeps
  (1 - a)/2 of such a component, which the next step's rotated bond vectors
  turn into a second-order difference.
"""
import copy
import math
import os

import numpy as np

from oracle import energy
from oracle.ewald import PME
from oracle import integrate as ointeg
from oracle.integrate import ACCEL, KB, constrain_velocities, langevin_middle_step, normals, philox4x32_10
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


def _rigid_projection(x, v, waters, mass):
    """Mass-weighted projection onto rigid-body motions, molecule by molecule:
    centre-of-mass velocity plus omega x r with I omega = L (an independent
    statement of the same projection the oracle solves by multipliers)."""
    out = np.array(v, np.float64, copy=True)
    m = np.asarray(mass, np.float64)
    for w in waters:
        idx = list(w)
        mm = m[idx]
        M = mm.sum()
        r = x[idx] - (mm[:, None] * x[idx]).sum(0) / M
        V = (mm[:, None] * v[idx]).sum(0) / M
        L = (mm[:, None] * np.cross(r, v[idx] - V)).sum(0)
        inertia = sum(mm[i] * (r[i] @ r[i] * np.eye(3) - np.outer(r[i], r[i])) for i in range(3))
        out[idx] = V + np.cross(np.linalg.solve(inertia, L), r)
    return out


def test_velocity_constraint_is_rigid_body_projection():
    s = _water_box()
    rng = np.random.default_rng(4)
    x = s.pos.astype(np.float64)
    v = rng.normal(0, 5.0, x.shape)
    vc = constrain_velocities(x, v, s.waters, s.mass, s.box)
    m = s.mass.astype(np.float64)
    for a, b in ((0, 1), (0, 2), (1, 2)):
        ia, ib = s.waters[:, a], s.waters[:, b]
        rate = ((x[ia] - x[ib]) * (vc[ia] - vc[ib])).sum(1)
        assert np.max(np.abs(rate)) < 1e-11
    for w in s.waters:
        idx = list(w)
        p0 = (m[idx, None] * v[idx]).sum(0)
        p1 = (m[idx, None] * vc[idx]).sum(0)
        assert np.allclose(p0, p1, atol=1e-11)
        c = (m[idx, None] * x[idx]).sum(0) / m[idx].sum()
        L0 = (m[idx, None] * np.cross(x[idx] - c, v[idx])).sum(0)
        L1 = (m[idx, None] * np.cross(x[idx] - c, vc[idx])).sum(0)
        assert np.allclose(L0, L1, atol=1e-10)
    assert np.allclose(vc, _rigid_projection(x, v, s.waters, s.mass), atol=1e-10)
    assert np.allclose(constrain_velocities(x, vc, s.waters, s.mass, s.box), vc, atol=1e-12)
    free = np.setdiff1d(np.arange(len(x)), s.waters.ravel())
    assert np.array_equal(vc[free], v[free])


def test_rigid_water_kinetic_temperature():
    """Non-interacting rigid waters at gamma = 20/ps: the stored velocities,
    projected on each water's rigid-body motions, hold 3 kT per water."""
    s = _water_box()
    T, gamma = 300.0, 20.0
    x = s.pos.astype(np.float64)
    v = np.zeros_like(x)
    zero = lambda y: np.zeros_like(y)
    acc = []
    for step in range(900):
        x, v = langevin_middle_step(s, x, v, zero, 0.002, T, gamma, 17, 0, step)
        if step >= 100:
            vp = _rigid_projection(x, v, s.waters, s.mass)[s.waters.ravel()]
            m = s.mass[s.waters.ravel()].astype(np.float64)[:, None]
            acc.append(0.5 * (m * vp * vp).sum() / ACCEL)
    ratio = np.mean(acc) / (3 * len(s.waters) * KB * T)
    assert abs(ratio - 1) < 0.03, ratio


def _tethered(s, k=20.0, seed=1):
    rng = np.random.default_rng(seed)
    anchor = s.pos.astype(np.float64) + rng.normal(0, 0.3, (s.n_atoms, 3))
    return (lambda y: 0.5 * k * ((y - anchor) ** 2).sum()), (lambda y: -k * (y - anchor))


def test_smooth_nve_and_time_reversibility():
    """Rigid waters (and free ligand atoms) tethered by smooth harmonic springs:
    at gamma = 0 the total energy (potential + mean kinetic energy of the
    projected velocities on either side of the positions) has no drift above
    1e-4 kcal/mol/ps per degree of freedom and fluctuates by < 1e-3 per
    degree of freedom at 2 fs; running the step backwards from the negated
    velocity returns to the start."""
    s = _water_box()
    pot, force = _tethered(s)
    m = s.mass.astype(np.float64)[:, None]
    x = s.pos.astype(np.float64)
    v = np.zeros_like(x)
    for step in range(50):
        x, v = langevin_middle_step(s, x, v, force, 0.002, 300.0, 20.0, 3, 0, step)
    x_start = x.copy()
    dt = 0.002
    tot = []
    kin = lambda vv: 0.5 * (m * constrain_velocities(x, vv, s.waters, s.mass, s.box) ** 2).sum() / ACCEL
    for step in range(800):
        e, v_prev = pot(x), v
        x, v = langevin_middle_step(s, x, v, force, dt, 300.0, 0.0, 3, 0, 100 + step)
        tot.append(e + 0.5 * (kin(v_prev) + kin(v)))
    dof = 6 * len(s.waters) + 3 * (s.n_atoms - 3 * len(s.waters))
    slope = np.polyfit(np.arange(len(tot)) * dt, tot, 1)[0]
    assert abs(slope) / dof < 1e-4, slope / dof
    assert np.std(tot) / dof < 1e-3, np.std(tot) / dof
    # reversal: the next kick must give -v back
    vr = -v - dt * force(x) * ACCEL / m
    for step in range(800):
        x, vr = langevin_middle_step(s, x, vr, force, dt, 300.0, 0.0, 3, 0, step)
    assert np.max(np.abs(x - x_start)) < 1e-9


def test_positions_independent_of_kick_projection(monkeypatch):
    """At gamma = 0, SHAKE along the old bond vectors absorbs a velocity
    component along them before the drift: the trajectory with the
    projection switched off matches to rounding."""
    s = _water_box()
    pot, force = _tethered(s)
    runs = []
    for on in (True, False):
        if not on:
            monkeypatch.setattr(ointeg, 'constrain_velocities', lambda x, v, *a: np.array(v, np.float64))
        x = s.pos.astype(np.float64)
        v = np.random.default_rng(2).normal(0, 3.0, x.shape)
        for step in range(40):
            x, v = ointeg.langevin_middle_step(s, x, v, force, 0.002, 300.0, 0.0, 9, 0, step)
        runs.append(x)
    assert np.max(np.abs(runs[0] - runs[1])) < 1e-9
