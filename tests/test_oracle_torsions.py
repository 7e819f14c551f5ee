"""Pins of the oracle's rotatable-torsion term (section "Double annihilation
protocol": periodic torsions of rotatable bonds scaled linearly by the
alchemical parameter, read here as lambda_vdw).

* Hand-built geometries with known dihedral angles give the closed form
  k [1 + cos(n phi - delta)] (phi = +-60, 90, 180 degrees; both phases).
* Finite differences of the energy give the forces; net force and torque vanish.
* lambda_vdw = 0 gives exactly zero energy and force; the term is linear in lambda.
* u_kn of a frame differs between states by exactly the change of the window
  energies (the torsion term included).
"""
import numpy as np

from oracle import bonded, energy, ukn as U
from oracle.ewald import PME
from paper_2603_22274_amd import gen

from ._systems import point_charges


def _quad_system(phi_deg, k, n, delta):
    """Four atoms a-b-c-d with bond b-c along x and dihedral phi (IUPAC sign)."""
    ph = np.radians(phi_deg)
    pos = np.array([[10.0, 11.0, 10.0], [10.0, 10.0, 10.0], [11.5, 10.0, 10.0],
                    [11.5, 10.0 + np.cos(ph), 10.0 + np.sin(ph)]])
    s = point_charges(pos, np.zeros(4), [40.0] * 3, 5.0, 0.3)
    s.torsions = np.array([[0, 1, 2, 3]], np.int32)
    s.torsion_k = np.array([k], np.float32)
    s.torsion_n = np.array([n], np.int32)
    s.torsion_phase = np.array([delta], np.float32)
    return s, pos


def test_closed_form_on_hand_built_dihedrals():
    for phi in (60.0, -60.0, 90.0, 180.0):
        for n, delta in ((1, 0.0), (2, np.pi), (3, 0.0)):
            s, pos = _quad_system(phi, 2.0, n, delta)
            e, _ = bonded.torsions(pos, s, 1.0)
            # a = b + y, d = c + (0, cos phi, sin phi) with b -> c along x: the
            # dihedral is phi itself in the oracle's sign convention
            ref = 2.0 * (1.0 + np.cos(n * np.radians(phi) - float(np.float32(delta))))
            assert abs(e - ref) < 1e-12, (phi, n, delta, e, ref)


def _fd(fun, x, atoms, h=1e-5):
    out = np.zeros((len(atoms), 3))
    for k, a in enumerate(atoms):
        for d in range(3):
            xp = x.copy(); xp[a, d] += h
            xm = x.copy(); xm[a, d] -= h
            out[k, d] = -(fun(xp) - fun(xm)) / (2 * h)
    return out


def test_forces_finite_difference_newton_and_torque():
    s = gen.torsion_leg()
    rng = np.random.default_rng(2)
    x = s.pos.astype(np.float64)
    lig = np.where(s.is_ligand)[0]
    x[lig] += rng.normal(0, 0.2, (len(lig), 3))
    e, f = bonded.torsions(x, s, 0.6)
    assert e != 0.0
    fd = _fd(lambda y: bonded.torsions(y, s, 0.6)[0], x, list(lig))
    assert np.allclose(fd, f[lig], rtol=1e-6, atol=1e-7)
    assert np.abs(f.sum(0)).max() < 1e-10
    c = x[lig].mean(0)
    assert np.abs(np.cross(x[lig] - c, f[lig]).sum(0)).max() < 1e-9


def test_lambda_endpoints_and_linearity():
    s = gen.torsion_leg()
    x = s.pos.astype(np.float64)
    e0, f0 = bonded.torsions(x, s, 0.0)
    assert e0 == 0.0 and not f0.any()
    e1, f1 = bonded.torsions(x, s, 1.0)
    eh, fh = bonded.torsions(x, s, 0.25)
    assert abs(eh - 0.25 * e1) < 1e-12 * abs(e1) and np.allclose(fh, 0.25 * f1, rtol=1e-13, atol=0)


def test_ukn_differences_include_torsions():
    s = gen.torsion_leg()
    beta = 1.0 / (0.0019872043 * 300.0)
    pme = PME(s.box, s.grid, s.ewald_alpha)
    rng = np.random.default_rng(5)
    x = s.pos.astype(np.float64)
    lig = np.where(s.is_ligand)[0]
    x[lig] += rng.normal(0, 0.15, (len(lig), 3))
    windows = [0, 3, 4, 7, 11]
    u = U.ukn_frame(s, x, s.lambdas[windows], beta, pme)
    E = np.array([energy.window_energy(s, x, s.lambdas[w], pme=pme)[0]['total'] for w in windows])
    assert np.allclose((u - u[0]) / beta, E - E[0], rtol=1e-9, atol=1e-7)
    # the torsion term is a visible part of those differences
    et = np.array([bonded.torsions(x, s, s.lambdas[w][1])[0] for w in windows])
    assert np.ptp(et) > 1.0
