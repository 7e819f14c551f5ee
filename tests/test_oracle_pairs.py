"""Pins of the oracle's pair terms, list and bonded/restraint forces.

* Softcore at lambda = 1 reduces exactly to the textbook 12-6 LJ; at
  lambda = 0 it vanishes; at r -> 0 with lambda < 1 it stays finite.
* Lorentz-Berthelot mixing checked on hand-computed sigma_ij / eps_ij.
* System level: lambda_vdw = 1 equals treating no atom as alchemical;
  lambda_vdw = 0 equals switching the ligand's epsilon off.
* Neighbour list equals a periodic k-d tree query (scipy).
* Forces equal central finite differences; pair, bonded and restraint
  forces sum to zero (Newton's third law).
"""
import copy

import numpy as np
from scipy.spatial import cKDTree

from oracle import bonded, pairs
from paper_2603_22274_amd import gen

from ._systems import point_charges


def test_softcore_endpoints_and_textbook_lj():
    r = np.linspace(2.5, 9.5, 50)
    sig, eps = 3.3, 0.12
    e1, d1 = pairs.softcore_lj(r, sig, eps, 1.0, 0.5)
    lj = 4 * eps * ((sig / r) ** 12 - (sig / r) ** 6)
    dlj = 4 * eps * (-12 * sig ** 12 / r ** 13 + 6 * sig ** 6 / r ** 7)
    assert np.allclose(e1, lj, rtol=1e-13, atol=0)
    assert np.allclose(d1, dlj, rtol=1e-12, atol=0)
    e0, d0 = pairs.softcore_lj(r, sig, eps, 0.0, 0.5)
    assert np.all(e0 == 0) and np.all(d0 == 0)
    # finite at full overlap when lambda < 1: r_eff^6 = alpha (1 - lambda) sigma^6
    for lam in (0.2, 0.5, 0.9):
        e, de = pairs.softcore_lj(np.array([1e-12]), sig, eps, lam, 0.5)
        c = 0.5 * (1 - lam)
        assert np.isfinite(e[0]) and abs(e[0] - lam * 4 * eps * (1 / c ** 2 - 1 / c)) < 1e-9 * abs(e[0])
        assert abs(de[0]) < 1e-30


def test_lorentz_berthelot_two_atoms():
    # sigma 3.0 / 3.6 -> 3.3 ; eps 0.1 / 0.16 -> sqrt(0.016) = 0.12649110640673517
    s = point_charges([[1, 1, 1], [5.0, 1, 1]], [0.0, 0.0], [20.0] * 3, 9.0, 0.3,
                      sigma=[3.0, 3.6], eps=[0.1, 0.16])
    _, elj, f = pairs.real_space(s.pos, s, (1.0, 1.0, 0.0))
    r = 4.0
    ref = 4 * 0.12649110640673517 * ((3.3 / r) ** 12 - (3.3 / r) ** 6)
    assert abs(elj - ref) < 1e-6 * abs(ref)    # float32 parameters


def test_lambda_vdw_endpoints_system():
    s = gen.config0()
    lam1 = (0.3, 1.0, 0.0)
    ec_a, elj_a, f_a = pairs.real_space(s.pos, s, lam1)
    s_plain = copy.deepcopy(s)
    s_plain.is_ligand[:] = 0
    q64 = s.charge.astype(np.float64)
    s_plain.charge = np.where(s.is_ligand.astype(bool), q64 * 0.3, q64)
    ec_b, elj_b, f_b = pairs.real_space(s.pos, s_plain, (1.0, 1.0, 0.0))
    assert abs(elj_a - elj_b) < 1e-10 * abs(elj_a) and abs(ec_a - ec_b) < 1e-10 * abs(ec_a)
    assert np.allclose(f_a, f_b, rtol=1e-9, atol=1e-9)
    s_off = copy.deepcopy(s)
    s_off.epsilon = np.where(s.is_ligand.astype(bool), 0.0, s.epsilon).astype(np.float32)
    _, elj_c, _ = pairs.real_space(s.pos, s, (1.0, 0.0, 0.0))
    _, elj_d, _ = pairs.real_space(s.pos, s_off, (1.0, 1.0, 0.0))
    assert abs(elj_c - elj_d) < 1e-10 * abs(elj_d)


def test_neighbor_list_matches_kdtree():
    for s in (gen.config0(), gen.small_complex()):
        got = pairs.neighbor_pairs(s.pos, s.box, s, s.r_list)
        x = np.mod(s.pos.astype(np.float64), s.box)
        ref = cKDTree(x, boxsize=s.box).query_pairs(s.r_list, output_type='ndarray')
        ref = np.sort(ref, axis=1)
        ex = {tuple(e) for e in s.excl.tolist()}
        ref = {tuple(p) for p in ref.tolist() if tuple(p) not in ex}
        assert {tuple(p) for p in got.tolist()} == ref


def test_tree_list_equals_brute_force():
    """The k-d tree candidate form of the canonical list is the brute-force
    list itself (identical FP64 test), on jittered coordinates of two systems."""
    for s in (gen.config0(), gen.small_complex()):
        rng = np.random.default_rng(4)
        x = (s.pos + rng.normal(0, 0.05, s.pos.shape)).astype(np.float32)
        a = pairs.neighbor_pairs(x, s.box, s, s.r_list)
        b = pairs.neighbor_pairs_tree(x, s.box, s, s.r_list)
        assert a.shape == b.shape and np.array_equal(a, b)


def test_sampled_atoms_match_full_sum():
    s = gen.config0()
    lam = s.lambdas[7]
    ec, elj, f = pairs.real_space(s.pos, s, lam)
    atoms = np.array([0, 3, 19, 20, 300, 667])
    fo, eo = pairs.real_space_atoms(s.pos, s, lam, atoms)
    assert np.allclose(fo, f[atoms], rtol=1e-10, atol=1e-10)
    allf, alle = pairs.real_space_atoms(s.pos, s, lam, np.arange(s.n_atoms))
    assert abs(alle.sum() - (ec + elj)) < 1e-9 * abs(ec + elj)


def _fd(fun, x, atoms, h=1e-5):
    out = np.zeros((len(atoms), 3))
    for k, a in enumerate(atoms):
        for ax in range(3):
            xp = x.copy(); xp[a, ax] += h
            xm = x.copy(); xm[a, ax] -= h
            out[k, ax] = -(fun(xp) - fun(xm)) / (2 * h)
    return out


def test_pair_and_exclusion_forces_fd_and_newton():
    s = gen.config0()
    lam = (0.5, 0.4, 0.0)
    x = s.pos.astype(np.float64)
    ec, elj, f = pairs.real_space(x, s, lam)
    ex, fx = pairs.exclusion_correction(x, s, lam)
    atoms = [0, 1, 10, 19, 20, 21, 22, 500]
    fd = _fd(lambda y: sum(pairs.real_space(y, s, lam)[:2]) + pairs.exclusion_correction(y, s, lam)[0], x, atoms)
    assert np.allclose(fd, (f + fx)[atoms], rtol=1e-6, atol=2e-6)
    tot = f + fx
    assert np.abs(tot.sum(0)).max() < 1e-10 * np.abs(tot).sum()


def test_bonds_and_boresch_fd_and_newton():
    s = gen.small_complex()
    x = s.pos.astype(np.float64)
    eb, fb = bonded.bonds(x, s)
    er, fr = bonded.boresch(x, s, 0.7)
    # displace anchors so every restraint term has a non-zero gradient
    rng = np.random.default_rng(3)
    x[s.restraint_atoms] += rng.normal(0, 0.3, (6, 3))
    er, fr = bonded.boresch(x, s, 0.7)
    assert er > 0
    fd = _fd(lambda y: bonded.boresch(y, s, 0.7)[0], x, list(s.restraint_atoms))
    assert np.allclose(fd, fr[s.restraint_atoms], rtol=1e-6, atol=1e-7)
    assert np.abs(fr.sum(0)).max() < 1e-10
    atoms = [0, 1, 2, 200, int(s.restraint_atoms[3])]
    fd = _fd(lambda y: bonded.bonds(y, s)[0], x, atoms)
    eb, fb = bonded.bonds(x, s)
    assert np.allclose(fd, fb[atoms], rtol=1e-6, atol=1e-6)
    assert np.abs(fb.sum(0)).max() < 1e-9


def test_boresch_zero_at_reference_and_right_angle():
    s = gen.small_complex()
    e, f = bonded.boresch(s.pos.astype(np.float64), s, 1.0)
    assert abs(e) < 1e-8           # g0 is the initial geometry (float32 rounding only)
    # hand-built right-angle geometry (IUPAC sign, clockwise positive looking along
    # the central bond): thetaA = thetaB = 90 deg, phi(P2,P1,L1,L2) = -90 deg,
    # phi(P1,L1,L2,L3) = 180 deg, phi(L1,P1,P2,P3) = +90 deg
    t = copy.deepcopy(s)
    x = np.zeros((t.n_atoms, 3)) + 50.0
    p1, p2, p3, l1, l2, l3 = t.restraint_atoms
    x[p1] = [10, 10, 10]; x[l1] = [13, 10, 10]; x[l2] = [13, 12, 10]
    x[p2] = [10, 10, 12]; x[p3] = [10, 12, 12]; x[l3] = [15, 12, 10]
    t.restraint_g0 = np.array([3.0, np.pi / 2, np.pi / 2, -np.pi / 2, np.pi, np.pi / 2])
    e, _ = bonded.boresch(x, t, 1.0)
    assert abs(e) < 1e-12
