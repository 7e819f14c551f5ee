"""Pins of the oracle's Ewald pieces against values fixed by mathematics.

* NaCl rock-salt Madelung constant 1.747565 (real + reciprocal + self).
* Wigner constant xi = 2.837297 of a single charge with neutralising
  background in a cubic box (reciprocal + self + background).
* Independence of the total Ewald energy from the splitting parameter
  (pins the sign and weight of the excluded-pair correction and self term).
* Smooth PME converges to the direct Ewald sum as grid and order grow.
"""
import numpy as np

from oracle import energy, pairs
from oracle.ewald import PME, direct_ewald, bspline, bspline_moduli
from paper_2603_22274_amd import gen

from ._systems import point_charges, rocksalt

MADELUNG_NACL = 1.747565
WIGNER_SC = 2.837297


def _ewald_total(sysd, pos, alpha):
    sysd.ewald_alpha = alpha
    lam = (1.0, 1.0, 0.0)
    ec, _, f = pairs.real_space(pos, sysd, lam)
    ex, fx = pairs.exclusion_correction(pos, sysd, lam)
    es = pairs.self_and_background(sysd, lam)
    q = pairs.scaled_charges(sysd, 1.0)
    er, fr = direct_ewald(np.asarray(pos, np.float64), q, sysd.box, alpha)
    return ec + ex + es + er, f + fx + fr


def test_madelung_rocksalt():
    P, q, box = rocksalt(8, 2.82)
    s = point_charges(P, q, box, r_cut=9.0, alpha=0.5)
    e, f = _ewald_total(s, s.pos, 0.5)
    expect = -256 * MADELUNG_NACL * pairs.KE / 2.82
    assert abs(e / expect - 1) < 5e-7
    assert np.max(np.abs(f)) < 1e-4


def test_wigner_single_charge():
    s = point_charges([[1.0, 2.0, 3.0]], [1.0], [10.0] * 3, r_cut=4.9, alpha=0.8)
    e, f = _ewald_total(s, s.pos, 0.8)
    expect = -WIGNER_SC * pairs.KE / (2 * 10.0)
    assert abs(e / expect - 1) < 5e-7
    assert np.max(np.abs(f)) < 1e-9


def test_alpha_independence_with_exclusions():
    s = gen.config0()
    s.epsilon[:] = 0
    e1, f1 = _ewald_total(s, s.pos, 0.45)
    e2, f2 = _ewald_total(s, s.pos, 0.55)
    assert abs(e1 - e2) < 1e-7 * abs(e1)
    assert np.sqrt(((f1 - f2) ** 2).sum() / (f1 ** 2).sum()) < 1e-6


def test_net_force_zero_direct_ewald():
    s = gen.config0()
    _, f = _ewald_total(s, s.pos, s.ewald_alpha)
    assert np.abs(f.sum(0)).max() < 1e-8 * np.abs(f).sum()


def test_bspline_partition_of_unity_and_moduli():
    u = np.linspace(0, 1, 17)[:-1]
    for n in (4, 5, 6):
        tot = sum(bspline(u + j, n) for j in range(n))
        assert np.allclose(tot, 1.0, atol=1e-14)
    # order-4 moduli: |sum_k M4(k+1) e^{i w k}|^2 = ((2 + cos w) / 3)^2
    K = 20
    w = 2 * np.pi * np.arange(K) / K
    assert np.allclose(bspline_moduli(K, 4), 1.0 / ((2 + np.cos(w)) / 3) ** 2, rtol=1e-13)


def test_pme_converges_to_direct_ewald():
    s = gen.config0()
    x = s.pos.astype(np.float64)
    q = pairs.scaled_charges(s, 1.0)
    e_ref, f_ref = direct_ewald(x, q, s.box, s.ewald_alpha)
    errs = []
    for K, n in ((20, 4), (32, 4), (32, 6)):
        e, f = PME(s.box, (K, K, K), s.ewald_alpha, n).energy_forces(x, q)
        errs.append((abs(e - e_ref) / abs(e_ref), np.sqrt(((f - f_ref) ** 2).sum() / (f_ref ** 2).sum())))
    # configured grid (20^3, order 4) within the Ewald-tolerance level
    assert errs[0][1] < 5e-3 and errs[0][0] < 5e-3
    assert errs[1][1] < errs[0][1] and errs[2][1] < errs[1][1]
    assert errs[2][1] < 1e-5 and errs[2][0] < 1e-5


def test_pme_energy_equals_half_q_phi_and_translation():
    s = gen.config0()
    x = s.pos.astype(np.float64)
    q = pairs.scaled_charges(s, 1.0)
    pme = PME(s.box, s.grid, s.ewald_alpha)
    Q = pme.spread(x, q)
    phi = pme.potential(Q)
    assert abs(0.5 * (Q * phi).sum() / pme.energy_of_grids(Q) - 1) < 1e-12
    # translation by a whole grid spacing is exact
    shift = s.box / np.array(s.grid)
    e0, _ = pme.energy_forces(x, q)
    e1, _ = pme.energy_forces(x + shift, q)
    assert abs(e1 - e0) < 1e-9 * abs(e0)


def test_total_forces_finite_difference():
    s = gen.config0()
    lam = s.lambdas[6]          # lambda_elec 0, lambda_vdw 5/7: softcore active
    pme = PME(s.box, s.grid, s.ewald_alpha)
    x = s.pos.astype(np.float64)
    _, f = energy.window_energy(s, x, lam, pme=pme)
    h = 1e-5
    for a in (0, 5, 100, 401):
        for ax in range(3):
            xp = x.copy(); xp[a, ax] += h
            xm = x.copy(); xm[a, ax] -= h
            ep, _ = energy.window_energy(s, xp, lam, pme=pme)
            em, _ = energy.window_energy(s, xm, lam, pme=pme)
            fd = -(ep['total'] - em['total']) / (2 * h)
            assert abs(fd - f[a, ax]) < 2e-5 + 1e-6 * abs(f[a, ax]), (a, ax, fd, f[a, ax])
