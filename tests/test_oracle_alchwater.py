"""Pins of the oracle's alchemical waters (section "Double annihilation
protocol": charged ligands decoupled with designated waters taking up the
fractional charge, each offset within -0.4 ... +0.6 e, their number fixed
across windows).

* The net charge of every window equals the coupled state's (zero for the
  synthetic legs, whose counter-ion neutralises the ligand); every offset of
  every window lies within [-0.4, 0.6] e; the offsets vanish at lambda_elec = 1.
* The count is the fewest waters within that range at lambda_elec = 0.
* u_kn of a frame differs between states exactly as the direct window
  energies (charges scaled per window, offsets included) do, for ligands of
  either sign: this pins the bilinear decomposition E[a,a] + 2 lam E[a,b] +
  lam^2 E[b,b] against the plain definition.
* Forces at an intermediate lambda_elec are the energy's finite differences.
"""
import numpy as np
import pytest

from oracle import energy, pairs, ukn as U
from oracle.ewald import PME
from paper_2603_22274_amd import gen


@pytest.mark.parametrize('q_lig', [1.0, -1.0, 2.0])
def test_neutral_windows_and_offset_range(q_lig):
    s = gen.charged_leg(q_ligand=q_lig)
    n_aw = int(np.count_nonzero(s.alch_offset))
    assert n_aw == gen.alchemical_water_count(q_lig)
    assert n_aw == {1.0: 2, -1.0: 3, 2.0: 4}[q_lig]
    aw = np.nonzero(s.alch_offset)[0]
    assert all(a in s.waters[:, 0] for a in aw)                  # oxygens of waters
    q_coupled = pairs.scaled_charges(s, 1.0)
    assert np.array_equal(q_coupled, s.charge.astype(np.float64))
    assert abs(q_coupled.sum()) < 1e-5
    for lam_e in np.unique(s.lambdas[:, 0]):
        q = pairs.scaled_charges(s, lam_e)
        assert abs(q.sum() - q_coupled.sum()) < 1e-6, lam_e
        offs = q[aw] - s.charge[aw]
        assert np.all(offs >= -0.4 - 1e-7) and np.all(offs <= 0.6 + 1e-7), offs


@pytest.mark.parametrize('q_lig', [1.0, -1.0])
def test_ukn_differences_match_window_energies(q_lig):
    s = gen.charged_leg(q_ligand=q_lig)
    beta = 1.0 / (0.0019872043 * 300.0)
    pme = PME(s.box, s.grid, s.ewald_alpha)
    rng = np.random.default_rng(6)
    x = s.pos.astype(np.float64) + rng.normal(0, 0.02, (s.n_atoms, 3))
    u = U.ukn_frame(s, x, s.lambdas, beta, pme)
    E = np.array([energy.window_energy(s, x, lam, pme=pme)[0]['total'] for lam in s.lambdas])
    assert np.allclose((u - u[0]) / beta, E - E[0], rtol=1e-9, atol=1e-7)
    # the offsets change the electrostatic windows by a visible amount
    s0 = gen.charged_leg(q_ligand=q_lig)
    s0.alch_offset = np.zeros_like(s0.alch_offset)
    E0 = np.array([energy.window_energy(s0, x, lam, pme=pme)[0]['total'] for lam in s.lambdas[:5]])
    assert np.max(np.abs((E[:5] - E[0]) - (E0 - E0[0]))) > 1.0


def test_forces_finite_difference_intermediate_lambda():
    s = gen.charged_leg()
    pme = PME(s.box, s.grid, s.ewald_alpha)
    lam = (0.4, 1.0, 0.0)
    x = s.pos.astype(np.float64)
    _, f = energy.window_energy(s, x, lam, pme=pme)
    aw = np.nonzero(s.alch_offset)[0]
    atoms = list(aw) + [0, 5, int(s.waters[7, 1])]
    h = 1e-5
    for a in atoms:
        for d in range(3):
            xp = x.copy(); xp[a, d] += h
            xm = x.copy(); xm[a, d] -= h
            fd = -(energy.window_energy(s, xp, lam, pme=pme)[0]['total'] -
                   energy.window_energy(s, xm, lam, pme=pme)[0]['total']) / (2 * h)
            # PME forces are the analytic gradient of the PME energy
            assert abs(fd - f[a, d]) < 1e-5 * max(1.0, abs(f[a, d])), (a, d, fd, f[a, d])
