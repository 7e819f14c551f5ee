"""Pins of the oracle's Monte Carlo barostat (section "Simulation protocol":
NPT at 1.01325 bar, volume moves every 25 steps) against what does not come
from its own formulas: the ideal-gas isothermal-isobaric volume distribution
(a Gamma law), the gas constant at standard conditions, rigid-body invariants
of the molecule move, and the molecule count of the synthetic systems."""
import dataclasses

import numpy as np

from oracle import barostat as ob
from paper_2603_22274_amd import gen


def test_pressure_unit_gives_RT_for_a_molar_volume_of_ideal_gas():
    # 1 atm x 22.413969 L/mol = R x 273.15 K; per molecule: P V = kB T
    v_molecule = 22.413969e-3 / ob.AVOGADRO * 1e30          # A^3
    pv = 1.01325 * ob.BAR * v_molecule
    assert abs(pv - ob.KB * 273.15) <= 2e-5 * ob.KB * 273.15


def test_ideal_gas_volume_is_gamma_distributed():
    # With U = 0 the move samples p(V) ~ V^N exp(-beta P V): Gamma(N + 1,
    # beta P), mean (N + 1) kT / P, relative variance 1 / (N + 1).  A wrong
    # Jacobian count (atoms instead of molecules, or N + 1), a wrong sign of
    # P dV or an asymmetric proposal moves either moment far outside the bound.
    # The proposal width is held fixed: adapting it to the acceptance of a
    # volume that fluctuates by 50 % (an ideal gas of three molecules) makes
    # the width depend on the state and biases the chain; in a liquid the
    # volume moves by ~0.1 % and the adaptation only sets the step.
    rng = np.random.default_rng(11)
    n_mol, T, p_bar = 3, 300.0, 1.01325
    kT = ob.KB * T
    mean = (n_mol + 1) * kT / (p_bar * ob.BAR)
    chains, steps, burn = 4000, 2500, 500
    for width in (0.3, 0.6):
        v = np.full(chains, mean)
        samples = []
        for t in range(steps):
            v_new, _ = ob.propose(v, width * mean, rng.random(chains))
            ok = (v_new > 0) & ob.accepted(ob.work(0.0, v, np.where(v_new > 0, v_new, v), n_mol, p_bar, T),
                                            rng.random(chains), T)
            v = np.where(ok, v_new, v)
            if t >= burn:
                samples.append(v.copy())
        s = np.concatenate(samples)
        assert abs(s.mean() / mean - 1) < 0.01, (width, s.mean() / mean)
        assert abs(s.var() / s.mean() ** 2 * (n_mol + 1) - 1) < 0.04, (width, s.var() / s.mean() ** 2)


def test_molecules_of_the_synthetic_systems():
    s0 = gen.config0()
    mol, n = ob.molecules(s0)
    assert n == 216 + 1                                       # waters + the ligand chain
    lig = np.nonzero(s0.is_ligand)[0]
    assert len(set(mol[lig].tolist())) == 1
    sc = gen.small_complex()
    mol, n = ob.molecules(sc)
    n_ions = int(np.sum([1 for a in range(len(sc.charge)) if np.sum(mol == mol[a]) == 1]))
    assert n == len(sc.waters) + 2 + n_ions                  # protein chain, ligand, single-atom ions


def test_molecule_move_is_rigid_and_scales_centres():
    s = gen.config0()
    mol, n = ob.molecules(s)
    x = s.pos.astype(np.float64)
    y = ob.scale_molecules(x, mol, n, 1.013)
    for m in (0, 7, n - 1):
        a = np.nonzero(mol == m)[0]
        assert np.abs((y[a] - y[a[0]]) - (x[a] - x[a[0]])).max() < 1e-12
    c0, c1 = ob.centres(x, mol, n), ob.centres(y, mol, n)
    assert np.abs(c1 - 1.013 * c0).max() < 1e-11
    back = ob.scale_molecules(y, mol, n, 1.0 / 1.013)
    assert np.abs(back - x).max() < 1e-11


def test_zero_volume_change_is_accepted_and_changes_nothing():
    s = dataclasses.replace(gen.config0(), lambdas=gen.config0().lambdas[:1])
    r = ob.attempt(s, s.pos, s.box, s.lambdas[0], 100.0, 0.5, 0.999999)
    assert r['s'] == 1.0 and r['accepted'] and abs(r['w']) < 1e-9
    assert np.abs(r['x'] - s.pos.astype(np.float64)).max() == 0.0


def test_adaptation_steps():
    assert ob.adapt(10.0, 2, 10, 1e4) == 10.0 / 1.1
    assert ob.adapt(10.0, 8, 10, 1e4) == 11.0
    assert ob.adapt(2950.0, 8, 10, 1e4) == 3000.0
    assert ob.adapt(10.0, 5, 10, 1e4) == 10.0
    assert ob.adapt(10.0, 0, 9, 1e4) == 10.0


def test_draws_are_uniform_and_distinct_per_window_and_attempt():
    u = np.array([ob.draws(7, w, t) for w in range(20) for t in range(50)])
    assert u.min() >= 0 and u.max() < 1
    assert len(np.unique(u[:, 0])) == len(u)
    assert abs(u.mean() - 0.5) < 0.03
