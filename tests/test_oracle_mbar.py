"""Pins of the oracle's MBAR and reduced potentials.

* Harmonic-oscillator windows sampled exactly: Delta f = (d/2) ln(k_K / k_1)
  for d Gaussian degrees of freedom, within 4 sigma of the estimate.
* Two states reduce to Bennett's acceptance ratio; a state with no samples
  reduces to the Zwanzig (EXP) estimator; sum_n W_nk = 1 at convergence;
  f is invariant under u_kn += c_n.
* u_kn: differences between windows equal differences of the full window
  potential (the split into E_LE, E_LL, E_sc and U_B drops nothing that
  depends on lambda).
"""
import numpy as np

from oracle import energy, mbar as M, ukn as U
from oracle.ewald import PME
from paper_2603_22274_amd import gen


def _harmonic_samples(ks, n_per, d=3, seed=0):
    rng = np.random.default_rng(seed)
    xs = [rng.normal(0, 1 / np.sqrt(k), (n_per, d)) for k in ks]      # beta = 1
    x2 = np.concatenate([(x * x).sum(1) for x in xs])
    u = 0.5 * np.array(ks)[:, None] * x2[None, :]
    return u, np.full(len(ks), n_per)


def test_mbar_harmonic_analytic():
    ks = [1.0, 1.6, 2.5, 4.0, 6.4]
    u, N = _harmonic_samples(ks, 3000)
    f, it = M.mbar(u, N)
    exact = 1.5 * np.log(np.array(ks) / ks[0])
    # spread over independent replicates gives the statistical scale
    reps = [M.mbar(*_harmonic_samples(ks, 3000, seed=s))[0][-1] for s in range(1, 9)]
    sd = np.std(reps)
    assert abs(f[-1] - exact[-1]) < 4 * sd + 1e-3
    assert np.all(np.abs(f - exact) < 0.05)


def test_mbar_two_states_is_bar():
    u, N = _harmonic_samples([1.0, 1.8], 2000, seed=4)
    f, _ = M.mbar(u, N, tol=1e-13)
    wf = u[1, :2000] - u[0, :2000]
    wr = u[0, 2000:] - u[1, 2000:]
    assert abs(f[1] - M.bar(wf, wr)) < 1e-9


def test_mbar_unsampled_state_is_exp():
    u, _ = _harmonic_samples([1.0, 1.5], 4000, seed=5)
    u = u[:, :4000]
    f, _ = M.mbar(u, [4000, 0], tol=1e-13)
    assert abs(f[1] - M.exp_estimator(u[1] - u[0])) < 1e-10


def test_mbar_weights_and_shift_invariance():
    ks = [1.0, 1.4, 2.0]
    u, N = _harmonic_samples(ks, 1500, seed=6)
    f, _ = M.mbar(u, N, tol=1e-13)
    W = M.weights(u, N, f)
    assert np.allclose(W.sum(1), 1.0, atol=1e-9)
    c = np.random.default_rng(1).normal(0, 5, u.shape[1])
    f2, _ = M.mbar(u + c[None, :], N, tol=1e-13)
    assert np.allclose(f, f2, atol=1e-9)


def _check_ukn_vs_energy(s, windows, beta=1.0 / (0.0019872043 * 300.0)):
    pme = PME(s.box, s.grid, s.ewald_alpha)
    x = s.pos.astype(np.float64)
    u = U.ukn_frame(s, x, s.lambdas[windows], beta, pme)
    E = np.array([energy.window_energy(s, x, s.lambdas[w], pme=pme)[0]['total'] for w in windows])
    du = (u - u[0]) / beta
    dE = E - E[0]
    assert np.allclose(du, dE, rtol=1e-9, atol=1e-7), (du, dE)


def test_ukn_matches_window_energy_solvent():
    s = gen.config0()
    _check_ukn_vs_energy(s, [0, 2, 4, 6, 11])


def test_ukn_matches_window_energy_complex():
    s = gen.small_complex()
    _check_ukn_vs_energy(s, [0, 5, 12, 17, 25, 41])
