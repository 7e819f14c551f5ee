"""Pins of the free-energy assembly oracle against the mathematics: the
analytic restraint term against a direct quadrature of the restrained
partition function (exact Jacobian r^2 sin(thA) sin(thB), exact cosine
dihedrals) in the stiff limit where the harmonic form becomes exact, and the
segmented MBAR sum against the closed-form free energies of harmonic
oscillators."""
import math

import numpy as np
from scipy import integrate, special

from oracle import estimator as oest

KB = oest.KB


def _quadrature_dg(g0, k, T):
    """-kT ln(Z_restrained / (8 pi^2 V0)) by one-dimensional quadratures."""
    beta = 1.0 / (KB * T)
    r0, ta, tb = g0[:3]
    sr = 1.0 / math.sqrt(beta * k[0])
    zr, _ = integrate.quad(lambda r: r * r * math.exp(-0.5 * beta * k[0] * (r - r0) ** 2),
                           max(0.0, r0 - 12 * sr), r0 + 12 * sr, epsabs=0, epsrel=1e-12, limit=200)
    za, _ = integrate.quad(lambda t: math.sin(t) * math.exp(-0.5 * beta * k[1] * (t - ta) ** 2), 0.0, math.pi,
                           epsabs=0, epsrel=1e-12, limit=200, points=[ta])
    zb, _ = integrate.quad(lambda t: math.sin(t) * math.exp(-0.5 * beta * k[2] * (t - tb) ** 2), 0.0, math.pi,
                           epsabs=0, epsrel=1e-12, limit=200, points=[tb])
    # int_0^{2pi} exp(-beta k (1 - cos x)) dx = 2 pi exp(-beta k) I0(beta k) = 2 pi ive(0, beta k)
    zphi = [2.0 * math.pi * special.ive(0, beta * kk) for kk in k[3:]]
    z = zr * za * zb * zphi[0] * zphi[1] * zphi[2]
    return -KB * T * math.log(z / (8.0 * math.pi ** 2 * oest.V0))


def test_restraint_term_matches_quadrature_in_the_stiff_limit():
    g0 = np.array([6.2, 1.35, 1.9, 0.4, -2.1, 1.0])
    base = np.array([2.0, 80.0, 80.0, 80.0, 80.0, 80.0])        # the paper's universal constants
    T = 298.15
    diffs = []
    for s in (1.0, 10.0, 100.0, 1000.0):
        k = base * s
        a = oest.boresch_restraint_dg(g0, k, T)
        q = _quadrature_dg(g0, k, T)
        assert a > 0 and q > 0                                   # restraining costs free energy
        diffs.append(abs(a - q))
    assert diffs[0] < 5e-3 and diffs[-1] < 1e-5, diffs
    assert diffs[0] > diffs[1] > diffs[2] > diffs[3], diffs     # the harmonic form converges


def test_restraint_term_scaling_laws():
    g0 = np.array([5.0, math.pi / 2, math.pi / 2, 0.0, 0.0, 0.0])
    k = np.full(6, 50.0)
    T = 300.0
    d0 = oest.boresch_restraint_dg(g0, k, T)
    # doubling every force constant adds 3 kT ln 2 (sqrt of 2^6)
    assert math.isclose(oest.boresch_restraint_dg(g0, 2 * k, T) - d0, 3 * KB * T * math.log(2), rel_tol=1e-12)
    # doubling r0 subtracts 2 kT ln 2 (r0^2 in the Jacobian)
    g1 = g0.copy(); g1[0] *= 2
    assert math.isclose(oest.boresch_restraint_dg(g1, k, T) - d0, -2 * KB * T * math.log(2), rel_tol=1e-12)


def test_segments_cover_the_path_with_shared_boundaries():
    s = oest.segments(13, 3)
    assert s == [[0, 1, 2, 3, 4], [4, 5, 6, 7, 8], [8, 9, 10, 11, 12]]
    assert oest.segments(5, 1) == [[0, 1, 2, 3, 4]]
    for W in range(3, 40):
        for n in range(1, W):
            segs = oest.segments(W, n)
            assert segs[0][0] == 0 and segs[-1][-1] == W - 1
            assert all(a[-1] == b[0] for a, b in zip(segs, segs[1:]))
            assert all(len(x) >= 2 for x in segs)


def test_segmented_mbar_sum_matches_harmonic_closed_form():
    # states U_k(x) = kap_k/2 (x - mu_k)^2 in 1D: f_k = -ln sqrt(2 pi / kap_k) + const
    rng = np.random.default_rng(5)
    kap = np.geomspace(1.0, 9.0, 9)
    mu = np.linspace(0.0, 0.6, 9)
    n = 4000
    T = 300.0
    kT = KB * T
    exact = kT * 0.5 * math.log(kap[-1] / kap[0])
    us, nks = [], []
    for seg in oest.segments(9, 3):
        x = np.concatenate([rng.normal(mu[k], 1.0 / math.sqrt(kap[k]), n) for k in seg])
        us.append(np.array([0.5 * kap[k] * (x - mu[k]) ** 2 for k in seg]))
        nks.append(np.full(len(seg), n))
    got = oest.segmented_dg(us, nks, T)
    assert abs(got - exact) < 0.02 * kT * 3, (got, exact)
