"""Pins for the oracle's iteration statistics, combination and integrands.

* Combination: a hand-worked example; m = 1 gives the iteration itself and
  chi^2/dof = NaN; equal variances give the arithmetic mean.
* Integrands: the oracle's f integrates (scipy quad) to the closed forms of
  sec. 3.1 (erf products for the Gaussians, elementary ones for Genz), and the
  Gaussian is a product of one-dimensional factors.
* Estimator and variance: over many seeds the pulls (I_t - I_exact)/sigma_t are
  standard normal, and a full adaptive run lands within 5 sigma of erf(1/2a)^d.
"""
import os

import numpy as np
import pytest
from scipy import integrate, special

HERE = os.path.dirname(os.path.abspath(__file__))


def test_combine_worked_example(orc):
    with open(os.path.join(HERE, "golden", "combine_worked_example.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    I, v, want = [[float(x) for x in part.split()] for part in rows[0].split("|")]
    got = orc.combine(I, v)
    assert np.allclose(got, want, rtol=1e-14, atol=0)


def test_combine_special_cases(orc):
    I, s, c = orc.combine([0.7], [0.09])
    assert abs(I - 0.7) < 4e-16 and abs(s - 0.3) < 1e-16 and np.isnan(c)
    I, s, c = orc.combine([1.0, 2.0, 3.0, 6.0], [0.5] * 4)
    assert abs(I - 3.0) < 1e-15 and abs(s - np.sqrt(0.5 / 4)) < 1e-16


def test_iteration_stats_definition(orc):
    # 4 events with v = 1, 2, 3, 6: mean 3, sample variance 14/3, variance of the mean 7/6
    v = np.array([1.0, 2.0, 3.0, 6.0])
    I, var = orc.iteration_stats(v.sum(), (v * v).sum(), 4)
    assert I == 3.0 and abs(var - np.var(v, ddof=1) / 4) < 1e-15


def _c(mu, a):
    return 0.5 * (special.erf((1 - mu) / a) + special.erf(mu / a))


@pytest.mark.parametrize("mu,a", [(0.5, 0.1), (0.3, 0.05), (0.15, 0.2)])
def test_gauss_integral_1d(orc, mu, a):
    pr = orc.Problem(1, 50, orc.GAUSS, [a, mu])
    q, _ = integrate.quad(lambda x: orc.integrand(pr, [x]), 0, 1, points=[mu], epsabs=1e-15, epsrel=1e-13)
    assert abs(q - _c(mu, a)) < 1e-12


def test_gauss_separable(orc):
    rng = np.random.default_rng(0)
    mu = rng.uniform(0.3, 0.7, 3)
    pr3 = orc.Problem(3, 50, orc.GAUSS, [0.1, *mu])
    for _ in range(20):
        x = rng.uniform(0, 1, 3)
        f1 = [orc.integrand(orc.Problem(1, 50, orc.GAUSS, [0.1, mu[i]]), [x[i]]) for i in range(3)]
        assert abs(orc.integrand(pr3, x) - np.prod(f1)) <= 1e-14 * max(np.prod(f1), 1e-300)


def test_bimodal_integral_1d(orc):
    a = 0.05
    pr = orc.Problem(1, 100, orc.BIMODAL, [a, 1 / 3, 2 / 3])
    q, _ = integrate.quad(lambda x: orc.integrand(pr, [x]), 0, 1, points=[1 / 3, 2 / 3],
                          epsabs=1e-15, epsrel=1e-13)
    assert abs(q - 0.5 * (_c(1 / 3, a) + _c(2 / 3, a))) < 1e-12
    # d = 20 closed form: both terms give prod c = c^20
    c = 0.5 * (special.erf(40 / 3) + special.erf(20 / 3))
    assert abs(c ** 20 - 1.0) < 1e-15


def test_genz_integrals_1d(orc):
    c, a = 3.0, 0.3
    pr = orc.Problem(1, 50, orc.GENZ_DISC, [c, a])
    q, _ = integrate.quad(lambda x: orc.integrand(pr, [x]), 0, 1, points=[a], epsabs=1e-15, epsrel=1e-13)
    assert abs(q - 1.0) < 1e-12
    assert orc.integrand(pr, [a]) == 0.0 and orc.integrand(pr, [a - 1e-9]) == 0.0
    assert abs(orc.integrand(pr, [0.9]) - c * np.exp(c * 0.9) / (np.exp(c) - np.exp(c * a))) < 1e-12
    pr = orc.Problem(1, 50, orc.GENZ_PEAK, [5.0, 0.4])
    q, _ = integrate.quad(lambda x: orc.integrand(pr, [x]), 0, 1, points=[0.4], epsabs=1e-15, epsrel=1e-13)
    assert abs(q - 1.0) < 1e-12


def test_pulls_are_standard_normal(orc):
    """(I_t - I)/sigma_t over 200 seeds, d = 2, M = 1e4, fixed uniform grid."""
    d, a, M = 2, 0.1, 10000
    exact = _c(0.5, a) ** d
    E = orc.uniform_edges(d, 50)
    pulls = []
    for seed in range(200):
        pr = orc.Problem(d, 50, orc.GAUSS, [a, 0.5, 0.5], seed=seed)
        S1, S2, _ = orc.accumulate(pr, E, 0, M)
        I, var = orc.iteration_stats(S1, S2, M)
        pulls.append((I - exact) / np.sqrt(var))
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 0.25
    assert 0.85 < pulls.std(ddof=1) < 1.15


def test_adaptive_run_hits_closed_form(orc):
    """Plain FP64 Vegas at d = 4, a = 0.1, N = 50, alpha = 1.5, 10 x 1e5 events,
    refining after every iteration and combining all ten."""
    d = 4
    pr = orc.Problem(d, 50, orc.GAUSS, [0.1] + [0.5] * d)
    res = orc.run(pr, orc.uniform_edges(d, 50), 10, 100000, [1] * 10, [1] * 10)
    I, sigma, chi2 = res["final"]
    exact = _c(0.5, 0.1) ** d
    assert abs(I - exact) < 5 * sigma
    assert sigma < 2e-3                       # adaptation worked: plain MC gives ~1.2e-2
    assert chi2 < 5.0
    E = res["edges"]
    assert np.all(np.diff(E, axis=1) > 0) and np.all(E[:, 0] == 0) and np.all(E[:, -1] == 1)
    # the adapted grid concentrates bins around the peak at 0.5
    w = np.diff(E, axis=1)
    assert np.all(w[:, 25] < 0.5 / 50) and np.all(w[:, 0] > 2.0 / 50)


# ---------------------------------------------------------------------------
# Parameter layouts at d > 1 (sec. 3.1: Eq. lepage and its two-centre form,
# Eq. genzdisc, Eq. productpeak), with a different value in every dimension so
# that a parameter read from the wrong slot changes the result.

MU_A3 = [0.2, 0.35, 0.6]
MU_B3 = [0.7, 0.55, 0.25]
GENZ3 = {"disc": ([0.7, 1.9, 1.2], [0.12, 0.31, 0.05]),
         "peak": ([4.0, 2.5, 6.0], [0.45, 0.62, 0.3])}


def _nested_quad(f, pts0, pts1):
    """Integral over [0,1]^2 of f(x0, x1), as two nested adaptive quadratures
    with the integrand's break points."""
    inner = lambda x0: integrate.quad(lambda x1: f(x0, x1), 0, 1, points=pts1, epsabs=1e-14,
                                      epsrel=1e-12, limit=200)[0]
    return integrate.quad(inner, 0, 1, points=pts0, epsabs=1e-14, epsrel=1e-12, limit=200)[0]


def test_bimodal_is_mean_of_two_gaussians_d3(orc):
    """The two-centre integrand equals the mean of the one-centre Gaussians
    (each pinned by separability and quadrature) at its two centres."""
    d, a = 3, 0.13
    pr = orc.Problem(d, 50, orc.BIMODAL, [a, *MU_A3, *MU_B3])
    ga = orc.Problem(d, 50, orc.GAUSS, [a, *MU_A3])
    gb = orc.Problem(d, 50, orc.GAUSS, [a, *MU_B3])
    rng = np.random.default_rng(5)
    pts = np.concatenate([rng.uniform(0, 1, (30, d)),
                          np.array(MU_A3) + rng.normal(0, 0.05, (15, d)),
                          np.array(MU_B3) + rng.normal(0, 0.05, (15, d))]).clip(0, 1)
    for x in pts:
        want = 0.5 * (orc.integrand(ga, x) + orc.integrand(gb, x))
        got = orc.integrand(pr, x)
        assert abs(got - want) <= 1e-14 * want, (x, got, want)


def test_bimodal_integral_d2(orc):
    """d = 2, distinct centres per dimension: quadrature of the oracle's f equals
    1/2 [c(muA_0) c(muA_1) + c(muB_0) c(muB_1)] (each Gaussian term integrates to
    a product of erf factors)."""
    a, mA, mB = 0.11, [0.3, 0.62], [0.71, 0.18]
    pr = orc.Problem(2, 50, orc.BIMODAL, [a, *mA, *mB])
    q = _nested_quad(lambda x0, x1: orc.integrand(pr, [x0, x1]), [mA[0], mB[0]], [mA[1], mB[1]])
    want = 0.5 * (_c(mA[0], a) * _c(mA[1], a) + _c(mB[0], a) * _c(mB[1], a))
    assert abs(q - want) < 1e-10, (q, want)


@pytest.mark.parametrize("kind", ["disc", "peak"])
def test_genz_separable_d3(orc, kind):
    """The d = 3 Genz integrand (normalisation included) is the product of the
    one-dimensional ones with each dimension's own c_i, a_i."""
    kid = orc.GENZ_DISC if kind == "disc" else orc.GENZ_PEAK
    c, th = GENZ3[kind]
    d = 3
    pr = orc.Problem(d, 50, kid, [*c, *th])
    ones = [orc.Problem(1, 50, kid, [c[i], th[i]]) for i in range(d)]
    rng = np.random.default_rng(9)
    for _ in range(40):
        x = rng.uniform(0, 1, d)
        if kind == "disc":   # mostly inside, where f > 0
            x = np.array(th) + (1 - np.array(th)) * rng.uniform(0, 1, d) if rng.uniform() < 0.8 else x
        want = np.prod([orc.integrand(ones[i], [x[i]]) for i in range(d)])
        got = orc.integrand(pr, x)
        assert abs(got - want) <= 1e-14 * max(want, 1e-300), (x, got, want)
    if kind == "disc":
        # zero exactly when some x_i <= a_i, for each dimension separately
        for i in range(d):
            x = np.array(th) + 0.5 * (1 - np.array(th))
            x[i] = th[i]
            assert orc.integrand(pr, x) == 0.0
            x[i] = th[i] + 1e-9
            assert orc.integrand(pr, x) > 0.0


@pytest.mark.parametrize("kind", ["disc", "peak"])
def test_genz_integral_d2(orc, kind):
    """d = 2 with distinct c_i, a_i: the normalisation makes the integral one."""
    kid = orc.GENZ_DISC if kind == "disc" else orc.GENZ_PEAK
    c, th = ([1.4, 0.6], [0.22, 0.08]) if kind == "disc" else ([3.5, 5.0], [0.35, 0.7])
    pr = orc.Problem(2, 50, kid, [*c, *th])
    q = _nested_quad(lambda x0, x1: orc.integrand(pr, [x0, x1]), [th[0]], [th[1]])
    assert abs(q - 1.0) < 1e-10, q
