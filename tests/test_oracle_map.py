"""Pins for the oracle's binning, map and Jacobian.

* Binning against exact rational arithmetic (y = (k + 1/2)/2^32, b = floor(yN)).
* Uniform grid: the map is the identity and the Jacobian is one.
* Change of variables: with the random points replaced by a midpoint lattice in
  y, the oracle's estimator is a quadrature of f(x(y)) w(y) over [0,1]^d, which
  equals the integral of f over x for ANY grid; compared with scipy quadrature
  and with the erf closed form.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate, special


@pytest.mark.parametrize("N", [2, 7, 50, 100, 255])
def test_binning_exact(orc, N):
    ks = list(range(0, 2**32, 2**32 // 4099)) + [0, 1, 2**32 - 2, 2**32 - 1]
    # words whose y N lands next to an integer
    for b in range(1, N):
        k0 = (b * 2**32) // N
        ks += [max(0, k0 - 1), k0, min(2**32 - 1, k0 + 1)]
    for k in ks:
        y = (k + 0.5) / 2**32
        assert Fraction(y) == Fraction(2 * k + 1, 2**33)
        b, delta = orc.bin_of(y, N)
        exact = Fraction((2 * k + 1) * N, 2**33)
        assert b == exact.numerator // exact.denominator
        assert Fraction(delta) == exact - b
        assert 0 <= b < N


@pytest.mark.parametrize("N", [49, 50, 100])
def test_uniform_grid_is_identity(orc, N):
    d = 6
    E = orc.uniform_edges(d, N)
    rng = np.random.default_rng(1)
    for _ in range(200):
        y = (rng.integers(0, 2**32, d) + 0.5) / 2**32
        b, delta, x, w = orc.map_point(E, y)
        assert np.all(np.abs(x - y) <= 4 * np.finfo(float).eps)
        # each width fl((b+1)/N) - fl(b/N) is within eps of 1/N, i.e. N eps relative
        assert abs(w - 1.0) <= d * (N + 1) * np.finfo(float).eps


def _random_grid(rng, d, N):
    E = np.zeros((d, N + 1))
    for i in range(d):
        widths = rng.uniform(0.2, 3.0, N)
        c = np.concatenate([[0.0], np.cumsum(widths)])
        E[i] = c / c[-1]
        E[i, 0], E[i, -1] = 0.0, 1.0
    return E


def test_map_is_monotone_and_covers(orc):
    rng = np.random.default_rng(2)
    E = _random_grid(rng, 1, 13)
    ys = (np.arange(0, 2**32, 2**20) + 0.5) / 2**32
    xs = [orc.map_point(E, [y])[2][0] for y in ys]
    assert np.all(np.diff(xs) > 0)
    assert 0 < xs[0] < E[0, 1] and E[0, -2] < xs[-1] < 1


def _lattice_1d(K):
    return ((np.arange(K) + 0.5) / K).reshape(-1, 1)


@pytest.mark.parametrize("mu,a", [(0.5, 0.1), (0.3, 0.2), (0.15, 0.1)])
def test_lattice_quadrature_1d_any_grid(orc, mu, a):
    """sum over a midpoint lattice of f(x(y)) w(y) -> integral of f dx on a
    random non-uniform grid; reference is scipy quad and the erf closed form."""
    rng = np.random.default_rng(3)
    N = 50
    pr = orc.Problem(1, N, orc.GAUSS, [a, mu])
    exact = 0.5 * (special.erf((1 - mu) / a) + special.erf(mu / a))
    q, _ = integrate.quad(lambda x: np.exp(-((x - mu) / a) ** 2) / (a * np.sqrt(np.pi)), 0, 1,
                          epsabs=1e-14, epsrel=1e-14, limit=200)
    assert abs(q - exact) < 1e-12
    for E in (orc.uniform_edges(1, N), _random_grid(rng, 1, N)):
        K = 1000 * N                       # lattice aligned with the bins in y
        S1, S2, H = orc.accumulate_points(pr, E, _lattice_1d(K))
        est = S1 / K
        assert abs(est - exact) < 2e-8, (est, exact)
        # H sums v^2 per bin, so it adds up to S2
        assert abs(H.sum() - S2) <= 1e-12 * S2


def test_lattice_quadrature_2d_refined_grid(orc):
    rng = np.random.default_rng(4)
    N, a, mu = 20, 0.2, (0.4, 0.6)
    pr = orc.Problem(2, N, orc.GAUSS, [a, *mu])
    E = _random_grid(rng, 2, N)
    K = 40 * N
    g = (np.arange(K) + 0.5) / K
    Y = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    S1, S2, H = orc.accumulate_points(pr, E, Y)
    est = S1 / len(Y)
    exact = np.prod([0.5 * (special.erf((1 - m) / a) + special.erf(m / a)) for m in mu])
    q, _ = integrate.dblquad(lambda x2, x1: orc.integrand(pr, [x1, x2]), 0, 1, 0, 1,
                             epsabs=1e-12, epsrel=1e-12)
    assert abs(q - exact) < 1e-9
    assert abs(est - exact) < 5e-6
    assert np.allclose(H.sum(axis=1), S2, rtol=1e-12)


def test_jacobian_is_product_of_bin_widths(orc):
    """w = prod N (E_{b+1} - E_b): on a grid where one dimension's bins are
    halved/doubled, w scales accordingly, and the lattice estimate of a
    constant integrand is exactly one (the map covers [0,1]^d once)."""
    rng = np.random.default_rng(5)
    E = _random_grid(rng, 3, 8)
    pr = orc.Problem(3, 8, orc.GENZ_PEAK, [1e-6] * 3 + [0.5] * 3)   # ~constant (c tiny)
    K = 16
    g = (np.arange(K) + 0.5) / K
    Y = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    tot = 0.0
    for y in Y:
        b, de, x, w = orc.map_point(E, y)
        widths = [E[i, b[i] + 1] - E[i, b[i]] for i in range(3)]
        assert abs(w - np.prod(8 * np.array(widths))) < 1e-13 * w
        tot += w
    assert abs(tot / len(Y) - 1.0) < 1e-12
