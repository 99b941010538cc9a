"""Pins of oracle.accumulate_fn, the accumulator for integrands given as NumPy
functions (user integrands): it must reduce to counting on the uniform grid,
agree with the oracle's own Gaussian accumulator, and hit closed forms."""
import numpy as np

import oracle


def test_constant_integrand_counts_events():
    """f = 1 on the uniform grid: w = 1 up to the rounding of the widths
    (k+1)/N - k/N, so S1 = S2 = n and H[i][b] is the number of events whose
    coordinate i falls in bin b, counted here from the Philox points alone."""
    d, N, n, seed = 3, 7, 2000, 5
    E = oracle.uniform_edges(d, N)
    S1, S2, H = oracle.accumulate_fn(d, N, seed, 0, E, 2, n, lambda x: np.ones(len(x)))
    tol = 8 * d * np.finfo(float).eps * n
    assert abs(S1 - n) <= tol and abs(S2 - n) <= 2 * tol
    counts = np.zeros((d, N))
    for e in range(n):
        y = oracle.point(seed, 2, 0, e, d)
        for i in range(d):
            counts[i, int(np.floor(y[i] * N))] += 1
    assert np.all(np.abs(H - counts) <= 1e-12 * n)


def test_gaussian_as_numpy_equals_builtin_accumulator():
    """The Gaussian written as a NumPy function gives the oracle's own
    Gaussian accumulator (C, compensated sums) on an adapted grid."""
    d, N, n = 4, 30, 20000
    params = [0.15, 0.3, 0.45, 0.6, 0.7]
    pr = oracle.Problem(d, N, oracle.GAUSS, params, seed=9, problem=2)
    E = oracle.run(pr, oracle.uniform_edges(d, N), 3, 5000, [1] * 3, [1] * 3)["edges"]
    nu = oracle.norm(pr)
    mu = np.array(params[1:])

    def f(x):
        return nu * np.exp(-((x - mu) ** 2).sum(axis=1) / params[0] ** 2)

    a1, a2, Ha = oracle.accumulate_fn(d, N, 9, 2, E, 4, n, f)
    b1, b2, Hb = oracle.accumulate(pr, E, 4, n)
    assert abs(a1 - b1) <= 1e-13 * b1 and abs(a2 - b2) <= 1e-13 * b2
    assert np.all(np.abs(Ha - Hb) <= 1e-13 * Hb.sum(axis=1, keepdims=True))


def test_product_integrand_closed_form_on_refined_grid():
    """prod x_i over [0,1]^3 is 1/8: the estimate S1/n on a refined grid lies
    within 5 standard errors, and sum |v| equals S1 for a positive f."""
    d, N, n = 3, 20, 50000
    pr = oracle.Problem(d, N, oracle.GAUSS, [0.2, 0.7, 0.7, 0.7])
    E = oracle.run(pr, oracle.uniform_edges(d, N), 2, 5000, [1, 1], [1, 1])["edges"]
    S1, S2, H, A = oracle.accumulate_fn(d, N, 0, 0, E, 0, n, lambda x: x.prod(axis=1), with_abs=True)
    I, var = oracle.iteration_stats(S1, S2, n)
    assert abs(I - 0.125) < 5 * var ** 0.5
    assert A == S1
    assert np.allclose(H.sum(axis=1), S2, rtol=1e-13)
