"""Pins for the oracle's adjoint (d estimate / d integrand parameters).

* At fixed samples and a fixed grid the adjoint is the exact derivative of the
  estimator: central finite differences of the oracle's own estimate (FP64,
  h = 1e-4, denominator = the represented step) agree with it.
* Statistically it estimates the closed-form gradient of prod_i c(mu_i; a),
  c = [erf((1-mu)/a) + erf(mu/a)]/2 (within 5 sigma over independent batches).
"""
import numpy as np
import pytest
from scipy import special


def _c(mu, a):
    return 0.5 * (special.erf((1 - mu) / a) + special.erf(mu / a))


def _dc_dmu(mu, a):
    return (np.exp(-mu ** 2 / a ** 2) - np.exp(-(1 - mu) ** 2 / a ** 2)) / (a * np.sqrt(np.pi))


def _dc_da(mu, a):
    return -((1 - mu) * np.exp(-(1 - mu) ** 2 / a ** 2) + mu * np.exp(-mu ** 2 / a ** 2)) / (a ** 2 * np.sqrt(np.pi))


def _closed_grad(mu, a):
    c = np.array([_c(m, a) for m in mu])
    g = []
    for j in range(len(mu)):
        g.append(_dc_dmu(mu[j], a) * np.prod(np.delete(c, j)))
    g.append(sum(_dc_da(mu[j], a) * np.prod(np.delete(c, j)) for j in range(len(mu))))
    return np.array(g)


def test_closed_form_values():
    """Spot values of the one-dimensional factors at a = 0.1."""
    assert abs(_c(0.3, 0.1) - 0.99998895475150) < 1e-13
    assert abs(_dc_dmu(0.3, 0.1) - 6.96265259733739e-4) < 1e-15
    assert abs(_dc_dmu(0.15, 0.1) - 0.59465144611815) < 1e-12
    assert _dc_dmu(0.5, 0.1) == 0.0


def _adapted(orc, pr, n=100000, iters=5):
    res = orc.run(pr, orc.uniform_edges(pr.dim, pr.n_bins), iters, n, [1] * iters, [1] * iters)
    return res["edges"]


def test_fd_matches_adjoint(orc):
    d, a = 8, np.float32(0.1)
    mu = np.random.default_rng(0).uniform(0.3, 0.7, 8).astype(np.float32)
    pr = orc.Problem(d, 50, orc.GAUSS, [float(a), *map(float, mu)])
    E = _adapted(orc, pr, n=50000)
    M, t = 20000, 5
    G, Gabs = orc.adjoint(pr, E, t, M)
    h = 1e-4
    for j in range(d + 1):
        p_plus = np.array(pr.params, dtype=np.float64)
        p_minus = p_plus.copy()
        idx = 1 + j if j < d else 0
        p_plus[idx] += h
        p_minus[idx] -= h
        step = p_plus[idx] - p_minus[idx]
        Sp, _, _ = orc.accumulate(orc.Problem(d, 50, orc.GAUSS, p_plus), E, t, M)
        Sm, _, _ = orc.accumulate(orc.Problem(d, 50, orc.GAUSS, p_minus), E, t, M)
        fd = (Sp - Sm) / step
        assert abs(fd - G[j]) <= 1e-6 * Gabs[j], (j, fd, G[j], Gabs[j])


@pytest.mark.parametrize("mu0", [0.15, 0.3])
def test_statistical_vs_closed_form(orc, mu0):
    d, a = 4, 0.1
    mu = [mu0, 0.45, 0.5, 0.62]
    pr = orc.Problem(d, 50, orc.GAUSS, [a, *mu])
    E = _adapted(orc, pr)
    M, B = 50000, 20
    batches = np.array([orc.adjoint(pr, E, 100 + b, M)[0] / M for b in range(B)])
    est = batches.mean(axis=0)
    se = batches.std(axis=0, ddof=1) / np.sqrt(B)
    want = _closed_grad(np.array(mu), a)
    assert np.all(np.abs(est - want) <= 5 * se + 1e-12), (est, want, se)
    if mu0 == 0.15:
        assert abs(est[0] - want[0]) < 0.05 * abs(want[0])
