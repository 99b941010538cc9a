"""Pins for the oracle's grid refinement.

Hand-worked examples (tests/golden/refine_worked_examples.txt) and invariants
that hold for the refinement whatever the input: end edges are kept exactly,
edges increase strictly, a flat histogram leaves ANY grid unchanged, the
result is invariant under scaling of the histogram, mirror-symmetric under
reversing it, alpha = 0 with no empty smoothed bin is a fixed point, an
all-zero histogram leaves the grid alone, and with alpha = 0 the new edges
split the support of the smoothed histogram into N parts of equal "old-bin"
count (a closed form).
"""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _examples():
    rows = []
    with open(os.path.join(HERE, "golden", "refine_worked_examples.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, h, e = line.split("|")
            rows.append((float(a), [float(v) for v in h.split()], [float(v) for v in e.split()]))
    return rows


def test_worked_examples(orc):
    rows = _examples()
    assert len(rows) == 3
    for alpha, h, want in rows:
        E = orc.uniform_edges(1, 4)
        got = orc.refine(np.array([h]), E, alpha)[0]
        assert np.allclose(got, want, rtol=0, atol=1e-14), (got, want)


def test_damping_limits(orc):
    assert orc.damp(0.0, 1.5) == 0.0
    assert orc.damp(1.0, 1.5) == 1.0
    # continuous at s -> 1 (limit of (s-1)/ln s is 1) and increasing
    assert abs(orc.damp(1 - 1e-9, 1.5) - 1.0) < 1e-8
    s = np.linspace(1e-6, 0.999, 200)
    r = [orc.damp(v, 1.5) for v in s]
    assert np.all(np.diff(r) > 0)
    # (s - 1)/ln s at s = 1/e is (1 - 1/e)
    assert abs(orc.damp(np.exp(-1.0), 1.0) - (1 - np.exp(-1.0))) < 1e-15


def _random_grid(rng, d, N):
    E = np.zeros((d, N + 1))
    for i in range(d):
        c = np.concatenate([[0.0], np.cumsum(rng.uniform(0.1, 4.0, N))])
        E[i] = c / c[-1]
        E[i, 0], E[i, -1] = 0.0, 1.0
    return E


@pytest.mark.parametrize("N", [2, 3, 7, 50, 100, 255])
def test_invariants(orc, N):
    rng = np.random.default_rng(N)
    d = 5
    E = _random_grid(rng, d, N)
    H = rng.exponential(1.0, (d, N)) ** 3
    H[1, : N // 2] = 0.0                        # empty bins
    H[2] = 0.0
    H[2, N // 3] = 1.0                          # one non-empty bin
    En = orc.refine(H, E, 1.5)
    assert np.all(En[:, 0] == 0.0) and np.all(En[:, -1] == 1.0)
    assert np.all(np.diff(En, axis=1) > 0)
    # scale invariance
    assert np.allclose(orc.refine(H * 1e-30, E, 1.5), En, rtol=0, atol=1e-15)
    assert np.allclose(orc.refine(H * 7.5e20, E, 1.5), En, rtol=0, atol=1e-15)
    # flat histogram: fixed point for any grid (up to the rounding of the
    # cumulative sum of N equal terms, which grows like N eps)
    tol = 4 * N * np.finfo(float).eps
    assert np.allclose(orc.refine(np.full((d, N), 3.0), E, 1.5), E, rtol=0, atol=tol)
    # alpha = 0 and every smoothed bin non-empty: fixed point
    Hp = rng.uniform(0.5, 2.0, (d, N))
    assert np.allclose(orc.refine(Hp, E, 0.0), E, rtol=0, atol=tol)
    # all-zero histogram: grid unchanged, bit for bit
    Z = np.zeros((d, N))
    assert np.array_equal(orc.refine(Z, E, 1.5), E)


@pytest.mark.parametrize("N", [4, 10, 50])
def test_reflection(orc, N):
    rng = np.random.default_rng(7)
    H = rng.exponential(1.0, (3, N))
    E = orc.uniform_edges(3, N)
    A = orc.refine(H, E, 1.5)
    B = orc.refine(H[:, ::-1].copy(), E, 1.5)
    assert np.allclose(A, 1.0 - B[:, ::-1], rtol=0, atol=1e-14)


def test_alpha0_equal_count_closed_form(orc):
    """alpha = 0: r = 1 on bins whose smoothed value is non-zero, 0 elsewhere.
    The new edge k then sits at old-bin coordinate lo + k (hi - lo)/N, mapped
    linearly through the old grid, where [lo, hi) is the run of non-empty
    smoothed bins."""
    rng = np.random.default_rng(11)
    N = 20
    E = _random_grid(rng, 1, N)
    H = np.zeros((1, N))
    H[0, 6:9] = [1.0, 5.0, 2.0]                 # smoothed support: bins 5..9
    lo, hi = 5, 10
    En = orc.refine(H, E, 0.0)[0]
    for k in range(1, N):
        u = lo + k * (hi - lo) / N              # position in old-bin units
        b = int(np.floor(u))
        if u == b and b > lo:                   # left-most crossing: end of bin b-1
            b -= 1
        want = E[0, b] + (u - b) * (E[0, b + 1] - E[0, b])
        assert abs(En[k] - want) < 1e-14, (k, En[k], want)


def test_nonfinite_histogram_keeps_the_grid(orc):
    """A dimension whose histogram holds an infinity or a NaN (an integrand that
    overflowed) has nothing finite to adapt to and keeps its edges, as an empty
    one does; the other dimensions refine as usual."""
    rng = np.random.default_rng(3)
    d, N = 4, 20
    E = _random_grid(rng, d, N)
    H = rng.exponential(1.0, (d, N))
    H[0, 3] = np.inf
    H[1, 7] = np.nan
    H[2, :] = 0.0
    En = orc.refine(H, E, 1.5)
    assert np.array_equal(En[:3], E[:3])
    ref3 = orc.refine(H[3:], E[3:], 1.5)
    assert np.array_equal(En[3], ref3[0]) and not np.array_equal(En[3], E[3])
    # a finite total that is too large to smooth (the smoothed sum overflows)
    H2 = np.full((1, N), 1.7e308)
    assert np.array_equal(orc.refine(H2, E[:1], 1.5), E[:1])
