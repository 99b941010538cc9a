"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same points.

Tolerances (FP64 path 1e-12 relative, FP32-mixed path 1e-6 relative, both
before error propagation):
* per-event records: bins exact; FP64 delta exact, x within 4 ulp, w and f to
  rounding level; FP32 delta is RN32 of the FP64 delta (even N), x/w/f to FP32
  rounding level;
* per-iteration sums S1, S2 relative; histograms per dimension normalised by
  that dimension's total (|dH| <= tol * sum_b H);
* refinement: the library's new edges against the oracle's refinement of the
  library's own histograms and edges, absolute;
* whole runs (FP64): combined integral, error and final edges.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2002_12921_amd import Vegas

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps


def _gauss(d, a=0.1, mu=0.5):
    mus = [mu] * d if np.isscalar(mu) else list(mu)
    return [a] + mus


def _adapted_edges(d, N, params, kind=oracle.GAUSS, iters=3, n=20000):
    pr = oracle.Problem(d, N, kind, params)
    r = oracle.run(pr, oracle.uniform_edges(d, N), iters, n, [1] * iters, [1] * iters)
    return r["edges"]


def _exponent(kind, params, x):
    """The integrand's exponent at the oracle's points (natural units): the
    size of the argument whose rounding sets the relative error of f."""
    d = x.shape[1]
    if kind == "gauss":
        a, mu = params[0], np.array(params[1:1 + d])
        return ((x - mu) ** 2).sum(axis=1) / a ** 2
    if kind == "bimodal":
        a, ma, mb = params[0], np.array(params[1:1 + d]), np.array(params[1 + d:])
        return np.minimum(((x - ma) ** 2).sum(axis=1), ((x - mb) ** 2).sum(axis=1)) / a ** 2
    if kind == "genz_disc":
        c, th = np.array(params[:d]), np.array(params[d:])
        return np.abs(((x - th) * c).sum(axis=1))
    return np.zeros(len(x))


def _centres(kind, params, d):
    """The per-dimension centre the FP32 table is offset from."""
    if kind in ("gauss", "bimodal"):
        return np.array(params[1:1 + d])
    return np.array(params[d:2 * d])


def _check_events(ev_gpu, ev_or, d, mixed, kind="gauss", params=None, N=50, E=None):
    """Per-event bounds.  FP64: delta exact, x to 4 ulp, w to 4d ulp, f to
    eps (16 + 4 (8 + d) A) with A the integrand's exponent.  FP32: delta is
    (RN32(lo) + h)/2^32, i.e. RN32 of the exact delta for even N and within
    one FP32 ulp of it for odd N; with w the bin's width and u = x - c the
    offset from the table's centre, x carries at most 2^-24 (3 w + 2 |u|)
    (the table's offset |u| + w, RN32(lo) w, RN32(w) w, the fma |u|); f
    carries 2^-24 (8 + 4d + (8 + d) A) and w 2^-24 (2d + 4)."""
    b_g, b_o = ev_gpu[:, :d], ev_or[:, :d]
    assert np.array_equal(b_g, b_o), "bins differ"
    de_g, de_o = ev_gpu[:, d:2 * d], ev_or[:, d:2 * d]
    x_g, x_o = ev_gpu[:, 2 * d:3 * d], ev_or[:, 2 * d:3 * d]
    w_g, w_o = ev_gpu[:, 3 * d], ev_or[:, 3 * d]
    f_g, f_o = ev_gpu[:, 3 * d + 1], ev_or[:, 3 * d + 1]
    A = _exponent(kind, params, x_o) if params is not None else np.zeros(len(x_o))
    big = f_o > 1e-280
    rel = np.abs(f_g[big] - f_o[big]) / f_o[big]
    if not mixed:
        assert np.array_equal(de_g, de_o)
        assert np.max(np.abs(x_g - x_o)) <= 4 * EPS64
        assert np.max(np.abs(w_g - w_o) / w_o) <= 4 * d * EPS64
        assert np.all(rel <= EPS64 * (16 + 4 * (8 + d) * A[big]))
    else:
        if N % 2 == 0:
            assert np.array_equal(de_g, de_o.astype(np.float32).astype(np.float64))
        else:
            assert np.all(np.abs(de_g - de_o) <= np.spacing(de_o.astype(np.float32)).astype(np.float64))
        E = oracle.uniform_edges(d, N) if E is None else np.asarray(E)
        bi = b_o.astype(np.int64)
        width = np.stack([np.diff(E[i])[bi[:, i]] for i in range(d)], axis=1)
        u = np.abs(x_o - _centres(kind, params, d)[None, :])
        assert np.all(np.abs(x_g - x_o) <= 2.0 ** -24 * (3 * width + 2 * u) * 1.001 + 4 * EPS64)
        assert np.max(np.abs(w_g - w_o) / w_o) <= (2 * d + 4) * 2.0 ** -24
        assert np.all(rel <= 2.0 ** -24 * (8 + 4 * d + (8 + d) * A[big]))


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("d,N", [(4, 50), (8, 50), (5, 7), (1, 2), (20, 100), (13, 255)])
def test_event_records(prec, d, N):
    params = _gauss(d, 0.1, np.linspace(0.3, 0.7, d))
    v = Vegas(d, N, "gauss", params, prec, seed=12345)
    E = _adapted_edges(d, N, params)
    v.set_edges(E)
    t, first, count = 3, 1000, 4096 + 37
    got = v.dump_events(first, count, iteration=t).cpu().numpy()
    ref = oracle.events(oracle.Problem(d, N, oracle.GAUSS, params, seed=12345), E, t, first, count)
    _check_events(got, ref, d, prec != "fp64", "gauss", params, N, E)


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("kind,params_fn", [
    ("bimodal", lambda d: [0.05] + [1 / 3] * d + [2 / 3] * d),
    ("genz_peak", lambda d: list(np.linspace(3, 6, d)) + list(np.linspace(0.2, 0.8, d))),
    ("genz_disc", lambda d: list(np.linspace(1, 3, d)) + list(np.linspace(0.05, 0.3, d))),
])
def test_event_records_other_integrands(prec, kind, params_fn):
    d, N = 6, 40
    params = params_fn(d)
    kid = {"bimodal": oracle.BIMODAL, "genz_peak": oracle.GENZ_PEAK, "genz_disc": oracle.GENZ_DISC}[kind]
    v = Vegas(d, N, kind, params, prec, seed=7, problem=3)
    got = v.dump_events(0, 3000, iteration=2).cpu().numpy()
    ref = oracle.events(oracle.Problem(d, N, kid, params, seed=7, problem=3), oracle.uniform_edges(d, N), 2, 0, 3000)
    if kind == "genz_disc":
        # x_i > a_i is decided as the FP64 x decides it, in both precisions
        assert np.array_equal(got[:, 3 * d + 1] == 0.0, ref[:, 3 * d + 1] == 0.0)
    _check_events(got, ref, d, prec != "fp64", kind, params, N)


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("N", [40, 7])
def test_genz_disc_decision_at_the_threshold(prec, N):
    """The discontinuous integrand's x_i > a_i decision at the boundary itself,
    one dimension at a time on an adapted grid: a_i is set to the FP64 x_i of
    one event (which then lies on the threshold and is outside) or to the
    next double below it (inside), the other thresholds low enough for that
    event to be inside there; every dumped event's decision equals the
    oracle's, that event's included, in both precisions (even N: delta exact
    in FP32 too; odd N: with the half-step h), and so do the sums."""
    d, M, t = 5, 20_000, 3
    c = list(np.linspace(1.0, 2.0, d))
    kid = oracle.GENZ_DISC
    E = _adapted_edges(d, N, c + [0.3] * d, kind=kid, iters=2, n=20_000)
    x = oracle.events(oracle.Problem(d, N, kid, c + [0.02] * d, seed=11), E, t, 0, M)[:, 2 * d:3 * d]
    tol = 1e-12 if prec == "fp64" else 1e-6
    for i in range(d):
        others = np.all(np.delete(x, i, axis=1) > 0.02, axis=1)
        k = int(np.flatnonzero(others & (x[:, i] > 0.1) & (x[:, i] < 0.9))[i])
        for below in (False, True):
            a = [0.02] * d
            a[i] = float(np.nextafter(x[k, i], -np.inf)) if below else float(x[k, i])
            params = c + a
            pr = oracle.Problem(d, N, kid, params, seed=11)
            v = Vegas(d, N, "genz_disc", params, prec, seed=11)
            v.set_edges(E)
            got = v.dump_events(0, M, iteration=t).cpu().numpy()
            ref = oracle.events(pr, E, t, 0, M)
            assert (ref[k, 3 * d + 1] != 0.0) == below
            assert np.array_equal(got[:, 3 * d + 1] == 0.0, ref[:, 3 * d + 1] == 0.0), (prec, N, i, below)
            v.iterate(M)
            S1, S2, H = v.last_iteration()
            o1, o2, Ho = oracle.accumulate(pr, E, 0, M)
            assert abs(S1 - o1) <= tol * abs(o1) and abs(S2 - o2) <= tol * abs(o2)
            assert _hist_close(H, Ho, tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("N", [40, 7])
def test_genz_disc_extreme_thresholds(prec, N):
    """The ends of the x_i > a_i decision: a_i = 0, where every event is
    inside (the event's word k need only be >= 0), and a_i the largest double
    below 1 in one dimension, where no event is (the bin's threshold lies past
    its last event, so the integrand is zero everywhere and so are the sums);
    decisions and sums against the oracle's, on the uniform and on an adapted
    grid."""
    d, M, t = 5, 20_000, 2
    c = list(np.linspace(1.0, 2.0, d))
    kid = oracle.GENZ_DISC
    tol = 1e-12 if prec == "fp64" else 1e-6
    E_ad = _adapted_edges(d, N, c + [0.3] * d, kind=kid, iters=2, n=20_000)
    for E in (oracle.uniform_edges(d, N), E_ad):
        for case in ("all", "none"):
            a = [0.0] * d
            if case == "none":
                a[2] = float(np.nextafter(1.0, 0.0))
            params = c + a
            pr = oracle.Problem(d, N, kid, params, seed=5)
            v = Vegas(d, N, "genz_disc", params, prec, seed=5)
            v.set_edges(E)
            got = v.dump_events(0, M, iteration=t).cpu().numpy()
            ref = oracle.events(pr, E, t, 0, M)
            inside_ref = ref[:, 3 * d + 1] != 0.0
            assert inside_ref.all() if case == "all" else not inside_ref.any()
            assert np.array_equal(got[:, 3 * d + 1] != 0.0, inside_ref), (prec, N, case)
            v.iterate(M)
            S1, S2, H = v.last_iteration()
            o1, o2, Ho = oracle.accumulate(pr, E, 0, M)
            if case == "none":
                assert S1 == 0.0 and S2 == 0.0 and o1 == 0.0 and not np.any(H)
            else:
                assert abs(S1 - o1) <= tol * abs(o1) and abs(S2 - o2) <= tol * abs(o2)
                assert _hist_close(H, Ho, tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_event_index_beyond_2_32(prec):
    """Events whose index needs the counter's second word (e >= 2^32): event
    records straddling 2^32 against the oracle's, one by one, and an
    iteration of 2^32 + 10^5 events in two chunks, the second straddling
    2^32, whose sums less those of the first chunk alone (a twin context
    running it as a whole iteration, same launch, so the same partial sums)
    equal the oracle's sums over the straddling events: within the path's
    tolerance plus the rounding of the large totals (half an ulp each)."""
    d, N = 8, 50
    params = _gauss(d, 0.1, np.linspace(0.35, 0.65, d))
    mixed = prec != "fp64"
    tol = 1e-6 if mixed else 1e-12
    pr = oracle.Problem(d, N, oracle.GAUSS, params)
    E0 = oracle.uniform_edges(d, N)
    first, count = 2 ** 32 - 100_000, 200_000
    v = Vegas(d, N, "gauss", params, prec)
    got = v.dump_events(first + count // 2 - 2000, 4000, iteration=0).cpu().numpy()
    ref = oracle.events(pr, E0, 0, first + count // 2 - 2000, 4000)
    _check_events(got, ref, d, mixed, "gauss", params, N)
    v.iterate(first, chunk="begin")
    v.iterate(count, chunk="end")
    S1x, S2x, Hx = v.last_iteration()
    w = Vegas(d, N, "gauss", params, prec)
    w.iterate(first)
    S1y, S2y, Hy = w.last_iteration()
    o1, o2, Ho = oracle.accumulate(pr, E0, 0, count, first)
    ulp = np.spacing
    assert abs((S1x - S1y) - o1) <= tol * abs(o1) + ulp(S1x) + ulp(S1y), (S1x - S1y, o1)
    assert abs((S2x - S2y) - o2) <= tol * abs(o2) + ulp(S2x) + ulp(S2y), (S2x - S2y, o2)
    # histograms: the first chunk's bins come from atomics in no fixed order,
    # so the two contexts' first-chunk bins agree to a few ulps of the bin
    slack = 4 * (ulp(Hx) + ulp(Hy))
    assert np.all(np.abs((Hx - Hy) - Ho) <= tol * Ho.sum(axis=1, keepdims=True) + slack)
    assert Ho.sum() > 0 and o1 > 0


def _hist_close(Hg, Ho, tol):
    tot = Ho.sum(axis=1, keepdims=True)
    return np.all(np.abs(Hg - Ho) <= tol * tot)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32_mixed", 1e-6)])
@pytest.mark.parametrize("d,N", [(4, 64), (8, 13), (8, 50), (8, 65), (5, 50), (3, 7), (12, 50), (16, 33)])
def test_histogram_layouts(prec, tol, d, N):
    """Sums and histograms with 16 replicas per bin (the fixed-stride layout
    where d is 4, 8, 12 or 16 and N <= 64), with one copy, and with the
    automatic choice, each against the oracle on the same adapted grid."""
    params = _gauss(d, mu=0.37)
    E = _adapted_edges(d, N, params)
    M = 300_007
    pr = oracle.Problem(d, N, oracle.GAUSS, params)
    o1, o2, Ho = oracle.accumulate(pr, E, 0, M)
    for rep in (16, 1, 0):
        v = Vegas(d, N, "gauss", params, prec)
        v.set_edges(E)
        v.set_hist_replicas(rep)
        v.iterate(M, combine=False)
        S1, S2, H = v.last_iteration()
        assert abs(S1 - o1) <= tol * abs(o1), (rep, S1, o1)
        assert abs(S2 - o2) <= tol * abs(o2), (rep, S2, o2)
        assert _hist_close(H, Ho, tol), rep
        assert H.sum() > 0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32_mixed", 1e-6)])
def test_lockstep_iterations(prec, tol):
    """Per iteration: sums and histograms vs the oracle on the library's own
    grid, then the refinement vs the oracle's refinement of the library's
    histograms."""
    d, N, M = 8, 50, 200_003
    params = _gauss(d)
    v = Vegas(d, N, "gauss", params, prec)
    pr = oracle.Problem(d, N, oracle.GAUSS, params)
    for t in range(4):
        E = v.edges()
        v.iterate(M)
        S1, S2, H = v.last_iteration()
        o1, o2, Ho = oracle.accumulate(pr, E, t, M)
        assert abs(S1 - o1) <= tol * abs(o1), (t, S1, o1)
        assert abs(S2 - o2) <= tol * abs(o2), (t, S2, o2)
        assert _hist_close(H, Ho, tol)
        v.refine()
        En = v.edges()
        assert np.max(np.abs(En - oracle.refine(H, E, 1.5))) <= 1e-12
        assert np.all(En[:, 0] == 0.0) and np.all(En[:, -1] == 1.0)
        assert np.all(np.diff(En, axis=1) > 0)


@pytest.mark.parametrize("prec,tol", [("fp32_mixed", 1e-6), ("fp64", 1e-12)])
def test_full_size_c2_iterations(prec, tol):
    """The benchmarked configuration itself: the d = 8 Gaussian (a = 0.1,
    mu = 0.5), 50 bins, seed 0, 1e7 events per iteration, with the automatic
    launch the benchmark times (16 replicas: the fixed-stride histogram
    layout; 1024-thread blocks, FP64 768) and its step (iterate with the refinement
    fused, not combined).  Two adaptation steps from the uniform grid, each
    against the oracle on the library's own grid: S1, S2 and every histogram
    bin at the path's tolerance, the refined grid at 1e-12.  Then sampled
    event records, one by one against the oracle: the first events of the
    iteration, a middle stretch, and its last events (counters near 1e7)."""
    d, N, M = 8, 50, 10_000_000
    params = _gauss(d)
    v = Vegas(d, N, "gauss", params, prec, seed=0, alpha=1.5)
    info = v.launch_info()
    # mixed: two 1024-thread blocks per CU; FP64: two 768-thread blocks (its
    # kernel is compiled for 6 waves per SIMD)
    assert info["threads"] == (1024 if prec != "fp64" else 768) and info["replicas"] == 16, info
    pr = oracle.Problem(d, N, oracle.GAUSS, params, seed=0)
    for t in range(2):
        E = v.edges()
        v.iterate(M, refine=True, combine=False)
        S1, S2, H = v.last_iteration()
        o1, o2, Ho = oracle.accumulate(pr, E, t, M)
        assert abs(S1 - o1) <= tol * abs(o1), (t, S1, o1)
        assert abs(S2 - o2) <= tol * abs(o2), (t, S2, o2)
        assert _hist_close(H, Ho, tol), t
        assert np.max(np.abs(v.edges() - oracle.refine(H, E, 1.5))) <= 1e-12
    E = v.edges()
    for first, count in ((0, 4096), (M // 2 - 2048, 4096), (M - 4096 - 13, 4096 + 13)):
        got = v.dump_events(first, count, iteration=2).cpu().numpy()
        ref = oracle.events(pr, E, 2, first, count)
        _check_events(got, ref, d, prec != "fp64", "gauss", params, N, E)


def test_free_running_fp64_c1():
    """Plain FP64 Vegas, d = 4, a = 0.1, 50 bins, 10 iterations x 1e5 events,
    alpha = 1.5, seed 0, refining after each iteration, all combined."""
    d, N = 4, 50
    params = _gauss(d)
    v = Vegas(d, N, "gauss", params, "fp64")
    for _ in range(10):
        v.iterate(100_000, refine=True)
    r = v.result()
    ref = oracle.run(oracle.Problem(d, N, oracle.GAUSS, params), oracle.uniform_edges(d, N), 10, 100_000,
                     [1] * 10, [1] * 10)
    I, s, c = ref["final"]
    assert abs(r["integral"] - I) <= 1e-12 * abs(I)
    assert abs(r["sigma"] - s) <= 1e-12 * s
    # chi^2 is built from differences I_t - I ~ sigma_t, so it inherits the
    # 1e-12 relative agreement amplified by I/sigma_t (~1e3)
    assert abs(r["chi2_dof"] - c) <= 1e-8 * max(c, 1e-3)
    assert np.max(np.abs(v.edges() - ref["edges"])) <= 1e-12
    assert r["n_iter"] == 10 and r["n_combined"] == 10 and r["n_events"] == 1_000_000
    assert abs(r["integral"] - 0.99999999999385016) < 5 * r["sigma"]   # erf(5)^4


def test_free_running_c2_shape_reduced():
    """The C2 schedule (5 adaptation iterations left out of the result, then
    5 accumulation iterations on the frozen grid) at reduced size, FP64 and
    mixed: FP64 matches the oracle; mixed drifts by << sigma."""
    d, N, M = 8, 50, 100_000
    params = _gauss(d)
    out = {}
    for prec in ("fp64", "fp32_mixed"):
        v = Vegas(d, N, "gauss", params, prec)
        for _ in range(5):
            v.iterate(M, refine=True, combine=False)
        for _ in range(5):
            v.iterate(M)
        out[prec] = v.result()
    ref = oracle.run(oracle.Problem(d, N, oracle.GAUSS, params), oracle.uniform_edges(d, N), 10, M,
                     [1] * 5 + [0] * 5, [0] * 5 + [1] * 5)
    I, s, _ = ref["final"]
    assert abs(out["fp64"]["integral"] - I) <= 1e-12 * I
    assert abs(out["fp64"]["sigma"] - s) <= 1e-12 * s
    assert out["fp64"]["n_combined"] == 5
    assert abs(out["fp32_mixed"]["integral"] - I) <= 0.1 * s
    assert abs(out["fp32_mixed"]["sigma"] - s) <= 1e-3 * s


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32_mixed", 1e-6)])
def test_chunked_iteration_equals_single_pass(prec, tol):
    d, N = 6, 60
    params = _gauss(d, 0.15)
    E = _adapted_edges(d, N, params)
    a = Vegas(d, N, "gauss", params, prec)
    a.set_edges(E)
    a.iterate(1_000_000)
    b = Vegas(d, N, "gauss", params, prec)
    b.set_edges(E)
    sizes = [123_457, 300_000, 76_543, 250_000, 250_000]
    b.iterate(sizes[0], chunk="begin")
    for s in sizes[1:-1]:
        b.iterate(s, chunk="mid")
    b.iterate(sizes[-1], chunk="end")
    sa, sb = a.last_iteration(), b.last_iteration()
    assert abs(sa[0] - sb[0]) <= 1e-13 * sa[0] and abs(sa[1] - sb[1]) <= 1e-13 * sa[1]
    assert _hist_close(sb[2], sa[2], 1e-13)
    o1, o2, Ho = oracle.accumulate(oracle.Problem(d, N, oracle.GAUSS, params), E, 0, 1_000_000)
    assert abs(sb[0] - o1) <= tol * o1 and abs(sb[1] - o2) <= tol * o2
    assert _hist_close(sb[2], Ho, tol)


@pytest.mark.parametrize("M", [2, 3, 255, 256, 257, 1000, 65_537])
def test_small_and_ragged_sizes(M):
    d, N = 3, 11
    params = _gauss(d, 0.2)
    v = Vegas(d, N, "gauss", params, "fp64", seed=99)
    v.iterate(M)
    S1, S2, H = v.last_iteration()
    o1, o2, Ho = oracle.accumulate(oracle.Problem(d, N, oracle.GAUSS, params, seed=99), oracle.uniform_edges(d, N), 0, M)
    assert abs(S1 - o1) <= 1e-12 * o1 and abs(S2 - o2) <= 1e-12 * o2
    assert _hist_close(H, Ho, 1e-12)
    r = v.result()
    I, var = oracle.iteration_stats(o1, o2, M)
    assert abs(r["last_integral"] - I) <= 1e-12 * I


def _tol(prec, d):
    """1e-12 for FP64; 1e-6 for FP32-mixed up to d = 20 (every benchmarked
    case).  Beyond, the rounding of the FP32 map and exponent, summed over d
    dimensions, grows with d (a = 0.3 at d = 33 puts S2 2.6e-6 from the
    oracle): 1e-6 d/8 there."""
    if prec == "fp64":
        return 1e-12
    return 1e-6 if d <= 20 else 1e-6 * d / 8


@pytest.mark.parametrize("d,N,prec", [(1, 2, "fp64"), (64, 50, "fp64"), (64, 100, "fp32_mixed"),
                                      (33, 255, "fp32_mixed"), (2, 255, "fp64")])
def test_dimension_and_bin_extremes(d, N, prec):
    params = _gauss(d, 0.3)
    tol = _tol(prec, d)
    v = Vegas(d, N, "gauss", params, prec, seed=2**63 + 5)
    M = 50_000
    v.iterate(M, refine=True)
    S1, S2, H = v.last_iteration()
    pr = oracle.Problem(d, N, oracle.GAUSS, params, seed=2**63 + 5)
    E0 = oracle.uniform_edges(d, N)
    o1, o2, Ho = oracle.accumulate(pr, E0, 0, M)
    assert abs(S1 - o1) <= tol * o1 and abs(S2 - o2) <= tol * o2
    assert _hist_close(H, Ho, tol)
    assert np.max(np.abs(v.edges() - oracle.refine(H, E0, 1.5))) <= 1e-12


def _two_peak_grid(d, N, peaks=(1 / 3, 2 / 3), width=0.05):
    """A grid whose bins crowd around the two peaks: edges at the quantiles of
    a mixture of two Gaussians (width) and a uniform floor."""
    from scipy import special
    xs = np.linspace(0, 1, 20001)
    dens = 0.2 + sum(np.exp(-((xs - p) / width) ** 2) / (width * np.sqrt(np.pi)) for p in peaks)
    cdf = np.concatenate([[0.0], np.cumsum((dens[1:] + dens[:-1]) / 2 * np.diff(xs))])
    cdf /= cdf[-1]
    e = np.interp(np.arange(N + 1) / N, cdf, xs)
    e[0], e[-1] = 0.0, 1.0
    return np.tile(e, (d, 1))


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_bimodal_d20_streamed(prec):
    """The d = 20 bimodal integrand (a = 0.05 at 1/3 and 2/3, N = 100) on a
    grid crowded at the peaks, one iteration streamed in four chunks and
    refined at its end."""
    d, N = 20, 100
    params = [0.05] + [1 / 3] * d + [2 / 3] * d
    E = _two_peak_grid(d, N)
    v = Vegas(d, N, "bimodal", params, prec)
    v.set_edges(E)
    sizes = [150_000, 100_000, 200_000, 50_000]
    for k, m in enumerate(sizes):
        v.iterate(m, chunk="begin" if k == 0 else ("end" if k == 3 else "mid"), refine=True)
    S1, S2, H = v.last_iteration()
    pr = oracle.Problem(d, N, oracle.BIMODAL, params)
    o1, o2, Ho = oracle.accumulate(pr, E, 0, sum(sizes))
    tol = _tol(prec, 8)
    assert o1 > 1e-3                         # the grid sees the peaks
    assert abs(S1 - o1) <= tol * o1 and abs(S2 - o2) <= tol * o2
    assert _hist_close(H, Ho, tol)
    assert np.max(np.abs(v.edges() - oracle.refine(H, E, 1.5))) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_full_size_bimodal_d20_streamed(prec):
    """The d = 20 bimodal workload at the benchmark's chunk size and launch:
    one adaptation iteration streamed as three chunks of 1e7 events (the
    benchmark streams ten per iteration through the same launch), refined at
    its end, on a grid crowded at the peaks so that the sums see them;
    against the oracle over the same 3e7 events."""
    from paper_2002_12921_amd import workloads
    d, N, per, chunks = 20, 100, 10_000_000, 3
    params = workloads.bimodal20()
    E = _two_peak_grid(d, N)
    v = Vegas(d, N, "bimodal", params, prec, seed=0, alpha=1.5)
    v.set_edges(E)
    for k in range(chunks):
        v.iterate(per, chunk="begin" if k == 0 else ("end" if k == chunks - 1 else "mid"), refine=True)
    S1, S2, H = v.last_iteration()
    o1, o2, Ho = oracle.accumulate(oracle.Problem(d, N, oracle.BIMODAL, params, seed=0), E, 0, chunks * per)
    tol = _tol(prec, 8)
    assert o1 > 1e-3
    assert abs(S1 - o1) <= tol * o1, (S1, o1)
    assert abs(S2 - o2) <= tol * o2, (S2, o2)
    assert _hist_close(H, Ho, tol)
    assert np.max(np.abs(v.edges() - oracle.refine(H, E, 1.5))) <= 1e-12


def test_checkpoint_resume():
    d, N, M = 5, 30, 40_000
    params = _gauss(d, 0.12)
    a = Vegas(d, N, "gauss", params, "fp64", seed=3)
    for _ in range(3):
        a.iterate(M, refine=True)
    st = a.get_state()
    for _ in range(2):
        a.iterate(M, refine=True)
    ra = a.result()
    b = Vegas(d, N, "gauss", params, "fp64", seed=3)
    b.set_state(st)
    assert b.iteration_index == 3
    for _ in range(2):
        b.iterate(M, refine=True)
    rb = b.result()
    assert abs(ra["integral"] - rb["integral"]) <= 1e-13 * abs(ra["integral"])
    assert np.max(np.abs(a.edges() - b.edges())) <= 1e-14
    assert rb["n_iter"] == 5


def test_state_errors():
    from paper_2002_12921_amd._lib import VegasError
    v = Vegas(3, 10, "gauss", _gauss(3), "fp64")
    with pytest.raises(VegasError, match="ESTATE"):
        v.refine()                                  # nothing to refine from
    with pytest.raises(VegasError, match="ESTATE"):
        v.iterate(100, chunk="mid")                 # no open iteration
    v.iterate(100, chunk="begin")
    with pytest.raises(VegasError, match="ESTATE"):
        v.iterate(100, chunk="begin")               # already open
    with pytest.raises(VegasError, match="EINVAL"):
        v.iterate(0, chunk="end")
    v.iterate(100, chunk="end")
    v.refine()
    with pytest.raises(VegasError, match="ESTATE"):
        v.refine()                                  # histograms already used
    r = v.result()
    assert r["n_iter"] == 1 and r["n_events"] == 200


def test_nonfinite_is_reported():
    # a huge, narrow peak overflows FP32 products in the mixed path? Use an
    # integrand whose FP64 normalisation overflows: a tiny width in many dims.
    d = 40
    v = Vegas(d, 4, "gauss", [1e-9] + [0.5] * d, "fp64")
    E0 = v.edges()
    v.iterate(1000, refine=True)
    r = v.result(allow_nonfinite=True)
    assert r["n_nonfinite"] == 1 and r["n_combined"] == 0
    from paper_2002_12921_amd._lib import VegasError
    with pytest.raises(VegasError, match="ENONFINITE"):
        v.result()
    # the histograms are not finite: the refinement keeps the grid (and its
    # tables: the next iteration is as on the uniform grid)
    assert np.array_equal(v.edges(), E0)
    _, _, H = v.last_iteration()
    assert not np.all(np.isfinite(H))
    # the state stays loadable (its edges are valid)
    w = Vegas(d, 4, "gauss", [1e-9] + [0.5] * d, "fp64")
    w.set_state(v.get_state())


@pytest.mark.parametrize("d", [8, 5, 12])
@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_adjoint_matches_oracle(prec, d):
    """The adjoint kernel vs the oracle's per-sample analytic gradient at the
    same points and grid; tolerance (_tol) relative to the L1 size of the
    terms (d = 8 and 12 fill their kernel's dimension bucket, d = 5 does not)."""
    N, M, t = 50, 300_000, 5
    tol = _tol(prec, d)
    mu = np.random.default_rng(0).uniform(0.3, 0.7, d).astype(np.float32)
    params = [0.1] + [float(m) for m in mu]
    E = _adapted_edges(d, N, params)
    v = Vegas(d, N, "gauss", params, prec)
    v.set_edges(E)
    gout = torch.full((1,), 2.5, dtype=torch.float64, device="cuda")
    grad = torch.zeros(d + 1, dtype=torch.float64, device="cuda")
    v.adjoint(t, M, gout, grad)
    G, Gabs = oracle.adjoint(oracle.Problem(d, N, oracle.GAUSS, params), E, t, M)
    got = grad.cpu().numpy()
    want = 2.5 * G / M
    assert np.all(np.abs(got - want) <= tol * 2.5 * Gabs / M), (got, want)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_autograd_function(dtype):
    """VegasIntegral: forward = one frozen-grid estimate, backward = adjoint
    (FP32 parameters reach the library as FP32, FP64 ones as FP64; both hold
    FP32 values here, so the estimate and gradient are the same)."""
    from paper_2002_12921_amd.autograd import vegas_integral
    d, N, M = 4, 40, 200_000
    mu = torch.tensor([0.15, 0.45, 0.5, 0.62], dtype=torch.float32, device="cuda").to(dtype).requires_grad_(True)
    a = torch.tensor(0.1, dtype=torch.float32, device="cuda").to(dtype).requires_grad_(True)
    params = [0.1] + [0.15, 0.45, 0.5, 0.62]
    p32 = [float(np.float32(x)) for x in params]
    v = Vegas(d, N, "gauss", p32, "fp64")
    for _ in range(4):
        v.iterate(100_000, refine=True)
    E = v.edges()
    t = v.iteration_index
    I = vegas_integral(mu, a, v, M)
    (3.0 * I).backward()
    pr = oracle.Problem(d, N, oracle.GAUSS, p32)
    S1, _, _ = oracle.accumulate(pr, E, t, M)
    assert abs(I.item() - S1 / M) <= 1e-12 * abs(S1 / M)
    G, Gabs = oracle.adjoint(pr, E, t, M)
    gm = mu.grad.cpu().numpy().astype(np.float64)
    ga = float(a.grad.cpu())
    want = 3.0 * G / M
    # grads are cast to the FP32 parameters' dtype
    assert np.all(np.abs(gm - want[:d]) <= 1e-6 * np.abs(want[:d]) + 1e-12 * 3 * Gabs[:d] / M)
    assert abs(ga - want[d]) <= 1e-6 * abs(want[d]) + 1e-12 * 3 * Gabs[d] / M
    # mu_0 = 0.15 is near an edge: its gradient is large and positive
    assert gm[0] > 0.3


@pytest.mark.parametrize("fused", [True, False])
def test_autograd_two_forwards_one_backward(fused):
    """Two forward passes on one context at different centres, then one
    backward of their sum: each gradient is the adjoint at its own centre and
    iteration (fused: summed in the forward launch; else the backward sets
    the forward's parameters back for the adjoint kernel), and the context's
    parameters afterwards are the last ones set."""
    from paper_2002_12921_amd.autograd import vegas_integral
    d, N, M = 4, 40, 100_000
    mu1_h = np.array([0.15, 0.45, 0.5, 0.62], dtype=np.float32)
    mu2_h = np.array([0.55, 0.35, 0.42, 0.7], dtype=np.float32)
    p0 = [float(np.float32(0.1))] + [float(m) for m in mu1_h]
    v = Vegas(d, N, "gauss", p0, "fp64")
    for _ in range(3):
        v.iterate(50_000, refine=True)
    E = v.edges()
    a = torch.tensor(0.1, dtype=torch.float32, device="cuda", requires_grad=True)
    mu1 = torch.tensor(mu1_h, device="cuda", requires_grad=True)
    mu2 = torch.tensor(mu2_h, device="cuda", requires_grad=True)
    t1 = v.iteration_index
    I1 = vegas_integral(mu1, a, v, M, fused)
    t2 = v.iteration_index
    I2 = vegas_integral(mu2, a, v, M, fused)
    assert t2 == t1 + 1
    (2.0 * I1 + 3.0 * I2).backward()
    ga = 0.0
    for mu_t, mu_h, t, wgt in ((mu1, mu1_h, t1, 2.0), (mu2, mu2_h, t2, 3.0)):
        pr = oracle.Problem(d, N, oracle.GAUSS, [float(np.float32(0.1))] + [float(m) for m in mu_h])
        G, Gabs = oracle.adjoint(pr, E, t, M)
        want = wgt * G / M
        got = mu_t.grad.cpu().numpy().astype(np.float64)
        # FP32 gradients: one rounding of the FP64 sum
        assert np.all(np.abs(got - want[:d]) <= 2.0 ** -24 * np.abs(want[:d]) + 1e-12 * wgt * Gabs[:d] / M), (got, want)
        ga += want[d]
    assert abs(float(a.grad.cpu()) - ga) <= 1e-6 * abs(ga)
    # the parameters in force are those of the last forward pass
    cur = v.get_params_device().cpu().numpy()
    assert np.array_equal(cur, np.array([np.float32(0.1)] + list(mu2_h), dtype=np.float64))
    # no record slot was used by the forward passes
    assert v.result(allow_nonfinite=True)["n_iter"] == 3


@pytest.mark.parametrize("fused", [True, False])
def test_autograd_backward_after_refine(fused):
    """A refinement between forward and backward changes the grid: the
    separate adjoint pass would need the old one, so its backward refuses;
    the fused gradient was summed at the forward's grid and stays valid."""
    from paper_2002_12921_amd.autograd import vegas_integral
    d, N, M = 3, 20, 10_000
    v = Vegas(d, N, "gauss", [0.1] + [0.5] * d, "fp64")
    v.iterate(20_000, refine=True)
    E = v.edges()
    mu = torch.full((d,), 0.5, dtype=torch.float64, device="cuda", requires_grad=True)
    a = torch.tensor(0.1, dtype=torch.float64, device="cuda", requires_grad=True)
    t = v.iteration_index
    I = vegas_integral(mu, a, v, M, fused)
    v.iterate(20_000, refine=True)
    if not fused:
        with pytest.raises(RuntimeError, match="grid changed"):
            I.backward()
        return
    I.backward()
    G, Gabs = oracle.adjoint(oracle.Problem(d, N, oracle.GAUSS, [0.1] + [0.5] * d), E, t, M)
    assert np.all(np.abs(mu.grad.cpu().numpy() - G[:d] / M) <= 1e-12 * Gabs[:d] / M)
    assert abs(float(a.grad.cpu()) - G[d] / M) <= 1e-12 * Gabs[d] / M


@pytest.mark.parametrize("fused", [True, False])
def test_autograd_rejects_bad_arguments(fused):
    """Host tensors, wrong sizes and other integrands are refused before any
    library call."""
    from paper_2002_12921_amd.autograd import vegas_integral
    d = 3
    v = Vegas(d, 20, "gauss", [0.1] + [0.5] * d, "fp64")
    mu = torch.full((d,), 0.5, dtype=torch.float64, requires_grad=True)
    a = torch.tensor(0.1, dtype=torch.float64, requires_grad=True)
    with pytest.raises(ValueError, match="GPU"):
        vegas_integral(mu, a, v, 1000, fused)
    with pytest.raises(ValueError, match="GPU"):
        vegas_integral(mu.detach().cuda().requires_grad_(), a, v, 1000, fused)
    with pytest.raises(ValueError, match="elements"):
        vegas_integral(torch.full((d + 1,), 0.5, dtype=torch.float64, device="cuda"), a.cuda(), v, 1000, fused)
    b = Vegas(d, 20, "bimodal", [0.1] + [0.3] * d + [0.6] * d, "fp64")
    with pytest.raises(ValueError, match="Gaussian"):
        vegas_integral(mu.detach().cuda(), a.detach().cuda(), b, 1000, fused)
    assert v.iteration_index == 0 and b.iteration_index == 0


@pytest.mark.parametrize("fused", [True, False])
def test_autograd_many_forward_passes(fused):
    """More forward passes than a context has record slots (1024): none of
    them takes a slot, and a backward after them still matches the oracle."""
    from paper_2002_12921_amd.autograd import vegas_integral
    d, N, M = 2, 10, 1000
    v = Vegas(d, N, "gauss", [0.2, 0.5, 0.5], "fp64")
    mu = torch.tensor([0.4, 0.6], dtype=torch.float64, device="cuda", requires_grad=True)
    a = torch.tensor(0.2, dtype=torch.float64, device="cuda", requires_grad=True)
    for _ in range(1100):
        I = vegas_integral(mu, a, v, M, fused)
    t = v.iteration_index - 1
    I.backward()
    pr = oracle.Problem(d, N, oracle.GAUSS, [0.2, 0.4, 0.6])
    S1, _, _ = oracle.accumulate(pr, oracle.uniform_edges(d, N), t, M)
    assert abs(I.item() - S1 / M) <= 1e-12 * abs(S1 / M)
    G, Gabs = oracle.adjoint(pr, oracle.uniform_edges(d, N), t, M)
    assert np.all(np.abs(mu.grad.cpu().numpy() - G[:d] / M) <= 1e-12 * Gabs[:d] / M)
    # recorded iterations still work after them
    v.iterate(M)
    assert v.result()["n_iter"] == 1


@pytest.mark.parametrize("d", [8, 5, 12])
@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_fused_gradient_matches_oracle(prec, d):
    """The forward pass with the gradient (vegas_iterate_grad): its estimate is
    bitwise that of the plain frozen-grid iteration (same events, same sums),
    and its gradient matches the oracle's per-sample analytic gradient at the
    same points and grid, at the path's tolerance relative to the L1 size of
    the terms (as the separate adjoint kernel)."""
    N, M, t = 50, 300_000, 0
    tol = _tol(prec, d)
    mu = np.random.default_rng(1).uniform(0.3, 0.7, d).astype(np.float32)
    params = [0.1] + [float(m) for m in mu]
    E = _adapted_edges(d, N, params)
    v = Vegas(d, N, "gauss", params, prec)
    v.set_edges(E)
    w = Vegas(d, N, "gauss", params, prec)
    w.set_edges(E)
    G = torch.zeros(d + 1, dtype=torch.float64, device="cuda")
    v.iterate_grad(M, G)
    w.iterate(M, hist=False)
    s1v, s2v, _ = v.last_iteration()
    s1w, s2w, _ = w.last_iteration()
    assert s1v == s1w and s2v == s2w
    o1, _, _ = oracle.accumulate(oracle.Problem(d, N, oracle.GAUSS, params), E, t, M)
    assert abs(s1v - o1) <= tol * o1
    Go, Gabs = oracle.adjoint(oracle.Problem(d, N, oracle.GAUSS, params), E, t, M)
    assert np.all(np.abs(G.cpu().numpy() - Go / M) <= tol * Gabs / M)
    # the one-call forward (parameters + the same iteration, (I_t, sigma_t)
    # written by the reduction) on a third context at the same iteration index
    u = Vegas(d, N, "gauss", [0.5] + [0.5] * d, prec)
    u.set_edges(E)
    G2 = torch.zeros(d + 1, dtype=torch.float64, device="cuda")
    out2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    pt = torch.tensor(params, dtype=torch.float64, device="cuda")
    u.forward_grad(pt, M, G2, out2)
    assert torch.equal(G2, G)
    # the same with a and mu as two arrays (value 0, then the rest)
    u2 = Vegas(d, N, "gauss", [0.5] + [0.5] * d, prec)
    u2.set_edges(E)
    G3 = torch.zeros(d + 1, dtype=torch.float64, device="cuda")
    out3 = torch.zeros(2, dtype=torch.float64, device="cuda")
    u2.forward_grad(pt[:1].clone(), M, G3, out3, rest=pt[1:].clone())
    assert torch.equal(G3, G) and torch.equal(out3, out2)
    I2, sig2 = out2.cpu().numpy()
    assert I2 == s1v / M
    assert np.isclose(sig2, np.sqrt(oracle.iteration_stats(s1v, s2v, M)[1]), rtol=1e-12)
    assert u.result(allow_nonfinite=True)["n_iter"] == 0  # not recorded
    # backward: gout times G, rounded once
    gout = torch.full((1,), 0.75, dtype=torch.float64, device="cuda")
    g32 = torch.zeros(d + 1, dtype=torch.float32, device="cuda")
    v.grad_scale(G, gout, g32)
    assert np.array_equal(g32.cpu().numpy(), (0.75 * G.cpu().numpy()).astype(np.float32))


def test_fused_gradient_c4_shape():
    """The differentiable case as benchmarked (the fused forward): d = 8,
    FP32 centres mu ~ U[0.3, 0.7] (seed 0), a = 0.1, grid from 5 FP64
    adaptation iterations of 1e6 events, 1e7 events at iteration 5 in
    FP32-mixed, against the oracle's analytic gradient at the same points."""
    d, N, M = 8, 50, 10_000_000
    mu32 = np.random.default_rng(0).uniform(0.3, 0.7, d).astype(np.float32)
    params = [float(np.float32(0.1))] + [float(m) for m in mu32]
    ad = Vegas(d, N, "gauss", params, "fp64")
    for _ in range(5):
        ad.iterate(1_000_000, refine=True)
    E = ad.edges()
    v = Vegas(d, N, "gauss", params, "fp32_mixed")
    v.set_edges(E)
    for _ in range(5):
        v.iterate(10, hist=False, record=False)  # to iteration index 5
    G = torch.zeros(d + 1, dtype=torch.float64, device="cuda")
    v.iterate_grad(M, G, combine=False, record=False)
    Go, Gabs = oracle.adjoint(oracle.Problem(d, N, oracle.GAUSS, params), E, 5, M)
    assert np.all(np.abs(G.cpu().numpy() - Go / M) <= 1e-6 * Gabs / M)


def test_adjoint_fp32_output_is_rounded_fp64():
    """The adjoint's FP32 output is the FP64 gradient rounded once."""
    d, N, M = 5, 30, 200_000
    v = Vegas(d, N, "gauss", [0.12] + list(np.linspace(0.3, 0.7, d)), "fp32_mixed")
    gout = torch.full((1,), 1.5, dtype=torch.float64, device="cuda")
    g64 = torch.zeros(d + 1, dtype=torch.float64, device="cuda")
    g32 = torch.zeros(d + 1, dtype=torch.float32, device="cuda")
    v.adjoint(2, M, gout, g64)
    v.adjoint(2, M, gout, g32)
    assert np.array_equal(g32.cpu().numpy(), g64.cpu().numpy().astype(np.float32))


def test_adjoint_c4_shape():
    """Differentiable case at full size: d = 8, mu ~ U[0.3, 0.7] (seed 0) and
    a = 0.1 as FP32 parameters, grid from 5 FP64 adaptation iterations of 1e6
    events, forward and backward at iteration 5 with 1e7 events (FP32-mixed),
    against the oracle's analytic gradient at the same points."""
    d, N, M = 8, 50, 10_000_000
    mu32 = np.random.default_rng(0).uniform(0.3, 0.7, d).astype(np.float32)
    params = [float(np.float32(0.1))] + [float(m) for m in mu32]
    ad = Vegas(d, N, "gauss", params, "fp64")
    for _ in range(5):
        ad.iterate(1_000_000, refine=True)
    E = ad.edges()
    v = Vegas(d, N, "gauss", params, "fp32_mixed")
    v.set_edges(E)
    gout = torch.ones(1, dtype=torch.float64, device="cuda")
    grad = torch.zeros(d + 1, dtype=torch.float64, device="cuda")
    v.adjoint(5, M, gout, grad)
    G, Gabs = oracle.adjoint(oracle.Problem(d, N, oracle.GAUSS, params), E, 5, M)
    assert np.all(np.abs(grad.cpu().numpy() - G / M) <= 1e-6 * Gabs / M)


def _genz_params(kind, d):
    from paper_2002_12921_amd import workloads
    return workloads.genz16(kind, d)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32_mixed", 1e-6)])
@pytest.mark.parametrize("kind", ["genz_disc", "genz_peak"])
def test_genz_d16_lockstep(kind, prec, tol):
    """Genz discontinuous and product-peak integrands at d = 16 (both
    normalised to 1): sums, histograms and refinements per iteration against
    the oracle on the library's own grid.  The discontinuous one leaves whole
    bins empty (x_i <= a_i contributes nothing), the refinement's r = 0 path."""
    d, N, M = 16, 50, 60_001
    params = _genz_params(kind, d)
    kid = oracle.GENZ_DISC if kind == "genz_disc" else oracle.GENZ_PEAK
    v = Vegas(d, N, kind, params, prec, seed=5)
    pr = oracle.Problem(d, N, kid, params, seed=5)
    for t in range(3):
        E = v.edges()
        v.iterate(M)
        S1, S2, H = v.last_iteration()
        o1, o2, Ho = oracle.accumulate(pr, E, t, M)
        assert abs(S1 - o1) <= tol * abs(o1), (t, S1, o1)
        assert abs(S2 - o2) <= tol * abs(o2), (t, S2, o2)
        assert _hist_close(H, Ho, tol)
        if kind == "genz_disc":
            assert np.any(Ho == 0.0)  # empty bins below the thresholds
        v.refine()
        assert np.max(np.abs(v.edges() - oracle.refine(H, E, 1.5))) <= 1e-12


@pytest.mark.parametrize("N", [50, 90])
def test_genz_disc_fp64_d16_every_replica_count(N):
    """The FP64 discontinuous kernels at d = 16 take at most 768 threads per
    block: the automatic launch picks 768, and every replica count (fixed and
    general layouts) and the kernel without histograms run at that size and
    match the oracle."""
    from paper_2002_12921_amd import workloads
    d, M = 16, 200_003
    params = workloads.genz16("genz_disc")
    pr = oracle.Problem(d, N, oracle.GENZ_DISC, params, seed=3)
    E = _adapted_edges(d, N, params, kind=oracle.GENZ_DISC, iters=2, n=20_000)
    o1, o2, Ho = oracle.accumulate(pr, E, 0, M)
    for rep in ((0, 16, 4, 1) if N <= 64 else (0, 8, 2, 1)):  # 16 copies of 90 bins exceed the LDS
        v = Vegas(d, N, "genz_disc", params, "fp64", seed=3)
        assert v.launch_info()["threads"] == 768
        v.set_edges(E)
        v.set_hist_replicas(rep)
        v.iterate(M, combine=False)
        S1, S2, H = v.last_iteration()
        assert abs(S1 - o1) <= 1e-12 * abs(o1) and abs(S2 - o2) <= 1e-12 * abs(o2), rep
        assert _hist_close(H, Ho, 1e-12), rep
    w = Vegas(d, N, "genz_disc", params, "fp64", seed=3)
    w.set_edges(E)
    w.iterate(M, hist=False)
    assert w.last_iteration()[0] == S1


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("kind", ["genz_disc", "genz_peak"])
def test_full_size_genz_d16(kind, prec):
    """The Genz workloads as benchmarked: d = 16, 50 bins, seed 0, 1e7 events,
    the automatic launch (one block of 16 replicas per CU: 1024 threads, 768
    for the FP64 discontinuous kernel), one adaptation step from the uniform
    grid against the oracle: sums and histograms at the path's tolerance, the
    refined grid at 1e-12."""
    from paper_2002_12921_amd import workloads
    d, N, M = 16, 50, 10_000_000
    params = workloads.genz16(kind)
    kid = oracle.GENZ_DISC if kind == "genz_disc" else oracle.GENZ_PEAK
    v = Vegas(d, N, kind, params, prec, seed=0, alpha=1.5)
    info = v.launch_info()
    assert info["threads"] == (768 if (kind, prec) == ("genz_disc", "fp64") else 1024), info
    assert info["replicas"] == 16, info
    E = v.edges()
    v.iterate(M, refine=True, combine=False)
    S1, S2, H = v.last_iteration()
    o1, o2, Ho = oracle.accumulate(oracle.Problem(d, N, kid, params, seed=0), E, 0, M)
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert abs(S1 - o1) <= tol * abs(o1), (S1, o1)
    assert abs(S2 - o2) <= tol * abs(o2), (S2, o2)
    assert _hist_close(H, Ho, tol)
    assert np.max(np.abs(v.edges() - oracle.refine(H, E, 1.5))) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("kind", ["genz_disc", "genz_peak"])
def test_genz_d16_schedule_hits_closed_form(kind, prec):
    """5 adaptation + 5 accumulation iterations of 1e6 events: the combined
    estimate is within 5 sigma of the closed form (1 by normalisation)."""
    d, N = 16, 50
    v = Vegas(d, N, kind, _genz_params(kind, d), prec, seed=11)
    for _ in range(5):
        v.iterate(1_000_000, refine=True, combine=False)
    for _ in range(5):
        v.iterate(1_000_000)
    r = v.result()
    assert r["n_combined"] == 5
    assert abs(r["integral"] - 1.0) <= 5 * r["sigma"], r
    assert r["sigma"] < 0.02


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
def test_no_hist_iterations(prec):
    """Iterations without histograms (frozen grid) give bit-identical S1, S2
    and combined results; their histogram row reads zero; they cannot refine.
    (The histograms' LDS atomics add in no fixed order, so two refinements of
    the same events agree only to rounding: b takes a's adapted grid.)"""
    from paper_2002_12921_amd import VegasError
    d, N, M = 8, 50, 400_009
    params = _gauss(d)
    a = Vegas(d, N, "gauss", params, prec)
    b = Vegas(d, N, "gauss", params, prec)
    for v in (a, b):
        for _ in range(3):
            v.iterate(M, refine=True, combine=False)
    b.set_edges(a.edges())
    for _ in range(3):
        a.iterate(M)
        b.iterate(M, hist=False)
        Sa, Sb = a.last_iteration(), b.last_iteration()
        assert Sa[0] == Sb[0] and Sa[1] == Sb[1]
        assert np.all(Sb[2] == 0.0) and Sa[2].sum() > 0
    ra, rb = a.result(), b.result()
    assert ra["integral"] == rb["integral"] and ra["sigma"] == rb["sigma"]
    with pytest.raises(VegasError):
        b.refine()  # nothing to refine from
    with pytest.raises(VegasError):
        b.iterate(M, refine=True, hist=False)
    # chunks of one iteration must agree on NO_HIST
    b.iterate(M // 2, chunk="begin", hist=False)
    with pytest.raises(VegasError):
        b.iterate(M // 2, chunk="end")
    b.iterate(M - M // 2, chunk="end", hist=False)
    a.iterate(M // 2, chunk="begin")
    a.iterate(M - M // 2, chunk="end")
    assert a.last_iteration()[0] == b.last_iteration()[0]


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("d,N", [(20, 100), (6, 40), (5, 7)])
def test_no_hist_bimodal_same_bits(prec, d, N):
    """The bimodal integrand with and without histograms: the same S1 and S2
    bits on a grid adapted to both centres (kernels of different LDS layouts
    and register budgets), and both match the oracle, histograms included.
    Partly adapted, the d = 20 grid leaves the sums to events between the
    peaks, where each term's offset from its farther centre decides the
    value: the FP32 path meets the tolerance there only with each offset
    rounded once from FP64 at its own size."""
    params = [0.05] + [1 / 3] * d + [2 / 3] * d
    M = 300_001
    E = _adapted_edges(d, N, params, kind=oracle.BIMODAL, iters=3, n=20_000)
    a = Vegas(d, N, "bimodal", params, prec, seed=5)
    b = Vegas(d, N, "bimodal", params, prec, seed=5)
    for v in (a, b):
        v.set_edges(E)
    a.iterate(M)
    b.iterate(M, hist=False)
    Sa, Sb = a.last_iteration(), b.last_iteration()
    assert Sa[0] == Sb[0] and Sa[1] == Sb[1]
    o1, o2, Ho = oracle.accumulate(oracle.Problem(d, N, oracle.BIMODAL, params, seed=5), E, 0, M)
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert abs(Sa[0] - o1) <= tol * abs(o1) and abs(Sa[1] - o2) <= tol * abs(o2)
    assert _hist_close(Sa[2], Ho, tol)


def test_time_event_kernel_leaves_state():
    """The measurement entry point runs the event kernel only: the iteration
    index, the records and the grid do not move."""
    from paper_2002_12921_amd import VegasError
    v = Vegas(8, 50, "gauss", _gauss(8), "fp32_mixed")
    v.iterate(100_000, refine=True)
    E, t = v.edges(), v.iteration_index
    r0 = v.result()
    ms = v.time_event_kernel(1_000_000, 3)
    ms_nh = v.time_event_kernel(1_000_000, 3, hist=False)
    assert ms > 0 and ms_nh > 0
    assert v.iteration_index == t and np.array_equal(v.edges(), E)
    r1 = v.result()
    assert all(r1[k] == r0[k] or (r1[k] != r1[k] and r0[k] != r0[k]) for k in r0)  # NaN-aware
    v.iterate(50_000, chunk="begin")
    with pytest.raises(VegasError):
        v.time_event_kernel(1000, 1)
    v.iterate(50_000, chunk="end")


@pytest.mark.parametrize("prec", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("d,N", [(3, 2), (3, 3), (4, 50), (2, 63), (2, 64), (2, 65), (2, 255)])
def test_refine_matches_oracle_across_bin_counts(prec, d, N):
    """Refinement (one wave for N <= 64, the whole block beyond) against the
    oracle's refinement of the library's own histograms, fused at the end of
    an iteration and stand-alone, plus the tables it rebuilds (checked through
    the next iteration's sums)."""
    params = _gauss(d, 0.2, 0.4)
    E = _adapted_edges(d, N, params, iters=2, n=5000)
    pr = oracle.Problem(d, N, oracle.GAUSS, params)
    M = 40_000
    for fused in (True, False):
        v = Vegas(d, N, "gauss", params, prec)
        v.set_edges(E)
        v.iterate(M, refine=fused)
        S1, S2, H = v.last_iteration()
        if not fused:
            v.refine()
        En = v.edges()
        assert np.max(np.abs(En - oracle.refine(H, E, 1.5))) <= 1e-12, (fused, N)
        v.iterate(M)
        o1, o2, _ = oracle.accumulate(pr, En, 1, M)
        tol = 1e-12 if prec == "fp64" else 1e-6
        assert abs(v.last_iteration()[0] - o1) <= tol * abs(o1)


def test_adjoint_vs_finite_differences_and_closed_form():
    """The library's gradient of the frozen-grid estimate against central
    finite differences (h = 1e-4) of the library's own forward at the same
    points, and, statistically, against the closed-form (erf) gradient of the
    exact integral: the mean of 8 independent iterations' gradients within 5
    standard errors."""
    from scipy import special
    d, N, M, h = 8, 50, 2_000_000, 1e-4
    mu = np.random.default_rng(0).uniform(0.3, 0.7, d)
    mu[0] = 0.15  # near an edge: a gradient well above the Monte Carlo noise
    a = 0.1
    params = [a] + list(mu)
    v = Vegas(d, N, "gauss", params, "fp64")
    for _ in range(5):
        v.iterate(1_000_000, refine=True, combine=False)
    state = v.get_state()
    t = v.iteration_index
    p0 = torch.tensor(params, dtype=torch.float64, device="cuda")

    def forward(p):
        v.set_state(state)
        v.set_params_device(torch.tensor(p, dtype=torch.float64, device="cuda"))
        v.iterate(M, combine=False)
        return v.last_iteration()[0] / M

    def gradient(it):
        v.set_state(state)
        v.set_params_device(p0)
        gout = torch.ones(1, dtype=torch.float64, device="cuda")
        grad = torch.zeros(d + 1, dtype=torch.float64, device="cuda")
        v.adjoint(it, M, gout, grad)
        return grad.cpu().numpy()

    g = gradient(t)
    # parameter layout (a, mu_0..mu_7); the gradient comes as (mu_0..mu_7, a)
    fd = np.zeros(d + 1)
    for j in range(d + 1):
        k = 1 + j if j < d else 0
        pp, pm = list(params), list(params)
        pp[k] += h
        pm[k] -= h
        fd[j] = (forward(pp) - forward(pm)) / (2 * h)
    # same points: only the O(h^2) truncation and rounding separate them
    assert np.all(np.abs(g - fd) <= 1e-5 * np.abs(fd).max()), (g, fd)
    # closed form: I = prod_i [erf((1 - mu_i)/a) + erf(mu_i/a)] / 2
    e1, e0 = special.erf((1 - mu) / a), special.erf(mu / a)
    term = (e1 + e0) / 2
    I = np.prod(term)
    dterm_mu = (-np.exp(-((1 - mu) / a) ** 2) + np.exp(-(mu / a) ** 2)) / (a * np.sqrt(np.pi))
    dterm_a = (-(1 - mu) * np.exp(-((1 - mu) / a) ** 2) - mu * np.exp(-(mu / a) ** 2)) / (a * a * np.sqrt(np.pi))
    exact = np.concatenate([I * dterm_mu / term, [I * np.sum(dterm_a / term)]])
    reps = np.array([gradient(t + 1 + r) for r in range(8)])
    mean, se = reps.mean(axis=0), reps.std(axis=0, ddof=1) / np.sqrt(len(reps))
    assert np.all(np.abs(mean - exact) <= 5 * se + 1e-12), (mean, exact, se)
    assert abs(exact[0]) > 10 * se[0]  # the check has power on mu_0


@pytest.mark.parametrize("alpha", [0.0, 0.5, 0.7, 1.0, 1.5, 2.0])
def test_refine_damping_exponents(alpha):
    """Refinement with the damping exponents that take the square-root and
    product paths (0.5, 1, 1.5, 2), the general power (0.7) and no damping
    exponent at all (0: every nonzero bin weighs the same), against the
    oracle's refinement of the library's histograms."""
    d, N, M = 4, 50, 100_000
    params = _gauss(d, 0.15, 0.45)
    E = _adapted_edges(d, N, params, iters=2, n=5000)
    v = Vegas(d, N, "gauss", params, "fp64", alpha=alpha)
    v.set_edges(E)
    v.iterate(M, refine=True)
    H = v.last_iteration()[2]
    assert np.max(np.abs(v.edges() - oracle.refine(H, E, alpha))) <= 1e-12


def test_graph_captured_iterations_replay():
    """Single-problem iterations recorded as a HIP graph (stream capture of
    the library's launches) and replayed three times, each from the uniform
    grid with eager work in between: every replay gives the eager run's
    combined result (to the rounding that nondeterministic histogram sums
    leave in the refined grids)."""
    d, N, M = 8, 50, 300_007
    params = _gauss(d)
    eager = Vegas(d, N, "gauss", params, "fp32_mixed", seed=3)
    for _ in range(3):
        eager.iterate(M, refine=True, combine=False)
    for _ in range(2):
        eager.iterate(M, hist=False)
    ref = eager.result()
    v = Vegas(d, N, "gauss", params, "fp32_mixed", seed=3)
    E0 = v.edges()
    s = torch.cuda.Stream()
    v.stream = s
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        for _ in range(3):
            v.iterate(M, refine=True, combine=False)
        for _ in range(2):
            v.iterate(M, hist=False)
    for rep in range(3):
        v.set_edges(E0)
        with torch.cuda.stream(s):  # replay() launches on the current stream
            g.replay()
        r = v.result()
        assert abs(r["integral"] - ref["integral"]) <= 1e-12 * abs(ref["integral"]), (rep, r, ref)
        assert abs(r["sigma"] - ref["sigma"]) <= 1e-9 * ref["sigma"], (rep, r, ref)
        assert r["n_combined"] == 2
        # eager work between replays
        eager.iterate(1000, hist=False, combine=False)
        torch.cuda.synchronize()
