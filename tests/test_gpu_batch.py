"""GPU parity of the batched path: many problems in one recorded graph.

Each problem of a batch is an independent Vegas run; its points carry the
problem index in the Philox counter.  FP64 batches match the oracle run of
each problem (1e-12); FP32-mixed batches match the single-problem mixed path
on the same points (reduction order only) and the oracle within the mixed
tolerance.  Graph replays give the same results; the tile size chosen by the
tuner does not change them beyond reduction-order rounding.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2002_12921_amd import Vegas
from paper_2002_12921_amd.batch import VegasBatch
from paper_2002_12921_amd import workloads

pytestmark = pytest.mark.gpu


def _small_batch(prec, n=9, seed=7):
    rng = np.random.default_rng(seed)
    probs = []
    for p in range(n):
        d = int(rng.integers(2, 17))
        a = float(rng.uniform(0.08, 0.3))
        probs.append({"dim": d, "n_bins": int(rng.choice([20, 50])), "params": [a] + [0.5] * d,
                      "n_events": int(rng.integers(5_000, 60_000)), "precision": prec, "problem": 3 * p + 1})
    return probs


def _oracle_run(q, n_iter, n_adapt):
    pr = oracle.Problem(q["dim"], q["n_bins"], oracle.GAUSS, q["params"], seed=0, problem=q["problem"])
    return oracle.run(pr, oracle.uniform_edges(q["dim"], q["n_bins"]), n_iter, q["n_events"],
                      [1] * n_adapt + [0] * (n_iter - n_adapt), [0] * n_adapt + [1] * (n_iter - n_adapt))


def test_batch_fp64_matches_oracle():
    probs = _small_batch("fp64")
    n_iter, n_adapt = 5, 3
    b = VegasBatch(probs, n_iter, n_adapt)
    b.run()
    res = b.results()
    for p, q in enumerate(probs):
        ref = _oracle_run(q, n_iter, n_adapt)
        I, s, c = ref["final"]
        assert abs(res[p]["integral"] - I) <= 1e-12 * abs(I), p
        assert abs(res[p]["sigma"] - s) <= 1e-12 * s, p
        assert res[p]["n_iter"] == n_iter and res[p]["n_combined"] == n_iter - n_adapt
        assert np.max(np.abs(b.edges(p) - ref["edges"])) <= 1e-12, p


@pytest.mark.parametrize("kind", ["genz_disc", "genz_peak", "bimodal"])
def test_batch_other_integrands_fp64_match_oracle(kind):
    """Batches of the other integrands (each dimension guarded against the
    problem's d; the fixed histogram layout where N <= 64): d across the three
    smallest buckets, FP64, every problem against its oracle run at 1e-12."""
    kid = {"genz_disc": oracle.GENZ_DISC, "genz_peak": oracle.GENZ_PEAK, "bimodal": oracle.BIMODAL}[kind]
    probs = []
    for p, (d, N, n) in enumerate([(3, 20, 20_000), (7, 50, 30_000), (12, 20, 25_000), (16, 50, 40_000)]):
        if kind == "bimodal":
            params = [0.2] + [0.35] * d + [0.65] * d
        else:
            params = workloads.genz16(kind, d)
        probs.append({"dim": d, "n_bins": N, "integrand": kind, "params": params, "n_events": n,
                      "precision": "fp64", "problem": p})
    n_iter, n_adapt = 4, 2
    b = VegasBatch(probs, n_iter, n_adapt)
    b.run()
    res = b.results()
    for p, q in enumerate(probs):
        pr = oracle.Problem(q["dim"], q["n_bins"], kid, q["params"], seed=0, problem=q["problem"])
        ref = oracle.run(pr, oracle.uniform_edges(q["dim"], q["n_bins"]), n_iter, q["n_events"],
                         [1] * n_adapt + [0] * (n_iter - n_adapt), [0] * n_adapt + [1] * (n_iter - n_adapt))
        I, s, c = ref["final"]
        assert abs(res[p]["integral"] - I) <= 1e-12 * abs(I), (kind, p)
        assert abs(res[p]["sigma"] - s) <= 1e-12 * s, (kind, p)
        assert np.max(np.abs(b.edges(p) - ref["edges"])) <= 1e-12, (kind, p)
    b.close()


@pytest.mark.parametrize("kind", ["genz_disc", "genz_peak", "bimodal"])
def test_batch_other_integrands_mixed_lockstep(kind):
    """FP32-mixed batches of the other integrands, stepped one iteration at a
    time: every problem's S1, S2 and (adaptation iterations) every histogram
    bin against the oracle on the batch's own grid at 1e-6, and every
    refinement against the oracle's refinement of the batch's histograms at
    1e-12; d across the three smallest buckets, even and odd N."""
    kid = {"genz_disc": oracle.GENZ_DISC, "genz_peak": oracle.GENZ_PEAK, "bimodal": oracle.BIMODAL}[kind]
    probs = []
    for p, (d, N, n) in enumerate([(3, 21, 20_000), (7, 50, 30_000), (12, 20, 25_000), (16, 50, 40_000)]):
        if kind == "bimodal":
            params = [0.2] + [0.35] * d + [0.65] * d
        else:
            params = workloads.genz16(kind, d)
        probs.append({"dim": d, "n_bins": N, "integrand": kind, "params": params, "n_events": n,
                      "precision": "fp32_mixed", "problem": p})
    n_iter, n_adapt = 4, 2
    b = VegasBatch(probs, n_iter, n_adapt)
    tol = 1e-6
    for k in range(n_iter):
        before = [b.edges(p) for p in range(len(probs))]
        b.step(k)
        for p, q in enumerate(probs):
            pr = oracle.Problem(q["dim"], q["n_bins"], kid, q["params"], seed=0, problem=q["problem"])
            S1, S2, H = b.last_iteration(p)
            o1, o2, Ho = oracle.accumulate(pr, before[p], k, q["n_events"])
            assert abs(S1 - o1) <= tol * abs(o1), (kind, p, k, S1, o1)
            assert abs(S2 - o2) <= tol * abs(o2), (kind, p, k, S2, o2)
            E = b.edges(p)
            if k < n_adapt:
                assert _hist_close(H, Ho, tol), (kind, p, k)
                assert np.max(np.abs(E - oracle.refine(H, before[p], 1.5))) <= 1e-12, (kind, p, k)
            else:
                assert np.array_equal(E, before[p])
    b.close()


def test_batch_wide_grids_general_layout():
    """Grids of more than 64 bins (the batch kernel's general histogram
    layout, with whatever replicas the tuner keeps) with the Gaussian's
    exact-d loops: FP64, every problem against its oracle run at 1e-12."""
    probs = [{"dim": d, "n_bins": N, "params": [0.2] + [0.5] * d, "n_events": n, "precision": "fp64",
              "problem": p}
             for p, (d, N, n) in enumerate([(2, 100, 20_000), (6, 80, 30_000), (11, 100, 25_000), (16, 80, 30_000)])]
    n_iter, n_adapt = 4, 2
    b = VegasBatch(probs, n_iter, n_adapt)
    b.run()
    res = b.results()
    for p, q in enumerate(probs):
        ref = _oracle_run(q, n_iter, n_adapt)
        I, s, c = ref["final"]
        assert abs(res[p]["integral"] - I) <= 1e-12 * abs(I), p
        assert abs(res[p]["sigma"] - s) <= 1e-12 * s, p
        assert np.max(np.abs(b.edges(p) - ref["edges"])) <= 1e-12, p
    b.close()


def test_batch_mixed_matches_single_problem_path():
    probs = _small_batch("fp32_mixed", n=6, seed=11)
    n_iter, n_adapt = 4, 2
    b = VegasBatch(probs, n_iter, n_adapt)
    b.run()
    res = b.results()
    for p, q in enumerate(probs):
        v = Vegas(q["dim"], q["n_bins"], "gauss", q["params"], "fp32_mixed", problem=q["problem"])
        for k in range(n_iter):
            v.iterate(q["n_events"], refine=k < n_adapt, combine=k >= n_adapt)
        r = v.result()
        # same points; the batch kernel (compiled for the batch's largest d)
        # sums the exponent in FP64 where the single-problem kernel for d <= 8
        # sums it in FP32, and the reduction order differs: the paths agree to
        # the FP32-mixed tolerance
        assert abs(res[p]["integral"] - r["integral"]) <= 1e-6 * abs(r["integral"]), p
        assert abs(res[p]["sigma"] - r["sigma"]) <= 1e-5 * r["sigma"], p
        ref = _oracle_run(q, n_iter, n_adapt)
        I, s, _ = ref["final"]
        assert abs(res[p]["integral"] - I) <= 0.1 * s, p


def test_graph_replay_and_tile_independence(monkeypatch):
    probs = _small_batch("fp64", n=5, seed=3)
    b = VegasBatch(probs, 3, 2)
    b.run()
    r1 = b.results()
    b.run()
    r2 = b.results()
    for x, y in zip(r1, r2):
        assert abs(x["integral"] - y["integral"]) <= 1e-13 * abs(x["integral"])
    tile = b.schedule()["tile_events"]
    other = 8192 if tile != 8192 else 131072
    monkeypatch.setenv("VEGAS_BATCH_TILE", str(other))
    c = VegasBatch(probs, 3, 2)
    assert c.schedule()["tile_events"] == other
    c.run()
    r3 = c.results()
    for x, y in zip(r1, r3):
        assert abs(x["integral"] - y["integral"]) <= 1e-12 * abs(x["integral"])


def test_batch256_shape_sampled():
    """The 256-problem batch (d in 2..16, a in [0.05, 0.3], events
    log-uniform in [1e4, 1e7], 5 adaptation + 5 accumulation iterations,
    FP32-mixed): every result is finite and near its closed form, and the
    smallest problems match the oracle run of the same problem."""
    from scipy import special
    probs = workloads.batch256()
    b = VegasBatch(probs, 10, 5)
    b.run()
    res = b.results()
    assert len(res) == 256
    pulls = []
    for p, q in enumerate(probs):
        a, d = q["params"][0], q["dim"]
        exact = special.erf(0.5 / a) ** d
        assert np.isfinite(res[p]["integral"]) and res[p]["n_combined"] == 5
        pulls.append((res[p]["integral"] - exact) / res[p]["sigma"])
    pulls = np.array(pulls)
    # a narrow peak in many dimensions seen by few events can make Vegas lock
    # onto the wrong region (a property of the method, checked below against
    # the oracle); the bulk of the problems land within 5 sigma
    assert np.mean(np.abs(pulls) < 5) > 0.9
    order = list(np.argsort([q["n_events"] for q in probs])[:4])
    worst = int(np.argmax(np.abs(pulls)))
    if probs[worst]["n_events"] <= 2_000_000:
        order.append(worst)
    for p in order:
        q = dict(probs[p])
        ref = _oracle_run(q, 10, 5)
        I, s, _ = ref["final"]
        assert abs(res[p]["integral"] - I) <= 0.1 * s, (p, res[p]["integral"], I, s)


def _hist_close(Hg, Ho, tol):
    return np.all(np.abs(Hg - Ho) <= tol * Ho.sum(axis=1, keepdims=True))


def test_batch256_lockstep_against_oracle():
    """The benchmarked 256-problem FP32-mixed batch, stepped one iteration at
    a time with the kernels the graph records: for two problems of each
    dimension bucket (d <= 4, <= 8, <= 16; the largest event count of the
    bucket and a middling one), every iteration's S1, S2 and (adaptation
    iterations) every histogram bin against the oracle on the batch's own
    grid at 1e-6, and every refinement against the oracle's refinement of the
    batch's histograms at 1e-12.  After the last step the combined results
    equal those of a graph replay."""
    probs = workloads.batch256()
    n_iter, n_adapt = 10, 5
    b = VegasBatch(probs, n_iter, n_adapt)
    sel = []
    for lo, hi in ((2, 4), (5, 8), (9, 16)):
        ps = [p for p, q in enumerate(probs) if lo <= q["dim"] <= hi]
        ps.sort(key=lambda p: probs[p]["n_events"])
        sel += [ps[-1], ps[len(ps) // 2]]
    assert len(set(sel)) == 6
    with pytest.raises(Exception):
        b.step(3)  # steps run in order from 0
    for p in sel:  # the plan leaves every problem at its start
        assert np.array_equal(b.edges(p), oracle.uniform_edges(probs[p]["dim"], 50))
    tol = 1e-6
    for k in range(n_iter):
        before = {p: b.edges(p) for p in sel}
        b.step(k)
        for p in sel:
            q = probs[p]
            pr = oracle.Problem(q["dim"], 50, oracle.GAUSS, q["params"], seed=0, problem=q["problem"])
            S1, S2, H = b.last_iteration(p)
            o1, o2, Ho = oracle.accumulate(pr, before[p], k, q["n_events"])
            assert abs(S1 - o1) <= tol * abs(o1), (p, k, S1, o1)
            assert abs(S2 - o2) <= tol * abs(o2), (p, k, S2, o2)
            E = b.edges(p)
            if k < n_adapt:
                assert _hist_close(H, Ho, tol), (p, k)
                assert np.max(np.abs(E - oracle.refine(H, before[p], 1.5))) <= 1e-12, (p, k)
            else:
                assert np.all(H == 0.0) and np.array_equal(E, before[p])
    stepped = b.results()
    b.run()
    replay = b.results()
    for x, y in zip(stepped, replay):
        # the histograms' LDS atomics add in no fixed order, so the grids (and
        # what follows) agree to rounding
        assert abs(x["integral"] - y["integral"]) <= 1e-10 * abs(y["integral"])
        assert x["n_combined"] == y["n_combined"] == n_iter - n_adapt


def test_forced_launch_shape_gives_the_same_results(monkeypatch):
    """The tuner's choice only changes the speed: a batch planned with a shape
    it did not choose (threads and histogram replicas forced for every
    bucket) gives the same per-problem results up to the reduction order."""
    probs = _small_batch("fp32_mixed", n=8, seed=5)
    b = VegasBatch(probs, 4, 2)
    sched = b.schedule()
    assert len(sched["buckets"]) >= 1 and sched["tuned_ms"] > 0
    b.run()
    r1 = b.results()
    bk = sched["buckets"][0]
    th = 256 if bk["threads"] != 256 else 1024
    rp = 2 if bk["replicas"] != 2 else 8
    monkeypatch.setenv("VEGAS_BATCH_THREADS", str(th))
    monkeypatch.setenv("VEGAS_BATCH_REPLICAS", str(rp))
    c = VegasBatch(probs, 4, 2)
    s2 = c.schedule()
    assert all(x["threads"] == th and x["replicas"] == rp for x in s2["buckets"]), s2
    c.run()
    r2 = c.results()
    for x, y in zip(r1, r2):
        assert abs(x["integral"] - y["integral"]) <= 1e-10 * abs(y["integral"])
        assert abs(x["sigma"] - y["sigma"]) <= 1e-8 * y["sigma"]


def test_tuning_cache_round_trip(monkeypatch, tmp_path):
    """With VEGAS_BATCH_TUNE_CACHE set, the first plan tunes and stores its
    choice; a second plan of the same batch on the same device reads it back
    (no tuning) and gets the same schedule."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("VEGAS_BATCH_TUNE_CACHE", str(path))
    probs = _small_batch("fp64", n=5, seed=9)
    a = VegasBatch(probs, 3, 2)
    sa = a.schedule()
    assert not sa["from_cache"] and path.exists()
    b = VegasBatch(probs, 3, 2)
    sb = b.schedule()
    assert sb["from_cache"]
    assert sb["tile_events"] == sa["tile_events"] and sb["buckets"] == sa["buckets"]
    a.run()
    b.run()
    for x, y in zip(a.results(), b.results()):
        assert abs(x["integral"] - y["integral"]) <= 1e-12 * abs(y["integral"])
