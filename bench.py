"""Throughput of one Vegas iteration on one MI355X.

Workload (the d = 8 Gaussian case): f(x) = prod_i exp(-(x_i - 1/2)^2/a^2)/(a sqrt(pi)),
a = 0.1, on [0,1]^8, 50 bins per dimension, alpha = 1.5, Philox seed 0,
1e7 events per iteration.  One step = one adaptation iteration of the whole hot
path: points -> map -> integrand -> sums and histograms -> merge ->
statistics -> refinement, all on the device.  The headline value is events/s
of the FP32-mixed path; the FP64 path is timed the same way beside it.

Also reported: the event kernel's roofline (VALU issue bound, with the HBM
traffic of its counter summary), the whole 5 adaptation + 5 accumulation
schedule for both precisions (eager and as a HIP graph), accumulation and
plain Monte Carlo iterations, the d = 4 FP64 case, the d = 20 bimodal
integrand streamed in 1e7-event chunks, the 256-problem batch, the
differentiable forward + backward, the same Gaussian as a user integrand
compiled at run time (both precisions), the Genz discontinuous and
product-peak integrands at d = 16, the VALU issue-rate probe, and the CPU
oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       python bench.py --profile-legs | --issue-probe
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# worker processes of the CPU baseline (at most; the host's cores otherwise)
CPU_WORKERS = 12
# untimed event-kernel launches (about 0.1 s of load) before a timed path
CLOCK_WARM_LAUNCHES = 2000
METRIC = "events/s per Vegas iteration (d=8 Gaussian, 1e7 evts), FP32-mixed vs FP64"
D, NBINS, A, ALPHA, EVENTS = 8, 50, 0.1, 1.5, 10_000_000

# Peak VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz,
# in lane-slots per second (one full-rate wave64 VALU instruction takes four
# cycles of one SIMD).
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9


def alg_slots_per_event(d: int) -> int:
    """VALU issue slots per event that the method needs for the Gaussian at
    dimension d, from a fixed table of its steps (written from the method,
    not read from this kernel's instruction counts, so a wasteful kernel
    cannot raise its own ceiling):
      Philox4x32-10: ceil(d/4) calls x 10 rounds x (2 wide multiplies
        + 2 XORs)                                            40 ceil(d/4)
      binning: per dimension 1 wide multiply-add + 1 integer op       2d
      map: per dimension convert + fma + table address                3d
      integrand: per dimension subtract + fma, 3 more, and one
        exponential at 4 slots (a quarter-rate transcendental)    2d + 7
      Jacobian: per dimension 1 multiply                               d
      sums: convert, square and two compensated updates               10
      histograms: per dimension 1 address                              d
    = 40 ceil(d/4) + 9d + 17, 169 at d = 8.  The table reads and histogram
    atomics run on the LDS pipe and are not counted.  Every VALU instruction
    is one slot except the exponential; the 32x32->64 multiply-add issues at
    the full rate on gfx950 (bench.py --issue-probe measures both)."""
    return 40 * math.ceil(d / 4) + 9 * d + 17


# Counter summary of the event kernel (HBM bytes per launch from FETCH_SIZE and
# WRITE_SIZE, scaled by the same counters on a plain copy of known size).  It
# holds for the kernel built from these sources only.
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_sample_gauss_d8_1e7_mixed_pmc.md")
KERNEL_SOURCES = ("k_sample.hip", "device_common.hpp", "vegas_internal.hpp")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2002_12921_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters():
    """(bytes per launch, VALU busy, note): the counter-derived HBM traffic of
    the event kernel and the share of its SIMD cycles that issued VALU
    instructions, or Nones when there is no summary or the kernel changed
    since the counters were taken."""
    try:
        with open(PMC_SUMMARY) as fh:
            text = fh.read()
    except OSError:
        return None, None, "no counter summary"
    vals = dict(re.findall(r"^- (\w+): (\S+)$", text, re.M))
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return None, None, "kernel changed since the counters were taken"
    busy = float(vals["valu_busy"]) if "valu_busy" in vals else None
    return float(vals["traffic_bytes_per_launch"]), busy, (
        f"FETCH_SIZE x {vals['fetch_scale']} + WRITE_SIZE x {vals['write_scale']} (copy-calibrated), "
        f"{os.path.relpath(PMC_SUMMARY, ROOT)}")


_CLOCK_CTX = []


def warm_clock():
    """About 0.1 s of back-to-back d = 8 event-kernel launches, untimed (the
    context's state stays as it was): the GPU's clock drops within half a
    second of idling and needs tens of ms of load to come back, so every
    timed leg starts after this burst, whatever its own warm-up."""
    from paper_2002_12921_amd import Vegas

    if not _CLOCK_CTX:
        _CLOCK_CTX.append(Vegas(D, NBINS, "gauss", [A] + [0.5] * D, "fp32_mixed", seed=0, alpha=ALPHA))
    _CLOCK_CTX[0].time_event_kernel(EVENTS, CLOCK_WARM_LAUNCHES)


def _events_per_s(ms_per_step: float) -> float:
    return EVENTS / (ms_per_step * 1e-3)


def time_accumulation(precision: str, steps: int, warmup: int, adapt: int = 5):
    """Accumulation iterations on a frozen (adapted) grid: no histograms and
    no refinement, the rest of the path as in the adaptation step.  With
    adapt = 0 the grid stays uniform: plain Monte Carlo."""
    import torch
    from paper_2002_12921_amd import Vegas

    v = Vegas(D, NBINS, "gauss", [A] + [0.5] * D, precision, seed=0, alpha=ALPHA)
    for _ in range(adapt):
        v.iterate(EVENTS, refine=True, combine=False)
    warm_clock()
    for _ in range(warmup):
        v.iterate(EVENTS, hist=False)
    v.reset_results()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        v.iterate(EVENTS, hist=False)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    return {"ms_per_iteration": ms, "events_per_s": _events_per_s(ms)}


def time_path(precision: str, steps: int, warmup: int, blocks: int = 0, replicas: int = 0,
              source: str | None = None):
    """Two timed passes over `steps` adaptation iterations: the first with
    nothing but the HIP events around the whole region (the headline), the
    second with the library's events around each kernel of each step (their
    durations within a step; the event records themselves add a few
    microseconds each).  Then the event kernel alone: `steps` launches back
    to back between two events on its stream, whose duration per launch sets
    the roofline figure.  source: the same Gaussian as a user integrand
    (compiled at run time, in the given precision), timed the same way."""
    import torch
    from paper_2002_12921_amd import Vegas

    params = [A] + [0.5] * D
    t_init = time.perf_counter()
    if source is None:
        v = Vegas(D, NBINS, "gauss", params, precision, seed=0, alpha=ALPHA)
    else:
        v = Vegas(D, NBINS, params=params, source=source, precision=precision, seed=0, alpha=ALPHA)
    init_s = time.perf_counter() - t_init
    if blocks:
        v.set_launch(blocks)
    if replicas:
        v.set_hist_replicas(replicas)
    stream = torch.cuda.current_stream()
    # The GPU's clock drops within half a second of idle and comes back after
    # tens of milliseconds of sustained load: a step measured straight after
    # idle takes ~56 us instead of ~48.  So the event kernel first runs for
    # about 0.1 s, untimed (it leaves the context's state as it was), before
    # the warm-up steps and the timed ones.
    v.time_event_kernel(EVENTS, CLOCK_WARM_LAUNCHES)
    for k in range(warmup):
        v.iterate(EVENTS, refine=True, combine=False)
        if k % 1000 == 999:
            v.reset_results()  # at most 1024 recorded iterations per context
    v.reset_results()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        v.iterate(EVENTS, refine=True, combine=False)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(stop)

    v.reset_results()
    v.timing_enable(True)
    for _ in range(steps):
        v.iterate(EVENTS, refine=True, combine=False)
    sample_ms, merge_ms, n = v.timing_read()
    v.timing_enable(False)
    # the event kernel alone: `steps` launches back to back between two events
    kernel_ms = v.time_event_kernel(EVENTS, steps)
    # one more adaptation step, kept for the comparison with the oracle
    E_before = v.edges()
    t = v.iteration_index
    v.iterate(EVENTS, refine=True, combine=False)
    S1, S2, H = v.last_iteration()
    lockstep = {"t": t, "edges": E_before, "edges_after": v.edges(), "S1": S1, "S2": S2, "H": H}
    return {
        "lockstep": lockstep,
        "ms_per_step": total_ms / steps,
        "wall_ms_per_step": wall * 1e3 / steps,
        "events_per_s": _events_per_s(total_ms / steps),
        "event_kernel_ms": kernel_ms,
        "event_kernel_ms_in_step": sample_ms / n,
        "merge_kernel_ms_in_step": merge_ms / n,
        "launch": v.launch_info(),
        "init_s": init_s,
    }


def c2_schedule(precision: str):
    """5 adaptation iterations (refined after, left out of the result), then
    5 accumulation iterations on the frozen grid (no histograms), 1e7 events each."""
    import torch
    from paper_2002_12921_amd import Vegas

    v = Vegas(D, NBINS, "gauss", [A] + [0.5] * D, precision, seed=0, alpha=ALPHA)
    warm_clock()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        v.iterate(EVENTS, refine=True, combine=False)
    for _ in range(5):
        v.iterate(EVENTS, hist=False)
    r = v.result()
    wall = time.perf_counter() - t0
    out = {"integral": r["integral"], "sigma": r["sigma"], "chi2_dof": r["chi2_dof"],
           "rel_err": r["sigma"] / r["integral"], "wall_ms": wall * 1e3}
    try:
        out.update(c2_schedule_graph(precision, r["integral"], r["sigma"]))
    except RuntimeError as e:  # capture refused, or a replay that disagreed
        out["graph_error"] = str(e)
    return out


def c2_schedule_graph(precision: str, integral: float, sigma: float, reps: int = 5):
    """The same 10 iterations recorded once as a HIP graph (stream capture of
    the library's launches) and replayed `reps` times, each replay from the
    uniform grid: GPU time of the whole schedule without host launch gaps.
    Every replay's combined result is checked against the eager run (equal
    up to the rounding that the nondeterministic histogram sums leave in the
    refined grids)."""
    import torch
    from paper_2002_12921_amd import Vegas

    v = Vegas(D, NBINS, "gauss", [A] + [0.5] * D, precision, seed=0, alpha=ALPHA)
    E0 = v.edges()
    s = torch.cuda.Stream()
    v.stream = s
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        for _ in range(5):
            v.iterate(EVENTS, refine=True, combine=False)
        for _ in range(5):
            v.iterate(EVENTS, hist=False)
    ms, worst = [], 0.0
    warm_clock()
    for _ in range(reps):
        v.set_edges(E0)  # on s, before the replay
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        with torch.cuda.stream(s):  # replay() launches on the current stream
            g.replay()
        e1.record(s)
        r = v.result()
        ms.append(e0.elapsed_time(e1))
        worst = max(worst, abs(r["integral"] - integral) / sigma)
        if not worst <= 1e-6:
            raise RuntimeError(f"graph replay differs from the eager schedule by {worst} sigma")
    return {"graph_ms": min(ms), "graph_ms_all": ms, "graph_replay_minus_eager_in_sigma_max": worst}


def batch_c5(reps: int):
    """The 256-problem batch (d in 2..16, a in [0.05, 0.3], events log-uniform
    in [1e4, 1e7], 50 bins, FP32-mixed), 5 adaptation + 5 accumulation
    iterations per problem, as one recorded graph replayed `reps` times; beside
    it the same problems run one after another through the single-problem
    entry points."""
    import torch
    from paper_2002_12921_amd import Vegas, workloads
    from paper_2002_12921_amd.batch import VegasBatch

    probs = workloads.batch256()
    n_iter, n_adapt = 10, 5
    total = n_iter * sum(q["n_events"] for q in probs)
    t0 = time.perf_counter()
    b = VegasBatch(probs, n_iter, n_adapt)
    plan_s = time.perf_counter() - t0
    b.run()
    warm_clock()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        b.run()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    res = b.results()
    sched = b.schedule()
    b.close()

    ctxs = [Vegas(q["dim"], q["n_bins"], "gauss", q["params"], q["precision"], seed=q["seed"],
                  alpha=q["alpha"], problem=q["problem"]) for q in probs]
    warm_clock()
    torch.cuda.synchronize()
    start.record()
    for v, q in zip(ctxs, probs):
        for _ in range(n_adapt):
            v.iterate(q["n_events"], refine=True, combine=False)
        for _ in range(n_iter - n_adapt):
            v.iterate(q["n_events"])
    stop.record()
    torch.cuda.synchronize()
    seq_ms = start.elapsed_time(stop)
    return {"events_per_s": total / (ms * 1e-3), "ms_per_run": ms, "events_per_run": total,
            "tile_events": sched["tile_events"], "blocks": sched["blocks"], "n_items": sched["n_items"],
            "buckets": sched["buckets"], "tuned_ms": sched["tuned_ms"], "plan_s": plan_s,
            "sequential_ms": seq_ms, "batch_over_sequential": seq_ms / ms,
            "finite_results": int(sum(1 for r in res if math.isfinite(r["integral"])))}


def c3_streamed():
    """The d = 20 bimodal workload (a = 0.05 at 1/3 and 2/3, N = 100, FP32-mixed):
    10 iterations of 1e8 events, each streamed as 10 chunks of 1e7 (5
    adaptation iterations, then 5 accumulation iterations without histograms)."""
    import torch
    from paper_2002_12921_amd import Vegas, workloads

    v = Vegas(20, 100, "bimodal", workloads.bimodal20(), "fp32_mixed", seed=0, alpha=ALPHA)
    chunks, per = 10, 10_000_000

    def iteration(adapt: bool):
        for k in range(chunks):
            ch = "begin" if k == 0 else ("end" if k == chunks - 1 else "mid")
            v.iterate(per, chunk=ch, refine=adapt, combine=not adapt, hist=adapt)

    iteration(True)  # warm-up (its own grid step)
    warm_clock()
    v.reset_results()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for it in range(10):
        iteration(it < 5)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    r = v.result()
    return {"events_per_s": 10 * chunks * per / (ms * 1e-3), "ms_total": ms, "integral": r["integral"],
            "sigma": r["sigma"], "chi2_dof": r["chi2_dof"], "exact": 1.0}


def differentiable_c4(steps: int, warmup: int):
    """The differentiable d = 8 case: centres mu ~ U[0.3, 0.7] (seed 0) and
    a = 0.1 as FP32 parameters, FP32-mixed, a grid adapted by 5 iterations of
    1e6 events; one forward + backward = an iteration of 1e7 events on the
    frozen grid (VegasIntegral.forward) and the adjoint over the same points
    (VegasIntegral.backward), through torch.autograd."""
    import torch
    from paper_2002_12921_amd import Vegas, workloads
    from paper_2002_12921_amd.autograd import vegas_integral

    mu0, a0 = workloads.c4_params()
    params = [float(a0)] + [float(m) for m in mu0]
    v = Vegas(D, NBINS, "gauss", params, "fp32_mixed", seed=0, alpha=ALPHA)
    for _ in range(5):
        v.iterate(1_000_000, refine=True, combine=False)
    mu = torch.tensor(mu0, device="cuda", requires_grad=True)
    a = torch.tensor(a0, device="cuda", requires_grad=True)

    def step():
        mu.grad = None
        a.grad = None
        vegas_integral(mu, a, v, EVENTS).backward()

    warm_clock()
    for _ in range(max(2, warmup)):
        step()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    return {"ms_per_forward_backward": ms, "events_per_s": EVENTS / (ms * 1e-3),
            "grad_mu0": float(mu.grad[0]), "grad_a": float(a.grad)}


def genz_d16(steps: int, warmup: int):
    """The paper's second workload: the Genz discontinuous and product-peak
    integrands at d = 16 (workloads.genz16), 50 bins, 1e7 events per
    adaptation iteration, in both precisions: events/s of the adaptation
    step and the event kernel alone (back-to-back launches)."""
    import torch
    from paper_2002_12921_amd import Vegas, workloads

    out = {}
    for kind in ("genz_disc", "genz_peak"):
        for prec in ("fp32_mixed", "fp64"):
            v = Vegas(16, NBINS, kind, workloads.genz16(kind), prec, seed=0, alpha=ALPHA)
            warm_clock()
            for _ in range(warmup):
                v.iterate(EVENTS, refine=True, combine=False)
            v.reset_results()
            torch.cuda.synchronize()
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record()
            for _ in range(steps):
                v.iterate(EVENTS, refine=True, combine=False)
            stop.record()
            torch.cuda.synchronize()
            v.reset_results()
            ms = start.elapsed_time(stop) / steps
            out[f"{kind}_{prec}"] = {"ms_per_step": ms, "events_per_s": _events_per_s(ms),
                                     "event_kernel_ms": v.time_event_kernel(EVENTS, steps),
                                     "launch": v.launch_info()}
    return out


def c1_small(reps: int):
    """The d = 4 FP64 case: 10 iterations of 1e5 events, each refined after and
    all combined, call by call (best of `reps` runs; at this size the launches,
    not the events, set the time)."""
    import torch
    from paper_2002_12921_amd import Vegas

    d, n_ev, n_iter = 4, 100_000, 10
    params = [A] + [0.5] * d
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run():
        v = Vegas(d, NBINS, "gauss", params, "fp64", seed=0, alpha=ALPHA)
        warm_clock()
        torch.cuda.synchronize()
        start.record()
        for _ in range(n_iter):
            v.iterate(n_ev, refine=True)
        stop.record()
        torch.cuda.synchronize()
        return start.elapsed_time(stop), v.result()

    run()
    ms, r = min((run() for _ in range(reps)), key=lambda x: x[0])

    # the same 10 iterations recorded once as a HIP graph and replayed from
    # the uniform grid: the launches' GPU time without the host's gaps
    v = Vegas(d, NBINS, "gauss", params, "fp64", seed=0, alpha=ALPHA)
    E0 = v.edges()
    s = torch.cuda.Stream()
    v.stream = s
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        for _ in range(n_iter):
            v.iterate(n_ev, refine=True)
    gms, worst = [], 0.0
    for _ in range(reps + 1):
        v.set_edges(E0)  # on s, before the replay
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        with torch.cuda.stream(s):  # replay() launches on the current stream
            g.replay()
        e1.record(s)
        rg = v.result()
        gms.append(e0.elapsed_time(e1))
        worst = max(worst, abs(rg["integral"] - r["integral"]) / r["sigma"])
        if not worst <= 1e-6:
            raise RuntimeError(f"graph replay differs from the eager run by {worst} sigma")
    return {"ms_total": ms, "events_per_s": n_iter * n_ev / (ms * 1e-3), "integral": r["integral"],
            "sigma": r["sigma"], "exact": 0.99999999999385016,
            "graph_ms": min(gms[1:]), "graph_replay_minus_eager_in_sigma_max": worst}


def phase_split(steps: int):
    """Event- and reduction-kernel times of three kinds of iteration on the
    d = 8 workload (after 3 adaptation iterations): with refinement, without
    refinement, and without histograms; per-kernel HIP events on the stream."""
    import torch
    from paper_2002_12921_amd import Vegas

    out = {}
    for prec in ("fp32_mixed", "fp64"):
        v = Vegas(D, NBINS, "gauss", [A] + [0.5] * D, prec, seed=0, alpha=ALPHA)
        for _ in range(3):
            v.iterate(EVENTS, refine=True, combine=False)
        torch.cuda.synchronize()
        res = {}
        for label, kw in (("refine", {"refine": True, "combine": False}), ("no_refine", {"combine": False}),
                          ("no_hist", {"hist": False})):
            v.timing_enable(True)
            for _ in range(steps):
                v.iterate(EVENTS, **kw)
            s_ms, m_ms, n = v.timing_read()
            v.timing_enable(False)
            res[label] = {"event_kernel_ms": s_ms / n, "merge_kernel_ms": m_ms / n}
        out[prec] = res
    return out


def _oracle_chunk(args):
    """Worker of the CPU baseline: the oracle's sums over one contiguous range
    of events of one iteration (the oracle as it stands, one call)."""
    import numpy as np
    import oracle
    params, E, t, e0, n = args
    pr = oracle.Problem(D, NBINS, oracle.GAUSS, params, seed=0, alpha=ALPHA)
    return oracle.accumulate(pr, np.asarray(E), t, n, e0)


def _oracle_iteration(pool, workers: int, params, E, t: int, n: int):
    """The oracle's (S1, S2, H) of one iteration, its events split into one
    contiguous range per worker process; the ranges' sums are added in
    order (S1, S2 with math.fsum)."""
    import numpy as np
    step = -(-n // workers)
    jobs = [(params, E.tolist(), t, e0, min(step, n - e0)) for e0 in range(0, n, step)]
    parts = pool.map(_oracle_chunk, jobs)
    S1 = math.fsum(p[0] for p in parts)
    S2 = math.fsum(p[1] for p in parts)
    H = np.sum(np.stack([p[2] for p in parts]), axis=0)
    return S1, S2, H


def cpu_baseline(pool, workers: int, iters: int, lockstep: dict):
    """The FP64 oracle (plain C, as it stands) on the same workload, on the
    host's cores: `iters` adaptation iterations of 1e7 events with
    refinement, seed 0, each iteration's events split over `workers`
    processes.  Also the error of each GPU path against the oracle on one
    adaptation iteration of the benchmark, run in lockstep on the path's own
    grid (the same points): |dS1|/S1, |dS2|/S2, the largest histogram
    difference over its dimension's total, and the refined grid against the
    oracle's refinement of the path's histograms."""
    import numpy as np
    import oracle
    params = [A] + [0.5] * D
    E = oracle.uniform_edges(D, NBINS)
    _oracle_iteration(pool, workers, params, E, 0, 2 * workers)  # workers load the oracle
    t0 = time.perf_counter()
    for t in range(iters):
        S1, S2, H = _oracle_iteration(pool, workers, params, E, t, EVENTS)
        E = oracle.refine(H, E, ALPHA)
    dt = time.perf_counter() - t0
    errors = {}
    for prec, rec in lockstep.items():
        o1, o2, Ho = _oracle_iteration(pool, workers, params, rec["edges"], rec["t"], EVENTS)
        tot = Ho.sum(axis=1, keepdims=True)
        errors[prec] = {
            "iteration": rec["t"],
            "S1_rel": abs(rec["S1"] - o1) / abs(o1),
            "S2_rel": abs(rec["S2"] - o2) / abs(o2),
            "hist_max_rel_to_dim_total": float(np.max(np.abs(rec["H"] - Ho) / tot)),
            "refined_edges_max_abs": float(np.max(np.abs(rec["edges_after"] -
                                                         oracle.refine(rec["H"], rec["edges"], ALPHA)))),
        }
        # I_t = S1/M (relative error that of S1) and its error sigma_t
        sg = math.sqrt(oracle.iteration_stats(rec["S1"], rec["S2"], EVENTS)[1])
        so = math.sqrt(oracle.iteration_stats(o1, o2, EVENTS)[1])
        errors[prec]["sigma_t_rel"] = abs(sg - so) / so
    affinity = len(os.sched_getaffinity(0))
    return {"value": iters * EVENTS / dt, "unit": "events/s", "cores": workers, "kind": "oracle",
            "host_cores_available": affinity,
            "sample": f"{iters} iterations x {EVENTS:.0e} events of the d=8 workload (accumulate + refine), "
                      f"FP64, each iteration's events split over {workers} processes, {dt:.1f} s",
            "error_vs_oracle": errors}


# VALU instructions per step of each issue-probe kernel's loop (eight chains;
# counted in the gfx950 code this build emits), and the 64-bit multiply-adds
# among them: mad: 8 v_mad_u64_u32 + 8 v_bitop3_b32 + 8 v_mov_b32; xor:
# 16 v_bitop3_b32; fma: 8 v_fma_f32; exp: 8 v_exp_f32.
PROBE_KERNELS = (("mad_bitop3", 24), ("bitop3", 16), ("fma_f32", 8), ("exp_f32", 8))
PROBE_ITERS = 32768


def issue_probe():
    """Issue rates of the instruction classes the VALU bound weighs
    (vegas_probe_issue_rates): lane-instructions per second of each probe
    kernel against the chip's VALU issue peak, and from them the issue slots
    one v_mad_u64_u32 and one v_exp_f32 take, with the XOR probe's rate as
    that of a full-rate instruction."""
    import ctypes
    import torch
    from paper_2002_12921_amd import _lib

    L = _lib.lib()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    scratch = torch.empty(4 * 256 * cus * 8, dtype=torch.uint8, device="cuda")
    ms = (ctypes.c_double * 4)()
    blocks = ctypes.c_int32()
    _lib.check(L.vegas_probe_issue_rates(ctypes.c_void_p(scratch.data_ptr()), scratch.numel(), PROBE_ITERS, ms,
                                         ctypes.byref(blocks), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
               "probe_issue_rates")
    threads = blocks.value * 256
    out = {"blocks": blocks.value, "iters": PROBE_ITERS}
    rates = {}
    for i, (name, per_step) in enumerate(PROBE_KERNELS):
        rate = PROBE_ITERS * threads * per_step / (ms[i] * 1e-3)
        rates[name] = rate
        out[name] = {"ms": ms[i], "lane_instr_per_s": rate, "frac_of_peak": rate / PEAK_SLOTS}
    full = rates["bitop3"]
    steps = PROBE_ITERS * threads
    # mad kernel: 16 full-rate instructions and 8 multiply-adds of w slots each
    out["mad_u64_u32_slots"] = (ms[0] * 1e-3 * full / steps - 16) / 8
    out["exp_f32_slots"] = ms[3] * 1e-3 * full / steps / 8
    out["fma_f32_slots"] = ms[2] * 1e-3 * full / steps / 8
    return out


def profile_legs():
    """Short runs of every benchmarked kernel, for rocprofv3 (traces and
    counters): the issue probe; the d = 8 Gaussian in both precisions (10
    adaptation steps, 5 accumulation iterations); the d = 20 bimodal (one
    adaptation and one accumulation iteration, each 10 chunks of 1e7); the
    Genz integrands at d = 16 (3 adaptation steps per kind and precision);
    the 256-problem batch (one graph replay; the plan reads its schedule from
    VEGAS_BATCH_TUNE_CACHE when set, so no tuning launches are traced); the
    differentiable d = 8 case (5 fused forward + backward passes, 3 separate
    adjoints); the d = 8 Gaussian as a user integrand (3 adaptation steps per
    precision); and the 256 MiB copy that scales the HBM counters."""
    import torch
    from paper_2002_12921_amd import Vegas, workloads
    from paper_2002_12921_amd.autograd import vegas_integral
    from paper_2002_12921_amd.batch import VegasBatch

    issue_probe()
    for prec in ("fp32_mixed", "fp64"):
        v = Vegas(D, NBINS, "gauss", [A] + [0.5] * D, prec, seed=0, alpha=ALPHA)
        for _ in range(10):
            v.iterate(EVENTS, refine=True, combine=False)
        for _ in range(5):
            v.iterate(EVENTS, hist=False)
    v = Vegas(20, 100, "bimodal", workloads.bimodal20(), "fp32_mixed", seed=0, alpha=ALPHA)
    for adapt in (True, False):
        for k in range(10):
            ch = "begin" if k == 0 else ("end" if k == 9 else "mid")
            v.iterate(EVENTS, chunk=ch, refine=adapt, combine=not adapt, hist=adapt)
    for kind in ("genz_disc", "genz_peak"):
        for prec in ("fp32_mixed", "fp64"):
            v = Vegas(16, NBINS, kind, workloads.genz16(kind), prec, seed=0, alpha=ALPHA)
            for _ in range(3):
                v.iterate(EVENTS, refine=True, combine=False)
    b = VegasBatch(workloads.batch256(), 10, 5)
    b.run()
    torch.cuda.synchronize()
    b.close()
    mu0, a0 = workloads.c4_params()
    v = Vegas(D, NBINS, "gauss", [float(a0)] + [float(m) for m in mu0], "fp32_mixed", seed=0, alpha=ALPHA)
    for _ in range(5):
        v.iterate(1_000_000, refine=True, combine=False)
    mu = torch.tensor(mu0, device="cuda", requires_grad=True)
    a = torch.tensor(a0, device="cuda", requires_grad=True)
    for _ in range(5):
        vegas_integral(mu, a, v, EVENTS).backward()
    for _ in range(3):
        vegas_integral(mu, a, v, EVENTS, False).backward()
    from paper_2002_12921_amd import user_integrands
    for prec in ("fp64", "fp32_mixed"):
        v = Vegas(D, NBINS, params=[A] + [0.5] * D, source=user_integrands.GAUSSIAN, precision=prec, seed=0,
                  alpha=ALPHA)
        for _ in range(3):
            v.iterate(EVENTS, refine=True, combine=False)
    copy_probe()
    torch.cuda.synchronize()


def copy_probe():
    """A plain device copy of known size (256 MiB), used to scale the HBM
    counters of a profiled run."""
    import torch
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the GPU's clock ramps over the first ~30 ms of sustained load (a d = 8
    # step drops from ~55 to ~48 us): the default warm-up covers that ramp
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=800)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--mixed-only", action="store_true")
    ap.add_argument("--fp64-only", action="store_true",
                    help="only time the FP64 adaptation step (for profiling the FP64 event kernel)")
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--profile-legs", action="store_true",
                    help="only run every benchmarked kernel briefly (for rocprofv3)")
    ap.add_argument("--issue-probe", action="store_true",
                    help="only run the VALU issue-rate probe")
    ap.add_argument("--phase-split", action="store_true",
                    help="only time iterations with/without refinement and without histograms")
    args = ap.parse_args()
    if not 1 <= args.steps <= 1000 or args.warmup < 0:
        print("--steps must be in [1, 1000] (a context records at most 1024 iterations) and --warmup >= 0",
              file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); the path is "
              "single-device by design", file=sys.stderr)
        sys.exit(2)

    # the CPU baseline's worker processes start before anything touches the GPU
    pool, workers = None, 0
    if not (args.no_cpu_baseline or args.copy_probe or args.phase_split or args.fp64_only or args.issue_probe
            or args.profile_legs):
        import multiprocessing as mp
        workers = max(1, min(len(os.sched_getaffinity(0)), CPU_WORKERS))
        pool = mp.get_context("spawn").Pool(workers)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()
    if args.phase_split:
        print(json.dumps({"phase_split": phase_split(args.steps)}), flush=True)
        return
    if args.issue_probe:
        print(json.dumps({"issue_probe": issue_probe()}), flush=True)
        return
    if args.profile_legs:
        profile_legs()
        print(json.dumps({"profile_legs": "done"}), flush=True)
        return
    if args.fp64_only:
        r = time_path("fp64", args.steps, args.warmup)
        print(json.dumps({"fp64_only": {k: r[k] for k in ("ms_per_step", "events_per_s", "event_kernel_ms")}}),
              flush=True)
        return

    # the issue probe first: ~40 ms of sustained load, which also brings the
    # GPU's clock up before the headline (a cold clock runs the first tens of
    # milliseconds of load ~15 % slower)
    probe = None if args.mixed_only else issue_probe()
    mixed = time_path("fp32_mixed", args.steps, args.warmup)
    fp64 = None if args.mixed_only else time_path("fp64", args.steps, args.warmup)
    sched = {} if args.mixed_only else {p: c2_schedule(p) for p in ("fp32_mixed", "fp64")}
    batch = None if args.mixed_only or args.batch_reps <= 0 else batch_c5(args.batch_reps)
    c3 = None if args.mixed_only else c3_streamed()
    c4 = None if args.mixed_only else differentiable_c4(args.steps, min(args.warmup, 300))
    c1 = None if args.mixed_only else c1_small(5)
    genz = None if args.mixed_only else genz_d16(min(args.steps, 100), min(args.warmup, 100))
    accum = None if args.mixed_only else {p: time_accumulation(p, args.steps, args.warmup)
                                          for p in ("fp32_mixed", "fp64")}
    plain = None if args.mixed_only else {p: time_accumulation(p, args.steps, args.warmup, adapt=0)
                                          for p in ("fp32_mixed", "fp64")}
    user = None
    if not args.mixed_only:
        from paper_2002_12921_amd import user_integrands
        user = {p: time_path(p, args.steps, args.warmup, source=user_integrands.GAUSSIAN)
                for p in ("fp64", "fp32_mixed")}

    slots = alg_slots_per_event(D)
    t_k = mixed["event_kernel_ms"] * 1e-3
    achieved = slots * EVENTS / t_k / 1e12
    peak = PEAK_SLOTS / 1e12
    traffic, valu_busy, traffic_note = measured_counters()
    out = {
        "metric": METRIC,
        "value": mixed["events_per_s"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "vegas_gauss_d8_1e7", "dim": D, "n_bins": NBINS, "a": A, "alpha": ALPHA,
                   "events_per_iteration": EVENTS, "seed": 0, "precision": "fp32_mixed (f64 sums)",
                   "step": "one adaptation iteration: sample+map+integrand+sums+histograms+merge+stats+refine"},
        "roofline": {"bound": "alu", "kernel": "k_sample (event kernel)", "achieved": achieved,
                     "peak": peak, "unit": "Tslot/s", "frac": achieved / peak, "traffic": traffic,
                     "traffic_unit": "bytes per launch", "traffic_note": traffic_note,
                     "alg_slots_per_event": slots, "kernel_ms": mixed["event_kernel_ms"],
                     "valu_busy_counters": valu_busy},
        "event_kernel_ms_in_step": mixed["event_kernel_ms_in_step"],
        "merge_kernel_ms_in_step": mixed["merge_kernel_ms_in_step"],
        "wall_ms_per_step": mixed["wall_ms_per_step"],
        "launch": mixed["launch"],
    }
    if fp64 is not None:
        out["fp64"] = {"value": fp64["events_per_s"], "ms_per_step": fp64["ms_per_step"],
                       "event_kernel_ms": fp64["event_kernel_ms"],
                       "event_kernel_ms_in_step": fp64["event_kernel_ms_in_step"],
                       "merge_kernel_ms_in_step": fp64["merge_kernel_ms_in_step"],
                       "launch": fp64["launch"]}
        out["mixed_over_fp64"] = mixed["events_per_s"] / fp64["events_per_s"]
    if sched:
        m, f = sched["fp32_mixed"], sched["fp64"]
        out["c2_schedule"] = {"fp32_mixed": m, "fp64": f,
                              "mixed_minus_fp64_in_sigma": (m["integral"] - f["integral"]) / f["sigma"],
                              "exact": 0.99999999998770032}
    if accum is not None:
        out["accumulation_iteration"] = accum
    if plain is not None:
        out["plain_mc_uniform_grid"] = plain
    if batch is not None:
        out["batch256"] = batch
    if c3 is not None:
        out["bimodal_d20_streamed"] = c3
    if c4 is not None:
        out["differentiable_d8"] = c4
    if c1 is not None:
        out["gauss_d4_fp64_small"] = c1
    if genz is not None:
        out["genz_d16"] = genz
    if user is not None:
        for p, builtin in (("fp64", fp64), ("fp32_mixed", mixed)):
            u = user[p]
            out["user_integrand_gauss_d8_" + p] = {
                "value": u["events_per_s"], "ms_per_step": u["ms_per_step"],
                "event_kernel_ms": u["event_kernel_ms"], "launch": u["launch"],
                "compile_and_init_s": u["init_s"],
                "over_builtin": u["events_per_s"] / builtin["events_per_s"] if builtin else None}
    if probe is not None:
        out["issue_probe"] = probe
    if pool is not None:
        lock = {"fp32_mixed": mixed["lockstep"]}
        if fp64 is not None:
            lock["fp64"] = fp64["lockstep"]
        out["cpu_baseline"] = cpu_baseline(pool, workers, args.cpu_iters, lock)
        out["cpu_baseline"]["gpu_over_cpu"] = mixed["events_per_s"] / out["cpu_baseline"]["value"]
        pool.close()
        pool.join()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
