"""Plain FP64 CPU reference ("oracle") for one Vegas iteration.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_2002_12921_amd``) never imports it and shares no code with it.

The arithmetic lives in ``vegas_oracle.c`` (plain C, gcc, FP64,
``-ffp-contract=off``); this module only compiles it and marshals arguments.
What each function computes, and which passage of the paper or of the Vegas
method it follows, is documented in ``vegas_oracle.h``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vegas_oracle.c")
_LIB = os.path.join(_HERE, "libvegas_oracle.so")

GAUSS, BIMODAL, GENZ_DISC, GENZ_PEAK = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable flags: no -march=native, no FMA
    contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("kind", ctypes.c_int32), ("problem", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("alpha", ctypes.c_double),
                ("params", ctypes.POINTER(ctypes.c_double))]


_lib = None


def lib():
    """The compiled oracle; VEGAS_ORACLE_LIB names another build of the same
    source to load instead (the sanitizer build of paper_2002_12921_amd/sanitize.py)."""
    global _lib
    if _lib is None:
        path = os.environ.get("VEGAS_ORACLE_LIB")
        if not path:
            build(force=False)
            path = _LIB
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        d, u32, u64, i32 = ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        pd, pi32, pu32, pp = P(d), P(i32), P(u32), P(_Problem)
        sig = {
            "vo_philox4x32_10": (None, [pu32, pu32, pu32]),
            "vo_point": (None, [u64, u32, u32, u64, ctypes.c_int, pd]),
            "vo_bin": (None, [d, ctypes.c_int, pi32, pd]),
            "vo_map": (d, [pd, ctypes.c_int, ctypes.c_int, pd, pi32, pd, pd]),
            "vo_norm": (d, [pp]),
            "vo_integrand": (d, [pp, pd]),
            "vo_gauss_grad": (None, [pp, pd, pd]),
            "vo_accumulate": (None, [pp, pd, u32, u64, u64, pd, pd]),
            "vo_accumulate_points": (None, [pp, pd, pd, u64, pd, pd]),
            "vo_events": (None, [pp, pd, u32, u64, u64, pd]),
            "vo_iteration_stats": (None, [d, d, d, pd, pd]),
            "vo_refine": (None, [pd, pd, ctypes.c_int, ctypes.c_int, d, pd]),
            "vo_damp": (d, [d, d]),
            "vo_combine": (None, [pd, pd, ctypes.c_int, pd]),
            "vo_adjoint": (None, [pp, pd, u32, u64, u64, pd, pd]),
            "vo_run": (None, [pp, pd, u32, ctypes.c_int, u64, pi32, pi32, pd, pd, pd]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class Problem:
    """One integration problem; ``params`` layout as in vegas_oracle.h."""
    dim: int
    n_bins: int
    kind: int
    params: Sequence[float]
    seed: int = 0
    alpha: float = 1.5
    problem: int = 0
    _keep: list = field(default_factory=list, repr=False)

    def c(self) -> _Problem:
        p = _f64(self.params)
        self._keep = [p]
        return _Problem(self.dim, self.n_bins, self.kind, self.problem, self.seed,
                        self.alpha, _dp(p))


def uniform_edges(dim: int, n_bins: int) -> np.ndarray:
    """Uniform starting grid E_k = k/N in every dimension, shape (dim, N+1)."""
    e = np.arange(n_bins + 1, dtype=np.float64) / n_bins
    return np.tile(e, (dim, 1))


def philox(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().vo_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def point(seed: int, t: int, p: int, e: int, d: int) -> np.ndarray:
    y = np.zeros(d)
    lib().vo_point(seed, t, p, e, d, _dp(y))
    return y


def bin_of(y: float, n_bins: int):
    b = ctypes.c_int32()
    de = ctypes.c_double()
    lib().vo_bin(y, n_bins, ctypes.byref(b), ctypes.byref(de))
    return b.value, de.value


def map_point(edges: np.ndarray, y: np.ndarray):
    edges = _f64(edges)
    d, n1 = edges.shape
    y = _f64(y)
    b = np.zeros(d, dtype=np.int32)
    de = np.zeros(d)
    x = np.zeros(d)
    w = lib().vo_map(_dp(edges), d, n1 - 1, _dp(y),
                     b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(de), _dp(x))
    return b, de, x, w


def norm(pr: Problem) -> float:
    return lib().vo_norm(ctypes.byref(pr.c()))


def integrand(pr: Problem, x) -> float:
    x = _f64(x)
    return lib().vo_integrand(ctypes.byref(pr.c()), _dp(x))


def gauss_grad(pr: Problem, x) -> np.ndarray:
    x = _f64(x)
    g = np.zeros(pr.dim + 1)
    lib().vo_gauss_grad(ctypes.byref(pr.c()), _dp(x), _dp(g))
    return g


def accumulate(pr: Problem, edges: np.ndarray, t: int, n: int, e0: int = 0):
    """Returns (S1, S2, H[d, N])."""
    edges = _f64(edges)
    sums = np.zeros(2)
    H = np.zeros((pr.dim, pr.n_bins))
    lib().vo_accumulate(ctypes.byref(pr.c()), _dp(edges), t, e0, n, _dp(sums), _dp(H))
    return sums[0], sums[1], H


def accumulate_points(pr: Problem, edges: np.ndarray, y: np.ndarray):
    edges = _f64(edges)
    y = _f64(y)
    n = y.shape[0]
    sums = np.zeros(2)
    H = np.zeros((pr.dim, pr.n_bins))
    lib().vo_accumulate_points(ctypes.byref(pr.c()), _dp(edges), _dp(y), n, _dp(sums), _dp(H))
    return sums[0], sums[1], H


def events(pr: Problem, edges: np.ndarray, t: int, e0: int, n: int) -> np.ndarray:
    """Per-event rows: b[d], delta[d], x[d], w, f."""
    edges = _f64(edges)
    out = np.zeros((n, 3 * pr.dim + 2))
    lib().vo_events(ctypes.byref(pr.c()), _dp(edges), t, e0, n, _dp(out))
    return out


def accumulate_fn(dim: int, n_bins: int, seed: int, problem: int, edges: np.ndarray, t: int, n: int, f,
                  e0: int = 0, with_abs: bool = False):
    """(S1, S2, H[d, N]) of one iteration for an integrand given as a NumPy
    function f(x) -> values, x of shape (n, d) in FP64 (a user integrand).

    The points, bins and weights are the oracle's (``events``: Philox point,
    bin and offset, the piecewise-linear map and its Jacobian w = prod N W_b,
    none of which depends on the integrand, so the Gaussian integrand serves
    only as a carrier); then v = f(x) w, S1 = sum v, S2 = sum v^2 and
    H[i][b] = sum of v^2 over the events with b_i = b, the accumulators of the
    per-event stage of the Vegas iteration (sec. 2.2), each sum rounded once
    (math.fsum).  with_abs: also return sum |v| (the scale of S1's rounding
    when f changes sign)."""
    carrier = Problem(dim, n_bins, GAUSS, [0.1] + [0.5] * dim, seed=seed, problem=problem)
    ev = events(carrier, edges, t, e0, n)
    b = ev[:, :dim].astype(np.int64)
    x = ev[:, 2 * dim:3 * dim]
    w = ev[:, 3 * dim]
    v = np.asarray(f(x), dtype=np.float64) * w
    v2 = v * v
    H = np.zeros((dim, n_bins))
    for i in range(dim):
        order = np.argsort(b[:, i], kind="stable")
        bs, vs = b[order, i], v2[order]
        cuts = np.searchsorted(bs, np.arange(n_bins + 1))
        for k in range(n_bins):
            H[i, k] = math.fsum(vs[cuts[k]:cuts[k + 1]])
    if with_abs:
        return math.fsum(v), math.fsum(v2), H, math.fsum(np.abs(v))
    return math.fsum(v), math.fsum(v2), H


def iteration_stats(S1: float, S2: float, M: float):
    I = ctypes.c_double()
    v = ctypes.c_double()
    lib().vo_iteration_stats(S1, S2, float(M), ctypes.byref(I), ctypes.byref(v))
    return I.value, v.value


def refine(H: np.ndarray, edges: np.ndarray, alpha: float) -> np.ndarray:
    H = _f64(H)
    edges = _f64(edges)
    d, n1 = edges.shape
    out = np.zeros_like(edges)
    lib().vo_refine(_dp(H), _dp(edges), d, n1 - 1, alpha, _dp(out))
    return out


def damp(s: float, alpha: float) -> float:
    return lib().vo_damp(s, alpha)


def combine(I, var):
    I = _f64(I)
    var = _f64(var)
    out = np.zeros(3)
    lib().vo_combine(_dp(I), _dp(var), len(I), _dp(out))
    return out[0], out[1], out[2]


def adjoint(pr: Problem, edges: np.ndarray, t: int, n: int, e0: int = 0):
    """Returns (G[d+1], Gabs[d+1]), unscaled sums of w df/dtheta."""
    edges = _f64(edges)
    G = np.zeros(pr.dim + 1)
    Ga = np.zeros(pr.dim + 1)
    lib().vo_adjoint(ctypes.byref(pr.c()), _dp(edges), t, e0, n, _dp(G), _dp(Ga))
    return G, Ga


def run(pr: Problem, edges: np.ndarray, n_iter: int, n_events: int, refine_after, combine_mask,
        t0: int = 0):
    """Whole run.  Returns dict(edges, iters[n_iter, 2], final(I, sigma, chi2dof), H_last)."""
    E = _f64(edges).copy()
    ra = np.ascontiguousarray(np.asarray(refine_after, dtype=np.int32))
    cm = np.ascontiguousarray(np.asarray(combine_mask, dtype=np.int32))
    it = np.zeros((n_iter, 2))
    fin = np.zeros(3)
    H = np.zeros((pr.dim, pr.n_bins))
    P32 = ctypes.POINTER(ctypes.c_int32)
    lib().vo_run(ctypes.byref(pr.c()), _dp(E), t0, n_iter, n_events,
                 ra.ctypes.data_as(P32), cm.ctypes.data_as(P32), _dp(it), _dp(fin), _dp(H))
    return {"edges": E, "iters": it, "final": tuple(fin), "H_last": H}
