"""Seeded synthetic workloads (inputs only; no Vegas arithmetic here).

These are the problem specifications the tests and the benchmark share:
  gaussian(d)      the symmetric Gaussian of sec. 3.1 (a = 0.1, centre 1/2)
  bimodal20()      two Gaussians (a = 0.05) at 1/3 and 2/3 in d = 20, N = 100
  c4_params()      trainable centres mu ~ U[0.3, 0.7]^8 (seed 0) and a = 0.1, FP32
  batch256()       256 Gaussian problems: d ~ U{2..16}, a ~ U[0.05, 0.3],
                   events ~ 10^U[4, 7], 50 bins, seed 0, problem index = position
  genz16(kind)     the Genz integrands at d = 16 (the paper gives no c_i, a_i):
                   discontinuous c_i = 0.5..1.5, a_i = 0.05..0.3; product peak
                   c_i = 2..4, a_i = 0.3..0.7 (evenly spaced over i)
"""
from __future__ import annotations

import numpy as np


def gaussian(d: int = 8, a: float = 0.1, mu: float = 0.5) -> list:
    return [a] + [mu] * d


def bimodal20(a: float = 0.05) -> list:
    d = 20
    return [a] + [1.0 / 3.0] * d + [2.0 / 3.0] * d


def c4_params():
    mu = np.random.default_rng(0).uniform(0.3, 0.7, 8).astype(np.float32)
    return mu, np.float32(0.1)


def batch256(n: int = 256, seed: int = 2002, precision: str = "fp32_mixed") -> list:
    rng = np.random.default_rng(seed)
    dims = rng.integers(2, 17, n)
    widths = rng.uniform(0.05, 0.3, n)
    events = np.round(10.0 ** rng.uniform(4, 7, n)).astype(np.int64)
    return [{"dim": int(dims[p]), "n_bins": 50, "integrand": "gauss",
             "params": [float(widths[p])] + [0.5] * int(dims[p]),
             "n_events": int(events[p]), "precision": precision, "seed": 0, "alpha": 1.5,
             "problem": p} for p in range(n)]


def genz16(kind: str, d: int = 16) -> list:
    if kind == "genz_disc":
        return list(np.linspace(0.5, 1.5, d)) + list(np.linspace(0.05, 0.3, d))
    if kind == "genz_peak":
        return list(np.linspace(2.0, 4.0, d)) + list(np.linspace(0.3, 0.7, d))
    raise ValueError(kind)
