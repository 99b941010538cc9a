"""Many independent Vegas integrations run as one recorded HIP graph.

Argument marshalling only: the library plans the work items, tunes the tile
size, records the run and replays it (include/vegas.h, vegas_batch_*).
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check, lib
from .integrator import make_desc


class VegasBatch:
    """problems: sequence of dicts with keys dim, n_bins, params, n_events and
    optionally integrand, precision, seed, alpha, problem (Philox problem
    index; defaults to the position in the batch)."""

    def __init__(self, problems: Sequence[dict], n_iter: int, n_adapt: int, device=None,
                 stream: Optional[torch.cuda.Stream] = None):
        n = len(problems)
        self.n = n
        self.stream = stream
        descs = (_lib.Desc * n)()
        self._keep = []
        self.dims, self.bins = [], []
        for p, q in enumerate(problems):
            d, keep = make_desc(q["dim"], q.get("n_bins", 50), q.get("integrand", "gauss"), q["params"],
                                q.get("precision", "fp32_mixed"), q.get("seed", 0), q.get("alpha", 1.5),
                                q.get("problem", p))
            descs[p] = d
            self._keep.append(keep)
            self.dims.append(q["dim"])
            self.bins.append(q.get("n_bins", 50))
        self._descs = descs
        ev = np.ascontiguousarray(np.array([int(q["n_events"]) for q in problems], dtype=np.int64))
        self._events = ev
        P = ctypes.POINTER
        evp = ev.ctypes.data_as(P(ctypes.c_int64))
        nbytes = ctypes.c_size_t()
        L = lib()
        check(L.vegas_batch_workspace_size(descs, evp, n, ctypes.byref(nbytes)), "batch_workspace_size")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            self._b = ctypes.c_void_p()
            check(L.vegas_batch_plan(ctypes.byref(self._b), descs, evp, n, ctypes.c_void_p(self.ws.data_ptr()),
                                     nbytes.value, n_iter, n_adapt, self._s()), "batch_plan")

    def _s(self):
        s = self.stream if self.stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    def run(self):
        check(lib().vegas_batch_run(self._b, self._s()), "batch_run")

    def step(self, k: int):
        """Iteration k of every problem, eagerly (k = 0 restarts; in order)."""
        check(lib().vegas_batch_step(self._b, int(k), self._s()), "batch_step")

    def last_iteration(self, p: int):
        """(S1, S2, H[d_p, N_p]) of problem p's last iteration."""
        sums = np.zeros(2)
        H = np.zeros((self.dims[p], self.bins[p]))
        P = ctypes.POINTER(ctypes.c_double)
        check(lib().vegas_batch_get_iteration(self._b, p, sums.ctypes.data_as(P), H.ctypes.data_as(P),
                                              self._s()), "batch_get_iteration")
        return sums[0], sums[1], H

    def results(self, allow_nonfinite: bool = False) -> list:
        out = (_lib.Result * self.n)()
        st = lib().vegas_batch_results(self._b, out, self._s())
        if not (allow_nonfinite and st == _lib.VEGAS_ENONFINITE):
            check(st, "batch_results")
        return [r.as_dict() for r in out]

    def edges(self, p: int) -> np.ndarray:
        e = np.zeros((self.dims[p], self.bins[p] + 1))
        check(lib().vegas_batch_get_edges(self._b, p, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          self._s()), "batch_get_edges")
        return e

    def schedule(self) -> dict:
        t, b, n, ms = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        check(lib().vegas_batch_schedule(self._b, ctypes.byref(t), ctypes.byref(b), ctypes.byref(n),
                                         ctypes.byref(ms)), "batch_schedule")
        out = {"tile_events": t.value, "blocks": b.value, "n_items": n.value, "tuned_ms": ms.value}
        L = lib()
        nb, fc = ctypes.c_int32(), ctypes.c_int32()
        check(L.vegas_batch_bucket(self._b, -1, ctypes.byref(nb), None, None, None, None, None, ctypes.byref(fc)),
              "batch_bucket")
        buckets = []
        for q in range(nb.value):
            dm, th, rp, bl, tm = (ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
                                  ctypes.c_double())
            check(L.vegas_batch_bucket(self._b, q, None, ctypes.byref(dm), ctypes.byref(th), ctypes.byref(rp),
                                       ctypes.byref(bl), ctypes.byref(tm), None), "batch_bucket")
            buckets.append({"dmax": dm.value, "threads": th.value, "replicas": rp.value, "blocks": bl.value,
                            "tuned_ms": tm.value})
        out["buckets"] = buckets
        out["from_cache"] = bool(fc.value)
        return out

    def close(self):
        if getattr(self, "_b", None):
            lib().vegas_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
