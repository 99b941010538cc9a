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
        return {"tile_events": t.value, "blocks": b.value, "n_items": n.value, "tuned_ms": ms.value}

    def close(self):
        if getattr(self, "_b", None):
            lib().vegas_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
