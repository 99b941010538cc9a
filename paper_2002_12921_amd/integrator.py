"""Python face of libvegas: argument marshalling only.

PyTorch provides the device workspace (one uint8 tensor) and the stream; every
step of an iteration runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

INTEGRANDS = {"gauss": _lib.GAUSS, "bimodal": _lib.BIMODAL,
              "genz_disc": _lib.GENZ_DISC, "genz_peak": _lib.GENZ_PEAK, "user": _lib.USER}
PRECISIONS = {"fp64": _lib.FP64, "fp32_mixed": _lib.FP32_MIXED, "mixed": _lib.FP32_MIXED}


# the current stream's handle without building a Stream object (a few
# microseconds per call otherwise, which a training loop pays on every step)
_raw_current_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> int:
    if stream is not None:
        return stream.cuda_stream
    if _raw_current_stream is not None:
        return _raw_current_stream(torch.cuda.current_device())
    return torch.cuda.current_stream().cuda_stream


def make_desc(dim: int, n_bins: int, integrand, params: Sequence[float], precision="fp64",
              seed: int = 0, alpha: float = 1.5, problem: int = 0):
    """Returns (Desc, keep-alive params array)."""
    kind = INTEGRANDS[integrand] if isinstance(integrand, str) else int(integrand)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64)).reshape(-1)
    d = _lib.Desc(dim, n_bins, kind, prec, seed, alpha,
                  p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(p), problem)
    return d, p


def compile_user(source: str, dim: int, precision="fp64") -> tuple[bool, str]:
    """Compile a user integrand for dimension dim and a precision without a
    device (see vegas_user_compile): (compiled?, compiler messages)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    buf = ctypes.create_string_buffer(1 << 16)
    st = lib().vegas_user_compile(source.encode(), int(dim), prec, buf, len(buf))
    if st not in (_lib.VEGAS_OK, _lib.VEGAS_ECOMPILE):
        check(st, "user_compile")
    return st == _lib.VEGAS_OK, buf.value.decode(errors="replace")


class Vegas:
    """One adaptive Vegas integration on the current HIP device.

    source: HIP device code defining
    ``__device__ vegas_real vegas_integrand(const vegas_real* x, int dim, const double* params)``
    (a user integrand, compiled at run time; vegas_real is double for
    precision "fp64" and float for "fp32_mixed"; integrand then defaults to
    "user" and params to none).

    static_workspace: use the device's one static context
    (vegas_init_grid_noalloc: no allocation; a later static Vegas on the same
    device takes it over)."""

    def __init__(self, dim: int, n_bins: int = 50, integrand=None,
                 params: Optional[Sequence[float]] = None, precision="fp64", seed: int = 0,
                 alpha: float = 1.5, problem: int = 0, device=None,
                 stream: Optional[torch.cuda.Stream] = None, source: Optional[str] = None,
                 static_workspace: bool = False):
        if integrand is None:
            integrand = "user" if source is not None else "gauss"
        if params is None:
            params = [] if source is not None else [0.1] + [0.5] * dim
        self.dim, self.n_bins = dim, n_bins
        self.desc, self._params = make_desc(dim, n_bins, integrand, params, precision, seed,
                                            alpha, problem)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream
        L = lib()
        if static_workspace:
            if source is not None:
                raise ValueError("user integrands need their own workspace")
            self.ws = None
            self._ctx = ctypes.c_void_p()
            with torch.cuda.device(self.device):
                check(L.vegas_init_grid_noalloc(ctypes.byref(self._ctx), ctypes.byref(self.desc), self._s()),
                      "init_grid_noalloc")
            return
        nbytes = ctypes.c_size_t()
        check(L.vegas_workspace_size(ctypes.byref(self.desc), ctypes.byref(nbytes)), "workspace_size")
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            self._ctx = ctypes.c_void_p()
            if source is not None:
                check(L.vegas_init_user(ctypes.byref(self._ctx), ctypes.byref(self.desc), source.encode(),
                                        ctypes.c_void_p(self.ws.data_ptr()), nbytes.value,
                                        self._s()), "init_user")
            else:
                check(L.vegas_init_grid(ctypes.byref(self._ctx), ctypes.byref(self.desc),
                                        ctypes.c_void_p(self.ws.data_ptr()), nbytes.value,
                                        self._s()), "init_grid")

    # -- helpers -----------------------------------------------------------
    def _s(self):
        return _stream_handle(self.stream)

    def close(self):
        if getattr(self, "_ctx", None):
            lib().vegas_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the hot path ------------------------------------------------------
    def iterate(self, n_events: int, refine: bool = False, combine: bool = True,
                chunk: Optional[str] = None, hist: bool = True, record: bool = True):
        """One iteration (or one chunk of one: chunk in {"begin", "mid", "end"}).
        hist=False skips the histograms (a frozen grid; every chunk alike);
        record=False keeps the estimate as the last iteration's only (no
        record slot, not combined)."""
        flags = {None: _lib.ITER_FULL, "begin": _lib.CHUNK_BEGIN, "mid": 0,
                 "end": _lib.CHUNK_END, "begin_end": _lib.ITER_FULL}[chunk]
        if flags & _lib.CHUNK_END:
            if refine:
                flags |= _lib.REFINE
            if not combine:
                flags |= _lib.NO_COMBINE
            if not record:
                flags |= _lib.NO_RECORD
        if not hist:
            flags |= _lib.NO_HIST
        check(lib().vegas_iterate(self._ctx, int(n_events), flags, self._s()), "iterate")

    def iterate_grad(self, n_events: int, G: torch.Tensor, combine: bool = True, record: bool = True):
        """One whole iteration on the frozen grid (no histograms) that also
        writes the estimate's gradient (1/M) sum w df/d(mu, a) into G (FP64,
        d + 1 values, on the device).  Gaussian integrand only."""
        assert G.is_cuda and G.dtype == torch.float64 and G.is_contiguous() and G.numel() >= self.dim + 1
        flags = _lib.ITER_FULL | _lib.NO_HIST
        if not combine:
            flags |= _lib.NO_COMBINE
        if not record:
            flags |= _lib.NO_RECORD
        check(lib().vegas_iterate_grad(self._ctx, int(n_events), flags, ctypes.c_void_p(G.data_ptr()), self._s()),
              "iterate_grad")

    def forward_grad(self, params: torch.Tensor, n_events: int, G: torch.Tensor, out: torch.Tensor,
                     rest: Optional[torch.Tensor] = None):
        """New parameters, then one frozen-grid iteration (no histograms, not
        recorded or combined) that writes the gradient of its estimate into G
        (FP64, d + 1) and (I_t, sigma_t) into out (FP64, 2): one library call.
        rest: None (all parameters in params), or the parameters after the
        first, with params holding only the first (a, then mu), same dtype."""
        assert params.is_cuda and params.is_contiguous() and params.dtype in (torch.float32, torch.float64)
        assert rest is None or (rest.is_cuda and rest.is_contiguous() and rest.dtype == params.dtype
                                and params.numel() == 1)
        assert G.is_cuda and G.dtype == torch.float64 and G.is_contiguous() and G.numel() >= self.dim + 1
        assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= 2
        self._forward_grad(params, n_events, G, out, rest)

    def _forward_grad(self, params, n_events, G, out, rest=None):
        """forward_grad without the argument checks (for callers that built
        the tensors themselves: the autograd function, whose step is
        host-paced)."""
        n = params.numel() if rest is None else 1 + rest.numel()
        check(lib().vegas_forward_grad(self._ctx, params.data_ptr(), None if rest is None else rest.data_ptr(), n,
                                       1 if params.dtype == torch.float32 else 0, int(n_events),
                                       _lib.ITER_FULL | _lib.NO_HIST | _lib.NO_COMBINE | _lib.NO_RECORD,
                                       G.data_ptr(), out.data_ptr(), self._s()),
              "forward_grad")

    def refine(self):
        check(lib().vegas_refine(self._ctx, self._s()), "refine")

    def result(self, allow_nonfinite: bool = False) -> dict:
        r = _lib.Result()
        st = lib().vegas_result(self._ctx, ctypes.byref(r), self._s())
        if not (allow_nonfinite and st == _lib.VEGAS_ENONFINITE):
            check(st, "result")
        return r.as_dict()

    def reset_results(self):
        check(lib().vegas_reset_results(self._ctx, self._s()), "reset_results")

    # -- parameters, adjoint -------------------------------------------------
    def set_params_device(self, params: torch.Tensor):
        assert params.is_cuda and params.is_contiguous() and params.dtype in (torch.float32, torch.float64)
        check(lib().vegas_set_params_device(self._ctx, ctypes.c_void_p(params.data_ptr()), params.numel(),
                                            1 if params.dtype == torch.float32 else 0, self._s()),
              "set_params_device")

    def get_params_device(self) -> torch.Tensor:
        """The context's current integrand parameters (FP64, on the device)."""
        n = self.desc.n_params
        out = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        check(lib().vegas_get_params_device(self._ctx, ctypes.c_void_p(out.data_ptr()), self._s()),
              "get_params_device")
        return out[:n]

    def versions(self) -> tuple[int, int]:
        """(grid version, parameter version): counters that advance whenever the
        edges or the integrand parameters change."""
        g, p = ctypes.c_int64(), ctypes.c_int64()
        check(lib().vegas_get_versions(self._ctx, ctypes.byref(g), ctypes.byref(p)), "get_versions")
        return g.value, p.value

    def last_iteration_device(self, out: torch.Tensor):
        assert out.is_cuda and out.dtype == torch.float64 and out.numel() >= 2
        check(lib().vegas_last_iteration_device(self._ctx, ctypes.c_void_p(out.data_ptr()), self._s()),
              "last_iteration_device")

    def grad_scale(self, G: torch.Tensor, gout: torch.Tensor, grad: torch.Tensor):
        """grad = gout * G (d + 1 values), one rounding to grad's dtype."""
        assert G.is_cuda and G.dtype == torch.float64 and G.is_contiguous() and G.numel() >= self.dim + 1
        assert gout.is_cuda and gout.dtype == torch.float64
        assert grad.is_cuda and grad.dtype in (torch.float64, torch.float32) and grad.is_contiguous()
        assert grad.numel() >= self.dim + 1
        self._grad_scale(G, gout, grad)

    def _grad_scale(self, G, gout, grad):
        """grad_scale without the argument checks (see _forward_grad)."""
        check(lib().vegas_grad_scale(G.data_ptr(), gout.data_ptr(), grad.data_ptr(), self.dim + 1,
                                     1 if grad.dtype == torch.float32 else 0, self._s()), "grad_scale")

    def adjoint(self, iteration: int, n_events: int, gout: torch.Tensor, grad: torch.Tensor):
        """grad (d + 1 values, FP64 or FP32) = gout (1/M) sum_e w_e df/d(mu, a)."""
        assert gout.is_cuda and gout.dtype == torch.float64
        assert grad.is_cuda and grad.dtype in (torch.float64, torch.float32) and grad.numel() >= self.dim + 1
        assert grad.is_contiguous()
        check(lib().vegas_adjoint(self._ctx, iteration, n_events, ctypes.c_void_p(gout.data_ptr()),
                                  ctypes.c_void_p(grad.data_ptr()), 1 if grad.dtype == torch.float32 else 0,
                                  self._s()), "adjoint")

    # -- inspection ------------------------------------------------------------
    @property
    def iteration_index(self) -> int:
        t = ctypes.c_int64()
        check(lib().vegas_get_iteration_index(self._ctx, ctypes.byref(t)), "get_iteration_index")
        return t.value

    def dump_events(self, first: int, count: int, iteration: Optional[int] = None) -> torch.Tensor:
        it = self.iteration_index if iteration is None else iteration
        out = torch.empty((count, 3 * self.dim + 2), dtype=torch.float64, device=self.device)
        check(lib().vegas_dump_events(self._ctx, it, first, count, ctypes.c_void_p(out.data_ptr()),
                                      self._s()), "dump_events")
        return out

    def edges(self) -> np.ndarray:
        e = np.zeros((self.dim, self.n_bins + 1))
        check(lib().vegas_get_edges(self._ctx, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    self._s()), "get_edges")
        return e

    def set_edges(self, edges: np.ndarray):
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
        assert e.shape == (self.dim, self.n_bins + 1)
        check(lib().vegas_set_edges(self._ctx, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    self._s()), "set_edges")

    def last_iteration(self):
        """(S1, S2, H[d, N]) of the last completed iteration."""
        sums = np.zeros(2)
        H = np.zeros((self.dim, self.n_bins))
        P = ctypes.POINTER(ctypes.c_double)
        check(lib().vegas_get_iteration(self._ctx, sums.ctypes.data_as(P), H.ctypes.data_as(P),
                                        self._s()), "get_iteration")
        return sums[0], sums[1], H

    def set_launch(self, n_blocks: int):
        check(lib().vegas_set_launch(self._ctx, n_blocks), "set_launch")

    def launch_info(self) -> dict:
        a, b, t, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().vegas_get_launch(self._ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(t), ctypes.byref(r)),
              "get_launch")
        return {"auto_blocks": a.value, "blocks_per_cu": b.value, "threads": t.value, "replicas": r.value}

    def set_hist_replicas(self, replicas: int):
        check(lib().vegas_set_hist_replicas(self._ctx, replicas), "set_hist_replicas")

    def time_event_kernel(self, n_events: int, reps: int, hist: bool = True) -> float:
        """Milliseconds per launch of the event kernel alone (reps launches
        back to back on the stream, between two HIP events)."""
        ms = ctypes.c_double()
        check(lib().vegas_time_event_kernel(self._ctx, int(n_events), int(reps), 0 if hist else 1,
                                            ctypes.byref(ms), self._s()), "time_event_kernel")
        return ms.value

    def timing_enable(self, enable: bool = True):
        check(lib().vegas_timing_enable(self._ctx, 1 if enable else 0), "timing_enable")

    def timing_read(self):
        """(summed event-kernel ms, summed reduction-kernel ms, calls) since the last read."""
        a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        check(lib().vegas_timing_read(self._ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)),
              "timing_read")
        return a.value, b.value, n.value

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        check(lib().vegas_state_size(self._ctx, ctypes.byref(n)), "state_size")
        buf = ctypes.create_string_buffer(n.value)
        check(lib().vegas_get_state(self._ctx, buf, n.value, self._s()), "get_state")
        return buf.raw

    def set_state(self, state: bytes):
        buf = ctypes.create_string_buffer(state, len(state))
        check(lib().vegas_set_state(self._ctx, buf, len(state), self._s()), "set_state")
