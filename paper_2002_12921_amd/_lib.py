"""ctypes loader for libvegas (the C ABI declared in include/vegas.h).

The library is the in-tree ``libvegas_gfx950.so`` built by ``build.py``.  There
is no fallback: if it is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# VEGAS_LIB names another build of the same sources to load instead (the
# host-sanitizer build of sanitize.py)
LIB_PATH = os.environ.get("VEGAS_LIB") or os.path.join(HERE, "libvegas_gfx950.so")

VEGAS_OK, VEGAS_EINVAL, VEGAS_ESTATE, VEGAS_EWORKSPACE = 0, -1, -2, -3
VEGAS_EHIP, VEGAS_ENONFINITE, VEGAS_EUNSUPPORTED, VEGAS_ECOMPILE = -4, -5, -6, -7
STATUS_NAMES = {0: "VEGAS_OK", -1: "VEGAS_EINVAL", -2: "VEGAS_ESTATE", -3: "VEGAS_EWORKSPACE",
                -4: "VEGAS_EHIP", -5: "VEGAS_ENONFINITE", -6: "VEGAS_EUNSUPPORTED",
                -7: "VEGAS_ECOMPILE"}

GAUSS, BIMODAL, GENZ_DISC, GENZ_PEAK, USER = 0, 1, 2, 3, 4
FP64, FP32_MIXED = 0, 1
CHUNK_BEGIN, CHUNK_END, ITER_FULL, NO_COMBINE, REFINE, NO_HIST, NO_RECORD = 1, 2, 3, 4, 8, 16, 32

# every symbol include/vegas.h declares
EXPORTS = [
    "vegas_workspace_size", "vegas_init_grid", "vegas_init_grid_noalloc", "vegas_init_user", "vegas_user_compile", "vegas_iterate",
    "vegas_iterate_grad", "vegas_forward_grad", "vegas_grad_scale", "vegas_refine", "vegas_result",
    "vegas_reset_results", "vegas_set_params_device", "vegas_get_params_device", "vegas_get_versions",
    "vegas_last_iteration_device",
    "vegas_adjoint", "vegas_dump_events", "vegas_get_edges", "vegas_set_edges",
    "vegas_get_iteration", "vegas_state_size", "vegas_get_state", "vegas_set_state",
    "vegas_get_iteration_index", "vegas_set_launch", "vegas_set_hist_replicas", "vegas_get_launch",
    "vegas_timing_enable", "vegas_timing_read", "vegas_time_event_kernel", "vegas_probe_issue_rates",
    "vegas_destroy", "vegas_last_error",
    "vegas_batch_workspace_size", "vegas_batch_plan", "vegas_batch_run", "vegas_batch_step",
    "vegas_batch_get_iteration", "vegas_batch_results",
    "vegas_batch_get_edges", "vegas_batch_schedule", "vegas_batch_bucket", "vegas_batch_destroy",
]


class VegasError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


class Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("integrand", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("alpha", ctypes.c_double),
                ("params", ctypes.POINTER(ctypes.c_double)), ("n_params", ctypes.c_int32),
                ("problem", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("integral", ctypes.c_double), ("sigma", ctypes.c_double),
                ("chi2_dof", ctypes.c_double), ("last_integral", ctypes.c_double),
                ("last_sigma", ctypes.c_double), ("n_iter", ctypes.c_int64),
                ("n_combined", ctypes.c_int64), ("n_events", ctypes.c_int64),
                ("n_nonfinite", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load libvegas (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libvegas is not built ({LIB_PATH} missing): run "
                           "`python -m paper_2002_12921_amd.build` or __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    P = ctypes.POINTER
    pd = P(ctypes.c_double)
    sig = {
        "vegas_workspace_size": [P(Desc), P(sz)],
        "vegas_init_grid": [P(vp), P(Desc), vp, sz, vp],
        "vegas_init_grid_noalloc": [P(vp), P(Desc), vp],
        "vegas_init_user": [P(vp), P(Desc), ctypes.c_char_p, vp, sz, vp],
        "vegas_user_compile": [ctypes.c_char_p, i32, i32, ctypes.c_char_p, sz],
        "vegas_iterate": [vp, i64, u32, vp],
        "vegas_iterate_grad": [vp, i64, u32, vp, vp],
        "vegas_forward_grad": [vp, vp, vp, i32, i32, i64, u32, vp, vp, vp],
        "vegas_grad_scale": [vp, vp, vp, i32, i32, vp],
        "vegas_refine": [vp, vp],
        "vegas_result": [vp, P(Result), vp],
        "vegas_reset_results": [vp, vp],
        "vegas_set_params_device": [vp, vp, i32, i32, vp],
        "vegas_last_iteration_device": [vp, vp, vp],
        "vegas_get_params_device": [vp, vp, vp],
        "vegas_get_versions": [vp, P(i64), P(i64)],
        "vegas_adjoint": [vp, i64, i64, vp, vp, i32, vp],
        "vegas_dump_events": [vp, i64, i64, i64, vp, vp],
        "vegas_get_edges": [vp, pd, vp],
        "vegas_set_edges": [vp, pd, vp],
        "vegas_get_iteration": [vp, pd, pd, vp],
        "vegas_state_size": [vp, P(sz)],
        "vegas_get_state": [vp, vp, sz, vp],
        "vegas_set_state": [vp, vp, sz, vp],
        "vegas_get_iteration_index": [vp, P(i64)],
        "vegas_set_launch": [vp, i32],
        "vegas_get_launch": [vp, P(i32), P(i32), P(i32), P(i32)],
        "vegas_set_hist_replicas": [vp, i32],
        "vegas_timing_enable": [vp, i32],
        "vegas_timing_read": [vp, pd, pd, P(i64)],
        "vegas_time_event_kernel": [vp, i64, i32, i32, pd, vp],
        "vegas_probe_issue_rates": [vp, sz, i32, pd, P(i32), vp],
        "vegas_destroy": [vp],
        "vegas_batch_workspace_size": [P(Desc), P(i64), i32, P(sz)],
        "vegas_batch_plan": [P(vp), P(Desc), P(i64), i32, vp, sz, i32, i32, vp],
        "vegas_batch_run": [vp, vp],
        "vegas_batch_step": [vp, i32, vp],
        "vegas_batch_get_iteration": [vp, i32, pd, pd, vp],
        "vegas_batch_results": [vp, P(Result), vp],
        "vegas_batch_get_edges": [vp, i32, pd, vp],
        "vegas_batch_schedule": [vp, P(i64), P(i32), P(i32), pd],
        "vegas_batch_bucket": [vp, i32, P(i32), P(i32), P(i32), P(i32), P(i32), pd, P(i32)],
        "vegas_batch_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.vegas_last_error.argtypes = []
    L.vegas_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int, where: str) -> int:
    if status != VEGAS_OK:
        msg = lib().vegas_last_error().decode(errors="replace")
        raise VegasError(status, where, msg)
    return status
