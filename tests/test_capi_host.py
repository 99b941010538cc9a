"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/vegas.h declares, and rejects bad arguments before
making any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2002_12921_amd import _lib
from paper_2002_12921_amd.integrator import make_desc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vegas.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vegas_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = _lib.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(_lib.EXPORTS)


def _size(desc):
    n = ctypes.c_size_t()
    st = _lib.lib().vegas_workspace_size(ctypes.byref(desc), ctypes.byref(n))
    return st, n.value


def test_workspace_size_valid():
    d, keep = make_desc(8, 50, "gauss", [0.1] + [0.5] * 8, "fp32_mixed")
    st, n = _size(d)
    assert st == 0 and n > 0
    d2, keep2 = make_desc(20, 100, "bimodal", [0.05] + [1 / 3] * 20 + [2 / 3] * 20, "fp32_mixed")
    st, n2 = _size(d2)
    assert st == 0 and n2 > n


@pytest.mark.parametrize("kw,code", [
    (dict(dim=0), _lib.VEGAS_EINVAL),
    (dict(dim=65), _lib.VEGAS_EINVAL),
    (dict(n_bins=1), _lib.VEGAS_EINVAL),
    (dict(n_bins=256), _lib.VEGAS_EINVAL),
    (dict(alpha=-1.0), _lib.VEGAS_EINVAL),
    (dict(alpha=float("nan")), _lib.VEGAS_EINVAL),
    (dict(params=[0.0] + [0.5] * 4), _lib.VEGAS_EINVAL),          # a = 0
    (dict(params=[0.1] + [0.5] * 3), _lib.VEGAS_EINVAL),          # wrong count
    (dict(params=[0.1, 0.5, float("inf"), 0.5, 0.5]), _lib.VEGAS_EINVAL),
    (dict(problem=1 << 24), _lib.VEGAS_EINVAL),
    (dict(integrand=7), _lib.VEGAS_EINVAL),
    (dict(precision=3), _lib.VEGAS_EINVAL),
])
def test_workspace_size_rejects(kw, code):
    base = dict(dim=4, n_bins=50, integrand=0, params=[0.1] + [0.5] * 4, precision=0,
                seed=0, alpha=1.5, problem=0)
    base.update(kw)
    if "params" not in kw and base["dim"] != 4:
        base["params"] = [0.1] + [0.5] * max(base["dim"], 0)
    d, keep = make_desc(**base)
    st, _ = _size(d)
    assert st == code
    assert len(_lib.lib().vegas_last_error()) > 0


def test_lds_limit_is_unsupported():
    d, keep = make_desc(64, 255, "gauss", [0.1] + [0.5] * 64, "fp64")
    st, _ = _size(d)
    assert st == _lib.VEGAS_EUNSUPPORTED


def _event_lds(prec, kind, d, N):
    """Bytes of LDS the event kernel asks for with one histogram copy: the
    grid table (16 bytes per bin in FP64 and for the bimodal FP32 table, else
    8), aligned to 128, the FP64 histogram, and 16 doubles of wave partials."""
    tab = d * N * (16 if (prec == "fp64" or kind == "bimodal") else 8)
    return ((tab + 127) // 128) * 128 + d * N * 8 + 16 * 8


@pytest.mark.parametrize("prec,kind,d,N", [("fp64", "gauss", 31, 220), ("fp64", "gauss", 44, 155),
                                           ("fp64", "gauss", 62, 110), ("fp32_mixed", "gauss", 53, 193),
                                           ("fp32_mixed", "gauss", 53, 192), ("fp64", "gauss", 64, 104)])
def test_lds_limit_matches_the_launch(prec, kind, d, N):
    """Sizes are admitted exactly when the event kernel's smallest launch fits
    the 160 KiB of LDS of a compute unit (near-limit cases on both sides)."""
    params = [0.1] + [0.5] * d
    desc, keep = make_desc(d, N, kind, params, prec)
    st, _ = _size(desc)
    fits = _event_lds(prec, kind, d, N) <= 160 * 1024
    assert st == (_lib.VEGAS_OK if fits else _lib.VEGAS_EUNSUPPORTED), (_event_lds(prec, kind, d, N), st)


def test_genz_parameter_checks():
    d, keep = make_desc(2, 50, "genz_disc", [1.0, 1.0, 0.5, 1.0], "fp64")   # a = 1 not < 1
    assert _size(d)[0] == _lib.VEGAS_EINVAL
    d, keep = make_desc(2, 50, "genz_peak", [1.0, -2.0, 0.5, 0.5], "fp64")  # c < 0
    assert _size(d)[0] == _lib.VEGAS_EINVAL


def test_init_rejects_before_hip():
    L = _lib.lib()
    d, keep = make_desc(4, 50, "gauss", [0.1] + [0.5] * 4)
    ctx = ctypes.c_void_p()
    assert L.vegas_init_grid(ctypes.byref(ctx), ctypes.byref(d), None, 0, None) == _lib.VEGAS_EWORKSPACE
    assert L.vegas_init_grid(ctypes.byref(ctx), ctypes.byref(d), ctypes.c_void_p(4096 + 8), 1 << 30, None) == _lib.VEGAS_EWORKSPACE
    assert L.vegas_init_grid(ctypes.byref(ctx), ctypes.byref(d), ctypes.c_void_p(4096), 16, None) == _lib.VEGAS_EWORKSPACE
    bad, keep2 = make_desc(4, 50, "gauss", [0.1] + [0.5] * 3)
    assert L.vegas_init_grid(ctypes.byref(ctx), ctypes.byref(bad), ctypes.c_void_p(4096), 1 << 30, None) == _lib.VEGAS_EINVAL
    assert ctx.value is None


def test_null_context_calls():
    L = _lib.lib()
    r = _lib.Result()
    assert L.vegas_iterate(None, 10, 3, None) == _lib.VEGAS_EINVAL
    assert L.vegas_refine(None, None) == _lib.VEGAS_EINVAL
    assert L.vegas_result(None, ctypes.byref(r), None) == _lib.VEGAS_EINVAL
    assert L.vegas_destroy(None) == _lib.VEGAS_OK
    assert L.vegas_batch_destroy(None) == _lib.VEGAS_OK
    # the differentiable entry points refuse NULL arguments before any HIP call
    fake = ctypes.c_void_p(4096)
    assert L.vegas_forward_grad(None, fake, None, 9, 1, 1000, _lib.ITER_FULL | _lib.NO_HIST, fake, fake, None) == _lib.VEGAS_EINVAL
    assert L.vegas_forward_grad(None, fake, fake, 9, 1, 1000, _lib.ITER_FULL | _lib.NO_HIST, fake, None, None) == _lib.VEGAS_EINVAL
    assert L.vegas_grad_scale(None, fake, fake, 9, 0, None) == _lib.VEGAS_EINVAL
    assert L.vegas_grad_scale(fake, fake, fake, 0, 0, None) == _lib.VEGAS_EINVAL
    assert L.vegas_iterate_grad(None, 1000, _lib.ITER_FULL | _lib.NO_HIST, fake, None) == _lib.VEGAS_EINVAL


GOOD_SRC = """
__device__ double vegas_integrand(const double* x, int dim, const double* p)
{
    double s = p[0];
    for (int i = 0; i < dim; ++i) s += x[i] * x[i];
    return exp(-s);
}
"""


def test_user_compile_on_host():
    """The runtime compiler needs no device: a valid integrand compiles for
    every dimension class; a broken one reports VEGAS_ECOMPILE with the
    compiler's message located in the caller's own line numbering."""
    from paper_2002_12921_amd import compile_user
    for d in (1, 4, 13, 64):
        ok, log = compile_user(GOOD_SRC, d)
        assert ok, log
    ok, log = compile_user("__device__ double vegas_integrand(const double* x, int d, const double* p)\n"
                           "{\n    return x[0] +* 2;\n}\n", 3)
    assert not ok and "integrand:3:" in log and "error" in log
    ok, log = compile_user("__device__ double not_the_entry(const double* x) { return 1.0; }\n", 2)
    assert not ok and "vegas_integrand" in log
    # FP32-mixed contexts hand f float coordinates: a source written for
    # vegas_real compiles in both precisions, one written for double* does not
    from paper_2002_12921_amd import user_integrands as ui
    for src in (ui.GAUSSIAN, ui.OSCILLATORY, ui.SINE_PRODUCT):
        for prec in ("fp64", "fp32_mixed"):
            ok, log = compile_user(src, 5, prec)
            assert ok, (prec, log)
    ok, log = compile_user(GOOD_SRC, 5, "fp32_mixed")
    assert not ok and "error" in log
    L = _lib.lib()
    assert L.vegas_user_compile(None, 3, 0, None, 0) == _lib.VEGAS_EINVAL
    assert L.vegas_user_compile(GOOD_SRC.encode(), 0, 0, None, 0) == _lib.VEGAS_EINVAL
    assert L.vegas_user_compile(GOOD_SRC.encode(), 65, 0, None, 0) == _lib.VEGAS_EINVAL
    assert L.vegas_user_compile(GOOD_SRC.encode(), 3, 7, None, 0) == _lib.VEGAS_EINVAL
    buf = ctypes.create_string_buffer(8)  # the log is cut to the buffer, NUL-terminated
    assert L.vegas_user_compile(b"garbage(", 2, 0, buf, 8) == _lib.VEGAS_ECOMPILE
    assert len(buf.value) <= 7


def test_user_desc_checks():
    L = _lib.lib()
    d, keep = make_desc(5, 40, "user", [], "fp64")
    st, n = _size(d)
    assert st == _lib.VEGAS_OK and n > 0
    d, keep = make_desc(5, 40, "user", [1.0] * 129, "fp64")
    assert _size(d)[0] == _lib.VEGAS_OK
    d, keep = make_desc(5, 40, "user", [1.0] * 130, "fp64")
    assert _size(d)[0] == _lib.VEGAS_EINVAL
    d, keep = make_desc(5, 40, "user", [], "fp32_mixed")
    assert _size(d)[0] == _lib.VEGAS_OK
    ctx = ctypes.c_void_p()
    u, keep = make_desc(5, 40, "user", [], "fp64")
    g, keep2 = make_desc(4, 50, "gauss", [0.1] + [0.5] * 4)
    # a user kind needs vegas_init_user, and vegas_init_user a user kind and a source
    assert L.vegas_init_grid(ctypes.byref(ctx), ctypes.byref(u), ctypes.c_void_p(4096), 1 << 30, None) == _lib.VEGAS_EINVAL
    assert L.vegas_init_user(ctypes.byref(ctx), ctypes.byref(g), GOOD_SRC.encode(), ctypes.c_void_p(4096), 1 << 30,
                             None) == _lib.VEGAS_EINVAL
    assert L.vegas_init_user(ctypes.byref(ctx), ctypes.byref(u), None, ctypes.c_void_p(4096), 1 << 30,
                             None) == _lib.VEGAS_EINVAL
    assert ctx.value is None
    # batches take built-in integrands only
    n_ev = (ctypes.c_int64 * 1)(1000)
    nb = ctypes.c_size_t()
    assert L.vegas_batch_workspace_size(ctypes.byref(u), n_ev, 1, ctypes.byref(nb)) == _lib.VEGAS_EUNSUPPORTED


def test_noalloc_rejects_before_hip():
    """The allocation-free init validates before any HIP call: NULL out, a bad
    description, and user integrands (which are compiled and loaded at init)."""
    L = _lib.lib()
    d, keep = make_desc(4, 50, "gauss", [0.1] + [0.5] * 4)
    assert L.vegas_init_grid_noalloc(None, ctypes.byref(d), None) == _lib.VEGAS_EINVAL
    ctx = ctypes.c_void_p()
    bad, keep2 = make_desc(4, 50, "gauss", [0.1] + [0.5] * 3)
    assert L.vegas_init_grid_noalloc(ctypes.byref(ctx), ctypes.byref(bad), None) == _lib.VEGAS_EINVAL
    u, keep3 = make_desc(4, 50, "user", [], "fp64")
    assert L.vegas_init_grid_noalloc(ctypes.byref(ctx), ctypes.byref(u), None) == _lib.VEGAS_EUNSUPPORTED
    assert ctx.value is None


def test_static_workspace_covers_every_admissible_size():
    """Every (dim, n_bins) the library admits needs at most the 4 MiB static
    workspace of the allocation-free context (FP64 and FP32 tables, one- and
    two-centre integrands)."""
    L = _lib.lib()
    worst = 0
    for prec in ("fp64", "fp32_mixed"):
        for kind, pf in (("gauss", lambda d: [0.1] + [0.5] * d),
                         ("bimodal", lambda d: [0.1] + [0.3] * d + [0.6] * d)):
            for d in range(1, 65):
                for N in range(2, 256, 3):
                    desc, keep = make_desc(d, N, kind, pf(d), prec)
                    n = ctypes.c_size_t()
                    if L.vegas_workspace_size(ctypes.byref(desc), ctypes.byref(n)) == _lib.VEGAS_OK:
                        worst = max(worst, n.value)
    assert 0 < worst <= 4 << 20
