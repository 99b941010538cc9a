"""The allocation-free context (vegas_init_grid_noalloc: the workspace is the
library's static device array) against a context in a caller-allocated
workspace (vegas_init_grid): same kernels, so the same results up to the
order of the FP64 histogram atomics.  Two calls in a row on one device, the
second with a smaller problem; both go through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2002_12921_amd import Vegas

pytestmark = pytest.mark.gpu


def _run(v, M, n_adapt, n_acc):
    for _ in range(n_adapt):
        v.iterate(M, refine=True, combine=False)
    for _ in range(n_acc):
        v.iterate(M, hist=False)
    return v.result(), v.edges()


def test_noalloc_matches_workspace_context():
    handles = []
    for d, N, prec, M in ((8, 50, "fp32_mixed", 400_000), (4, 20, "fp64", 60_000)):
        params = [0.1] + list(np.linspace(0.35, 0.65, d))
        ref = Vegas(d, N, "gauss", params, prec)
        st = Vegas(d, N, "gauss", params, prec, static_workspace=True)
        assert st.ws is None
        handles.append(st._ctx.value)
        # the state starts clean: uniform grid, nothing recorded
        assert np.array_equal(st.edges(), ref.edges())
        r_ref, E_ref = _run(ref, M, 3, 2)
        r_st, E_st = _run(st, M, 3, 2)
        assert np.max(np.abs(E_st - E_ref)) <= 1e-12
        for k in ("integral", "sigma", "last_integral", "last_sigma"):
            assert abs(r_st[k] - r_ref[k]) <= 1e-12 * abs(r_ref[k]), (k, r_st[k], r_ref[k])
        for k in ("n_iter", "n_combined", "n_events", "n_nonfinite"):
            assert r_st[k] == r_ref[k], k
        # one more iteration with histograms: sums and histograms of the last iteration
        ref.iterate(M)
        st.iterate(M)
        s1r, s2r, Hr = ref.last_iteration()
        s1s, s2s, Hs = st.last_iteration()
        assert abs(s1s - s1r) <= 1e-12 * abs(s1r) and abs(s2s - s2r) <= 1e-12 * abs(s2r)
        assert np.all(np.abs(Hs - Hr) <= 1e-12 * Hr.sum(axis=1, keepdims=True))
        # checkpoints without a pinned staging buffer
        w = Vegas(d, N, "gauss", params, prec)
        w.set_state(st.get_state())
        assert np.array_equal(w.edges(), st.edges())
        st.close()  # does nothing to the static context
        ref.close()
    # one static context per device: the second call re-initialised the first's
    assert handles[0] == handles[1]
