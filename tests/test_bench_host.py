"""Host-side pieces of bench.py: the algorithmic work count and the
counter-summary lookup (no GPU)."""
import bench


def test_alg_slots_table():
    # the method's step table: Philox 40 per group of four dimensions;
    # binning 2, map 3, integrand 2, Jacobian 1, histogram address 1 per
    # dimension; 3 + 4 (one quarter-rate exponential) + 10 (sums) per event
    assert bench.alg_slots_per_event(8) == 169
    assert bench.alg_slots_per_event(5) == 80 + 45 + 17
    assert bench.alg_slots_per_event(4) == 40 + 36 + 17
    assert bench.alg_slots_per_event(20) == 200 + 180 + 17


def test_gpus_above_one_is_refused(monkeypatch, capsys):
    import sys
    import pytest
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code != 0
    assert "one GPU" in capsys.readouterr().err


def test_counters_only_for_the_profiled_kernel(monkeypatch):
    t, busy, note = bench.measured_counters()
    if t is not None:
        assert 1.0e6 < t < 1.0e8
    if busy is not None:
        assert 0.0 < busy <= 1.0
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 64)
    t, busy, note = bench.measured_counters()
    assert t is None and busy is None and "changed" in note
