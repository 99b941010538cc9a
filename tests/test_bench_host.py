"""Host-side pieces of bench.py: the algorithmic work count and the
counter-summary lookup (no GPU)."""
import bench


def test_alg_slots_table():
    # Philox 40 ceil(d/4) - (ceil(d/4) - 1), 7 per dimension, 20 per event
    assert bench.alg_slots_per_event(8) == 79 + 56 + 20
    assert bench.alg_slots_per_event(5) == 79 + 35 + 20
    assert bench.alg_slots_per_event(4) == 40 + 28 + 20


def test_gpus_above_one_is_refused(monkeypatch, capsys):
    import sys
    import pytest
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code != 0
    assert "one GPU" in capsys.readouterr().err


def test_traffic_only_for_the_profiled_kernel(monkeypatch):
    t, note = bench.measured_traffic()
    if t is not None:
        assert 1.0e6 < t < 1.0e8
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 64)
    t, note = bench.measured_traffic()
    assert t is None and "changed" in note
