"""Host checks of bench.py's reporting: the measured HBM traffic is taken
from the counter summary only when that summary was recorded on the same
sources, workload and step (method and transfer-function form)."""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_measured_traffic_needs_matching_sources_workload_and_step(tmp_path, monkeypatch):
    step = {"method": "exact", "transfer_function": "compact, 7 floats per row"}
    (tmp_path / "profiles").mkdir()
    summary = {"workload": "w", "step": step, "source_sha256": "abc",
               "kernels": {"spread_tiles": {"traffic_bytes_per_launch": 123}}}
    (tmp_path / "profiles" / "counters.json").write_text(json.dumps(summary))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: "abc")
    assert bench.measured_traffic("spread_tiles", "w", dict(step)) == 123
    assert bench.measured_traffic("build_interp", "w", dict(step)) is None
    assert bench.measured_traffic("spread_tiles", "other", dict(step)) is None
    assert bench.measured_traffic("spread_tiles", "w", {"method": "fast",
                                                        "transfer_function": "27 floats per row"}) is None
    monkeypatch.setattr(bench, "source_hash", lambda: "changed")
    assert bench.measured_traffic("spread_tiles", "w", dict(step)) is None


def test_contract_byte_model():
    """The roofline's bytes per marker follow the hot-path contract: build
    12 + 12 + 324, interpolation 336 + 12 + 4T, spreading 336 + 12 + 4 + 8T;
    the fused build-and-interpolate kernel carries both phases."""
    T = 3.5
    contract, own = bench.byte_models(0, True, 7, T, False)
    assert contract["build_exact"] == 348.0
    assert contract["interp"] == 348.0 + 4 * T
    assert contract["spread_tiles"] == 352.0 + 8 * T
    assert contract["build_interp"] == contract["build_exact"] + contract["interp"]
    # compact rows of 7 floats per component move less than the 27-value rows
    assert own["build_interp"] < contract["build_interp"]
    assert own["spread_tiles"] == 12 + 84 + 12 + 8 * T
    _, own_full = bench.byte_models(0, False, 7, T, False)
    assert own_full["spread_tiles"] == 12 + 324 + 12 + 8 * T
