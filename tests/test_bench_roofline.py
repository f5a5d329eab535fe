"""Host logic of the bench line: which roofline ceiling a launch is reported against, and
the guard that drops the measured HBM traffic once the kernel sources change."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bound_follows_the_arithmetic_intensity():
    # 8 TB/s against 78.6 TFLOP/s: the ridge is 9.825 flop/B
    ms = 1.0
    alu = bench.roofline("k", ms, alg_bytes=1e9, alg_flops=14.5e9, peak_tflops=78.6, traffic=None)
    hbm = bench.roofline("k", ms, alg_bytes=1e9, alg_flops=7.2e9, peak_tflops=78.6, traffic=None)
    assert alu["ridge_flop_per_byte"] == pytest.approx(9.825)
    assert alu["bound"] == "alu" and alu["unit"] == "TFLOP/s"
    assert alu["achieved"] == pytest.approx(14.5) and alu["frac"] == pytest.approx(14.5 / 78.6)
    assert hbm["bound"] == "hbm" and hbm["unit"] == "GB/s"
    assert hbm["achieved"] == pytest.approx(1000.0) and hbm["frac"] == pytest.approx(1000.0 / 8000.0)
    # the other ceiling is always reported beside the bound one
    for rec in (alu, hbm):
        assert rec["hbm"]["achieved"] == pytest.approx(1000.0)
        assert rec["alu"]["peak"] == 78.6 and rec["hbm"]["peak"] == 8000.0


def test_traffic_is_dropped_when_a_profiled_source_changes(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    import hashlib
    rec = {"source_sha256": {"k.hip": hashlib.sha256(src.read_bytes()).hexdigest()},
           "a": {"bytes_per_launch": 100.0}, "b": {"bytes_per_launch": 20.0}}
    tf = tmp_path / "traffic.json"
    tf.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tf))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("a", "b") == 120.0
    assert bench.measured_traffic("missing") is None
    src.write_text("kernel v2\n")
    assert bench.measured_traffic("a") is None
