"""Host logic of bench.py (no GPU needed): the one-GPU guard and the rule that HBM traffic
from the profiler counters is reported only for the kernel sources, storage and tile shape
the counters were taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_for_the_profiled_configuration(monkeypatch):
    entry = {"sources_sha16": bench.kernel_sources_sha16(), "storage": "f32", "fetch_kib": 1.0e6, "fetch_scale": 2.0,
             "write_kib": 2.0e6, "write_scale": 1.0, "tile": [64, 4]}
    monkeypatch.setattr(bench, "COUNTERS", {"jet_256x256x1024": entry})
    t = bench.measured_traffic("f32", [64, 4, 64], "jet_256x256x1024")
    assert t == pytest.approx((1.0e6 * 2.0 + 2.0e6) * 1024.0)
    assert bench.measured_traffic("f16", [64, 4, 64], "jet_256x256x1024") is None
    assert bench.measured_traffic("f32", [32, 8, 64], "jet_256x256x1024") is None
    assert bench.measured_traffic("f32", [64, 4, 64], "rayleigh_taylor_128x128x512") is None
    entry["sources_sha16"] = "0" * 16
    assert bench.measured_traffic("f32", [64, 4, 64], "jet_256x256x1024") is None


def test_counters_are_plausible_for_the_state():
    """Stored counters describe one FP32 step of their workload: writes are the 128-byte state
    of every cell, reads at least that."""
    cells = {"jet_256x256x1024": 256 * 256 * 1024, "rayleigh_taylor_128x128x512": 128 * 128 * 512}
    for name, c in bench.COUNTERS.items():
        n = cells[name]
        assert c["write_kib"] * c["write_scale"] * 1024 == pytest.approx(128 * n, rel=0.01), name
        assert c["fetch_kib"] * c["fetch_scale"] * 1024 >= 128 * n, name
