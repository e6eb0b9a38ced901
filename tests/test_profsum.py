"""Host-side checks of the profiler summaries and of how bench.py reads measured HBM traffic."""
import os

import pytest

from paper_2607_17929_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_committed_traffic_summary_parses():
    t = profsum.load_traffic(os.path.join(ROOT, "profiles", "pm_step_512_clustered_traffic.md"))
    assert t is not None and t["n"] == 512
    assert abs(t["write_scale"] - 1.0) < 0.05 and t["read_scale"] > 0
    for stage in profsum.STAGE_KERNELS:
        e = t["stages"][f"fp32:{stage}"]
        assert e["traffic_bytes_per_launch"] == pytest.approx(e["read_bytes_per_launch"] + e["write_bytes_per_launch"],
                                                              abs=2)
        assert len(e["source_sha256"]) == 64


def test_bench_drops_traffic_when_sources_change(monkeypatch):
    import bench
    t = profsum.load_traffic(os.path.join(ROOT, "profiles", "pm_step_512_clustered_traffic.md"))
    e = t["stages"]["fp32:kick_drift"]
    monkeypatch.setattr(profsum, "source_hash", lambda stage, csrc=profsum.CSRC: e["source_sha256"])
    assert bench.measured_traffic(512, "kick_drift") == e["traffic_bytes_per_launch"]
    monkeypatch.setattr(profsum, "source_hash", lambda stage, csrc=profsum.CSRC: "0" * 64)
    assert bench.measured_traffic(512, "kick_drift") is None
    assert bench.measured_traffic(256, "kick_drift") is None
