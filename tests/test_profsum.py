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


def test_committed_512_summaries_leave_out_the_closure_legs():
    """The summaries average the last launches of each stage's kernels, which belong to the step legs only
    when no later leg of the profiled bench runs the same kernels: every 512^3 summary's bench command
    leaves out the closure's cost legs (a 1024^3 mesh and the closure step reuse the scan and scatter)."""
    for name in ("pm_step_512_clustered_kernel_trace.md", "pm_step_512_clustered_traffic.md",
                 "pm_step_512_clustered_counters.md"):
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            cmds = [ln for ln in fh.read().splitlines() if "rocprofv3" in ln and "bench.py" in ln]
        assert cmds, name
        assert all("--no-closure-cost" in c for c in cmds), name
