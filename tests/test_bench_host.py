"""Host logic of bench.py (no GPU): the algorithmic byte model behind the roofline figure, the parser of
the committed closure summary, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_stage_bytes_at_512():
    b = bench.stage_bytes(512, 512 ** 3, 4)
    F = 512 ** 3 * 4
    S = 512 * 512 * 257 * 8
    P = 24 + 12
    assert b["deposit"] == 512 ** 3 * P + 10 * F  # particles in, ten fields out
    assert b["kick_drift"] == 512 ** 3 * (2 * P + 4) + 5 * F
    assert b["kspace"] == 23 * S  # 10 sources in, 5 solutions out, tensor state in and out
    assert abs(b["deposit"] / 1e9 - 10.20) < 0.01 and abs(b["kick_drift"] / 1e9 - 12.88) < 0.01


def test_closure_summary_parses():
    cl = bench.closure_result()
    assert cl is not None
    assert 0.0 < cl["max_pk_deviation_to_half_nyquist"] < cl["plain_1x_deviation"]
    assert 0.0 < cl["cost_vs_2x"] < 1.0
    assert "not measured" in cl["source"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
