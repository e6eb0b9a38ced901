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
    # the increment solve: phi_{n-1} read, phi_n and the increment written besides chi and B
    assert b["fft_x_inv"] == 5 * S + 7 * F
    assert abs(b["deposit"] / 1e9 - 10.20) < 0.01 and abs(b["kick_drift"] / 1e9 - 12.88) < 0.01


def test_byte_model_matches_counted_traffic_of_single_pass_stages():
    """Stages that read each input once and write each output once (the inverse column pass and the C2R)
    move what the model says: the committed FETCH_SIZE + WRITE_SIZE bytes are within 10 % of it."""
    from paper_2607_17929_amd import profsum
    t = profsum.load_traffic(os.path.join(ROOT, "profiles", "pm_step_512_clustered_traffic.md"))
    b = bench.stage_bytes(512, 512 ** 3, 4)
    for stage in ("fft_y_inv", "fft_x_inv"):
        got = t["stages"][f"fp32:{stage}"]["traffic_bytes_per_launch"]
        assert 0.95 < got / b[stage] < 1.10, (stage, got / b[stage])


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
