"""The benchmark script's host logic (no GPU): the one-GPU guard, the
algorithmic byte count of one inner step that the roofline divides by, and
the reading of the committed rocprofv3 traffic summaries."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N, NH, K = 2097152, 24822528, 16  # 128^3 convection-diffusion, S on the pattern of Abar, k = 16


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_row():
    """Half-stored J_tilde entries at (v + 4) bytes, a 4-byte row pointer, the k
    deflation vectors and ten vector streams: 354.0 B (FP64) and 202.7 B (FP32)
    per row at 128^3, and 290.0 B for FP64 with a basis of 4-byte values."""
    assert round(bench.mrs_bytes_per_row(NH / N, K, 8), 1) == 354.0
    assert round(bench.mrs_bytes_per_row(NH / N, K, 4), 1) == 202.7
    assert round(bench.mrs_bytes_per_row(NH / N, K, 8, 4), 1) == 290.0
    assert bench.mrs_bytes_per_row(0.0, 0, 8) == 4 + 80


@pytest.mark.parametrize("order", ["natural", "x-line tiles 4x4", "library grid order"])
def test_committed_traffic_is_read_for_its_own_order_and_source(order):
    """Each committed summary is taken on the current kernel source, so the
    benchmark reports its HBM bytes; another workload size gets none."""
    fp64 = bench.measured_traffic("fp64", order, 128)
    fp32 = bench.measured_traffic("fp32", order, 128)
    assert fp64 is not None and fp32 is not None, \
        "the committed rocprofv3 summaries predate paper_2009_06954_amd/csrc/kernels.hip: retake them"
    alg64, alg32 = bench.mrs_bytes_per_row(NH / N, K, 8) * N, bench.mrs_bytes_per_row(NH / N, K, 4) * N
    # the stored form moves fewer bytes than the algorithmic count (no columns in the slot form)
    assert 0.7 * alg64 < fp64 < alg64 and 0.7 * alg32 < fp32 < alg32
    assert bench.measured_traffic("fp64", order, 192) is None


def test_traffic_summaries_name_their_command():
    d = os.path.join(ROOT, "profiles")
    for f in os.listdir(d):
        if f.endswith("_traffic.json"):
            rec = json.load(open(os.path.join(d, f)))
            assert set(rec["kernels"]) == {"fp64", "fp32"} and rec["calibration"]["fetch_factor"] > 0
        if f.endswith(".md"):
            assert "rocprofv3" in open(os.path.join(d, f)).read()
