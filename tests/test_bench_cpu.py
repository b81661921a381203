"""The benchmark script's host logic (no GPU): the one-GPU guard, the
algorithmic byte count of one inner step that the roofline divides by, the
reading of the committed rocprofv3 traffic summaries, and the CPU baseline's
fit and check."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N, NH, K = 2097152, 24822528, 16  # 128^3 convection-diffusion, S on the pattern of Abar, k = 16
N2, NH2 = 7077888, 84161664       # 192^3


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_row():
    """Half-stored J_tilde entries at (v + 4) bytes, a 4-byte row pointer, the k
    deflation vectors and ten vector streams: 354.0 B (FP64) and 202.7 B (FP32)
    per row at 128^3, and 290.0 B for FP64 with a basis of 4-byte values;
    355 B and 203 B at 192^3 (nh = 12 n - (21 m^2 - 6 m))."""
    assert round(bench.mrs_bytes_per_row(NH / N, K, 8), 1) == 354.0
    assert round(bench.mrs_bytes_per_row(NH / N, K, 4), 1) == 202.7
    assert round(bench.mrs_bytes_per_row(NH / N, K, 8, 4), 1) == 290.0
    assert bench.mrs_bytes_per_row(0.0, 0, 8) == 4 + 80
    assert NH2 == 12 * N2 - (21 * 192 ** 2 - 6 * 192)
    assert round(bench.mrs_bytes_per_row(NH2 / N2, K, 8)) == 355
    assert round(bench.mrs_bytes_per_row(NH2 / N2, K, 4)) == 203


def test_workload_keys():
    assert bench.workload_key(192, 1000.0, 16, "library grid order") == "convdiff3d_192_Pe1000_k16_gridorder"
    assert bench.workload_key(128, 100.0, 16, "natural") == "convdiff3d_128_Pe100_k16"


def _summaries():
    d = os.path.join(ROOT, "profiles")
    return [os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith("_traffic.json")]


def test_default_workload_has_committed_summaries():
    """The benchmark's default line (192^3, Pe 1000, library grid order) has a
    committed traffic summary and kernel trace."""
    key = bench.workload_key(192, 1000.0, 16, "library grid order")
    d = os.path.join(ROOT, "profiles")
    assert os.path.exists(os.path.join(d, f"k_mrs_iter_{key}_traffic.json"))
    assert os.path.exists(os.path.join(d, f"k_mrs_iter_{key}_trace.md"))


@pytest.mark.parametrize("path", _summaries(), ids=os.path.basename)
def test_traffic_summary_is_read_only_for_its_own_kernel_source(path, monkeypatch):
    """A summary's HBM bytes are reported while the kernel source is the one
    the counters were taken on, and never otherwise; they lie below the
    algorithmic bytes (the slot form stores no columns)."""
    rec = json.load(open(path))
    assert set(rec["kernels"]) == {"fp64", "fp32"} and rec["calibration"]["fetch_factor"] > 0
    key = os.path.basename(path)[len("k_mrs_iter_"):-len("_traffic.json")]
    defl = "explicit"
    if key.endswith("_fp32basis"):
        key, defl = key[:-len("_fp32basis")], "explicit_fp32_basis"
    monkeypatch.setattr(bench, "kernel_sha", lambda: rec["kernel_src_sha256"])
    for prec in ("fp64", "fp32"):
        got = bench.measured_traffic(prec, key, defl)
        k = rec["kernels"][prec]
        assert got == k["hbm_bytes"]
        assert 0.5 * k["algorithmic_bytes"] < got < 1.05 * k["algorithmic_bytes"]
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 64)
    assert bench.measured_traffic("fp64", key, defl) is None


def test_profile_summaries_name_their_command():
    d = os.path.join(ROOT, "profiles")
    for f in os.listdir(d):
        if f.endswith(".md"):
            assert "rocprofv3" in open(os.path.join(d, f)).read(), f


def test_cpu_baseline_fit_and_check():
    """Cost per (row x inner step) from the smaller run predicts the larger
    one; the larger one's cost extrapolates to the full problem."""
    small = {"n": 4096, "inner_its": 400, "solve_s": 0.16}
    large = {"n": 13824, "inner_its": 560, "solve_s": 0.45}
    c_small, c_large = bench.unit_cost(small), bench.unit_cost(large)
    assert c_small == pytest.approx(0.16 / (4096 * 400))
    assert c_small * large["n"] * large["inner_its"] / large["solve_s"] == pytest.approx(1.68, rel=1e-3)
    assert c_large * N2 * 3741 == pytest.approx(0.45 * (N2 / 13824) * (3741 / 560))
