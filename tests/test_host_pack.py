"""Host logic of the sliced skew storage (no GPU): the packer's output, read
back on the CPU, applies exactly the skew matrix of its CSR input (in-block
and off-block parts, ragged last block, several row-block sizes), and grid
patterns get the 16-bit off-block column form (the 32-bit form is exercised
on the GPU with a random pattern)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_06954_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("pack")
    exe = str(d / "check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", f"-I{CSRC}",
                    os.path.join(ROOT, "tests", "host_pack_check.cpp"),
                    os.path.join(CSRC, "host_setup.cpp"), "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("m,R", [(12, 64), (20, 128), (33, 512), (48, 2048)])
def test_packed_skew_storage_is_exact(checker, m, R):
    r = subprocess.run([checker, str(m), str(R)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "narrow=1" in r.stdout
