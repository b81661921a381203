"""Host logic of the sliced skew storage (no GPU): the packer's output, read
back on the CPU the way the kernels read it, applies exactly the skew matrix
of its CSR input (in-block and off-block parts, ragged last block, several
row-block sizes) in each column form: grid patterns get the offset-slot form
by default, and the 32-bit, 16-bit and slot forms can be forced; a random
pattern keeps per-entry columns and refuses the slot form.  In the slot form
every real entry's column must be reachable without the clamp that the
kernels apply to padding lanes."""
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


def _run(checker, *args):
    r = subprocess.run([checker, *map(str, args)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    return r


@pytest.mark.parametrize("m,R", [(12, 64), (20, 128), (33, 512), (48, 2048)])
def test_packed_skew_storage_is_exact(checker, m, R):
    r = _run(checker, m, R)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "form=3" in r.stdout  # offset slots for a grid pattern


@pytest.mark.parametrize("form,tag", [(1, "form=1 narrow=0"), (2, "form=2 narrow=1"), (3, "form=3")])
@pytest.mark.parametrize("m,R", [(12, 64), (33, 512)])
def test_forced_column_forms_are_exact(checker, m, R, form, tag):
    r = _run(checker, m, R, form)
    assert r.returncode == 0, r.stdout + r.stderr
    assert tag in r.stdout


def test_random_pattern_keeps_entry_columns(checker):
    r = _run(checker, 20, 128, 0, "random")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "form=3" not in r.stdout
    r = _run(checker, 20, 128, 3, "random")
    assert r.returncode == 3 and "rejected" in r.stdout


def test_host_code_under_sanitizers(tmp_path):
    """The host packer built with AddressSanitizer and UndefinedBehaviorSanitizer
    (g++, host code only) runs clean on grid and random patterns and each
    column form (the setup stages: tests/test_host_setup.py)."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    flags = ["-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=address,undefined",
             "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", f"-I{CSRC}"]
    pack = str(tmp_path / "pack")
    r = subprocess.run([gxx, *flags, os.path.join(ROOT, "tests", "host_pack_check.cpp"),
                        os.path.join(CSRC, "host_setup.cpp"), "-o", pack], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    for args, rc in (((12, 64, 0), 0), ((12, 64, 1), 0), ((12, 64, 2), 0), ((20, 128, 3), 0),
                     ((12, 64, 0, "random"), 0), ((12, 64, 3, "random"), 3)):
        r = subprocess.run([pack, *map(str, args)], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == rc, (args, r.stdout + r.stderr)
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
