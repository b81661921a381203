"""Build libasss.so (gfx950) in-tree with hipcc.

    python -m paper_2009_06954_amd.build        # or build() from Python

Host setup code is compiled with g++, the HIP sources with hipcc for gfx950,
and everything is linked into paper_2009_06954_amd/libasss.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libasss.so")
ARCH = os.environ.get("ASSS_OFFLOAD_ARCH", "gfx950")
ROCM_LIB = "/opt/rocm/lib"  # roctx (ranges for rocprofv3 --marker-trace)

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (plain scalar/vector FP32 code only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    gxx = shutil.which("g++") or "g++"
    with tempfile.TemporaryDirectory() as tmp:
        jobs = []
        for src in ("host_setup.cpp", "ildl_host.cpp"):
            o = os.path.join(tmp, src.replace(".cpp", ".o"))
            jobs.append(([gxx, *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", o], o))
        for src in ("kernels.hip", "ildl.hip", "ildl_setup.hip", "outer.hip", "asss.hip", "batch.hip"):
            o = os.path.join(tmp, src.replace(".hip", ".o"))
            jobs.append(([hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o], o))
        # the translation units compile independently: run them side by side
        with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
            list(ex.map(lambda j: _run(j[0]), jobs))
        objs = [o for _, o in jobs]
        out_tmp = LIB + ".tmp"
        _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp, *objs, "-lpthread",
              f"-L{ROCM_LIB}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}"])
        os.replace(out_tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
