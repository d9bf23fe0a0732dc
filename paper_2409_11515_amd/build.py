"""Build libcondest.so (the C-ABI library) in-tree with hipcc for gfx950.

    python -m paper_2409_11515_amd.build        # or: python paper_2409_11515_amd/build.py

Every HIP source is compiled with packed-FP32 instructions disabled; the
host-only C++ sources are compiled by hipcc too (no device code in them).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libcondest.so")

HIP_SOURCES = ["kernels.hip", "panels_upload.hip", "plan.hip", "batch_kernels.hip", "batch.hip", "cnn.hip",
               "noalloc.hip"]
HOST_SOURCES = ["host_csr.cpp", "host_order.cpp", "host_lu.cpp", "panels.cpp"]
ARCH = os.environ.get("CONDEST_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libcondest)")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC]
    jobs = []
    for s in HIP_SOURCES:
        obj = os.path.join(BUILD, s + ".o")
        jobs.append(
            [cc, *common, f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-c", os.path.join(CSRC, s), "-o", obj])
    for s in HOST_SOURCES:
        obj = os.path.join(BUILD, s + ".o")
        jobs.append([cc, *common, "-x", "c++", "-c", os.path.join(CSRC, s), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(_run, jobs))
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
