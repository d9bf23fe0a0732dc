"""The host set-up code under AddressSanitizer and UBSan (CPU only).

Builds tests/sanitize/host_driver.cpp with the library's host sources
(validation and transpose, nested dissection, the sparse LU, the panel
planner with its inverses, the joining of block schedules and the host
replay of the solves) by g++ with -fsanitize=address,undefined and no
recovery, and runs it: any out-of-bounds access, use after free, leak or
undefined behaviour aborts the run, and the driver's own checks (backward
errors of the replayed solves, the error codes of bad inputs) must pass.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_11515_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")] + [
    os.path.join(CSRC, f) for f in ("host_csr.cpp", "host_order.cpp", "host_lu.cpp", "panels.cpp")]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_setup_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_asan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, *SOURCES, "-o", exe, "-lpthread"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "host checks ok" in r.stdout
