"""bench.py's contract on the CPU: the multi-GPU refusal and its workloads."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_every_workload_kind_has_a_driver():
    sys.path.insert(0, ROOT)
    import bench

    drivers = {"hm": bench.make_matrix, "stokes": bench.make_matrix, "batch": bench.bench_batch,
               "warm": bench.bench_warm}
    for name, w in bench.WORKLOADS.items():
        assert w["kind"] in drivers, name
        assert callable(drivers[w["kind"]])
