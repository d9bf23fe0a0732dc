"""Write the extended-precision reference values stored next to this script.

Calls only the oracle's exact references and the seeded generators; nothing
from the GPU library. Run from the repository root:

    python tests/golden/make_golden.py

Outputs (JSON, one file per workload):
  c1_stokes_10x10_seed0.json   tiny Stokes system, 10x10 cells (n = 320):
                               sigma_max, sigma_min from mpmath's SVD at 50
                               digits and, independently, through an mpmath
                               inverse at 50 digits;
  hm_side6_seed1.json          six-field hydro-mechanical system on 6x6 nodes
                               (n = 216), mpmath inverse at 50 digits;
  hm_side201_seed1.json        the 201x201-node hydro-mechanical system
                               (n = 242406), start vectors seeds 11 and 12:
                               the oracle's sigma_max, sigma_min and kappa
                               with the benchmark's options (alpha 4e-2, step
                               floor 2.5e-3, stop rule 1e-6 over 25), and a
                               reference from 3000 updates at a constant
                               alpha of 1.25e-3.
"""

from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import PAOptions, estimate_cond  # noqa: E402
from oracle.exact import sv_extremes_mp_inverse, sv_extremes_mp_svd  # noqa: E402
from synth import hydromech2d, start_vector, stokes2d  # noqa: E402


def _write(name, payload):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(payload, f, indent=1, sort_keys=True)
        f.write("\n")


def _first_within(trace, rel):
    final = trace[-1]
    ok = np.nonzero(np.abs(trace - final) <= rel * abs(final))[0]
    return int(ok[0]) + 1


def main(which=("c1", "hm6")):
    if "c1" in which:
        a = stokes2d(10, 10, seed=0)
        d = a.to_scipy().toarray()
        t0 = time.time()
        smax_i, smin_i = sv_extremes_mp_inverse(d, dps=50)
        t1 = time.time()
        smax_s, smin_s = sv_extremes_mp_svd(d, dps=50)
        t2 = time.time()
        _write("c1_stokes_10x10_seed0.json", {
            "workload": "stokes2d(nx=10, ny=10, seed=0)", "n": a.n, "nnz": a.nnz,
            "sigma_max_svd": smax_s, "sigma_min_svd": smin_s, "kappa_svd": smax_s / smin_s,
            "sigma_max_inv": smax_i, "sigma_min_inv": smin_i, "kappa_inv": smax_i / smin_i,
            "method": "mpmath svd_r at 50 digits; mpmath inverse at 50 digits + LAPACK sigma_max",
            "seconds": {"inverse": t1 - t0, "svd": t2 - t1},
        })
    if "hm6" in which:
        a = hydromech2d(6, seed=1)
        d = a.to_scipy().toarray()
        smax, smin = sv_extremes_mp_inverse(d, dps=50)
        _write("hm_side6_seed1.json", {
            "workload": "hydromech2d(side=6, seed=1)", "n": a.n, "nnz": a.nnz,
            "sigma_max_inv": smax, "sigma_min_inv": smin, "kappa_inv": smax / smin,
            "method": "mpmath inverse at 50 digits + LAPACK sigma_max",
        })
    if "c2" in which:
        a = hydromech2d(201, seed=1)
        x0a = start_vector(a.n, 11)
        x0b = start_vector(a.n, 12)
        # (1) the benchmark's own options: step 4e-2 halving to a floor of
        #     2.5e-3, stop rule 1e-6 over 25 updates
        bench = PAOptions(alpha=4e-2, max_iter=6000, stop_rtol=1e-6, stop_window=25,
                          alpha_min=2.5e-3, alpha_decay=0.5)
        r = estimate_cond(a.n, a.rowptr, a.col, a.val, x0a, x0b, opts=bench)
        # (2) reference: a constant small step (1.25e-3) for 3000 updates, no stop rule
        ref = PAOptions(alpha=1.25e-3, max_iter=3000)
        q = estimate_cond(a.n, a.rowptr, a.col, a.val, x0a, x0b, opts=ref)
        _write("hm_side201_seed1.json", {
            "workload": "hydromech2d(side=201, seed=1)", "n": a.n, "nnz": a.nnz,
            "starts": {"sigma_max": "start_vector(n, 11)", "sigma_min": "start_vector(n, 12)"},
            "opts": {"alpha": 4e-2, "alpha_min": 2.5e-3, "alpha_decay": 0.5, "beta1": 0.9,
                     "beta2": 0.999, "eps": 1e-8, "stop_rtol": 1e-6, "stop_window": 25,
                     "max_iter": 6000},
            "sigma_max": r["sigma_max"], "sigma_min": r["sigma_min"], "kappa": r["kappa"],
            "iters": {"max": r["iters_max"], "min": r["iters_min"]},
            "reference": {"opts": {"alpha": 1.25e-3, "max_iter": 3000},
                          "sigma_max": q["sigma_max"], "sigma_min": q["sigma_min"],
                          "kappa": q["kappa"],
                          "iters_to_1e-3": {"max": _first_within(q["trace_max"], 1e-3),
                                            "min": _first_within(q["trace_min"], 1e-3)}},
            "oracle_seconds": {"max_run": r["time_max_s"], "lu": r["time_lu_s"],
                               "min_run": r["time_min_s"]},
            "superlu_nnz": {"L": r["nnz_l"], "U": r["nnz_u"]},
            "method": "oracle Projected Adam (float64, SciPy SuperLU for Algorithm 2)",
        })

if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("c1", "hm6"))
