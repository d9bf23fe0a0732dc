"""kappa_2(A) = ||A||_2 ||A^-1||_2 = sigma_max / sigma_min from two Projected Adam runs.

sigma_max: Algorithm 1 with M = A (equation ``nabla_loss``).
sigma_min: Algorithm 1 with M = A^-1 through Algorithm 2 (one LU), giving
||A^-1||_2 = 1/sigma_min (section "Computing the condition number of a
matrix", equation for kappa_2 via singular values).

Optional ablation, not the paper's method: ``min_method="spmv"`` minimises
||A x||/||x|| directly with the same optimiser (gradient sign flipped; see
``ablation``), which the paper does not do.
"""

from __future__ import annotations

import time

import numpy as np

from .csr import spmv, transpose_csr, validate_csr
from .inverse import LUInverse
from .ablation import minimise_by_spmv
from .padam import PAOptions, projected_adam

EPS_MACH = float(np.finfo(np.float64).eps)


def forward_apply(n, rowptr, col, val):
    """(apply, evaluate) for M = A: apply(x) = (A x, A^T (A x))."""
    t_rowptr, t_col, t_val = transpose_csr(n, rowptr, col, val)

    def evaluate(x):
        return spmv(rowptr, col, val, x)

    def apply(x):
        y = spmv(rowptr, col, val, x)
        return y, spmv(t_rowptr, t_col, t_val, y)

    return apply, evaluate


def estimate_cond(n, rowptr, col, val, x0_max, x0_min=None, opts: PAOptions | None = None,
                  opts_min: PAOptions | None = None, min_method: str = "lu") -> dict:
    """Estimate sigma_max, sigma_min and kappa_2 of the CSR matrix A.

    Returns a dict with sigma_max, sigma_min, kappa, iters_max, iters_min,
    traces, the best vectors, the LU fill and timings. sigma_min = 0 and
    kappa = inf are reported when the LU meets an exactly zero pivot.
    """
    validate_csr(n, rowptr, col, val)
    opts = opts or PAOptions()
    opts_min = opts_min or opts
    x0_min = x0_max if x0_min is None else x0_min
    out = {}
    apply_fwd, eval_fwd = forward_apply(n, rowptr, col, val)
    t0 = time.perf_counter()
    rmax = projected_adam(apply_fwd, eval_fwd, x0_max, opts)
    out["time_max_s"] = time.perf_counter() - t0
    out.update(sigma_max=rmax.sigma, iters_max=rmax.iters, trace_max=rmax.trace, x_max=rmax.x_best)
    if min_method == "lu":
        t0 = time.perf_counter()
        inv = LUInverse(n, rowptr, col, val)
        out["time_lu_s"] = time.perf_counter() - t0
        out["nnz_l"], out["nnz_u"] = inv.nnz_l, inv.nnz_u
        t0 = time.perf_counter()
        rinv = projected_adam(inv.apply, inv.evaluate, x0_min, opts_min)
        out["time_min_s"] = time.perf_counter() - t0
        out.update(sigma_min=1.0 / rinv.sigma, iters_min=rinv.iters, trace_min=rinv.trace,
                   x_min=rinv.x_best, inv_norm=rinv.sigma)
    elif min_method == "spmv":
        t0 = time.perf_counter()
        rmin = minimise_by_spmv(apply_fwd, eval_fwd, x0_min, opts_min)
        out["time_min_s"] = time.perf_counter() - t0
        out.update(sigma_min=rmin.sigma, iters_min=rmin.iters, trace_min=rmin.trace, x_min=rmin.x_best)
    else:
        raise ValueError("min_method must be 'lu' or 'spmv'")
    out["kappa"] = out["sigma_max"] / out["sigma_min"]
    out["numerically_singular"] = out["kappa"] >= 1.0 / EPS_MACH
    return out
