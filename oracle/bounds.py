"""Error bounds of an approximate solution from kappa_2 (section "Error
estimates and conditioning").

Given A, b, an approximate solution x_hat of A x = b, kappa = kappa_2(A) and
||A||_2 (= sigma_max; both from the estimator), the residual
b_hat - b = A x_hat - b gives:

* Theorem "Bounds on the relative error ||x_hat - x|| / ||x||":
  (1/kappa) ||b_hat - b||/||b|| <= ||x_hat - x||/||x|| <= kappa ||b_hat - b||/||b||;
* Theorem "Bounds on the relative error ||x_hat - x|| / ||x_hat||":
  ||b_hat - b||/(||A|| ||x_hat||) <= ||x_hat - x||/||x_hat||
  <= kappa ||b_hat - b||/(||A|| ||x_hat||) =: epsilon;
* Theorem "Tight upper bound of the error ||x_hat - x|| / ||x||":
  ||x_hat - x||/||x|| <= epsilon / (1 - epsilon) for epsilon < 1 (no bound
  otherwise: reported as +inf);
* Theorem "Numerical singularity of a matrix": the error that rounding the
  data to machine precision alone can cause, 2 eps kappa / (1 - kappa eps),
  finite only while kappa eps < 1 (+inf beyond: numerically singular).

All norms are 2-norms, the residual is formed in float64 from the oracle's
product, and each quantity is the formula written out.

TEST INFRASTRUCTURE ONLY (part of the oracle package).
"""

from __future__ import annotations

import math

import numpy as np

from .csr import spmv, validate_csr

EPS_MACH = float(np.finfo(np.float64).eps)


def error_bounds(n, rowptr, col, val, x_hat, b, kappa, norm_a, eps_mach=EPS_MACH) -> dict:
    validate_csr(n, rowptr, col, val)
    if not (kappa >= 1.0) or not (norm_a > 0.0):
        raise ValueError("kappa must be >= 1 and ||A|| > 0")
    x_hat = np.asarray(x_hat, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = spmv(rowptr, col, val, x_hat) - b  # b_hat - b
    res_norm = math.sqrt(float(r @ r))
    b_norm = math.sqrt(float(b @ b))
    x_norm = math.sqrt(float(x_hat @ x_hat))
    if not (b_norm > 0.0 and x_norm > 0.0):
        raise ValueError("b and x_hat must be non-zero")
    rel_res = res_norm / b_norm
    eps = kappa * res_norm / (norm_a * x_norm)
    out = {
        "res_norm": res_norm,
        "b_norm": b_norm,
        "x_norm": x_norm,
        "rel_residual": rel_res,
        "err_x_lower": rel_res / kappa,
        "err_x_upper": kappa * rel_res,
        "err_xhat_lower": res_norm / (norm_a * x_norm),
        "err_xhat_upper": eps,
        "err_x_tight": eps / (1.0 - eps) if eps < 1.0 else math.inf,
        "roundoff_floor": (2.0 * eps_mach * kappa / (1.0 - kappa * eps_mach)
                           if kappa * eps_mach < 1.0 else math.inf),
    }
    return out
