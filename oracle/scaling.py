"""Column scaling (section "Row and Column Scaling", paragraph "Column
Scaling"): right preconditioning with D_col = diag of the column 2-norms of
A, giving A D_col^-1, whose columns all have unit norm. The paper's figure
of condition numbers per iteration compares kappa_2(A) with
kappa_2(A D_col^-1).

The oracle forms A D_col^-1 explicitly (each entry divided by its column's
norm) and runs the unchanged estimator on it, with its own LU of the scaled
matrix.

TEST INFRASTRUCTURE ONLY (part of the oracle package).
"""

from __future__ import annotations

import math

import numpy as np

from .csr import transpose_csr, validate_csr
from .estimate import estimate_cond


def column_norms(n, rowptr, col, val) -> np.ndarray:
    """||A[:, j]||_2 for every column j, from the rows of A^T."""
    t_rowptr, _, t_val = transpose_csr(n, rowptr, col, val)
    out = np.empty(n)
    for j in range(n):
        seg = t_val[t_rowptr[j]:t_rowptr[j + 1]]
        out[j] = math.sqrt(float(np.dot(seg, seg)))
    return out


def scale_columns(n, rowptr, col, val):
    """(rowptr, col, val / d[col], d): the CSR of A D_col^-1 and the norms d.
    A zero column cannot be scaled: ValueError."""
    validate_csr(n, rowptr, col, val)
    d = column_norms(n, rowptr, col, val)
    if not np.all(d > 0.0):
        raise ValueError("a zero column has no column scaling")
    col = np.asarray(col)
    return rowptr, col, np.asarray(val, dtype=np.float64) / d[col], d


def estimate_cond_col_scaled(n, rowptr, col, val, x0_max, x0_min=None, **kw) -> dict:
    """kappa_2(A D_col^-1) by the estimator on the explicitly scaled matrix."""
    rp, c, v, _ = scale_columns(n, rowptr, col, val)
    return estimate_cond(n, rp, c, v, x0_max, x0_min, **kw)
