"""CSR helpers for the oracle: validation, explicit transpose, products.

The gradient of equation ``nabla_loss`` needs A x and A^T (A x); the oracle
forms A^T explicitly (a stable counting sort over columns) so that both
products are plain row-wise sums.
"""

from __future__ import annotations

import math

import numpy as np


class CsrError(ValueError):
    pass


def validate_csr(n, rowptr, col, val) -> None:
    """Square n x n CSR with monotone row pointers, in-range columns, finite values."""
    rowptr = np.asarray(rowptr)
    col = np.asarray(col)
    val = np.asarray(val)
    if n <= 0:
        raise CsrError("n must be positive")
    if rowptr.shape != (n + 1,):
        raise CsrError("rowptr must have n+1 entries")
    if rowptr[0] != 0 or np.any(np.diff(rowptr) < 0):
        raise CsrError("rowptr must start at 0 and be non-decreasing")
    nnz = int(rowptr[-1])
    if col.shape != (nnz,) or val.shape != (nnz,):
        raise CsrError("col/val length must equal rowptr[n]")
    if nnz and (col.min() < 0 or col.max() >= n):
        raise CsrError("column index out of range")
    if not np.all(np.isfinite(val)):
        raise CsrError("non-finite value")
    if nnz == 0 or not np.any(val != 0.0):
        raise CsrError("zero matrix")


def transpose_csr(n, rowptr, col, val):
    """CSR of A^T by a stable counting sort on the column index.

    Entries of each row of A^T come out in increasing original-row order.
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    counts = np.bincount(col, minlength=n)
    t_rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=t_rowptr[1:])
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    order = np.argsort(col, kind="stable")  # stable: keeps increasing row order
    t_col = rows[order].astype(np.int32)
    t_val = val[order]
    return t_rowptr, t_col, t_val


def spmv(rowptr, col, val, x):
    """y = A x, one float64 sum per row (entries in stored order)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    prod = np.asarray(val, dtype=np.float64) * np.asarray(x, dtype=np.float64)[np.asarray(col)]
    n = rowptr.size - 1
    y = np.zeros(n)
    nonempty = np.diff(rowptr) > 0
    if prod.size:
        sums = np.add.reduceat(prod, rowptr[:-1][nonempty])
        y[nonempty] = sums
    return y


def spmv_abs(rowptr, col, val, x):
    """(|A| |x|)_i, the scale of the componentwise rounding bound of y_i."""
    return spmv(rowptr, col, np.abs(val), np.abs(x))


def spmv_exact(rowptr, col, val, x):
    """y = A x with every row summed exactly (math.fsum), rounded once.

    Slow; for small inputs only.
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = rowptr.size - 1
    y = np.empty(n)
    for i in range(n):
        lo, hi = rowptr[i], rowptr[i + 1]
        y[i] = math.fsum(float(v) * float(x[c]) for v, c in zip(val[lo:hi], col[lo:hi]))
    return y
