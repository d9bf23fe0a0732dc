"""Algorithm 2: the operator M = A^-1 for Projected Adam, from one LU.

r = A^-1 x comes from solving L U r = x and s = A^-T r from solving
U^T L^T s = r; the gradient is then x/||x||^2 - s/||r||^2, the same form as
equation ``nabla_loss`` with M = A^-1 (section "Computing the condition
number", the algorithm computing the gradient for A^-1).

The paper writes the factorisation as A = L U without saying how it pivots.
Here it is SciPy's SuperLU (COLAMD column order, threshold partial
pivoting) for sparse input, or LAPACK's partial-pivoting dense LU for tiny
matrices; either way the factors are computed once and reused every step.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla_dense
import scipy.sparse as sp
import scipy.sparse.linalg as sla


class SingularMatrix(ArithmeticError):
    pass


class LUInverse:
    """Apply A^-1 and A^-T through one LU factorisation of A."""

    def __init__(self, n, rowptr, col, val, dense_below: int = 2000):
        a = sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col), np.asarray(rowptr)),
                          shape=(n, n))
        self.n = n
        self.dense = n < dense_below
        if self.dense:
            d = a.toarray()
            lu, piv = sla_dense.lu_factor(d, check_finite=True)
            if np.any(np.diag(lu) == 0.0):
                raise SingularMatrix("zero pivot")
            self._lu = (lu, piv)
            self.nnz_l = int(np.count_nonzero(np.tril(lu, -1)))
            self.nnz_u = int(np.count_nonzero(np.triu(lu)))
        else:
            try:
                self._slu = sla.splu(a.tocsc())
            except RuntimeError as e:  # SuperLU reports exact singularity this way
                raise SingularMatrix(str(e)) from e
            self.nnz_l = int(self._slu.L.nnz)
            self.nnz_u = int(self._slu.U.nnz)

    def solve(self, x):
        """r with L U r = x (with the factorisation's permutations)."""
        if self.dense:
            return sla_dense.lu_solve(self._lu, x, trans=0, check_finite=False)
        return self._slu.solve(np.asarray(x, np.float64))

    def solve_t(self, r):
        """s with U^T L^T s = r, i.e. s = A^-T r."""
        if self.dense:
            return sla_dense.lu_solve(self._lu, r, trans=1, check_finite=False)
        return self._slu.solve(np.asarray(r, np.float64), trans="T")

    def apply(self, x):
        r = self.solve(x)
        return r, self.solve_t(r)

    def evaluate(self, x):
        return self.solve(x)
