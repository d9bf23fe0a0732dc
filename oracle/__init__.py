"""Plain CPU oracle for the Projected Adam condition-number estimator.

TEST INFRASTRUCTURE ONLY. This package is the slow, obviously-correct
reference that the GPU library is checked against. Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
library and its Python binding never do, and it imports nothing from them.

Everything is float64, single thread, written in the order the paper states
the method:

* ``csr``      -- CSR validation, explicit transpose, reference products;
* ``padam``    -- Algorithm 1 (Projected Adam) with the gradient of
                  equation ``nabla_loss``;
* ``inverse``  -- Algorithm 2: the gradient for A^-1 from one LU
                  factorisation (SciPy's SuperLU, or a dense LU for tiny
                  matrices);
* ``estimate`` -- kappa_2 = sigma_max / sigma_min from the two runs;
* ``ablation`` -- not the paper's method: sigma_min by descending on
                  ||A x|| / ||x|| with products alone (the comparison that
                  shows why the paper needs Algorithm 2);
* ``scaling``  -- column scaling A D_col^-1 (section "Row and Column
                  Scaling") and kappa_2 of the scaled matrix;
* ``bounds``   -- the error bounds of an approximate solution that the paper
                  derives from kappa (section "Error estimates and
                  conditioning");
* ``exact``    -- closed forms and extended-precision singular values used to
                  pin the oracle itself.
"""

from .csr import validate_csr, transpose_csr, spmv, spmv_abs  # noqa: F401
from .padam import PAOptions, PAResult, projected_adam  # noqa: F401
from .inverse import LUInverse  # noqa: F401
from .estimate import estimate_cond, forward_apply  # noqa: F401
from .bounds import error_bounds  # noqa: F401
from .scaling import column_norms, scale_columns, estimate_cond_col_scaled  # noqa: F401
