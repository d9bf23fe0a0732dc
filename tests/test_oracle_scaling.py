"""Pins of the oracle's column scaling (section "Row and Column Scaling").

The scaled matrix must have unit column norms; column scaling removes any
column scaling already applied (A S for a positive diagonal S scales to the
same matrix); a diagonal matrix scales to a signed permutation (kappa = 1);
and on a matrix B D_c whose column norms D_c span many decades, kappa of the
scaled matrix is that of B with unit columns, checked in extended precision.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import PAOptions
from oracle.exact import sv_extremes_mp_inverse
from oracle.scaling import column_norms, estimate_cond_col_scaled, scale_columns
from synth import Csr, diag_csr, scaled_banded, start_vector


def test_column_norms_against_dense():
    a = scaled_banded(70, seed=2, col_decades=8, row_decades=2)
    d = np.linalg.norm(a.to_scipy().toarray(), axis=0)
    np.testing.assert_allclose(column_norms(a.n, a.rowptr, a.col, a.val), d, rtol=1e-15)


def test_scaled_columns_have_unit_norm_and_absorb_prior_scaling():
    a = scaled_banded(90, seed=3, col_decades=10, row_decades=3)
    rp, c, v, d = scale_columns(a.n, a.rowptr, a.col, a.val)
    np.testing.assert_allclose(column_norms(a.n, rp, c, v), 1.0, rtol=4e-16 * 8)
    s = 2.0 ** np.random.default_rng(4).integers(-40, 40, a.n)  # exact rescaling
    b = Csr.from_scipy(a.to_scipy() @ sp.diags(s))
    _, _, vb, db = scale_columns(b.n, b.rowptr, b.col, b.val)
    np.testing.assert_array_equal(db, d * s)
    np.testing.assert_array_equal(vb, v)


def test_diagonal_scales_to_kappa_one():
    rng = np.random.default_rng(5)
    dd = rng.choice([-1.0, 1.0], 30) * 10.0 ** rng.uniform(-10, 10, 30)
    a = diag_csr(dd, rng.permutation(30), rng.permutation(30))
    r = estimate_cond_col_scaled(a.n, a.rowptr, a.col, a.val, start_vector(30, 1),
                                 opts=PAOptions(max_iter=50))
    assert r["kappa"] == pytest.approx(1.0, abs=1e-14)


def test_scaled_kappa_against_extended_precision():
    a = scaled_banded(60, seed=7, col_decades=12, row_decades=0)
    dense = a.to_scipy().toarray()
    smax, smin = sv_extremes_mp_inverse(dense, dps=60)
    assert smax / smin > 1e10
    scaled = dense / np.linalg.norm(dense, axis=0)
    tmax, tmin = sv_extremes_mp_inverse(scaled, dps=40)
    r = estimate_cond_col_scaled(a.n, a.rowptr, a.col, a.val, start_vector(a.n, 2),
                                 opts=PAOptions(max_iter=6000))
    assert r["kappa"] == pytest.approx(tmax / tmin, rel=1e-8)
    assert r["kappa"] < 1e-6 * smax / smin


def test_zero_column_rejected():
    a = Csr.from_scipy(sp.csr_matrix(np.array([[1.0, 0.0], [2.0, 0.0]])))
    with pytest.raises(ValueError):
        scale_columns(a.n, a.rowptr, a.col, a.val)
