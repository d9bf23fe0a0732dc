"""Pins of the oracle's error-bound evaluator (section "Error estimates and
conditioning") against cases where the true error is known exactly.

On a diagonal matrix with power-of-two entries every quantity is exact, so
the theorems' bounds can be checked for equality where they are attained
(the error along the smallest singular direction attains the upper bound of
the first theorem, along the largest its lower bound), and on random
scaled matrices the true errors must lie inside every bound.
"""

import math

import numpy as np
import pytest

from oracle.bounds import EPS_MACH, error_bounds
from oracle.exact import sv_extremes_mp_inverse
from synth import diag_csr, scaled_banded, start_vector

D = np.array([8.0, 4.0, 0.5])  # kappa = 16, ||A|| = 8


def _b(a, x):
    return a.to_scipy() @ x


@pytest.mark.parametrize("t", [2.0**-10, 0.25])
def test_upper_bound_attained_along_smallest_direction(t):
    a = diag_csr(D)
    x = np.array([1.0, 0.0, 0.0])
    xh = x + t * np.array([0.0, 0.0, 1.0])
    r = error_bounds(3, a.rowptr, a.col, a.val, xh, _b(a, x), kappa=16.0, norm_a=8.0)
    true_rel = t  # ||x_hat - x|| / ||x||
    assert r["res_norm"] == t / 2 and r["b_norm"] == 8.0
    assert r["err_x_upper"] == true_rel
    assert r["err_x_lower"] == true_rel / 256
    # relative to x_hat: eps = kappa ||r|| / (||A|| ||x_hat||) = t / sqrt(1 + t^2) exactly
    assert r["err_xhat_upper"] == pytest.approx(t / math.sqrt(1 + t * t), rel=1e-15)
    assert r["err_xhat_lower"] == pytest.approx(r["err_xhat_upper"] / 16, rel=1e-15)
    assert true_rel <= r["err_x_tight"] * (1 + 1e-15)


def test_lower_bound_attained_along_largest_direction():
    a = diag_csr(D)
    x = np.array([0.0, 0.0, 1.0])
    t = 2.0**-6
    xh = x + t * np.array([1.0, 0.0, 0.0])
    r = error_bounds(3, a.rowptr, a.col, a.val, xh, _b(a, x), kappa=16.0, norm_a=8.0)
    assert r["err_x_lower"] == t
    assert r["err_x_upper"] == 256 * t
    # the second theorem's lower bound is attained too: ||r|| = ||A|| ||x_hat - x||
    assert r["err_xhat_lower"] == pytest.approx(t / math.sqrt(1 + t * t), rel=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_true_errors_inside_every_bound(seed):
    a = scaled_banded(40, seed=40 + seed, col_decades=3, row_decades=1)
    dense = a.to_scipy().toarray()
    smax, smin = sv_extremes_mp_inverse(dense, dps=40)
    kappa = smax / smin
    x = start_vector(a.n, seed)
    b = dense @ x
    rng = np.random.default_rng(seed)
    xh = x + 1e-6 * np.linalg.norm(x) * rng.standard_normal(a.n) / math.sqrt(a.n)
    r = error_bounds(a.n, a.rowptr, a.col, a.val, xh, b, kappa=kappa, norm_a=smax)
    e_x = np.linalg.norm(xh - x) / np.linalg.norm(x)
    e_xh = np.linalg.norm(xh - x) / np.linalg.norm(xh)
    tol = 1 + 1e-9
    assert r["err_x_lower"] <= e_x * tol and e_x <= r["err_x_upper"] * tol
    assert r["err_xhat_lower"] <= e_xh * tol and e_xh <= r["err_xhat_upper"] * tol
    assert e_x <= r["err_x_tight"] * tol
    # the second theorem's bracket is kappa wide, the first's kappa^2
    assert r["err_xhat_upper"] / r["err_xhat_lower"] == pytest.approx(kappa, rel=1e-12)
    assert r["err_x_upper"] / r["err_x_lower"] == pytest.approx(kappa * kappa, rel=1e-12)


def test_tight_bound_and_roundoff_limits():
    a = diag_csr(D)
    x = np.array([1.0, 0.0, 0.0])
    xh = x + np.array([0.0, 0.0, 4.0])  # eps = 4 / sqrt(17) > ... < 1; then a huge error
    r = error_bounds(3, a.rowptr, a.col, a.val, xh, _b(a, x), kappa=16.0, norm_a=8.0)
    assert r["err_xhat_upper"] < 1 and math.isfinite(r["err_x_tight"])
    r2 = error_bounds(3, a.rowptr, a.col, a.val, xh, _b(a, x), kappa=64.0, norm_a=8.0)
    assert r2["err_xhat_upper"] >= 1 and r2["err_x_tight"] == math.inf
    assert r["roundoff_floor"] == pytest.approx(2 * EPS_MACH * 16 / (1 - 16 * EPS_MACH), rel=1e-15)
    big = error_bounds(3, a.rowptr, a.col, a.val, xh, _b(a, x), kappa=2.0 / EPS_MACH, norm_a=8.0)
    assert big["roundoff_floor"] == math.inf
    with pytest.raises(ValueError):
        error_bounds(3, a.rowptr, a.col, a.val, xh, _b(a, x), kappa=0.5, norm_a=8.0)
