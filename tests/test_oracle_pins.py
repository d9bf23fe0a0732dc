"""Pins of the CPU oracle against facts fixed by the mathematics, not by itself.

Each test names the property it checks. Together they are meant to fail on a
plausible slip anywhere in the oracle: a wrong sign of the gradient
(maximising the wrong thing), A in place of A^T, a dropped bias correction,
a dropped projection or normalisation, a wrong best-iterate rule, a wrong
triangular solve.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import PAOptions, estimate_cond, forward_apply, projected_adam
from oracle.ablation import minimise_by_spmv
from oracle.csr import spmv, spmv_abs, spmv_exact, transpose_csr, validate_csr, CsrError
from oracle.exact import kappa_blockdiag2, sv_2x2, sv_extremes_mp_inverse
from oracle.inverse import LUInverse
from synth import Csr, csr_from_dense, diag_csr, scaled_banded, start_vector
from synth.matrices import block_diag_2x2


def _est(a: Csr, seed=0, iters=4000, **kw):
    x0 = start_vector(a.n, seed)
    return estimate_cond(a.n, a.rowptr, a.col, a.val, x0, opts=PAOptions(max_iter=iters, **kw))


# ----------------------------------------------------------- P1: diagonal
@pytest.mark.parametrize("seed", [0, 1])
def test_diagonal_closed_form(seed):
    rng = np.random.default_rng(100 + seed)
    n = 40
    d = rng.choice([-1.0, 1.0], n) * 10.0 ** rng.uniform(-12, 12, n)
    a = diag_csr(d)
    r = _est(a, seed)
    assert r["sigma_max"] == pytest.approx(np.abs(d).max(), rel=1e-12)
    assert r["sigma_min"] == pytest.approx(np.abs(d).min(), rel=1e-12)
    assert r["kappa"] == pytest.approx(np.abs(d).max() / np.abs(d).min(), rel=1e-11)


def test_permuted_diagonal_closed_form():
    rng = np.random.default_rng(7)
    n = 50
    d = rng.choice([-1.0, 1.0], n) * 10.0 ** rng.uniform(-8, 8, n)
    a = diag_csr(d, rng.permutation(n), rng.permutation(n))
    r = _est(a, 3)
    assert r["sigma_max"] == pytest.approx(np.abs(d).max(), rel=1e-12)
    assert r["sigma_min"] == pytest.approx(np.abs(d).min(), rel=1e-12)


# ------------------------------------------------------ P2: 2x2 blocks
def test_sv_2x2_against_textbook():
    # the closed form against numpy's SVD on well-conditioned blocks
    rng = np.random.default_rng(3)
    for _ in range(50):
        b = rng.standard_normal((2, 2))
        s = np.linalg.svd(b, compute_uv=False)
        s1, s2 = sv_2x2(*b.ravel())
        assert s1 == pytest.approx(s[0], rel=1e-13)
        assert s2 == pytest.approx(s[1], rel=1e-12)


def test_block_diagonal_closed_form_nonsymmetric():
    # non-symmetric blocks: using A where A^T belongs changes the answer
    rng = np.random.default_rng(11)
    nb = 20
    blocks = rng.standard_normal((nb, 2, 2)) * 10.0 ** rng.uniform(-6, 6, (nb, 1, 1))
    blocks[:, 0, 1] *= 5.0  # strongly non-symmetric
    a = block_diag_2x2(blocks)
    smax, smin, kap = kappa_blockdiag2(blocks)
    r = _est(a, 5, iters=6000)
    assert r["sigma_max"] == pytest.approx(smax, rel=1e-9)
    assert r["sigma_min"] == pytest.approx(smin, rel=1e-9)
    assert r["kappa"] == pytest.approx(kap, rel=1e-8)


# ------------------------------------------------------ P3: degenerate cI
@pytest.mark.parametrize("c", [1.0, 2.0**-30, -(2.0**17)])
def test_scaled_identity_is_a_fixed_point(c):
    n = 17
    a = diag_csr(np.full(n, c))
    x0 = start_vector(n, 9)
    apply, evaluate = forward_apply(a.n, a.rowptr, a.col, a.val)
    seen = []
    res = projected_adam(apply, evaluate, x0, PAOptions(max_iter=25),
                         observer=lambda t, xp, g, d, xn: seen.append((g.copy(), d.copy())))
    assert all(np.all(g == 0.0) and np.all(d == 0.0) for g, d in seen)
    assert res.sigma == abs(c)
    # x only goes through repeated renormalisation: same direction to rounding
    np.testing.assert_allclose(res.x_best, x0 / np.sqrt(x0 @ x0), rtol=0, atol=8e-16)


# --------------------------------------------------- P4: power-of-two scale
@pytest.mark.parametrize("k", [-40, 25])
def test_power_of_two_scaling_bitwise(k):
    a = scaled_banded(60, seed=2, col_decades=4, row_decades=2)
    b = Csr(a.n, a.rowptr, a.col, a.val * 2.0**k)
    x0 = start_vector(a.n, 4)
    o = PAOptions(max_iter=300)
    fa = forward_apply(a.n, a.rowptr, a.col, a.val)
    fb = forward_apply(b.n, b.rowptr, b.col, b.val)
    ra = projected_adam(*fa, x0, o)
    rb = projected_adam(*fb, x0, o)
    np.testing.assert_array_equal(ra.x_best, rb.x_best)
    assert rb.sigma == ra.sigma * 2.0**k
    np.testing.assert_array_equal(rb.trace, ra.trace * 2.0**k)


# ------------------------------------------------- P5: route independence
def test_transpose_and_permutation_invariance():
    rng = np.random.default_rng(5)
    a = scaled_banded(80, seed=6, col_decades=5, row_decades=2)
    s = a.to_scipy()
    at = Csr.from_scipy(s.T)
    p = sp.eye(a.n, format="csr")[rng.permutation(a.n)]
    q = sp.eye(a.n, format="csr")[:, rng.permutation(a.n)]
    paq = Csr.from_scipy(p @ s @ q)
    k0 = _est(a, 1, iters=8000)["kappa"]
    k1 = _est(at, 2, iters=8000)["kappa"]
    k2 = _est(paq, 3, iters=8000)["kappa"]
    assert k1 == pytest.approx(k0, rel=1e-7)
    assert k2 == pytest.approx(k0, rel=1e-7)


# ----------------------------------------------- P6: bounds and one-sidedness
def test_sanity_bounds_and_one_sided():
    a = scaled_banded(120, seed=8, col_decades=6, row_decades=2)
    d = a.to_scipy().toarray()
    smax_t, smin_t = sv_extremes_mp_inverse(d, dps=40)
    for its in (5, 40, 3000):
        r = _est(a, 4, iters=its)
        assert r["sigma_max"] <= smax_t * (1 + 1e-13)
        assert r["sigma_min"] >= smin_t * (1 - 1e-13)
    cn = np.sqrt((d * d).sum(0))
    rn = np.sqrt((d * d).sum(1))
    assert r["sigma_max"] >= max(cn.max(), rn.max()) * (1 - 1e-13)
    assert r["sigma_max"] <= math.sqrt((d * d).sum())
    assert r["sigma_min"] <= min(cn.min(), rn.min()) * (1 + 1e-13)
    assert r["sigma_max"] == pytest.approx(smax_t, rel=1e-9)
    assert r["sigma_min"] == pytest.approx(smin_t, rel=1e-9)


# ------------------------------------------------ P7: per-step invariants
def test_per_step_invariants():
    a = scaled_banded(64, seed=10, col_decades=3, row_decades=1)
    apply, evaluate = forward_apply(a.n, a.rowptr, a.col, a.val)
    eps = np.finfo(float).eps
    sig = []

    def obs(t, xp, g, d, xn):
        assert abs(np.sqrt(xp @ xp) - 1) <= 4 * eps
        assert abs(np.sqrt(xn @ xn) - 1) <= 4 * eps
        # gradient of a 0-homogeneous loss is orthogonal to x
        assert abs(xp @ g) <= 1e-12 * np.linalg.norm(g) + 1e-300
        # the projected step is tangent to the sphere at x
        assert abs(xp @ d) <= 1e-14 * max(np.linalg.norm(d), 1e-300)
        y = evaluate(xn)
        sig.append(np.sqrt((y @ y) / (xn @ xn)))

    res = projected_adam(apply, evaluate, start_vector(a.n, 1), PAOptions(max_iter=200), observer=obs)
    # best-iterate tracking = running max over x_1..x_T, never x_0
    np.testing.assert_allclose(res.trace, np.maximum.accumulate(sig), rtol=1e-13)
    assert np.all(np.diff(res.trace) >= 0)


def test_first_step_closed_form():
    # After one step the bias corrections cancel exactly: m_hat = g, v_hat = g^2,
    # so the raw step is alpha * g / (|g| + eps). Dropping either correction or
    # using the wrong moment breaks this.
    a = scaled_banded(30, seed=12, col_decades=2, row_decades=1)
    apply, evaluate = forward_apply(a.n, a.rowptr, a.col, a.val)
    x0 = start_vector(a.n, 2)
    got = {}
    projected_adam(apply, evaluate, x0, PAOptions(max_iter=1, alpha=0.05),
                   observer=lambda t, xp, g, d, xn: got.update(x=xp, g=g, d=d, xn=xn))
    x = x0 / np.linalg.norm(x0)
    dense = a.to_scipy().toarray()
    y = dense @ x
    g = x / (x @ x) - dense.T @ y / (y @ y)
    raw = 0.05 * g / (np.abs(g) + 1e-8)
    tangent = raw - (x @ raw) * x
    np.testing.assert_allclose(got["g"], g, rtol=1e-10, atol=1e-14 * np.abs(g).max())
    np.testing.assert_allclose(got["d"], tangent, rtol=1e-9, atol=1e-15)
    xn = (x - tangent) / np.linalg.norm(x - tangent)
    np.testing.assert_allclose(got["xn"], xn, rtol=1e-9, atol=1e-15)


def test_early_stop_rule():
    a = scaled_banded(50, seed=13, col_decades=3, row_decades=1)
    x0 = start_vector(a.n, 6)
    full = estimate_cond(a.n, a.rowptr, a.col, a.val, x0, opts=PAOptions(max_iter=3000))
    st = estimate_cond(a.n, a.rowptr, a.col, a.val, x0,
                       opts=PAOptions(max_iter=3000, stop_rtol=1e-12, stop_window=50))
    assert st["iters_max"] % 50 == 0 and st["iters_max"] < 3000
    T = st["iters_max"]
    # the stopped run is the full run cut at T
    np.testing.assert_array_equal(st["trace_max"], full["trace_max"][:T])
    assert full["trace_max"][T - 1] - full["trace_max"][T - 51] <= 1e-12 * full["trace_max"][T - 1]


# ---------------------------------------------- P8: tiny brute force (mpmath)
@pytest.mark.parametrize("seed", [0, 1])
def test_scaling_dominated_vs_extended_precision(seed):
    # kappa ~ 1e20+ : a float64 SVD of A would be wrong in sigma_min here
    a = scaled_banded(60, seed=20 + seed, col_decades=10, row_decades=3)
    smax, smin = sv_extremes_mp_inverse(a.to_scipy().toarray(), dps=60)
    assert smax / smin > 1e18
    r = _est(a, seed, iters=6000)
    assert r["sigma_max"] == pytest.approx(smax, rel=1e-9)
    assert r["sigma_min"] == pytest.approx(smin, rel=1e-9)


def test_mp_inverse_matches_mp_svd_tiny():
    # the two extended-precision references agree on a small scaled matrix
    from oracle.exact import sv_extremes_mp_svd

    a = scaled_banded(14, seed=4, col_decades=8, row_decades=2).to_scipy().toarray()
    s1 = sv_extremes_mp_svd(a, dps=50)
    s2 = sv_extremes_mp_inverse(a, dps=50)
    assert s2[0] == pytest.approx(s1[0], rel=1e-13)
    assert s2[1] == pytest.approx(s1[1], rel=1e-12)


# -------------------------------------------------- P9: products and transpose
def test_spmv_exact_on_integers():
    rng = np.random.default_rng(1)
    n = 300
    a = sp.random(n, n, density=0.03, random_state=2, format="csr")
    a.data = rng.integers(-(2**20), 2**20, a.nnz).astype(float)
    x = rng.integers(-(2**20), 2**20, n).astype(float)
    c = Csr.from_scipy(a)
    exact = (a.astype(np.int64) @ x.astype(np.int64)).astype(float)  # integer arithmetic
    np.testing.assert_array_equal(spmv(c.rowptr, c.col, c.val, x), exact)
    np.testing.assert_array_equal(spmv_exact(c.rowptr, c.col, c.val, x), exact)


def test_transpose_against_dense():
    a = scaled_banded(90, seed=3)
    t_rowptr, t_col, t_val = transpose_csr(a.n, a.rowptr, a.col, a.val)
    dt = sp.csr_matrix((t_val, t_col, t_rowptr), shape=(a.n, a.n)).toarray()
    np.testing.assert_array_equal(dt, a.to_scipy().toarray().T)
    # stable order: column indices of each row of A^T increase
    for i in range(a.n):
        seg = t_col[t_rowptr[i]:t_rowptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_empty_rows_in_spmv():
    a = csr_from_dense(np.array([[0.0, 0, 0], [1, 2, 0], [0, 0, 0]]))
    np.testing.assert_array_equal(spmv(a.rowptr, a.col, a.val, np.array([1.0, 1, 1])), [0, 3, 0])


# ------------------------------------------------------ P10: LU solves
@pytest.mark.parametrize("n,bound", [(300, 1e-10), (2500, 1e-8)])
def test_lu_solves_backward_error(n, bound):
    a = scaled_banded(n, seed=30, col_decades=8, row_decades=2)
    inv = LUInverse(a.n, a.rowptr, a.col, a.val)
    s = a.to_scipy()
    x = start_vector(n, 1)
    r = inv.solve(x)
    # componentwise backward error |A r - x| <= c eps (|A||r| + |x|); the bound
    # is loose (pivot growth) but a wrong or transposed solve misses it by far
    res = np.abs(s @ r - x)
    scale = abs(s) @ np.abs(r) + np.abs(x)
    assert np.max(res / scale) < bound
    st = inv.solve_t(r)
    res_t = np.abs(s.T @ st - r)
    scale_t = abs(s.T) @ np.abs(st) + np.abs(r)
    assert np.max(res_t / scale_t) < bound


# ------------------------------------------------------ validation
@pytest.mark.parametrize(
    "bad",
    [
        (2, [0, 1], [0], [1.0]),  # rowptr too short
        (2, [0, 1, 1], [2], [1.0]),  # column out of range
        (2, [0, 1, 2], [0, 1], [1.0, np.nan]),  # non-finite
        (2, [0, 2, 1], [0, 1], [1.0, 1.0]),  # decreasing rowptr
        (2, [0, 0, 0], [], []),  # zero matrix
    ],
)
def test_validation_rejects(bad):
    with pytest.raises(CsrError):
        validate_csr(bad[0], np.array(bad[1]), np.array(bad[2], dtype=np.int64), np.array(bad[3]))


def test_spmv_abs_on_integers():
    # (|A| |x|)_i is the scale of every componentwise SpMV bar: exact on
    # integer data against integer arithmetic, never below |A x|, and equal
    # to A x when A and x are non-negative
    rng = np.random.default_rng(21)
    n = 250
    a = sp.random(n, n, density=0.04, random_state=22, format="csr")
    a.data = rng.integers(-(2**20), 2**20, a.nnz).astype(float)
    x = rng.integers(-(2**20), 2**20, n).astype(float)
    c = Csr.from_scipy(a)
    exact = (abs(a).astype(np.int64) @ np.abs(x).astype(np.int64)).astype(float)
    got = spmv_abs(c.rowptr, c.col, c.val, x)
    np.testing.assert_array_equal(got, exact)
    assert np.all(got >= np.abs(spmv(c.rowptr, c.col, c.val, x)))
    pos = Csr(c.n, c.rowptr, c.col, np.abs(c.val))
    np.testing.assert_array_equal(spmv_abs(pos.rowptr, pos.col, pos.val, np.abs(x)),
                                  spmv(pos.rowptr, pos.col, pos.val, np.abs(x)))


# ------------------------------------- ablation: sigma_min by SpMV alone
def _min_spmv(a: Csr, seed, **kw):
    apply, evaluate = forward_apply(a.n, a.rowptr, a.col, a.val)
    return minimise_by_spmv(apply, evaluate, start_vector(a.n, seed), PAOptions(**kw))


def test_spmv_min_diagonal_kappa_1e2():
    # well-conditioned (kappa ~ 1e2, n = 60): the descent reaches min |d|
    # from above; a flipped gradient sign would climb to max |d| instead and
    # a ">" in the best rule would report the largest value seen
    rng = np.random.default_rng(200)
    n = 60
    d = rng.choice([-1.0, 1.0], n) * 10.0 ** rng.uniform(0, 2, n)
    a = diag_csr(d, rng.permutation(n), rng.permutation(n))
    r = _min_spmv(a, 1, max_iter=20000)
    assert np.abs(d).min() <= r.sigma <= np.abs(d).min() * (1 + 1e-5)
    assert np.all(np.diff(r.trace) <= 0)
    # with the step-size floor it lands on the closed form
    r2 = _min_spmv(a, 1, max_iter=20000, alpha_min=1e-4, stop_rtol=1e-9, stop_window=50)
    assert r2.sigma == pytest.approx(np.abs(d).min(), rel=1e-12)
    assert r2.iters < 20000 and r2.iters % 50 == 0


def test_spmv_min_block_diagonal_closed_form():
    # non-symmetric 2x2 blocks, moderate kappa: A^T in place of A changes the
    # smallest singular value of each block
    rng = np.random.default_rng(31)
    nb = 15
    blocks = rng.standard_normal((nb, 2, 2)) + 3.0 * np.eye(2)
    blocks[:, 0, 1] *= 4.0
    a = block_diag_2x2(blocks)
    smax, smin, _ = kappa_blockdiag2(blocks)
    r = _min_spmv(a, 2, max_iter=20000, alpha_min=1e-4, stop_rtol=1e-10, stop_window=50)
    assert r.sigma == pytest.approx(smin, rel=1e-9)


@pytest.mark.parametrize("c", [4.0, -(2.0**-12)])
def test_spmv_min_scaled_identity_fixed_point(c):
    a = diag_csr(np.full(23, c))
    r = _min_spmv(a, 4, max_iter=30)
    assert r.sigma == abs(c)
    x0 = start_vector(23, 4)
    np.testing.assert_allclose(r.x_best, x0 / np.sqrt(x0 @ x0), rtol=0, atol=8e-16)


def test_spmv_min_power_of_two_scaling_bitwise():
    a = scaled_banded(50, seed=3, col_decades=2, row_decades=1)
    b = Csr(a.n, a.rowptr, a.col, a.val * 2.0**-33)
    ra = _min_spmv(a, 5, max_iter=200)
    rb = _min_spmv(b, 5, max_iter=200)
    np.testing.assert_array_equal(ra.x_best, rb.x_best)
    np.testing.assert_array_equal(rb.trace, ra.trace * 2.0**-33)


def test_spmv_min_is_an_upper_bound_and_fails_at_large_kappa():
    # every iterate's ||A x|| / ||x|| is >= sigma_min; at kappa ~ 1e4 the
    # descent is still far from it after 20000 updates (the reason the paper
    # computes ||A^-1|| through an LU instead)
    rng = np.random.default_rng(201)
    n = 60
    d = rng.choice([-1.0, 1.0], n) * 10.0 ** rng.uniform(0, 4, n)
    a = diag_csr(d)
    r = _min_spmv(a, 1, max_iter=20000)
    assert r.sigma >= np.abs(d).min()
    assert r.sigma > 2.0 * np.abs(d).min()
    e = _est(a, 1, iters=4000)  # the LU route on the same matrix
    assert e["sigma_min"] == pytest.approx(np.abs(d).min(), rel=1e-9)


def test_estimate_cond_spmv_route_matches_ablation():
    a = scaled_banded(40, seed=9, col_decades=1, row_decades=1)
    x0 = start_vector(a.n, 7)
    o = PAOptions(max_iter=500)
    r = estimate_cond(a.n, a.rowptr, a.col, a.val, x0, opts=o, min_method="spmv")
    rr = _min_spmv(a, 7, max_iter=500)
    assert r["sigma_min"] == rr.sigma
    assert r["kappa"] == r["sigma_max"] / rr.sigma
