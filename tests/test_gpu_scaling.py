"""Column scaling on the device against the oracle (section "Row and Column
Scaling"): kappa_2(A D_col^-1) from the same plan as kappa_2(A).

The device scales on the fly and reuses A's LU for the sigma_min run
((A D^-1)^-1 = D A^-1); the oracle forms A D^-1 explicitly and factors it
again with SuperLU. Bars: column norms to 1e-14 relative; the scaled
products within 1e-12 of (|A D^-1| |x|)_i componentwise; kappa to 1e-3, the
first 50 traced values to 1e-10 (sigma_max) and 1e-8 (sigma_min, two
different factorisations).
"""

import numpy as np
import pytest

from oracle import PAOptions, estimate_cond as oracle_estimate
from oracle.csr import spmv as oracle_spmv, spmv_abs, transpose_csr
from oracle.scaling import column_norms, scale_columns
from synth import Csr, diag_csr, hydromech2d, start_vector, stokes2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2409_11515_amd as pa

    pa._binding.lib()
    return torch


def _dev(torch, x):
    return torch.as_tensor(np.ascontiguousarray(x, np.float64), device="cuda")


def test_column_norms_and_scaled_products(torch_cuda):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    a = hydromech2d(40, seed=3)
    p = pa.Plan(a.n, a.rowptr, a.col, a.val, sigma_min_method=pa.COND_MIN_NONE).bind()
    d = p.column_norms().cpu().numpy()
    np.testing.assert_allclose(d, column_norms(a.n, a.rowptr, a.col, a.val), rtol=1e-14)
    rp, c, v, _ = scale_columns(a.n, a.rowptr, a.col, a.val)
    x = start_vector(a.n, 2) * 10.0 ** np.random.default_rng(1).uniform(-4, 4, a.n)
    y = p.spmv(_dev(torch, x), col_scaled=True).cpu().numpy()
    assert np.all(np.abs(y - oracle_spmv(rp, c, v, x)) <= 1e-12 * spmv_abs(rp, c, v, x) + 1e-300)
    yt = p.spmv(_dev(torch, x), transpose=True, col_scaled=True).cpu().numpy()
    tr, tc, tv = transpose_csr(a.n, rp, c, v)
    assert np.all(np.abs(yt - oracle_spmv(tr, tc, tv, x)) <= 1e-12 * spmv_abs(tr, tc, tv, x) + 1e-300)
    p.close()


@pytest.mark.parametrize("mk,iters", [(lambda: stokes2d(10, 10, seed=0), 6000),
                                      (lambda: hydromech2d(13, seed=2), 3000),
                                      (lambda: hydromech2d(31, seed=5), 3000)])
def test_col_scaled_kappa_matches_oracle(torch_cuda, mk, iters):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    a = mk()
    p = pa.Plan(a.n, a.rowptr, a.col, a.val).bind()
    x0 = start_vector(a.n, 4)
    plain = p.run(_dev(torch, x0), max_iter=iters)
    g = p.run(_dev(torch, x0), max_iter=iters, trace=True, scaling=pa.COND_SCALE_COL)
    p.close()
    assert g["flags"] & pa._binding.COND_F_COLSCALED
    rp, c, v, _ = scale_columns(a.n, a.rowptr, a.col, a.val)
    o = oracle_estimate(a.n, rp, c, v, x0, opts=PAOptions(max_iter=iters))
    assert g["kappa"] == pytest.approx(o["kappa"], rel=1e-3)
    np.testing.assert_allclose(g["trace_max"][:50], o["trace_max"][:50], rtol=1e-10)
    np.testing.assert_allclose(g["trace_min"][:50], o["trace_min"][:50], rtol=1e-8)
    # the paper's observation: column scaling removes most of kappa
    assert g["kappa"] < 1e-6 * plain["kappa"]


def test_col_scaled_diagonal_is_kappa_one(torch_cuda):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    rng = np.random.default_rng(9)
    a = diag_csr(rng.choice([-1.0, 1.0], 300) * 10.0 ** rng.uniform(-9, 9, 300),
                 rng.permutation(300), rng.permutation(300))
    p = pa.Plan(a.n, a.rowptr, a.col, a.val).bind()
    r = p.run(_dev(torch, start_vector(a.n, 1)), max_iter=40, scaling=pa.COND_SCALE_COL)
    p.close()
    assert r["kappa"] == pytest.approx(1.0, abs=1e-13)


def test_zero_column_refuses_scaling(torch_cuda):
    import scipy.sparse as sp

    import paper_2409_11515_amd as pa

    torch = torch_cuda
    m = sp.random(50, 50, density=0.2, random_state=3, format="csr") + sp.eye(50)
    m = m.tolil()
    m[:, 7] = 0.0
    m[7, 7] = 0.0
    a = Csr.from_scipy(m.tocsr())
    p = pa.Plan(a.n, a.rowptr, a.col, a.val, sigma_min_method=pa.COND_MIN_NONE).bind()
    with pytest.raises(pa.CondError) as e:
        p.run(_dev(torch, start_vector(a.n, 1)), max_iter=10, scaling=pa.COND_SCALE_COL)
    assert e.value.status == pa._binding.COND_EINVAL
    assert p.column_norms().cpu().numpy()[7] == 0.0
    p.close()
