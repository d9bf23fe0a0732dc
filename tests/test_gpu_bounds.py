"""Error bounds of an approximate solution on the device against the oracle.

The device forms r = A x_hat - b and the three norms with its own summation
order; the oracle with numpy's. Bars: ||b|| and ||x_hat|| to 1e-13 relative
(sums of squares of identical values); ||r|| within 1e-12 ||(|A||x_hat| +
|b|)|| absolute (the componentwise product bar carried to the norm), so the
bounds, each linear in ||r||, agree to that bar divided by ||r||.
"""

import math

import numpy as np
import pytest

from oracle import PAOptions, estimate_cond as oracle_estimate
from oracle.bounds import error_bounds as oracle_bounds
from oracle.csr import spmv as oracle_spmv, spmv_abs
from oracle.inverse import LUInverse
from synth import diag_csr, hydromech2d, scaled_banded, start_vector

pytestmark = pytest.mark.gpu

RES_BAR = 1e-12


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2409_11515_amd as pa

    pa._binding.lib()
    return torch


def _check(g, o, scale):
    assert g["b_norm"] == pytest.approx(o["b_norm"], rel=1e-13)
    assert g["x_norm"] == pytest.approx(o["x_norm"], rel=1e-13)
    assert abs(g["res_norm"] - o["res_norm"]) <= RES_BAR * scale
    rel = RES_BAR * scale / o["res_norm"] + 1e-13
    for k in ("rel_residual", "err_x_lower", "err_x_upper", "err_xhat_lower", "err_xhat_upper"):
        assert g[k] == pytest.approx(o[k], rel=rel), k
    assert g["roundoff_floor"] == o["roundoff_floor"]
    if math.isinf(o["err_x_tight"]):
        assert math.isinf(g["err_x_tight"])
    else:
        assert g["err_x_tight"] == pytest.approx(o["err_x_tight"], rel=4 * rel)


@pytest.mark.parametrize("mk,noise", [(lambda: hydromech2d(30, seed=3), 1e-6),
                                      (lambda: hydromech2d(30, seed=3), 0.0),
                                      (lambda: scaled_banded(3001, seed=4, col_decades=3), 1e-3),
                                      (lambda: diag_csr(np.array([-2.5])), 0.25)])
def test_bounds_match_oracle(torch_cuda, mk, noise):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    a = mk()
    x = start_vector(a.n, 5)
    b = oracle_spmv(a.rowptr, a.col, a.val, x)
    # x_hat: an LU solve of A x = b (noise 0), or that solve perturbed
    xh = LUInverse(a.n, a.rowptr, a.col, a.val).solve(b) if a.n > 1 else b / a.val
    xh = xh + noise * np.linalg.norm(xh) * start_vector(a.n, 6) / math.sqrt(a.n)
    p = pa.Plan(a.n, a.rowptr, a.col, a.val).bind()
    x0 = torch.as_tensor(start_vector(a.n, 7), device="cuda")
    r = p.run(x0, max_iter=2000, stop_rtol=1e-9, stop_window=50)
    kappa, norm_a = max(r["kappa"], 1.0), r["sigma_max"]
    g = p.error_bounds(torch.as_tensor(xh, device="cuda"), torch.as_tensor(b, device="cuda"),
                       kappa, norm_a)
    p.close()
    o = oracle_bounds(a.n, a.rowptr, a.col, a.val, xh, b, kappa, norm_a)
    scale = np.linalg.norm(spmv_abs(a.rowptr, a.col, a.val, xh) + np.abs(b))
    _check(g, o, scale)
    if noise == 0.0 and a.n > 1:
        # an LU solve of a system with kappa > 1/eps: the relative residual
        # is tiny, yet the bound relative to x_hat is not small
        assert g["rel_residual"] < 1e-10
        assert g["err_xhat_upper"] > 1e3 * g["rel_residual"]


def test_bounds_errors(torch_cuda):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    a = hydromech2d(6, seed=1)
    p = pa.Plan(a.n, a.rowptr, a.col, a.val).bind()
    z = torch.zeros(a.n, dtype=torch.float64, device="cuda")
    one = torch.ones(a.n, dtype=torch.float64, device="cuda")
    with pytest.raises(pa.CondError) as e:
        p.error_bounds(one, z, 10.0, 1.0)  # b = 0
    assert e.value.status == pa._binding.COND_ENUMERIC
    with pytest.raises(pa.CondError) as e:
        p.error_bounds(one, one, 0.5, 1.0)  # kappa < 1
    assert e.value.status == pa._binding.COND_EINVAL
    with pytest.raises(pa.CondError) as e:
        p.error_bounds(one, one, 10.0, float("inf"))
    assert e.value.status == pa._binding.COND_EINVAL
    p.close()
