"""The allocation-free error-bounds entry point against the plan's.

cond_error_bounds_noalloc keeps the residual's partial sums in a fixed
scratch array inside the library instead of device memory from a plan. It
runs the same kernels with the same grid, so on the same canonical CSR it
must return exactly what cond_plan_error_bounds returns. Checked on two
calls in a row, the second on a smaller system, so that whatever the first
call left in the scratch array must not leak into the second.
"""

import ctypes as C
import math

import numpy as np
import pytest

from synth import hydromech2d, scaled_banded, start_vector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2409_11515_amd as pa

    pa._binding.lib()
    return torch


def _canonical(a):
    s = a.to_scipy().tocsr()
    s.sum_duplicates()
    s.sort_indices()
    return s


def _case(torch, a, seed):
    import paper_2409_11515_amd as pa

    s = _canonical(a)
    n = s.shape[0]
    x = start_vector(n, seed)
    b = s @ x
    xh = x + 1e-5 * start_vector(n, seed + 1) / math.sqrt(n)
    kappa, norm_a = 3.0e8 + seed, 17.5 + seed
    dev = lambda v, dt: torch.as_tensor(np.ascontiguousarray(v, dt), device="cuda")
    xh_d, b_d = dev(xh, np.float64), dev(b, np.float64)
    p = pa.Plan(n, s.indptr, s.indices, s.data, sigma_min_method=pa.COND_MIN_NONE).bind()
    ref = p.error_bounds(xh_d, b_d, kappa, norm_a)
    p.close()
    got = pa.error_bounds_noalloc(dev(s.indptr, np.int64), dev(s.indices, np.int32),
                                  dev(s.data, np.float64), xh_d, b_d, kappa, norm_a)
    return got, ref


def test_noalloc_matches_plan_twice(torch_cuda):
    # first a larger system (more blocks), then a smaller one
    big = hydromech2d(90, seed=2)
    small = scaled_banded(1000, seed=3, col_decades=2)
    for a, seed in ((big, 1), (small, 4)):
        got, ref = _case(torch_cuda, a, seed)
        for k in ref:
            assert got[k] == ref[k] or (math.isinf(got[k]) and math.isinf(ref[k])), (k, got[k], ref[k])
        assert 0 < ref["res_norm"] < ref["b_norm"]


def test_noalloc_rejects_bad_arguments(torch_cuda):
    import paper_2409_11515_amd as pa

    torch = torch_cuda
    L = pa._binding.lib()
    out = pa._binding.BoundsT()
    one = torch.ones(4, dtype=torch.float64, device="cuda")
    rp = torch.tensor([0, 1, 2, 3, 4], dtype=torch.int64, device="cuda")
    col = torch.arange(4, dtype=torch.int32, device="cuda")
    args = (rp.data_ptr(), col.data_ptr(), one.data_ptr(), one.data_ptr(), one.data_ptr())
    assert L.cond_error_bounds_noalloc(0, 4, *args, 2.0, 1.0, None, C.byref(out)) == pa._binding.COND_EINVAL
    assert L.cond_error_bounds_noalloc(4, -1, *args, 2.0, 1.0, None, C.byref(out)) == pa._binding.COND_EINVAL
    assert L.cond_error_bounds_noalloc(4, 4, *args, 0.5, 1.0, None, C.byref(out)) == pa._binding.COND_EINVAL
    assert L.cond_error_bounds_noalloc(4, 4, None, *args[1:], 2.0, 1.0, None,
                                       C.byref(out)) == pa._binding.COND_EINVAL
    # a valid call: identity, x_hat = b = 1, so r = 0
    assert L.cond_error_bounds_noalloc(4, 4, *args, 2.0, 1.0, None, C.byref(out)) == 0
    assert out.res_norm == 0.0 and out.b_norm == 2.0 and out.x_norm == 2.0
