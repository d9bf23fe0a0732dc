"""CPU checks of the C-ABI library: exported symbols and the host set-up steps.

These call only the host-side entry points (no device is touched): the
explicit transpose, the nested-dissection order and the sparse LU that the
plan builds before any kernel runs. They are checked against the oracle's
independent transpose and against mathematical properties of the factors.
"""

import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2409_11515_amd as pa
from paper_2409_11515_amd import _binding
from oracle.csr import transpose_csr
from synth import Csr, csr_from_dense, diag_csr, hydromech2d, scaled_banded, stokes2d, start_vector

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "condest.h")).read()
    declared = set(re.findall(r"\b(cond_[a-z_0-9]+)\s*\(", hdr))
    assert declared == set(_binding.EXPORTS)
    L = _binding.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert pa.version() >= 1


def test_transpose_matches_oracle_bitwise():
    a = hydromech2d(12, seed=3)
    tr, tc, tv = pa.csr_transpose(a.n, a.rowptr, a.col, a.val)
    orp, oc, ov = transpose_csr(a.n, a.rowptr, a.col, a.val)
    np.testing.assert_array_equal(tr, orp)
    np.testing.assert_array_equal(tc, oc)
    np.testing.assert_array_equal(tv, ov)


def test_transpose_empty_rows_and_unsorted_input():
    d = np.array([[0, 0, 0, 0], [3.0, 0, 1.0, 0], [0, 0, 0, 0], [0, 2.0, 0, 5.0]])
    rowptr = np.array([0, 0, 2, 2, 4])
    col = np.array([2, 0, 3, 1])  # unsorted within rows
    val = np.array([1.0, 3.0, 5.0, 2.0])
    tr, tc, tv = pa.csr_transpose(4, rowptr, col, val)
    t = sp.csr_matrix((tv, tc, tr), shape=(4, 4)).toarray()
    np.testing.assert_array_equal(t, d.T)


@pytest.mark.parametrize("bad", [
    (2, [0, 1], [0], [1.0]),
    (2, [0, 1, 1], [2], [1.0]),
    (2, [0, 1, 2], [0, 1], [1.0, np.inf]),
    (2, [0, 2, 1], [0, 1], [1.0, 1.0]),
    (2, [0, 0, 0], [], []),
    (0, [0], [], []),
])
def test_csr_check_rejects(bad):
    n, rp, col, val = bad
    rp = np.array(rp, np.int64)
    if rp.size != n + 1:
        # the binding sizes nnz from rowptr; pass a struct with a short rowptr on purpose
        h = _binding.HostCsr(max(n, 1), np.append(rp, rp[-1]), col, val)
        h.struct.n = n if n > 0 else 0
        h.struct.nnz = 99
        st = _binding.lib().cond_csr_check(C.byref(h.struct))
        assert st == _binding.COND_EINVAL
        return
    with pytest.raises(pa.CondError) as e:
        pa.csr_check(n, rp, col, val)
    assert e.value.status == _binding.COND_EINVAL


def test_nd_order_is_a_permutation():
    a = hydromech2d(20, seed=1)
    p = pa.order_nd(a.n, a.rowptr, a.col, a.val)
    assert sorted(p.tolist()) == list(range(a.n))


@pytest.mark.parametrize("mk", [
    lambda: stokes2d(10, 10, seed=0),
    lambda: scaled_banded(3000, seed=5),
    lambda: hydromech2d(30, seed=2),
])
def test_lu_factors_reproduce_pa_q(mk):
    a = mk()
    lu = pa.LU(a.n, a.rowptr, a.col, a.val)
    f = lu.export()
    n = a.n
    L = sp.csr_matrix((f["l_val"], f["l_col"], f["l_rowptr"]), shape=(n, n)) + sp.eye(n)
    U = sp.csr_matrix((f["u_val"], f["u_col"], f["u_rowptr"]), shape=(n, n)) + sp.diags(f["u_diag"])
    assert sp.triu(L, 1).nnz == 0 and sp.tril(U, -1).nnz == 0
    assert sorted(f["row_perm"].tolist()) == list(range(n))
    assert sorted(f["col_perm"].tolist()) == list(range(n))
    A = a.to_scipy()
    paq = A[f["row_perm"]][:, f["col_perm"]]
    # componentwise: |PAQ - LU| <= c eps |L||U|, checked on random vectors
    z = start_vector(n, 3)
    lhs = np.abs(paq @ z - L @ (U @ z))
    rhs = abs(L) @ (abs(U) @ np.abs(z))
    assert np.max(lhs / np.maximum(rhs, 1e-300)) < 1e-12


@pytest.mark.parametrize("trans", [False, True])
def test_lu_host_solve_backward_error(trans):
    a = hydromech2d(24, seed=4)
    lu = pa.LU(a.n, a.rowptr, a.col, a.val)
    A = a.to_scipy()
    M = A.T if trans else A
    x = start_vector(a.n, 8)
    r = lu.solve(x, trans=trans)
    be = np.max(np.abs(M @ r - x) / (abs(M) @ np.abs(r) + np.abs(x)))
    assert be < 1e-9


def test_lu_singular_matrix_reports_esingular():
    d = np.eye(5)
    d[3, 3] = 0.0
    d[3, 1] = 0.0
    a = Csr.from_scipy(sp.csr_matrix(d))
    with pytest.raises(pa.CondError) as e:
        pa.LU(a.n, a.rowptr, a.col, a.val)
    assert e.value.status == _binding.COND_ESINGULAR


def test_lu_rejects_bad_col_perm():
    a = scaled_banded(20, seed=1)
    with pytest.raises(pa.CondError) as e:
        pa.LU(a.n, a.rowptr, a.col, a.val, col_perm=np.zeros(20, np.int32))
    assert e.value.status == _binding.COND_EINVAL


def test_plan_create_on_host_reports_workspace():
    # plan_create does host work only; its workspace size must cover the data
    a = hydromech2d(10, seed=1)
    p = pa.Plan(a.n, a.rowptr, a.col, a.val)
    assert p.workspace_bytes >= 12 * 2 * a.nnz + 8 * 10 * a.n
    p.close()


def test_solve_schedule_on_host():
    # the panel schedule is host data: a panel holds 1..64 rows, a level at
    # least one panel, a panel at least one task (slices plus a finish step)
    a = hydromech2d(40, seed=2)
    p = pa.Plan(a.n, a.rowptr, a.col, a.val)
    info = p.solve_info()
    assert set(info) == {"L", "U", "Ut", "Lt"}
    for levels, tasks, panels in info.values():
        assert 1 <= levels <= panels <= tasks
        assert -(-a.n // 64) <= panels <= a.n
    p.close()
    q = pa.Plan(a.n, a.rowptr, a.col, a.val, sigma_min_method=pa.COND_MIN_NONE)
    with pytest.raises(_binding.CondError):
        q.solve_info()
    q.close()


def _dense(n, seed):
    rng = np.random.default_rng(seed)
    return csr_from_dense(rng.standard_normal((n, n)) + 2.0 * np.sqrt(n) * np.eye(n))


def _perm_diag(n, seed):
    rng = np.random.default_rng(seed)
    return diag_csr(10.0 ** rng.uniform(-6, 6, n), row_perm=rng.permutation(n),
                    col_perm=rng.permutation(n))


@pytest.mark.parametrize("mk,bound", [(lambda: csr_from_dense(np.array([[3.0]])), 1e-15),
                                      (lambda: _perm_diag(50, 1), 1e-15),
                                      (lambda: scaled_banded(300, seed=1), 1e-12),
                                      (lambda: _dense(300, 2), 1e-12),
                                      (lambda: stokes2d(10, 10, seed=0), 1e-9),
                                      (lambda: hydromech2d(30, seed=3), 1e-9),
                                      (lambda: hydromech2d(61, seed=5), 1e-9),
                                      (lambda: hydromech2d(201, seed=1), 1e-6)])
def test_solve_schedule_replayed_on_host(mk, bound):
    # the data the device solves run on (task records, slices and slots,
    # packed inverses of the panel triangles, gathers, scatters), with
    # the tasks taken in ticket order, solve the system: componentwise
    # backward errors, and agreement with the oracle's SuperLU solves (two
    # pivoted factorisations). The replay itself refuses a schedule in
    # which a task reads a value that a later ticket solves.
    # Edge cases: a 1x1 matrix, a permuted diagonal (one level, one panel),
    # banded and dense matrices (full panels, sliced panels at 300x300)
    from oracle.inverse import LUInverse

    a = mk()
    p = pa.Plan(a.n, a.rowptr, a.col, a.val)
    x = start_vector(a.n, 2)
    r, s = p.solve_replay(x)
    p.close()
    A = a.to_scipy()
    be_r = np.max(np.abs(A @ r - x) / (abs(A) @ np.abs(r) + np.abs(x)))
    be_s = np.max(np.abs(A.T @ s - r) / (abs(A.T) @ np.abs(s) + np.abs(r)))
    assert be_r < bound and be_s < bound, (be_r, be_s)
    if a.n <= 30000:
        r_ref, s_ref = LUInverse(a.n, a.rowptr, a.col, a.val).apply(x)
        assert np.linalg.norm(r - r_ref) <= 1e-6 * np.linalg.norm(r_ref)
        assert np.linalg.norm(s - s_ref) <= 1e-6 * np.linalg.norm(s_ref)


def test_batch_create_on_host():
    # batch set-up is host work: concatenation and workspace sizing
    mats = [hydromech2d(s, seed=s) for s in (5, 7, 6)]
    b = pa.Batch([(m.n, m.rowptr, m.col, m.val) for m in mats])
    assert list(b.row0) == [0, mats[0].n, mats[0].n + mats[1].n, sum(m.n for m in mats)]
    assert b.workspace_bytes >= 8 * 8 * 7 * b.row0[-1]
    b.close()


def test_interleave_starts_layout():
    s0 = np.arange(16.0).reshape(8, 2)
    s1 = 100 + np.arange(24.0).reshape(8, 3)
    v = pa.interleave_starts([s0, s1])
    # global row 0 = matrix 0 row 0: starts 0..7 are s0[:, 0]
    np.testing.assert_array_equal(v[:8], s0[:, 0])
    np.testing.assert_array_equal(v[8:16], s0[:, 1])
    np.testing.assert_array_equal(v[16:24], s1[:, 0])
    assert v.size == 8 * 5


def test_device_arguments_checked_before_the_library():
    # every pointer handed to the C ABI is checked first: a wrong dtype,
    # length, layout or device raises ValueError before any launch (the plan
    # is not even bound here, so a call that got through would fail with
    # COND_ESTATE from the library instead)
    import torch

    a = hydromech2d(5, seed=1)
    p = pa.Plan(a.n, a.rowptr, a.col, a.val, sigma_min_method=pa.COND_MIN_NONE)
    good = torch.zeros(a.n, dtype=torch.float64)
    bad = [torch.zeros(a.n, dtype=torch.float32),        # dtype
           torch.zeros(a.n - 1, dtype=torch.float64),    # too short
           torch.zeros(2 * a.n, dtype=torch.float64)[::2],  # strided
           good,                                         # host memory
           np.zeros(a.n)]                                # not a tensor
    for x in bad:
        with pytest.raises(ValueError):
            p.run(x)
        with pytest.raises(ValueError):
            p.spmv(x)
        with pytest.raises(ValueError):
            p.inverse_apply(x)
        with pytest.raises(ValueError):
            pa.estimate_cond(a.n, a.rowptr, a.col, a.val, x)
    with pytest.raises(ValueError):
        p.run(None, None)
    p.close()
    mats = [hydromech2d(s, seed=s) for s in (5, 6)]
    b = pa.Batch([(m.n, m.rowptr, m.col, m.val) for m in mats])
    rows = int(b.row0[-1])
    for x in (torch.zeros(rows, dtype=torch.float64), torch.zeros(8 * rows, dtype=torch.float64),
              torch.zeros(8 * rows, dtype=torch.float32)):
        with pytest.raises(ValueError):
            b.run(x)
    b.close()


def test_batch_merged_solves_replayed_on_host():
    # the batch's sigma_min route factors every matrix (parallel threads),
    # merges the factors block-diagonally and plans the four solves over
    # them; replayed on the host in ticket order, for every (matrix, start)
    # the solves give A_m^-1 x and A_m^-T r: backward errors per matrix and
    # agreement with the oracle's SuperLU solves
    from oracle.inverse import LUInverse
    from synth import hm_batch_specs, start_block

    specs = hm_batch_specs(count=5, side_range=(5, 24), seed_sides=11, seed_base=12)
    mats = [hydromech2d(s, log_eta=le, log_k=lk) for s, le, lk in specs]
    b = pa.Batch([(m.n, m.rowptr, m.col, m.val) for m in mats], sigma_min=True)
    f = b.fill()
    assert f["nnz_l"] > 0 and f["nnz_u"] >= b.row0[-1]
    starts = [start_block(m.n, 8, 70 + i) for i, m in enumerate(mats)]
    x = pa.interleave_starts(starts)
    r, s = b.solve_replay(x)
    b.close()
    for i, m in enumerate(mats):
        lo, hi = b.row0[i], b.row0[i + 1]
        A = m.to_scipy()
        inv = LUInverse(m.n, m.rowptr, m.col, m.val)
        for k in range(8):
            xk = starts[i][k]
            rk = r[lo * 8 + k:hi * 8:8]
            sk = s[lo * 8 + k:hi * 8:8]
            be_r = np.max(np.abs(A @ rk - xk) / (abs(A) @ np.abs(rk) + np.abs(xk)))
            be_s = np.max(np.abs(A.T @ sk - rk) / (abs(A.T) @ np.abs(sk) + np.abs(rk)))
            assert be_r < 1e-9 and be_s < 1e-9, (i, k, be_r, be_s)
            r_ref, s_ref = inv.apply(xk)
            assert np.linalg.norm(rk - r_ref) <= 1e-6 * np.linalg.norm(r_ref)
            assert np.linalg.norm(sk - s_ref) <= 1e-6 * np.linalg.norm(s_ref)


def test_batch_without_min_route_refuses_run_min():
    mats = [hydromech2d(s, seed=s) for s in (5, 6)]
    b = pa.Batch([(m.n, m.rowptr, m.col, m.val) for m in mats])
    with pytest.raises(_binding.CondError):
        b.fill()
    with pytest.raises(_binding.CondError):
        b.solve_replay(np.zeros(8 * b.row0[-1]))
    b.close()
