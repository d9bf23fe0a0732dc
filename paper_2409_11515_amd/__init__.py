"""MI355X Projected Adam condition-number estimator (arXiv 2409.11515).

Python face of the C-ABI library ``libcondest.so`` (declared in
``include/condest.h``). The functions here have the same names as the C
entry points without the ``cond_`` prefix and only marshal arguments:
numpy arrays for host data, torch tensors for device memory and streams.

    from paper_2409_11515_amd import estimate_cond
    r = estimate_cond(n, rowptr, col, val, x0_max=x0)   # x0: torch float64 on cuda
    r["kappa"], r["sigma_max"], r["sigma_min"]
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from ._binding import (  # noqa: F401
    COND_F_MAXITER,
    COND_F_NUMSING,
    COND_MIN_LU,
    COND_MIN_NONE,
    COND_MIN_SPMV,
    COND_SCALE_COL,
    COND_SCALE_NONE,
    CondError,
    HostCsr,
    ResultT,
    check,
    lib,
    make_opts,
)

__all__ = ["csr_check", "csr_transpose", "order_nd", "LU", "Plan", "Batch", "CNN", "interleave_starts",
           "estimate_cond", "estimate_batched", "CondError"]


def version() -> int:
    return lib().cond_version()


def csr_check(n, rowptr, col, val) -> None:
    h = HostCsr(n, rowptr, col, val)
    check(lib().cond_csr_check(C.byref(h.struct)), "csr_check")


def csr_transpose(n, rowptr, col, val):
    """(t_rowptr int64, t_col int32, t_val float64) of A^T, computed by the library."""
    h = HostCsr(n, rowptr, col, val)
    nnz = int(h.rowptr[-1])
    tr = np.empty(n + 1, np.int64)
    tc = np.empty(nnz, np.int32)
    tv = np.empty(nnz, np.float64)
    check(lib().cond_csr_transpose(C.byref(h.struct), tr.ctypes.data, tc.ctypes.data,
                                   tv.ctypes.data), "csr_transpose")
    return tr, tc, tv


def order_nd(n, rowptr, col, val) -> np.ndarray:
    h = HostCsr(n, rowptr, col, val)
    perm = np.empty(n, np.int32)
    check(lib().cond_order_nd(C.byref(h.struct), perm.ctypes.data), "order_nd")
    return perm


class LU:
    """Host LU of the library, P A Q = L U (for checks of the set-up step)."""

    def __init__(self, n, rowptr, col, val, col_perm=None, pivot_tol=1e-6):
        h = HostCsr(n, rowptr, col, val)
        cp = None if col_perm is None else np.ascontiguousarray(col_perm, np.int32)
        self._h = C.c_void_p()
        check(lib().cond_lu_factor(C.byref(h.struct), None if cp is None else cp.ctypes.data,
                                   float(pivot_tol), C.byref(self._h)), "lu_factor")
        n_ = C.c_int32()
        nl = C.c_int64()
        nu = C.c_int64()
        check(lib().cond_lu_info(self._h, C.byref(n_), C.byref(nl), C.byref(nu)), "lu_info")
        self.n, self.nnz_l, self.nnz_u = n_.value, nl.value, nu.value

    def export(self) -> dict:
        n = self.n
        nl = self.nnz_l
        nus = self.nnz_u - n
        out = dict(l_rowptr=np.empty(n + 1, np.int64), l_col=np.empty(nl, np.int32),
                   l_val=np.empty(nl), u_rowptr=np.empty(n + 1, np.int64),
                   u_col=np.empty(nus, np.int32), u_val=np.empty(nus), u_diag=np.empty(n),
                   row_perm=np.empty(n, np.int32), col_perm=np.empty(n, np.int32))
        keys = ["l_rowptr", "l_col", "l_val", "u_rowptr", "u_col", "u_val", "u_diag", "row_perm",
                "col_perm"]
        check(lib().cond_lu_export(self._h, *[out[k].ctypes.data for k in keys]), "lu_export")
        return out

    def solve(self, x, trans=False) -> np.ndarray:
        x = np.ascontiguousarray(x, np.float64)
        r = np.empty_like(x)
        check(lib().cond_lu_solve_host(self._h, 1 if trans else 0, x.ctypes.data, r.ctypes.data),
              "lu_solve_host")
        return r

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().cond_lu_destroy(self._h)
            self._h = C.c_void_p()


def _vec(x, n, name="x", dtype=None):
    """Device pointer of ``x`` after checking it is what the C ABI reads: a
    contiguous CUDA tensor of ``n`` elements of ``dtype`` (float64 unless
    given). Raises ValueError before any launch otherwise, so a host, short,
    strided or float32 tensor never reaches a kernel."""
    import torch

    dtype = torch.float64 if dtype is None else dtype
    if not isinstance(x, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor on the GPU")
    if x.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, not {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if x.numel() != n:
        raise ValueError(f"{name} must have {n} elements, not {x.numel()}")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must be on a CUDA (HIP) device, not {x.device}")
    return x.data_ptr()


def _stream_ptr(torch, stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Plan:
    """Device plan: host set-up at construction, device memory from torch.

    ``Plan(n, rowptr, col, val, **opts)`` validates the matrix, builds A^T
    and (unless ``sigma_min_method=COND_MIN_NONE``) the LU on the host;
    ``bind()`` allocates the workspace as a torch uint8 CUDA tensor and
    uploads; ``run()`` performs both Projected Adam runs.
    """

    def __init__(self, n, rowptr, col, val, col_perm=None, **opts):
        self._h = C.c_void_p()
        self.n = int(n)
        self.opts = make_opts(**opts)
        h = HostCsr(n, rowptr, col, val)
        cp = None if col_perm is None else np.ascontiguousarray(col_perm, np.int32)
        self.opts.col_perm = None if cp is None else cp.ctypes.data
        check(lib().cond_plan_create(C.byref(h.struct), C.byref(self.opts), C.byref(self._h)),
              "plan_create")
        self.opts.col_perm = None
        sz = C.c_size_t()
        check(lib().cond_plan_workspace_bytes(self._h, C.byref(sz)), "plan_workspace_bytes")
        self.workspace_bytes = sz.value
        self.workspace = None

    def bind(self, device="cuda", stream=None, own_memory=False):
        import torch

        if own_memory:
            ptr = None
        else:
            self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8,
                                         device=device)
            base = self.workspace.data_ptr()
            ptr = (base + 255) // 256 * 256
        check(lib().cond_plan_bind(self._h, ptr, self.workspace_bytes,
                                   _stream_ptr(torch, stream)), "plan_bind")
        return self

    def run(self, x0_max, x0_min=None, trace=False, x_best=False, **opts) -> dict:
        import torch

        o = make_opts(**{**self._opts_dict(), **opts})
        if x0_max is None and x0_min is None:
            raise ValueError("run needs x0_max, x0_min or both")
        p_max = None if x0_max is None else _vec(x0_max, self.n, "x0_max")
        p_min = None if x0_min is None else _vec(x0_min, self.n, "x0_min")
        dev = (x0_max if x0_max is not None else x0_min).device
        T = int(o.max_iter)
        tmax = torch.zeros(T, dtype=torch.float64, device=dev) if trace else None
        tmin = torch.zeros(T, dtype=torch.float64, device=dev) if trace else None
        bmax = torch.zeros(self.n, dtype=torch.float64, device=dev) if x_best else None
        bmin = torch.zeros(self.n, dtype=torch.float64, device=dev) if x_best else None
        res = ResultT()
        st = lib().cond_plan_run(self._h, C.byref(o), p_max, p_min, C.byref(res),
                                 None if tmax is None else tmax.data_ptr(),
                                 None if tmin is None else tmin.data_ptr(),
                                 None if bmax is None else bmax.data_ptr(),
                                 None if bmin is None else bmin.data_ptr())
        out = {f: getattr(res, f) for f, _ in ResultT._fields_}
        out["status"] = st
        if trace:
            out["trace_max"] = tmax[: max(res.iters_max, 0)].cpu().numpy()
            out["trace_min"] = tmin[: max(res.iters_min, 0)].cpu().numpy()
        if x_best:
            out["x_best_max"] = bmax
            out["x_best_min"] = bmin
        check(st, "plan_run")
        return out

    def _opts_dict(self):
        return {f: getattr(self.opts, f) for f, _ in self.opts._fields_ if f != "col_perm"}

    def kernel_stats(self) -> dict:
        """{kernel: (total_ms, launches, algorithmic_bytes_per_launch)} of the last profiled run."""
        from ._binding import KERNEL_NAMES

        k = len(KERNEL_NAMES)
        ms = np.zeros(k)
        cnt = np.zeros(k, np.int64)
        by = np.zeros(k)
        check(lib().cond_plan_kernel_stats(self._h, ms.ctypes.data, cnt.ctypes.data, by.ctypes.data),
              "plan_kernel_stats")
        return {name: (float(ms[i]), int(cnt[i]), float(by[i])) for i, name in enumerate(KERNEL_NAMES)}

    def solve_info(self) -> dict:
        """{solve: (levels, tasks, panels)} of the four triangular solves
        (L, U, Ut, Lt): the panel schedule the planner chose."""
        lv = np.zeros(4, np.int32)
        tk = np.zeros(4, np.int64)
        pn = np.zeros(4, np.int64)
        check(lib().cond_plan_solve_info(self._h, lv.ctypes.data, tk.ctypes.data, pn.ctypes.data),
              "plan_solve_info")
        return {name: (int(lv[i]), int(tk[i]), int(pn[i]))
                for i, name in enumerate(("L", "U", "Ut", "Lt"))}

    def solve_replay(self, x):
        """(r, s) = (A^-1 x, A^-T r) on the host from the device-ready solve
        schedule (numpy float64 in and out); needs no device."""
        x = np.ascontiguousarray(x, np.float64)
        r = np.empty_like(x)
        s = np.empty_like(x)
        check(lib().cond_plan_solve_replay(self._h, x.ctypes.data, r.ctypes.data, s.ctypes.data),
              "plan_solve_replay")
        return r, s

    def spmv(self, x, transpose=False, col_scaled=False):
        """y = A x (A^T x with transpose); with col_scaled the matrix is the
        column-scaled A D_col^-1."""
        import torch

        px = _vec(x, self.n)
        y = torch.empty_like(x)
        flags = (1 if transpose else 0) | (2 if col_scaled else 0)
        check(lib().cond_plan_spmv(self._h, flags, px, y.data_ptr()), "plan_spmv")
        return y

    def column_norms(self):
        """The column 2-norms of A (D_col of column scaling), on the device."""
        import torch

        d = torch.empty(self.n, dtype=torch.float64, device=self.workspace.device
                        if self.workspace is not None else "cuda")
        check(lib().cond_plan_column_norms(self._h, d.data_ptr()), "plan_column_norms")
        return d

    def inverse_apply(self, x):
        import torch

        px = _vec(x, self.n)
        r = torch.empty_like(x)
        s = torch.empty_like(x)
        check(lib().cond_plan_inverse_apply(self._h, px, r.data_ptr(), s.data_ptr()),
              "plan_inverse_apply")
        return r, s

    def error_bounds(self, x_hat, b, kappa, norm_a) -> dict:
        """Bounds on the error of x_hat as a solution of A x = b (CUDA float64
        tensors of n entries) from kappa and ||A|| = sigma_max: the four
        theorems of section "Error estimates and conditioning"."""
        from ._binding import BoundsT

        px = _vec(x_hat, self.n, "x_hat")
        pb = _vec(b, self.n, "b")
        out = BoundsT()
        check(lib().cond_plan_error_bounds(self._h, px, pb, float(kappa), float(norm_a),
                                           C.byref(out)), "plan_error_bounds")
        return {f: getattr(out, f) for f, _ in BoundsT._fields_}

    def inject_timeout(self):
        """Test hook: the next sigma_min run or inverse apply starts timed out."""
        check(lib().cond_plan_inject_timeout(self._h), "plan_inject_timeout")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().cond_plan_destroy(self._h)
            self._h = C.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may already be gone
            pass


class Batch:
    """Batched multi-start runs over many matrices (8 starts each).

    ``Batch([(n, rowptr, col, val), ...], sigma_min=False, **opts).bind()``
    concatenates the matrices block-diagonally (with ``sigma_min=True`` it
    also factors every matrix for the sigma_min run); ``run(x0)`` is the
    sigma_max run and ``run_min(x0)`` the sigma_min run, each taking a CUDA
    float64 tensor of ``rows * 8`` entries (row i, start k at index 8*i + k;
    see ``row0``).
    """

    K = 8

    def __init__(self, mats, sigma_min=False, **opts):
        from ._binding import CsrT

        self._h = C.c_void_p()
        opts.setdefault("sigma_min_method", COND_MIN_LU if sigma_min else COND_MIN_NONE)
        self.opts = make_opts(**opts)
        self._keep = [HostCsr(*m) for m in mats]
        arr = (CsrT * len(self._keep))(*[h.struct for h in self._keep])
        check(lib().cond_batch_create(C.cast(arr, C.c_void_p), len(self._keep), C.byref(self.opts),
                                      C.byref(self._h)), "batch_create")
        self.count = len(self._keep)
        self.row0 = np.zeros(self.count + 1, np.int64)
        sz = C.c_size_t()
        check(lib().cond_batch_info(self._h, self.row0.ctypes.data, C.byref(sz), None, None),
              "batch_info")
        self.workspace_bytes = sz.value
        self.workspace = None

    def bind(self, device="cuda", stream=None, tile_rows=0, grid=0):
        import torch

        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        check(lib().cond_batch_bind(self._h, ptr, self.workspace_bytes, _stream_ptr(torch, stream),
                                    int(tile_rows), int(grid)), "batch_bind")
        tr = C.c_int32()
        gr = C.c_int32()
        check(lib().cond_batch_info(self._h, None, None, C.byref(tr), C.byref(gr)), "batch_info")
        self.tile_rows, self.grid = tr.value, gr.value
        return self

    def fill(self) -> dict:
        """nnz of the merged factors and the host LU time (sigma_min batches)."""
        nl, nu, ms = C.c_int64(), C.c_int64(), C.c_double()
        check(lib().cond_batch_fill(self._h, C.byref(nl), C.byref(nu), C.byref(ms)), "batch_fill")
        return {"nnz_l": nl.value, "nnz_u": nu.value, "lu_s": ms.value / 1e3}

    def solve_replay(self, x):
        """(r, s) = (A_m^-1 x, A_m^-T r) per (matrix, start) on the host from
        the device-ready merged solve schedules (numpy, batch layout)."""
        x = np.ascontiguousarray(x, np.float64)
        r = np.empty_like(x)
        s = np.empty_like(x)
        check(lib().cond_batch_solve_replay(self._h, x.ctypes.data, r.ctypes.data, s.ctypes.data),
              "batch_solve_replay")
        return r, s

    def run_min(self, x0, trace=False, **opts) -> dict:
        """The sigma_min run (Algorithm 2) of every (matrix, start) pair;
        ``pair_best`` holds ||A^-1 x|| / ||x||, ``sigma_min`` 1 / its maximum."""
        return self.run(x0, trace=trace, _route=1, **opts)

    def run(self, x0, trace=False, _route=0, **opts) -> dict:
        import torch

        o = make_opts(**{**{f: getattr(self.opts, f) for f, _ in self.opts._fields_
                            if f != "col_perm"}, **opts})
        npairs = self.count * self.K
        px = _vec(x0, int(self.row0[-1]) * self.K, "x0")
        smax = np.zeros(self.count)
        best = np.zeros(npairs)
        iters = np.zeros(npairs, np.int64)
        status = np.zeros(npairs, np.int32)
        tr = torch.zeros(npairs * int(o.max_iter), dtype=torch.float64,
                         device=x0.device) if trace else None
        ms = C.c_double()
        fn = lib().cond_batch_run_min if _route == 1 else lib().cond_batch_run
        st = fn(self._h, C.byref(o), px, smax.ctypes.data, best.ctypes.data, iters.ctypes.data,
                status.ctypes.data, None if tr is None else tr.data_ptr(), None, C.byref(ms))
        out = dict(pair_best=best.reshape(self.count, self.K),
                   pair_iters=iters.reshape(self.count, self.K),
                   pair_status=status.reshape(self.count, self.K), ms=ms.value, status=st)
        out["sigma_min" if _route == 1 else "sigma_max"] = smax
        if trace:
            out["trace"] = tr.view(self.count, self.K, int(o.max_iter)).cpu().numpy()
        check(st, "batch_run_min" if _route == 1 else "batch_run")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().cond_batch_destroy(self._h)
            self._h = C.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may already be gone
            pass


def interleave_starts(starts_per_matrix) -> np.ndarray:
    """Per matrix an array of shape (8, n_m) (start k in row k) -> one float64
    vector in the batch layout: global row i, start k at index 8*i + k."""
    return np.ascontiguousarray(np.concatenate(
        [np.asarray(s, np.float64).T.reshape(-1) for s in starts_per_matrix]))


def stream_triad(n, grid=4096, reps=20, stream=None) -> dict:
    """The device's streaming ceiling: a = b + s c over n doubles (24 n bytes
    per launch) by the library's own kernel; average ms per launch and GB/s."""
    import torch

    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.rand(n, dtype=torch.float64, device="cuda")
    ms = C.c_double()
    check(lib().cond_stream_triad(int(n), a.data_ptr(), b.data_ptr(), c.data_ptr(), 0.5, int(grid),
                                  int(reps), _stream_ptr(torch, stream), C.byref(ms)), "stream_triad")
    ref = b + 0.5 * c
    if not torch.equal(a, ref):
        raise RuntimeError("triad kernel wrote wrong values")
    return {"ms": ms.value, "bytes": 24.0 * n, "gbs": 24.0 * n / (ms.value * 1e-3) / 1e9}


def estimate_batched(mats, x0_max, x0_min=None, stream=None, **opts) -> list:
    """cond_estimate_batched: kappa_2 of every matrix of [(n, rowptr, col,
    val), ...] from 8 starts each (x0 in the batch layout, CUDA float64);
    one result dict per matrix."""
    import torch

    from ._binding import CsrT

    keep = [HostCsr(*m) for m in mats]
    rows = sum(h.n for h in keep)
    arr = (CsrT * len(keep))(*[h.struct for h in keep])
    o = make_opts(**opts)
    outs = (ResultT * len(keep))()
    p_max = _vec(x0_max, rows * Batch.K, "x0_max")
    p_min = None if x0_min is None else _vec(x0_min, rows * Batch.K, "x0_min")
    check(lib().cond_estimate_batched(C.cast(arr, C.c_void_p), len(keep), C.byref(o), p_max, p_min,
                                      _stream_ptr(torch, stream), C.cast(outs, C.c_void_p)),
          "estimate_batched")
    return [{f: getattr(r, f) for f, _ in ResultT._fields_} for r in outs]


def estimate_cond(n, rowptr, col, val, x0_max, x0_min=None, stream=None, **opts) -> dict:
    """kappa_2 of the CSR matrix: create + bind (library memory) + run + destroy."""
    import torch

    h = HostCsr(n, rowptr, col, val)
    o = make_opts(**opts)
    res = ResultT()
    p_max = _vec(x0_max, int(n), "x0_max")
    p_min = None if x0_min is None else _vec(x0_min, int(n), "x0_min")
    st = lib().cond_estimate(C.byref(h.struct), C.byref(o), p_max, p_min,
                             _stream_ptr(torch, stream), C.byref(res))
    check(st, "estimate")
    return {f: getattr(res, f) for f, _ in ResultT._fields_}


def error_bounds_noalloc(rowptr, col, val, x_hat, b, kappa, norm_a, stream=None) -> dict:
    """cond_error_bounds_noalloc: the error bounds for A given on the device
    (rowptr int64 [n+1], col int32 [nnz], val float64 [nnz], all CUDA
    tensors) without any device allocation inside the library."""
    import torch

    from ._binding import BoundsT

    n = int(rowptr.numel()) - 1
    nnz = int(col.numel())
    prp = _vec(rowptr, n + 1, "rowptr", torch.int64)
    pc = _vec(col, nnz, "col", torch.int32)
    pv = _vec(val, nnz, "val")
    px = _vec(x_hat, n, "x_hat")
    pb = _vec(b, n, "b")
    out = BoundsT()
    check(lib().cond_error_bounds_noalloc(n, nnz, prp, pc, pv, px, pb, float(kappa),
                                          float(norm_a), _stream_ptr(torch, stream),
                                          C.byref(out)), "error_bounds_noalloc")
    return {f: getattr(out, f) for f, _ in BoundsT._fields_}


class CNN:
    """The warm-start network on the device (``cond_cnn_*``).

    ``CNN(max_batch, max_side, train=True)``; ``set_params(vec)`` takes the
    float32 parameter vector (layer by layer, W[ky][kx][ci][co] then b[co]);
    ``predict(fields)`` maps a CUDA float64 tensor [batch, 2, side-1, side-1]
    of per-cell (log10 eta, log10 k) to start vectors [batch, 6 side^2];
    ``gradients`` / ``train_step`` take float32 labels in that layout.
    """

    def __init__(self, max_batch, max_side, train=True, stream=None):
        import torch

        self._h = C.c_void_p()
        self.max_batch, self.max_side = int(max_batch), int(max_side)
        self.param_count = lib().cond_cnn_param_count()
        check(lib().cond_cnn_create(self.max_batch, self.max_side, 1 if train else 0,
                                    _stream_ptr(torch, stream), C.byref(self._h)), "cnn_create")

    def set_params(self, vec):
        v = np.ascontiguousarray(vec, np.float32)
        if v.size != self.param_count:
            raise ValueError(f"expected {self.param_count} parameters, got {v.size}")
        check(lib().cond_cnn_set_params(self._h, v.ctypes.data), "cnn_set_params")
        return self

    def get_params(self) -> np.ndarray:
        v = np.zeros(self.param_count, np.float32)
        check(lib().cond_cnn_get_params(self._h, v.ctypes.data), "cnn_get_params")
        return v

    @staticmethod
    def _shape(fields):
        import torch

        if not isinstance(fields, torch.Tensor) or fields.device.type != "cuda" \
                or fields.dtype != torch.float64 or fields.dim() != 4 or fields.shape[1] != 2 \
                or fields.shape[2] != fields.shape[3] or not fields.is_contiguous():
            raise ValueError("fields must be a contiguous float64 CUDA tensor [batch, 2, s-1, s-1]")
        return int(fields.shape[0]), int(fields.shape[2]) + 1

    def predict(self, fields):
        import torch

        b, s = self._shape(fields)
        x0 = torch.empty(b, 6 * s * s, dtype=torch.float64, device=fields.device)
        check(lib().cond_cnn_predict(self._h, fields.data_ptr(), b, s, x0.data_ptr()), "cnn_predict")
        return x0

    def gradients(self, fields, labels):
        import torch

        b, s = self._shape(fields)
        _vec(labels, b * 6 * s * s, "labels", torch.float32)
        g = np.zeros(self.param_count, np.float32)
        losses = np.zeros(b, np.float32)
        check(lib().cond_cnn_gradients(self._h, fields.data_ptr(), labels.data_ptr(), b, s,
                                       g.ctypes.data, losses.ctypes.data), "cnn_gradients")
        return g, losses

    def train_step(self, fields, labels, lr) -> float:
        import torch

        b, s = self._shape(fields)
        _vec(labels, b * 6 * s * s, "labels", torch.float32)
        ml = C.c_float()
        check(lib().cond_cnn_train_step(self._h, fields.data_ptr(), labels.data_ptr(), b, s,
                                        float(lr), C.byref(ml)), "cnn_train_step")
        return ml.value

    def activation(self, layer, batch, side) -> np.ndarray:
        ch = (8, 64, 64, 64, 16)[layer]
        a = np.zeros((batch, side, side, ch), np.float32)
        check(lib().cond_cnn_activation(self._h, int(layer), int(batch), int(side), a.ctypes.data),
              "cnn_activation")
        return a

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().cond_cnn_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may already be gone
            pass
