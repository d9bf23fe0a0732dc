// Sparse LU for Algorithm 2 ("Compute Gradient for A^-1"): the paper needs one
// factorisation A = L U, reused by every gradient evaluation. Here it is
// P A Q = L U computed on the host, once per matrix, by a left-looking
// column factorisation (Gilbert and Peierls, 1988): each column of A Q is
// solved against the columns of L found so far, visiting only the rows
// reachable in the graph of L (a depth-first search gives them in
// topological order), then a pivot is chosen by threshold partial pivoting
// that prefers the diagonal entry. The fill-reducing column order Q comes
// from the caller or from nested dissection.
//
// The factors are exported in four CSR orientations (L, U, L^T, U^T) so that
// every triangular solve on the device is a row-wise gather.

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.hpp"

namespace condest {

namespace {

struct ColFactors {
  std::vector<int64_t> lp{0}, up{0};
  std::vector<int32_t> li, ui;
  std::vector<double> lx, ux;
};

// CSC (columns of a matrix) -> CSR of the same matrix, columns sorted.
void csc_to_csr(int32_t n, const std::vector<int64_t>& cp, const std::vector<int32_t>& ci,
                const std::vector<double>& cx, HostCsr& out) {
  out.n = n;
  out.rowptr.assign(n + 1, 0);
  const int64_t nnz = cp[n];
  for (int64_t p = 0; p < nnz; ++p) out.rowptr[ci[p] + 1]++;
  for (int32_t i = 0; i < n; ++i) out.rowptr[i + 1] += out.rowptr[i];
  out.col.resize(nnz);
  out.val.resize(nnz);
  std::vector<int64_t> next(out.rowptr.begin(), out.rowptr.end() - 1);
  for (int32_t j = 0; j < n; ++j)
    for (int64_t p = cp[j]; p < cp[j + 1]; ++p) {
      int64_t q = next[ci[p]]++;
      out.col[q] = j;
      out.val[q] = cx[p];
    }
}

// CSC of a matrix viewed as the CSR of its transpose, with rows sorted.
void csc_as_transpose_csr(int32_t n, const std::vector<int64_t>& cp, std::vector<int32_t> ci,
                          std::vector<double> cx, HostCsr& out) {
  out.n = n;
  out.rowptr = cp;
  std::vector<std::pair<int32_t, double>> tmp;
  for (int32_t j = 0; j < n; ++j) {
    tmp.clear();
    for (int64_t p = cp[j]; p < cp[j + 1]; ++p) tmp.emplace_back(ci[p], cx[p]);
    std::sort(tmp.begin(), tmp.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t k = 0; k < tmp.size(); ++k) {
      ci[cp[j] + k] = tmp[k].first;
      cx[cp[j] + k] = tmp[k].second;
    }
  }
  out.col = std::move(ci);
  out.val = std::move(cx);
}

}  // namespace

int lu_factor(const HostCsr& a, const HostCsr& at, const int32_t* col_perm_in, double tol,
              cond_lu& lu) {
  const int32_t n = a.n;
  if (!(tol > 0.0 && tol <= 1.0)) tol = 1e-6;
  std::vector<int32_t> q(n);
  if (col_perm_in) {
    std::vector<char> seen(n, 0);
    for (int32_t k = 0; k < n; ++k) {
      int32_t j = col_perm_in[k];
      if (j < 0 || j >= n || seen[j]) return fail(COND_EINVAL, "col_perm is not a permutation");
      seen[j] = 1;
      q[k] = j;
    }
  } else {
    nested_dissection(a, at, q);
  }
  // Column j of A is row j of A^T.
  ColFactors f;
  const int64_t guess = 4 * a.nnz();
  f.li.reserve(guess);
  f.lx.reserve(guess);
  f.ui.reserve(guess);
  f.ux.reserve(guess);
  std::vector<double> udiag(n, 0.0), x(n, 0.0);
  std::vector<int32_t> pinv(n, -1), mark(n, -1), xi(n), stk(n);
  std::vector<int64_t> pstk(n);
  // Symmetric pruning (Eisenstat and Liu): the depth-first searches read
  // column kk of L only up to lpend[kk]. Once a later column k has kk in its
  // reach and its pivot row in L(:, kk), the rows of L(:, kk) not yet
  // pivotal are all in L(:, k) as well (stored even where their value is
  // zero), so a search reaching kk finds them through the pivot row and
  // column k: L(:, kk) is reordered with its pivotal rows first and the
  // search stops after them. The reach, and so the factors' structure, is
  // unchanged; only the order the searches list it in (and with it the
  // order of the numeric updates) can differ.
  std::vector<int64_t> lpend;
  lpend.reserve(n);
  std::vector<char> pruned(n, 0);
  for (int32_t k = 0; k < n; ++k) {
    const int32_t j = q[k];
    // --- symbolic: rows reachable from the pattern of A(:, j) through L
    int32_t top = n;
    for (int64_t pa = at.rowptr[j]; pa < at.rowptr[j + 1]; ++pa) {
      int32_t r0 = at.col[pa];
      if (mark[r0] == k) continue;
      int32_t head = 0;
      stk[0] = r0;
      while (head >= 0) {
        int32_t r = stk[head];
        int32_t kk = pinv[r];
        if (mark[r] != k) {
          mark[r] = k;
          pstk[head] = kk < 0 ? 0 : f.lp[kk];
        }
        bool done = true;
        if (kk >= 0) {
          const int64_t pend = lpend[kk];
          for (int64_t p = pstk[head]; p < pend; ++p) {
            int32_t w = f.li[p];
            if (mark[w] == k) continue;
            pstk[head] = p + 1;
            stk[++head] = w;
            done = false;
            break;
          }
        }
        if (done) {
          --head;
          xi[--top] = r;
        }
      }
    }
    // --- numeric: x = L \ A(:, j) over the reach, in topological order
    for (int64_t pa = at.rowptr[j]; pa < at.rowptr[j + 1]; ++pa) x[at.col[pa]] = at.val[pa];
    for (int32_t p = top; p < n; ++p) {
      int32_t r = xi[p];
      int32_t kk = pinv[r];
      if (kk < 0) continue;
      const double xr = x[r];
      if (xr == 0.0) continue;
      for (int64_t pl = f.lp[kk]; pl < f.lp[kk + 1]; ++pl) x[f.li[pl]] -= f.lx[pl] * xr;
    }
    // --- pivot: largest candidate, but keep the diagonal row j if within tol
    int32_t piv = -1;
    double amax = -1.0;
    for (int32_t p = top; p < n; ++p) {
      int32_t r = xi[p];
      if (pinv[r] >= 0) continue;
      double v = std::fabs(x[r]);
      if (v > amax) amax = v, piv = r;
    }
    if (piv < 0 || amax <= 0.0 || !std::isfinite(amax)) {
      for (int32_t p = top; p < n; ++p) x[xi[p]] = 0.0;
      return fail(COND_ESINGULAR, "zero pivot in column " + std::to_string(j));
    }
    if (pinv[j] < 0 && mark[j] == k && std::fabs(x[j]) >= tol * amax) piv = j;
    const double pv = x[piv];
    // --- store U(:, k) (pivotal rows) and L(:, k) (the rest, scaled)
    for (int32_t p = top; p < n; ++p) {
      int32_t r = xi[p];
      double v = x[r];
      x[r] = 0.0;
      if (r == piv) continue;
      int32_t kk = pinv[r];
      if (kk >= 0) {
        if (v != 0.0) {
          f.ui.push_back(kk);
          f.ux.push_back(v);
        }
      } else {
        // kept where zero too: the pruning relies on L(:, k) holding every
        // non-pivotal row of the reach
        f.li.push_back(r);
        f.lx.push_back(v / pv);
      }
    }
    udiag[k] = pv;
    pinv[piv] = k;
    f.lp.push_back(static_cast<int64_t>(f.li.size()));
    f.up.push_back(static_cast<int64_t>(f.ui.size()));
    lpend.push_back(f.lp[k + 1]);
    // --- prune the columns of the reach whose L holds this pivot row
    for (int32_t p = top; p < n; ++p) {
      const int32_t kk = pinv[xi[p]];
      if (kk < 0 || kk == k || pruned[kk]) continue;
      bool has = false;
      for (int64_t pl = f.lp[kk]; pl < lpend[kk] && !has; ++pl) has = f.li[pl] == piv;
      if (!has) continue;
      int64_t lo = f.lp[kk], hi = f.lp[kk + 1] - 1;
      while (lo <= hi) {
        if (pinv[f.li[lo]] >= 0) {
          ++lo;
        } else if (pinv[f.li[hi]] < 0) {
          --hi;
        } else {
          std::swap(f.li[lo], f.li[hi]);
          std::swap(f.lx[lo], f.lx[hi]);
          ++lo;
          --hi;
        }
      }
      lpend[kk] = lo;
      pruned[kk] = 1;
    }
  }
  // rows of L to pivot order
  for (auto& r : f.li) r = pinv[r];
  lu.n = n;
  lu.u_diag = std::move(udiag);
  lu.col_perm = q;
  lu.row_perm.assign(n, -1);
  for (int32_t i = 0; i < n; ++i) lu.row_perm[pinv[i]] = i;
  csc_to_csr(n, f.lp, f.li, f.lx, lu.l_rows);
  csc_to_csr(n, f.up, f.ui, f.ux, lu.u_rows);
  csc_as_transpose_csr(n, f.lp, std::move(f.li), std::move(f.lx), lu.l_cols);
  csc_as_transpose_csr(n, f.up, std::move(f.ui), std::move(f.ux), lu.u_cols);
  return COND_OK;
}

// Host reference triangular solves with the exported layout.
void lu_solve_host(const cond_lu& lu, int trans, const double* x, double* r) {
  const int32_t n = lu.n;
  std::vector<double> w(n);
  if (!trans) {
    // L c = P x, U z = c, r = Q z
    for (int32_t k = 0; k < n; ++k) w[k] = x[lu.row_perm[k]];
    for (int32_t k = 0; k < n; ++k) {
      double s = w[k];
      for (int64_t p = lu.l_rows.rowptr[k]; p < lu.l_rows.rowptr[k + 1]; ++p)
        s -= lu.l_rows.val[p] * w[lu.l_rows.col[p]];
      w[k] = s;
    }
    for (int32_t k = n - 1; k >= 0; --k) {
      double s = w[k];
      for (int64_t p = lu.u_rows.rowptr[k]; p < lu.u_rows.rowptr[k + 1]; ++p)
        s -= lu.u_rows.val[p] * w[lu.u_rows.col[p]];
      w[k] = s / lu.u_diag[k];
    }
    for (int32_t k = 0; k < n; ++k) r[lu.col_perm[k]] = w[k];
  } else {
    // U^T h = Q^T x, L^T v = h, s = P^T v
    for (int32_t k = 0; k < n; ++k) w[k] = x[lu.col_perm[k]];
    for (int32_t k = 0; k < n; ++k) {
      double s = w[k];
      for (int64_t p = lu.u_cols.rowptr[k]; p < lu.u_cols.rowptr[k + 1]; ++p)
        s -= lu.u_cols.val[p] * w[lu.u_cols.col[p]];
      w[k] = s / lu.u_diag[k];
    }
    for (int32_t k = n - 1; k >= 0; --k) {
      double s = w[k];
      for (int64_t p = lu.l_cols.rowptr[k]; p < lu.l_cols.rowptr[k + 1]; ++p)
        s -= lu.l_cols.val[p] * w[lu.l_cols.col[p]];
      w[k] = s;
    }
    for (int32_t k = 0; k < n; ++k) r[lu.row_perm[k]] = w[k];
  }
}

}  // namespace condest

using namespace condest;

extern "C" {

int cond_lu_factor(const cond_csr_t* A, const int32_t* col_perm, double pivot_tol, cond_lu_t** out) {
  if (!out) return fail(COND_EINVAL, "null output");
  *out = nullptr;
  HostCsr a, at;
  int st = canonical_copy(A, a);
  if (st) return st;
  transpose(a, at);
  auto* lu = new (std::nothrow) cond_lu();
  if (!lu) return fail(COND_ENOMEM, "allocation failed");
  try {
    st = lu_factor(a, at, col_perm, pivot_tol, *lu);
  } catch (const std::bad_alloc&) {
    st = fail(COND_ENOMEM, "host memory exhausted in LU");
  }
  if (st) {
    delete lu;
    return st;
  }
  *out = lu;
  return COND_OK;
}

void cond_lu_destroy(cond_lu_t* lu) { delete lu; }

int cond_lu_info(const cond_lu_t* lu, int32_t* n, int64_t* nnz_l, int64_t* nnz_u) {
  if (!lu) return fail(COND_EINVAL, "null lu");
  if (n) *n = lu->n;
  if (nnz_l) *nnz_l = lu->l_rows.nnz();
  if (nnz_u) *nnz_u = lu->u_rows.nnz() + lu->n;
  return COND_OK;
}

int cond_lu_export(const cond_lu_t* lu, int64_t* l_rowptr, int32_t* l_col, double* l_val,
                   int64_t* u_rowptr, int32_t* u_col, double* u_val, double* u_diag,
                   int32_t* row_perm, int32_t* col_perm) {
  if (!lu) return fail(COND_EINVAL, "null lu");
  if (l_rowptr) std::copy(lu->l_rows.rowptr.begin(), lu->l_rows.rowptr.end(), l_rowptr);
  if (l_col) std::copy(lu->l_rows.col.begin(), lu->l_rows.col.end(), l_col);
  if (l_val) std::copy(lu->l_rows.val.begin(), lu->l_rows.val.end(), l_val);
  if (u_rowptr) std::copy(lu->u_rows.rowptr.begin(), lu->u_rows.rowptr.end(), u_rowptr);
  if (u_col) std::copy(lu->u_rows.col.begin(), lu->u_rows.col.end(), u_col);
  if (u_val) std::copy(lu->u_rows.val.begin(), lu->u_rows.val.end(), u_val);
  if (u_diag) std::copy(lu->u_diag.begin(), lu->u_diag.end(), u_diag);
  if (row_perm) std::copy(lu->row_perm.begin(), lu->row_perm.end(), row_perm);
  if (col_perm) std::copy(lu->col_perm.begin(), lu->col_perm.end(), col_perm);
  return COND_OK;
}

int cond_lu_solve_host(const cond_lu_t* lu, int trans, const double* x, double* r) {
  if (!lu || !x || !r) return fail(COND_EINVAL, "null argument");
  lu_solve_host(*lu, trans, x, r);
  return COND_OK;
}

}  // extern "C"
