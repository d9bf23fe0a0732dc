// Host-side CSR handling: validation, canonical copy, explicit transpose.
//
// The gradient of equation nabla_loss needs A^T (A v). The transpose is
// stored explicitly so that both products are row-parallel gathers with no
// atomics on the device.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.hpp"

namespace condest {

static thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int check_csr(const cond_csr_t* A) {
  if (!A) return fail(COND_EINVAL, "null matrix");
  if (A->n <= 0) return fail(COND_EINVAL, "n must be positive");
  if (!A->rowptr) return fail(COND_EINVAL, "null rowptr");
  if (A->rowptr[0] != 0) return fail(COND_EINVAL, "rowptr[0] must be 0");
  const int64_t n = A->n;
  for (int64_t i = 0; i < n; ++i)
    if (A->rowptr[i + 1] < A->rowptr[i]) return fail(COND_EINVAL, "rowptr must be non-decreasing");
  if (A->rowptr[n] != A->nnz) return fail(COND_EINVAL, "rowptr[n] must equal nnz");
  if (A->nnz > 0 && (!A->col || !A->val)) return fail(COND_EINVAL, "null col/val");
  bool any_nonzero = false;
  for (int64_t p = 0; p < A->nnz; ++p) {
    if (A->col[p] < 0 || A->col[p] >= A->n) return fail(COND_EINVAL, "column index out of range");
    if (!std::isfinite(A->val[p])) return fail(COND_EINVAL, "non-finite matrix entry");
    any_nonzero |= (A->val[p] != 0.0);
  }
  if (!any_nonzero) return fail(COND_EINVAL, "zero matrix");
  return COND_OK;
}

int canonical_copy(const cond_csr_t* A, HostCsr& out) {
  int st = check_csr(A);
  if (st) return st;
  const int32_t n = A->n;
  out.n = n;
  out.rowptr.assign(n + 1, 0);
  out.col.clear();
  out.val.clear();
  out.col.reserve(A->nnz);
  out.val.reserve(A->nnz);
  std::vector<std::pair<int32_t, double>> row;
  for (int32_t i = 0; i < n; ++i) {
    row.clear();
    for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) row.emplace_back(A->col[p], A->val[p]);
    std::stable_sort(row.begin(), row.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t k = 0; k < row.size();) {
      size_t e = k;
      double s = 0.0;
      while (e < row.size() && row[e].first == row[k].first) s += row[e++].second;
      out.col.push_back(row[k].first);
      out.val.push_back(s);
      k = e;
    }
    out.rowptr[i + 1] = static_cast<int64_t>(out.col.size());
  }
  return COND_OK;
}

void transpose(const HostCsr& a, HostCsr& t) {
  const int32_t n = a.n;
  const int64_t nnz = a.nnz();
  t.n = n;
  t.rowptr.assign(n + 1, 0);
  for (int64_t p = 0; p < nnz; ++p) t.rowptr[a.col[p] + 1]++;
  for (int32_t i = 0; i < n; ++i) t.rowptr[i + 1] += t.rowptr[i];
  t.col.resize(nnz);
  t.val.resize(nnz);
  std::vector<int64_t> next(t.rowptr.begin(), t.rowptr.end() - 1);
  for (int32_t i = 0; i < n; ++i)
    for (int64_t p = a.rowptr[i]; p < a.rowptr[i + 1]; ++p) {
      int64_t q = next[a.col[p]]++;
      t.col[q] = i;
      t.val[q] = a.val[p];
    }
}

}  // namespace condest

using namespace condest;

extern "C" {

const char* cond_strerror(int status) {
  switch (status) {
    case COND_OK: return "ok";
    case COND_EINVAL: return "invalid argument";
    case COND_ESINGULAR: return "matrix is singular (zero pivot)";
    case COND_ENOMEM: return "out of memory or workspace too small";
    case COND_EHIP: return "HIP runtime error";
    case COND_ENUMERIC: return "norm became zero or non-finite, or a factor block has no finite inverse";
    case COND_ESTATE: return "call out of order";
    case COND_ETIMEOUT: return "triangular-solve wait exceeded its spin limit";
    default: return "unknown status";
  }
}

const char* cond_last_error(void) { return g_last_error.c_str(); }

int cond_version(void) { return 1; }

void cond_opts_default(cond_opts_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->alpha = 1e-2;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->eps = 1e-8;
  o->max_iter = 20000;
  o->stop_rtol = 0.0;
  o->stop_window = 0;
  o->sigma_min_method = COND_MIN_LU;
  o->chunk = 0;
  o->col_perm = nullptr;
  o->pivot_tol = 1e-6;
  o->alpha_min = 0.0;
  o->alpha_decay = 0.5;
}

int cond_csr_check(const cond_csr_t* A) { return check_csr(A); }

int cond_csr_transpose(const cond_csr_t* A, int64_t* t_rowptr, int32_t* t_col, double* t_val) {
  int st = check_csr(A);
  if (st) return st;
  if (!t_rowptr || (A->nnz && (!t_col || !t_val))) return fail(COND_EINVAL, "null output");
  // Transpose the caller's entries as given (no duplicate merging), stably.
  const int32_t n = A->n;
  std::fill(t_rowptr, t_rowptr + n + 1, 0);
  for (int64_t p = 0; p < A->nnz; ++p) t_rowptr[A->col[p] + 1]++;
  for (int32_t i = 0; i < n; ++i) t_rowptr[i + 1] += t_rowptr[i];
  std::vector<int64_t> next(t_rowptr, t_rowptr + n);
  for (int32_t i = 0; i < n; ++i)
    for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
      int64_t q = next[A->col[p]]++;
      t_col[q] = i;
      t_val[q] = A->val[p];
    }
  return COND_OK;
}

}  // extern "C"
