// Internal declarations shared by the host set-up and the device plan.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "condest.h"

namespace condest {

// Sets the thread's last-error text and returns status.
int fail(int status, const std::string& msg);

struct HostCsr {
  int32_t n = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  int64_t nnz() const { return rowptr.empty() ? 0 : rowptr.back(); }
};

// Validation of a caller CSR (square, monotone, in range, finite, non-zero).
int check_csr(const cond_csr_t* A);
// Copy with duplicates summed and columns sorted within each row.
int canonical_copy(const cond_csr_t* A, HostCsr& out);
// Stable counting-sort transpose.
void transpose(const HostCsr& a, HostCsr& t);
// Nested-dissection order of the pattern of a + a^T.
void nested_dissection(const HostCsr& a, const HostCsr& at, std::vector<int32_t>& perm);

}  // namespace condest

struct cond_lu;
namespace condest {
// P A Q = L U with threshold partial pivoting (col_perm_in: Q, or null for
// nested dissection). Thread-safe: no shared state.
int lu_factor(const HostCsr& a, const HostCsr& at, const int32_t* col_perm_in, double tol,
              cond_lu& lu);
}  // namespace condest

// LU factors, P A Q = L U, held in both orientations for the four solves.
struct cond_lu {
  int32_t n = 0;
  // L: unit lower, strictly-lower part; U: strictly-upper part + diagonal.
  condest::HostCsr l_rows, u_rows;  // CSR in pivot order
  condest::HostCsr l_cols, u_cols;  // CSR of L^T and U^T (= CSC of L and U)
  std::vector<double> u_diag;
  std::vector<int32_t> row_perm;  // row_perm[k] = row of A that is row k of P A
  std::vector<int32_t> col_perm;  // col_perm[k] = column of A that is column k of A Q
};
