// Host set-up of the estimator under AddressSanitizer and UBSan: validation,
// transpose, nested dissection, the sparse LU (P A Q = L U), the panel
// schedules of the four triangular solves (as the device plan builds them),
// schedules of independent blocks joined into one (as the batch builds
// them), and the host replay of the solves, on seeded grid matrices and the
// error cases. Exits non-zero on any failed check; the sanitizers abort on
// any memory or undefined-behaviour error.

#include <cmath>
#include <cstdio>
#include <vector>

#include "condest.h"
#include "internal.hpp"
#include "panels.hpp"

using namespace condest;

namespace {

int failures = 0;
#define EXPECT(cond, what)                                   \
  do {                                                       \
    if (!(cond)) {                                           \
      std::printf("FAILED: %s (line %d)\n", what, __LINE__); \
      ++failures;                                            \
    }                                                        \
  } while (0)

// 64-bit linear congruential generator (Knuth's MMIX constants), uniform in [0, 1).
struct Lcg {
  unsigned long long s;
  double next() {
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    return static_cast<double>(s >> 11) * (1.0 / 9007199254740992.0);
  }
};

// A non-symmetric 5-point grid operator on side x side nodes with scaled
// columns (values spread over 12 decades), so the LU pivots and fills.
HostCsr grid_matrix(int side, unsigned long long seed) {
  Lcg g{seed};
  const int n = side * side;
  std::vector<double> colscale(n);
  for (int j = 0; j < n; ++j) colscale[j] = std::pow(10.0, 12.0 * g.next() - 6.0);
  HostCsr a;
  a.n = n;
  a.rowptr.push_back(0);
  for (int i = 0; i < side; ++i)
    for (int j = 0; j < side; ++j) {
      const int r = i * side + j;
      const int nb[5] = {r - side, r - 1, r, r + 1, r + side};
      const bool ok[5] = {i > 0, j > 0, true, j + 1 < side, i + 1 < side};
      for (int k = 0; k < 5; ++k)
        if (ok[k]) {
          const double v = k == 2 ? 4.5 + g.next() : -1.0 + 0.6 * (g.next() - 0.5);
          a.col.push_back(nb[k]);
          a.val.push_back(v * colscale[nb[k]]);
        }
      a.rowptr.push_back(static_cast<int64_t>(a.col.size()));
    }
  return a;
}

cond_csr_t view(const HostCsr& a) {
  cond_csr_t c;
  c.n = a.n;
  c.nnz = a.nnz();
  c.rowptr = a.rowptr.data();
  c.col = a.col.data();
  c.val = a.val.data();
  return c;
}

// max_i |A r - x|_i / (|A| |r| + |x|)_i (transpose: A^T)
double backward_error(const HostCsr& a, bool transpose, const std::vector<double>& r,
                      const std::vector<double>& x) {
  const int n = a.n;
  std::vector<double> y(n, 0.0), s(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int64_t p = a.rowptr[i]; p < a.rowptr[i + 1]; ++p) {
      const int row = transpose ? a.col[p] : i, c = transpose ? i : a.col[p];
      y[row] += a.val[p] * r[c];
      s[row] += std::fabs(a.val[p] * r[c]);
    }
  double worst = 0.0;
  for (int i = 0; i < n; ++i) worst = std::fmax(worst, std::fabs(y[i] - x[i]) / (s[i] + std::fabs(x[i])));
  return worst;
}

// The device order: the slots are a permutation of the tasks, the lists
// partition them, and each list keeps the dependency order (its slots hold
// increasing task indices), which is what makes every wait of the solve end.
void check_lists(const PanelCsr& t) {
  const int32_t ntasks = static_cast<int32_t>(t.task_panel.size());
  EXPECT(static_cast<int>(t.list_off.size()) == kTaskLists + 1, "list count");
  EXPECT(t.list_off[0] == 0 && t.list_off[kTaskLists] == ntasks, "lists cover the tasks");
  std::vector<int32_t> seen(ntasks, 0);
  std::vector<int32_t> last(kTaskLists, -1);
  for (int32_t k = 0; k < ntasks; ++k) {
    const int32_t q = t.task_slot[k];
    EXPECT(q >= 0 && q < ntasks && !seen[q], "slot permutation");
    if (q < 0 || q >= ntasks) continue;
    seen[q] = 1;
    int l = 0;
    while (l < kTaskLists && q >= t.list_off[l + 1]) ++l;
    EXPECT(l < kTaskLists && q > last[l], "list keeps the dependency order");
    if (l < kTaskLists) last[l] = q;
    EXPECT(t.task_rec[8 * q] == t.task_panel[k] && t.task_rec[8 * q + 1] == t.task_kind[k], "record at slot");
  }
}

struct Schedules {
  PanelCsr t[4];
  std::vector<int32_t> row_perm, col_perm, rev;
};

// The four solves of Algorithm 2 as the device plan (prows = kMaxPanelRows)
// or the batch (prows = kPanel) schedules them.
Schedules schedule(const cond_lu& f, int32_t prows) {
  Schedules s;
  const int32_t n = f.n;
  std::vector<double> udiag_rev(n);
  for (int32_t k = 0; k < n; ++k) udiag_rev[k] = f.u_diag[n - 1 - k];
  s.t[0] = split_panels(f.l_rows, prows);
  invert_panels(s.t[0], nullptr);
  check_lists(s.t[0]);
  s.t[1] = split_panels(reverse_order(f.u_rows), prows);
  invert_panels(s.t[1], udiag_rev.data());
  check_lists(s.t[1]);
  s.t[2] = split_panels(f.u_cols, prows);
  invert_panels(s.t[2], f.u_diag.data());
  check_lists(s.t[2]);
  s.t[3] = split_panels(reverse_order(f.l_cols), prows);
  invert_panels(s.t[3], nullptr);
  check_lists(s.t[3]);
  s.row_perm = f.row_perm;
  s.col_perm = f.col_perm;
  s.rev.resize(n);
  for (int32_t k = 0; k < n; ++k) s.rev[k] = n - 1 - k;
  return s;
}

// r = A^-1 x and s = A^-T r by replaying the schedules.
bool solve(const Schedules& s, const std::vector<double>& x, std::vector<double>& r,
           std::vector<double>& t) {
  const size_t n = x.size();
  std::vector<double> c(n), z(n), h(n), wv(n);
  if (!replay_solve(s.t[0], s.row_perm.data(), x.data(), c.data())) return false;
  if (!replay_solve(s.t[1], s.rev.data(), c.data(), z.data())) return false;
  if (!replay_solve(s.t[2], s.rev.data(), z.data(), h.data())) return false;
  if (!replay_solve(s.t[3], s.rev.data(), h.data(), wv.data())) return false;
  r.assign(n, 0.0);
  t.assign(n, 0.0);
  for (size_t k = 0; k < n; ++k) r[s.col_perm[n - 1 - k]] = z[k];
  for (size_t k = 0; k < n; ++k) t[s.row_perm[n - 1 - k]] = wv[k];
  return true;
}

void check_system(const HostCsr& a, unsigned long long seed, double bound) {
  cond_csr_t c = view(a);
  EXPECT(cond_csr_check(&c) == COND_OK, "csr_check");
  HostCsr at;
  transpose(a, at);
  EXPECT(at.nnz() == a.nnz(), "transpose size");
  cond_lu f;
  EXPECT(lu_factor(a, at, nullptr, 1e-6, f) == COND_OK, "lu_factor");
  for (int32_t prows : {kMaxPanelRows, kPanel}) {
    Schedules s = schedule(f, prows);
    Lcg g{seed};
    std::vector<double> x(a.n), r, t;
    for (double& v : x) v = g.next() - 0.5;
    EXPECT(solve(s, x, r, t), "replay");
    const double be_r = backward_error(a, false, r, x), be_t = backward_error(a, true, t, r);
    std::printf("n=%d prows=%d fill=%lld+%lld backward errors %.2e %.2e\n", a.n, prows,
                static_cast<long long>(f.l_rows.nnz()), static_cast<long long>(f.u_rows.nnz()), be_r, be_t);
    EXPECT(be_r < bound && be_t < bound, "backward error");
  }
}

}  // namespace

int main() {
  // single systems: one row, small and mid-size grids
  HostCsr one;
  one.n = 1;
  one.rowptr = {0, 1};
  one.col = {0};
  one.val = {-3.0};
  check_system(one, 1, 1e-15);
  check_system(grid_matrix(7, 3), 4, 1e-10);
  check_system(grid_matrix(45, 5), 6, 1e-9);

  // three blocks scheduled separately and joined, as the batch does
  const int sides[3] = {9, 23, 14};
  std::vector<Schedules> parts;
  std::vector<HostCsr> blocks;
  int64_t total = 0;
  for (int k = 0; k < 3; ++k) {
    blocks.push_back(grid_matrix(sides[k], 10 + k));
    HostCsr at;
    transpose(blocks[k], at);
    cond_lu f;
    EXPECT(lu_factor(blocks[k], at, nullptr, 1e-6, f) == COND_OK, "block lu");
    parts.push_back(schedule(f, kPanel));
    total += blocks[k].n;
  }
  Schedules joined;
  std::vector<int64_t> row0 = {0};
  for (int k = 0; k < 3; ++k) row0.push_back(row0.back() + blocks[k].n);
  for (int f = 0; f < 4; ++f) {
    const bool reversed = f == 1 || f == 3;
    std::vector<const PanelCsr*> ps;
    std::vector<int64_t> offs;
    std::vector<int32_t> groups;
    for (int k = 0; k < 3; ++k) {
      const int m = reversed ? 2 - k : k;
      ps.push_back(&parts[m].t[f]);
      offs.push_back(reversed ? total - row0[m + 1] : row0[m]);
      groups.push_back(m);
    }
    joined.t[f] = merge_panels(ps, offs, groups);
    const PanelCsr& J = joined.t[f];
    check_lists(J);
    // every task carries its block's id
    for (size_t q = 0; q < J.task_panel.size(); ++q) {
      const int32_t row = J.pstart[J.task_panel[q]];
      const int32_t g = J.task_group[q];
      const int64_t lo = reversed ? total - row0[g + 1] : row0[g];
      const int64_t hi = reversed ? total - row0[g] : row0[g + 1];
      EXPECT(row >= lo && row < hi, "task group");
      EXPECT(J.slot_group[J.task_slot[q]] == g, "slot group");
    }
    // a list cut down to some blocks' slots still runs: each list is in
    // level order, and a block's rows read only columns of the same block
    std::vector<int32_t> slot_task(J.task_panel.size());
    for (size_t q = 0; q < J.task_panel.size(); ++q) slot_task[J.task_slot[q]] = static_cast<int32_t>(q);
    for (int l = 0; l < kTaskLists; ++l)
      for (int32_t q = J.list_off[l] + 1; q < J.list_off[l + 1]; ++q)
        EXPECT(J.task_level[slot_task[q - 1]] <= J.task_level[slot_task[q]], "list level order");
    for (size_t q = 0; q < J.task_panel.size(); ++q) {
      const int32_t g = J.task_group[q];
      const int64_t lo = reversed ? total - row0[g + 1] : row0[g];
      const int32_t p = J.task_panel[q];
      for (int32_t i = J.pstart[p]; i < J.pstart[p + 1]; ++i)
        for (int64_t e = J.off_rp[i]; e < J.off_rp[i + 1]; ++e)
          EXPECT(J.off_col[e] >= lo && J.off_col[e] < J.pstart[p], "block-local columns");
    }
  }
  joined.row_perm.resize(total);
  joined.col_perm.resize(total);
  joined.rev.resize(total);
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < blocks[k].n; ++i) {
      joined.row_perm[row0[k] + i] = static_cast<int32_t>(row0[k]) + parts[k].row_perm[i];
      joined.col_perm[row0[k] + i] = static_cast<int32_t>(row0[k]) + parts[k].col_perm[i];
    }
  for (int64_t k = 0; k < total; ++k) joined.rev[k] = static_cast<int32_t>(total - 1 - k);
  Lcg g{77};
  std::vector<double> x(total), r, t;
  for (double& v : x) v = g.next() - 0.5;
  EXPECT(solve(joined, x, r, t), "joined replay");
  for (int k = 0; k < 3; ++k) {
    std::vector<double> xk(x.begin() + row0[k], x.begin() + row0[k + 1]);
    std::vector<double> rk(r.begin() + row0[k], r.begin() + row0[k + 1]);
    std::vector<double> tk(t.begin() + row0[k], t.begin() + row0[k + 1]);
    const double be_r = backward_error(blocks[k], false, rk, xk), be_t = backward_error(blocks[k], true, tk, rk);
    EXPECT(be_r < 1e-10 && be_t < 1e-10, "joined block backward error");
  }

  // error cases: a zero column (singular), a malformed matrix, a bad order
  HostCsr sing = grid_matrix(6, 9);
  for (int64_t p = 0; p < sing.nnz(); ++p)
    if (sing.col[p] == 5) sing.val[p] = 0.0;
  HostCsr sat;
  transpose(sing, sat);
  cond_lu fs;
  EXPECT(lu_factor(sing, sat, nullptr, 1e-6, fs) == COND_ESINGULAR, "singular");
  HostCsr bad = grid_matrix(4, 2);
  bad.col[3] = 99;
  cond_csr_t cb = view(bad);
  EXPECT(cond_csr_check(&cb) == COND_EINVAL, "column out of range");
  std::vector<int32_t> perm(16, 0);
  HostCsr ok = grid_matrix(4, 2), okt;
  transpose(ok, okt);
  cond_lu fp;
  EXPECT(lu_factor(ok, okt, perm.data(), 1e-6, fp) == COND_EINVAL, "not a permutation");
  std::vector<int32_t> nd(ok.n);
  cond_csr_t co = view(ok);
  EXPECT(cond_order_nd(&co, nd.data()) == COND_OK, "nested dissection");

  std::printf(failures ? "host checks FAILED\n" : "host checks ok\n");
  return failures ? 1 : 0;
}
