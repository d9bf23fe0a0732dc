// Batch plan: block-diagonal concatenation of many matrices, K = 8 starts
// each, tile schedule chosen by a small autotuner, iterations captured in
// HIP graphs and replayed until every (matrix, start) pair has stopped.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <future>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "condest.h"
#include "internal.hpp"
#include "panels.hpp"
#include "panels_upload.hpp"

using namespace condest;

#define BCHK(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(COND_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

namespace {

constexpr size_t kAl = kAlign;
const int kTileCandidates[] = {32, 64, 128, 256};
const int kGridCandidates[] = {1024, 2048, 4096};

size_t take(size_t& off, size_t bytes) {
  size_t o = (off + kAl - 1) / kAl * kAl;
  off = o + bytes;
  return o;
}

struct BatchKey {
  const void* trace = nullptr;
  const void* xbest = nullptr;
  AdamParams p{};
  int chunk = 0;
  bool operator==(const BatchKey& o) const {
    return trace == o.trace && xbest == o.xbest && chunk == o.chunk &&
           std::memcmp(&p, &o.p, sizeof(p)) == 0;
  }
};

}  // namespace

struct cond_batch {
  int32_t nmat = 0;
  std::vector<int64_t> row0;  // nmat + 1
  std::vector<int32_t> a_rp, a_col, at_rp, at_col;
  std::vector<double> a_val, at_val;
  int64_t nrows = 0, nnz = 0;
  // schedule
  int tile_rows = 0, grid = 0;
  std::vector<int64_t> tiles;
  std::vector<int32_t> tile_mat, mat_tile0;
  int64_t max_tiles = 0;
  double setup_ms = 0.0;
  // device
  bool bound = false;
  hipStream_t user_stream = nullptr, stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, eva = nullptr, evb = nullptr;
  char* ws = nullptr;
  size_t need = 0;
  bool own = false;
  BatchArgs args;
  BatchPair* h_pairs = nullptr;  // pinned, two slots of nmat*K
  hipGraphExec_t exec = nullptr;
  BatchKey key;
  // sigma_min route: every matrix's LU (P_m A_m Q_m = L_m U_m, factored in
  // parallel threads), merged into block-diagonal factors whose pivot rows
  // keep each matrix's rows together, and the four solve schedules of them
  bool want_min = false;
  PanelCsr pL, pU, pUt, pLt;
  std::vector<int32_t> row_perm, rev, scat_s, scat_r;  // scat_r: host replay only
  DevTri dL, dU, dUt, dLt;
  BatchLists lists;  // the four solves' lists, compacted to the running matrices
  int64_t nnz_l = 0, nnz_u = 0;
  double lu_ms = 0.0;
  bool rearm_slots = false;  // a solve wait timed out: re-arm the slice slots first
  hipGraphExec_t exec_min = nullptr;
  BatchKey key_min;
  struct {
    size_t a_rp, a_col, a_val, at_rp, at_col, at_val, tiles, tile_mat, mat_tile0, live_mat,
        live_pref, mat_live;
    size_t vec[7], parts[4], pairs, g;
    size_t tri[4][kTriSlots];
    size_t row_perm, rev, scat_s, svec[4], tickets, cl_slots[4], cl_cnt;
  } o{};
};

namespace {

void make_schedule(cond_batch* b, int tile_rows) {
  b->tiles.assign(1, 0);
  b->tile_mat.clear();
  b->mat_tile0.assign(1, 0);
  for (int32_t m = 0; m < b->nmat; ++m) {
    for (int64_t r = b->row0[m]; r < b->row0[m + 1]; r += tile_rows) {
      b->tiles.push_back(std::min<int64_t>(r + tile_rows, b->row0[m + 1]));
      b->tile_mat.push_back(m);
    }
    b->mat_tile0.push_back(static_cast<int32_t>(b->tile_mat.size()));
  }
  b->tile_rows = tile_rows;
}

int upload_schedule(cond_batch* b) {
  BCHK(hipMemcpyAsync(b->ws + b->o.tiles, b->tiles.data(), b->tiles.size() * 8,
                      hipMemcpyHostToDevice, b->stream));
  BCHK(hipMemcpyAsync(b->ws + b->o.tile_mat, b->tile_mat.data(), b->tile_mat.size() * 4,
                      hipMemcpyHostToDevice, b->stream));
  BCHK(hipMemcpyAsync(b->ws + b->o.mat_tile0, b->mat_tile0.data(), b->mat_tile0.size() * 4,
                      hipMemcpyHostToDevice, b->stream));
  BCHK(hipStreamSynchronize(b->stream));
  b->args.ntiles = static_cast<int>(b->tile_mat.size());
  return COND_OK;
}

AdamParams bparams(const cond_opts_t& o) {
  AdamParams p{};
  p.alpha = o.alpha;
  p.beta1 = o.beta1;
  p.beta2 = o.beta2;
  p.eps = o.eps;
  p.stop_rtol = o.stop_rtol;
  p.stop_window = o.stop_window;
  p.max_iter = o.max_iter;
  p.alpha_min = o.alpha_min;
  p.alpha_decay = o.alpha_decay;
  return p;
}

// One update of the sigma_min run (Algorithm 2) for every pair: the solves
// take all K starts of every matrix at once over the block-diagonal factors.
void enqueue_batch_min_iteration(cond_batch* b, const BatchArgs& a, const AdamParams& p) {
  hipStream_t s = b->stream;
  const int K = kBatchK;
  int* stop = &a.g->stop_all;
  int* abort = &a.g->abort_wait;
  batch_launch_live(a, s);
  // once a matrix has stopped, the solves walk only the running matrices'
  // tasks: the lists are cut down whenever the set of running matrices
  // changes
  batch_launch_compact(a, b->lists, s);
  batch_launch_normalise(a, b->grid, s);
  batch_launch_rearm(a, b->grid, s);
  // r = A^-1 x: L c = P x, U z = c (z reversed); s = A^-T r: U^T h = z,
  // L^T wv = h, w = P^T wv
  const int* cut = &a.g->compact;  // set while the solves take the cut lists
  launch_trsv_multi(K, b->dL, a.x, reinterpret_cast<const int*>(b->ws + b->o.row_perm), a.c,
                    nullptr, nullptr, a.tickets, stop, abort, cut, s);
  const int* rev = reinterpret_cast<const int*>(b->ws + b->o.rev);
  launch_trsv_multi(K, b->dU, a.c, rev, a.z, nullptr, nullptr, tix(a.tickets, 1), stop, abort, cut,
                    s);
  batch_launch_sumsq_rev(a, b->grid, s);
  batch_launch_reduce(a, 1, p, s);
  launch_trsv_multi(K, b->dUt, a.z, rev, a.h, nullptr, nullptr, tix(a.tickets, 2), stop, abort, cut,
                    s);
  launch_trsv_multi(K, b->dLt, a.h, rev, a.wv, a.w, reinterpret_cast<const int*>(b->ws + b->o.scat_s),
                    tix(a.tickets, 3), stop, abort, cut, s);
  batch_launch_pass1(a, p, b->grid, s);
  batch_launch_reduce(a, 2, p, s);
  batch_launch_pass2(a, p, b->grid, s);
  batch_launch_reduce(a, 0, p, s);
}

void enqueue_batch_iteration(cond_batch* b, const BatchArgs& a, const AdamParams& p) {
  hipStream_t s = b->stream;
  batch_launch_live(a, s);  // drop the tiles of matrices whose starts have all stopped
  batch_launch_normalise(a, b->grid, s);
  batch_launch_spmm(a, 0, b->grid, s);
  batch_launch_reduce(a, 1, p, s);
  batch_launch_spmm(a, 1, b->grid, s);
  batch_launch_pass1(a, p, b->grid, s);
  batch_launch_reduce(a, 2, p, s);
  batch_launch_pass2(a, p, b->grid, s);
  batch_launch_reduce(a, 0, p, s);
}

}  // namespace

namespace {

// Every matrix's LU and its four solve schedules in parallel threads (one
// matrix per thread at a time, as the single-matrix plan builds them), then
// the schedules joined block-diagonally: matrix m's pivot rows at
// [row0[m], row0[m+1]) for the solves in pivot order (L, U^T), its reversed
// rows at [N - row0[m+1], N - row0[m]) for the reversed ones (U, L^T).
int batch_factor(cond_batch* b, std::vector<HostCsr>& as, std::vector<HostCsr>& ats, double tol) {
  const int32_t count = b->nmat;
  const int64_t n = b->row0.back();
  auto t0 = std::chrono::steady_clock::now();
  struct Part {
    PanelCsr t[4];  // L, U reversed, U^T, L^T reversed
    std::vector<int32_t> row_perm, col_perm;
    int64_t nnz_l = 0, nnz_u = 0;
  };
  std::vector<Part> parts(count);
  std::vector<int> status(count, COND_OK);
  std::vector<std::string> why(count);
  std::atomic<int32_t> next(0);
  unsigned hw = std::thread::hardware_concurrency();
  const int32_t nthreads = std::max<int32_t>(1, std::min<int32_t>(count, hw ? static_cast<int32_t>(hw) : 4));
  auto sched = [](const HostCsr& t, const double* diag) {
    PanelCsr p = split_panels(t, kPanel);  // the several-sides solves take 64-row panels
    invert_panels(p, diag);
    return p;
  };
  // CONDEST_PROGRESS=1: a line on stderr as each matrix is factored
  const char* env = std::getenv("CONDEST_PROGRESS");
  const bool progress = env && env[0] == '1';
  std::atomic<int32_t> done(0);
  auto worker = [&]() {
    for (int32_t m; (m = next.fetch_add(1)) < count;) {
      try {
        cond_lu f;
        status[m] = lu_factor(as[m], ats[m], nullptr, tol, f);
        as[m] = HostCsr();
        ats[m] = HostCsr();
        if (status[m]) {
          why[m] = cond_last_error();
          continue;
        }
        Part& q = parts[m];
        const int32_t nm = f.n;
        std::vector<double> udiag_rev(nm);
        for (int32_t k = 0; k < nm; ++k) udiag_rev[k] = f.u_diag[nm - 1 - k];
        q.t[0] = sched(f.l_rows, nullptr);
        q.t[1] = sched(reverse_order(f.u_rows), udiag_rev.data());
        q.t[2] = sched(f.u_cols, f.u_diag.data());
        q.t[3] = sched(reverse_order(f.l_cols), nullptr);
        q.row_perm = std::move(f.row_perm);
        q.col_perm = std::move(f.col_perm);
        q.nnz_l = f.l_rows.nnz();
        q.nnz_u = f.u_rows.nnz() + nm;
        for (const PanelCsr& t : q.t)
          for (double w : t.winv)
            if (!std::isfinite(w)) {
              status[m] = COND_ENUMERIC;
              why[m] = "a diagonal block of the LU factors has no finite float64 inverse";
            }
      } catch (const std::bad_alloc&) {
        status[m] = COND_ENOMEM;
        why[m] = "host memory exhausted";
      }
      const int32_t d = done.fetch_add(1) + 1;
      if (progress) std::fprintf(stderr, "[condest] batch set-up: %d of %d matrices factored\n", d, count);
    }
  };
  std::vector<std::thread> pool;
  for (int32_t k = 0; k < nthreads; ++k) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  for (int32_t m = 0; m < count; ++m)
    if (status[m]) return fail(status[m], "matrix " + std::to_string(m) + ": " + why[m]);
  b->lu_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  b->row_perm.resize(n);
  std::vector<int32_t> col_perm(n);
  for (int32_t m = 0; m < count; ++m) {
    const int32_t off = static_cast<int32_t>(b->row0[m]);
    const Part& q = parts[m];
    for (size_t k = 0; k < q.row_perm.size(); ++k) {
      b->row_perm[off + k] = off + q.row_perm[k];
      col_perm[off + k] = off + q.col_perm[k];
    }
    b->nnz_l += q.nnz_l;
    b->nnz_u += q.nnz_u;
  }
  PanelCsr* out[4] = {&b->pL, &b->pU, &b->pUt, &b->pLt};
  for (int f = 0; f < 4; ++f) {
    const bool reversed = f == 1 || f == 3;
    std::vector<const PanelCsr*> ps;
    std::vector<int64_t> offs;
    std::vector<int32_t> groups;
    for (int32_t k = 0; k < count; ++k) {
      const int32_t m = reversed ? count - 1 - k : k;
      ps.push_back(&parts[m].t[f]);
      offs.push_back(reversed ? n - b->row0[m + 1] : b->row0[m]);
      groups.push_back(m);
    }
    *out[f] = merge_panels(ps, offs, groups);
    for (int32_t m = 0; m < count; ++m) parts[m].t[f] = PanelCsr();
  }
  b->rev.resize(n);
  b->scat_s.resize(n);
  b->scat_r.resize(n);
  for (int64_t k = 0; k < n; ++k) {
    b->rev[k] = static_cast<int32_t>(n - 1 - k);
    b->scat_s[k] = b->row_perm[n - 1 - k];
    b->scat_r[k] = col_perm[n - 1 - k];
  }
  return COND_OK;
}

}  // namespace

extern "C" {

int cond_batch_create(const cond_csr_t* As, int32_t count, const cond_opts_t* o,
                      cond_batch_t** out) {
  if (!out || !As || count <= 0 || !o) return fail(COND_EINVAL, "invalid batch arguments");
  *out = nullptr;
  auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<cond_batch> b(new (std::nothrow) cond_batch());
  if (!b) return fail(COND_ENOMEM, "allocation failed");
  if (o->sigma_min_method != COND_MIN_LU && o->sigma_min_method != COND_MIN_NONE)
    return fail(COND_EINVAL, "a batch runs sigma_min by COND_MIN_LU or not at all");
  b->want_min = o->sigma_min_method == COND_MIN_LU;
  std::vector<HostCsr> keep_a, keep_at;  // for the LUs
  try {
    b->nmat = count;
    b->row0.assign(1, 0);
    b->a_rp.assign(1, 0);
    b->at_rp.assign(1, 0);
    if (b->want_min) {
      keep_a.resize(count);
      keep_at.resize(count);
    }
    for (int32_t m = 0; m < count; ++m) {
      HostCsr a, at;
      int st = canonical_copy(&As[m], a);
      if (st) return st;
      transpose(a, at);
      const int64_t off = b->row0.back();
      if (off + a.n > (1LL << 28) || b->nnz + a.nnz() >= (1LL << 31) - 1)
        return fail(COND_EINVAL, "batch too large for 32-bit indices");
      for (int32_t i = 0; i < a.n; ++i) {
        for (int64_t p = a.rowptr[i]; p < a.rowptr[i + 1]; ++p) {
          b->a_col.push_back(static_cast<int32_t>(a.col[p] + off));
          b->a_val.push_back(a.val[p]);
        }
        b->a_rp.push_back(static_cast<int32_t>(b->a_col.size()));
        for (int64_t p = at.rowptr[i]; p < at.rowptr[i + 1]; ++p) {
          b->at_col.push_back(static_cast<int32_t>(at.col[p] + off));
          b->at_val.push_back(at.val[p]);
        }
        b->at_rp.push_back(static_cast<int32_t>(b->at_col.size()));
      }
      b->row0.push_back(off + a.n);
      b->nnz += a.nnz();
      if (b->want_min) {
        keep_a[m] = std::move(a);
        keep_at[m] = std::move(at);
      }
    }
    if (b->want_min) {
      int st = batch_factor(b.get(), keep_a, keep_at, o->pivot_tol);
      if (st) return st;
    }
  } catch (const std::bad_alloc&) {
    return fail(COND_ENOMEM, "host memory exhausted in batch set-up");
  }
  b->nrows = b->row0.back();
  // the largest schedule (smallest tiles) sizes the workspace
  make_schedule(b.get(), kTileCandidates[0]);
  b->max_tiles = static_cast<int64_t>(b->tile_mat.size());
  size_t off = 0;
  const size_t n = b->nrows, K = kBatchK;
  b->o.a_rp = take(off, (n + 1) * 4);
  b->o.a_col = take(off, b->nnz * 4);
  b->o.a_val = take(off, b->nnz * 8);
  b->o.at_rp = take(off, (n + 1) * 4);
  b->o.at_col = take(off, b->nnz * 4);
  b->o.at_val = take(off, b->nnz * 8);
  b->o.tiles = take(off, (b->max_tiles + 1) * 8);
  b->o.tile_mat = take(off, b->max_tiles * 4);
  b->o.mat_tile0 = take(off, (count + 1) * 4);
  b->o.live_mat = take(off, static_cast<size_t>(count) * 4);
  b->o.live_pref = take(off, (count + 1) * 4);
  b->o.mat_live = take(off, static_cast<size_t>(count) * 4);
  for (int k = 0; k < 7; ++k) b->o.vec[k] = take(off, n * K * 8);
  for (int k = 0; k < 4; ++k) b->o.parts[k] = take(off, b->max_tiles * K * 8);
  b->o.pairs = take(off, static_cast<size_t>(count) * K * sizeof(BatchPair));
  b->o.g = take(off, sizeof(BatchGlobal));
  if (b->want_min) {
    Layout L;
    L.off = off;
    const PanelCsr* tris[4] = {&b->pL, &b->pU, &b->pUt, &b->pLt};
    for (int f = 0; f < 4; ++f) tri_layout(*tris[f], kBatchK, L, b->o.tri[f]);
    b->o.row_perm = L.take(n * 4);
    b->o.rev = L.take(n * 4);
    b->o.scat_s = L.take(n * 4);
    for (int k = 0; k < 4; ++k) b->o.svec[k] = L.take(n * K * 8);
    b->o.tickets = L.take(4 * kSolveTickets * sizeof(unsigned));  // four solves' counters
    for (int f = 0; f < 4; ++f) b->o.cl_slots[f] = L.take(tris[f]->task_slot.size() * 4);
    b->o.cl_cnt = L.take(4 * kTaskLists * 4);
    off = L.off;
  }
  b->need = off;
  b->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = b.release();
  return COND_OK;
}

int cond_batch_info(const cond_batch_t* b, int64_t* row0, size_t* workspace_bytes,
                    int32_t* tile_rows, int32_t* grid) {
  if (!b) return fail(COND_EINVAL, "null batch");
  if (row0) std::copy(b->row0.begin(), b->row0.end(), row0);
  if (workspace_bytes) *workspace_bytes = b->need;
  if (tile_rows) *tile_rows = b->tile_rows;
  if (grid) *grid = b->grid;
  return COND_OK;
}

int cond_batch_bind(cond_batch_t* b, void* workspace, size_t bytes, void* stream,
                    int32_t tile_rows, int32_t grid) {
  if (!b) return fail(COND_EINVAL, "null batch");
  if (b->bound) return fail(COND_ESTATE, "batch already bound");
  if (workspace && bytes < b->need) return fail(COND_ENOMEM, "workspace too small");
  if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAl))
    return fail(COND_EINVAL, "workspace must be 256-byte aligned");
  if (tile_rows < 0 || grid < 0) return fail(COND_EINVAL, "invalid schedule");
  b->user_stream = static_cast<hipStream_t>(stream);
  BCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
  BCHK(hipEventCreate(&b->ev0));
  BCHK(hipEventCreate(&b->ev1));
  BCHK(hipEventCreateWithFlags(&b->eva, hipEventDisableTiming));
  BCHK(hipEventCreateWithFlags(&b->evb, hipEventDisableTiming));
  BCHK(hipHostMalloc(reinterpret_cast<void**>(&b->h_pairs),
                     2 * static_cast<size_t>(b->nmat) * kBatchK * sizeof(BatchPair),
                     hipHostMallocDefault));
  if (workspace) {
    b->ws = static_cast<char*>(workspace);
    b->own = false;
  } else {
    BCHK(hipMalloc(reinterpret_cast<void**>(&b->ws), b->need));
    b->own = true;
  }
  if (b->user_stream) {
    hipEvent_t e;
    BCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    BCHK(hipEventRecord(e, b->user_stream));
    BCHK(hipStreamWaitEvent(b->stream, e, 0));
    BCHK(hipEventDestroy(e));
  }
  auto up = [&](size_t o, const void* src, size_t nb) -> int {
    if (!nb) return COND_OK;
    BCHK(hipMemcpyAsync(b->ws + o, src, nb, hipMemcpyHostToDevice, b->stream));
    return COND_OK;
  };
  int st;
  if ((st = up(b->o.a_rp, b->a_rp.data(), b->a_rp.size() * 4))) return st;
  if ((st = up(b->o.a_col, b->a_col.data(), b->a_col.size() * 4))) return st;
  if ((st = up(b->o.a_val, b->a_val.data(), b->a_val.size() * 8))) return st;
  if ((st = up(b->o.at_rp, b->at_rp.data(), b->at_rp.size() * 4))) return st;
  if ((st = up(b->o.at_col, b->at_col.data(), b->at_col.size() * 4))) return st;
  if ((st = up(b->o.at_val, b->at_val.data(), b->at_val.size() * 8))) return st;
  BatchArgs& a = b->args;
  a.nmat = b->nmat;
  a.tiles = reinterpret_cast<const long long*>(b->ws + b->o.tiles);
  a.tile_mat = reinterpret_cast<const int*>(b->ws + b->o.tile_mat);
  a.mat_tile0 = reinterpret_cast<const int*>(b->ws + b->o.mat_tile0);
  a.live_mat = reinterpret_cast<int*>(b->ws + b->o.live_mat);
  a.live_pref = reinterpret_cast<int*>(b->ws + b->o.live_pref);
  a.mat_live = reinterpret_cast<int*>(b->ws + b->o.mat_live);
  a.a_rowptr = reinterpret_cast<const int*>(b->ws + b->o.a_rp);
  a.a_col = reinterpret_cast<const int*>(b->ws + b->o.a_col);
  a.a_val = reinterpret_cast<const double*>(b->ws + b->o.a_val);
  a.at_rowptr = reinterpret_cast<const int*>(b->ws + b->o.at_rp);
  a.at_col = reinterpret_cast<const int*>(b->ws + b->o.at_col);
  a.at_val = reinterpret_cast<const double*>(b->ws + b->o.at_val);
  double** vecs[7] = {&a.x, &a.m, &a.v, &a.d, &a.y, &a.w, &a.xbest};
  for (int k = 0; k < 7; ++k) *vecs[k] = reinterpret_cast<double*>(b->ws + b->o.vec[k]);
  a.parts_x = reinterpret_cast<double*>(b->ws + b->o.parts[0]);
  a.parts_y = reinterpret_cast<double*>(b->ws + b->o.parts[1]);
  a.parts_xd = reinterpret_cast<double*>(b->ws + b->o.parts[2]);
  a.parts_xx = reinterpret_cast<double*>(b->ws + b->o.parts[3]);
  a.pairs = reinterpret_cast<BatchPair*>(b->ws + b->o.pairs);
  a.g = reinterpret_cast<BatchGlobal*>(b->ws + b->o.g);
  a.nrows = b->nrows;
  if (b->want_min) {
    const PanelCsr* tris[4] = {&b->pL, &b->pU, &b->pUt, &b->pLt};
    DevTri* devs[4] = {&b->dL, &b->dU, &b->dUt, &b->dLt};
    for (int f = 0; f < 4; ++f)
      if ((st = tri_upload(b->ws, b->o.tri[f], *tris[f], kBatchK, b->stream, *devs[f]))) return st;
    if ((st = up(b->o.row_perm, b->row_perm.data(), b->row_perm.size() * 4))) return st;
    if ((st = up(b->o.rev, b->rev.data(), b->rev.size() * 4))) return st;
    if ((st = up(b->o.scat_s, b->scat_s.data(), b->scat_s.size() * 4))) return st;
    double** sv[4] = {&a.c, &a.z, &a.h, &a.wv};
    for (int k = 0; k < 4; ++k) *sv[k] = reinterpret_cast<double*>(b->ws + b->o.svec[k]);
    a.tickets = reinterpret_cast<unsigned*>(b->ws + b->o.tickets);
    BCHK(hipMemsetAsync(a.tickets, 0, 4 * kSolveTickets * sizeof(unsigned), b->stream));
    BatchLists& l = b->lists;
    l.cl_cnt = reinterpret_cast<int*>(b->ws + b->o.cl_cnt);
    for (int f = 0; f < 4; ++f) {
      l.slot_group[f] = devs[f]->slot_group;
      std::copy(tris[f]->list_off.begin(), tris[f]->list_off.end(), l.list_off[f]);
      l.cl_slots[f] = reinterpret_cast<int*>(b->ws + b->o.cl_slots[f]);
      devs[f]->cl_slots = l.cl_slots[f];
      devs[f]->cl_cnt = l.cl_cnt + f * kTaskLists;
    }
  }
  BCHK(hipMemsetAsync(b->ws + b->o.vec[0], 0, b->nrows * kBatchK * 8, b->stream));
  // every pair running: the autotuner's products cover every tile
  BCHK(hipMemsetAsync(b->ws + b->o.pairs, 0, static_cast<size_t>(b->nmat) * kBatchK * sizeof(BatchPair),
                      b->stream));
  BCHK(hipStreamSynchronize(b->stream));
  // Autotuner: time the A-product for each (tile rows, grid) candidate on
  // this batch and keep the fastest, unless the caller fixed the schedule.
  int best_r = tile_rows, best_g = grid;
  if (!tile_rows || !grid) {
    float best_ms = 1e30f;
    for (int r : kTileCandidates) {
      if (tile_rows && r != tile_rows) continue;
      make_schedule(b, r);
      if ((st = upload_schedule(b))) return st;
      batch_launch_live(a, b->stream);
      for (int g : kGridCandidates) {
        if (grid && g != grid) continue;
        b->grid = g;
        batch_launch_spmm(a, 0, g, b->stream);  // warm-up
        BCHK(hipEventRecord(b->ev0, b->stream));
        for (int rep = 0; rep < 3; ++rep) batch_launch_spmm(a, 0, g, b->stream);
        BCHK(hipEventRecord(b->ev1, b->stream));
        BCHK(hipEventSynchronize(b->ev1));
        float ms = 0.f;
        BCHK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
        if (ms < best_ms) best_ms = ms, best_r = r, best_g = g;
      }
    }
  }
  make_schedule(b, best_r);
  if ((st = upload_schedule(b))) return st;
  b->grid = best_g;
  b->bound = true;
  return COND_OK;
}

void cond_batch_destroy(cond_batch_t* b) {
  if (!b) return;
  if (b->stream) hipStreamSynchronize(b->stream);
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->exec_min) hipGraphExecDestroy(b->exec_min);
  if (b->own && b->ws) hipFree(b->ws);
  if (b->h_pairs) hipHostFree(b->h_pairs);
  for (hipEvent_t e : {b->ev0, b->ev1, b->eva, b->evb})
    if (e) hipEventDestroy(e);
  if (b->stream) hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"

namespace {

// The run of one route for every pair: route 0 sigma_max (M = A), route 1
// the sigma_min run of Algorithm 2 (M = A^-1). sigma[m] is the route's
// result for matrix m from its best start: sigma_max, or sigma_min = 1 / the
// largest ||A^-1 x|| / ||x||.
int batch_run(cond_batch_t* b, int route, const cond_opts_t* o, const double* x0, double* sigma_out,
              double* pair_best, int64_t* pair_iters, int32_t* pair_status, double* trace,
              double* x_best, double* ms_out) {
  if (!b || !o || !x0) return fail(COND_EINVAL, "null argument");
  if (!b->bound) return fail(COND_ESTATE, "batch not bound");
  if (route == 1 && !b->want_min)
    return fail(COND_ESTATE, "the batch was created without the sigma_min route (COND_MIN_LU)");
  if (!(o->alpha > 0) || o->max_iter < 1 || o->stop_window < 0 || o->chunk < 0)
    return fail(COND_EINVAL, "invalid Projected Adam options");
  if (!(o->alpha_min >= 0) || o->alpha_min > o->alpha ||
      (o->alpha_min > 0 && !(o->alpha_decay > 0 && o->alpha_decay < 1)))
    return fail(COND_EINVAL, "invalid step-size floor or decay");
  const AdamParams p = bparams(*o);
  const int npairs = b->nmat * kBatchK;
  BatchArgs a = b->args;
  a.trace = trace;
  a.xbest = x_best ? x_best : b->args.xbest;
  if (b->user_stream) {
    hipEvent_t e;
    BCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    BCHK(hipEventRecord(e, b->user_stream));
    BCHK(hipStreamWaitEvent(b->stream, e, 0));
    BCHK(hipEventDestroy(e));
  }
  const int chunk = o->chunk > 0 ? o->chunk : 16;
  BatchKey k;
  k.trace = trace;
  k.xbest = a.xbest;
  k.p = p;
  k.chunk = chunk;
  hipGraphExec_t& exec = route == 1 ? b->exec_min : b->exec;
  BatchKey& key = route == 1 ? b->key_min : b->key;
  if (!exec || !(key == k)) {
    if (exec) {
      BCHK(hipGraphExecDestroy(exec));
      exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    BCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    for (int it = 0; it < chunk; ++it) {
      if (route == 1)
        enqueue_batch_min_iteration(b, a, p);
      else
        enqueue_batch_iteration(b, a, p);
    }
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (e != hipSuccess) return fail(COND_EHIP, std::string("capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(COND_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
    key = k;
  }
  if (route == 1 && b->rearm_slots) {
    const PanelCsr* tris[4] = {&b->pL, &b->pU, &b->pUt, &b->pLt};
    const DevTri* devs[4] = {&b->dL, &b->dU, &b->dUt, &b->dLt};
    for (int f = 0; f < 4; ++f)
      if (tris[f]->nslots > 0)
        launch_fill(static_cast<long long>(tris[f]->nslots) * tris[f]->prows * kBatchK, devs[f]->partials, kPending, b->stream);
    b->rearm_slots = false;
  }
  // initial per-pair state
  for (int q = 0; q < npairs; ++q) {
    BatchPair& s = b->h_pairs[q];
    std::memset(&s, 0, sizeof(s));
    s.best = -1.0;
    s.ckpt = -1.0;
    s.alpha = o->alpha;
  }
  BCHK(hipEventRecord(b->ev0, b->stream));
  BCHK(hipMemcpyAsync(a.pairs, b->h_pairs, npairs * sizeof(BatchPair), hipMemcpyHostToDevice,
                      b->stream));
  batch_launch_init(a, x0, b->grid, b->stream);
  batch_launch_reduce(a, 0, p, b->stream);
  BCHK(hipGetLastError());
  const long long total = o->max_iter + 1;
  long long launched = 0;
  BatchPair* slot[2] = {b->h_pairs, b->h_pairs + npairs};
  hipEvent_t ev[2] = {b->eva, b->evb};
  int cur = 0;
  auto launch_chunk = [&](int s) -> int {
    BCHK(hipGraphLaunch(exec, b->stream));
    launched += chunk;
    BCHK(hipMemcpyAsync(slot[s], a.pairs, npairs * sizeof(BatchPair), hipMemcpyDeviceToHost,
                        b->stream));
    BCHK(hipEventRecord(ev[s], b->stream));
    return COND_OK;
  };
  int st;
  const char* env = std::getenv("CONDEST_PROGRESS");
  const bool progress = env && env[0] == '1';
  auto t_last = std::chrono::steady_clock::now();
  if ((st = launch_chunk(0))) return st;
  for (;;) {
    const bool more = launched < total;
    if (more && (st = launch_chunk(cur ^ 1))) return st;
    BCHK(hipEventSynchronize(ev[cur]));
    bool all = true;
    int running = 0;
    for (int q = 0; q < npairs; ++q) running += slot[cur][q].stopped == 0;
    all = running == 0;
    if (all || !more) break;
    if (progress && std::chrono::steady_clock::now() - t_last > std::chrono::seconds(30)) {
      t_last = std::chrono::steady_clock::now();
      std::fprintf(stderr, "[condest] batch %s run: %lld updates, %d of %d pairs running\n",
                   route == 1 ? "sigma_min" : "sigma_max", launched - chunk, running, npairs);
    }
    cur ^= 1;
  }
  BCHK(hipEventRecord(b->ev1, b->stream));
  BCHK(hipMemcpyAsync(b->h_pairs, a.pairs, npairs * sizeof(BatchPair), hipMemcpyDeviceToHost,
                      b->stream));
  BCHK(hipStreamSynchronize(b->stream));
  float ms = 0.f;
  BCHK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  if (ms_out) *ms_out = ms;
  int status = COND_OK;
  for (int m = 0; m < b->nmat; ++m) {
    double best = -1.0;
    for (int kk = 0; kk < kBatchK; ++kk) {
      const BatchPair& s = b->h_pairs[m * kBatchK + kk];
      if (!s.stopped) return fail(COND_EHIP, "batch run ended before every pair stopped");
      if (pair_best) pair_best[m * kBatchK + kk] = s.best;
      if (pair_iters) pair_iters[m * kBatchK + kk] = s.iters;
      if (pair_status) pair_status[m * kBatchK + kk] = s.status;
      if (s.status && !status) status = s.status;
      if (s.status == COND_ETIMEOUT) b->rearm_slots = true;
      if (s.status == COND_OK) best = std::max(best, s.best);
    }
    // every start is a lower bound of ||M||_2: keep the largest
    if (sigma_out) sigma_out[m] = route == 1 ? 1.0 / best : best;
  }
  if (status) return fail(status, "a (matrix, start) pair failed");
  return COND_OK;
}

}  // namespace

extern "C" {

int cond_batch_run(cond_batch_t* b, const cond_opts_t* o, const double* x0, double* sigma_max,
                   double* pair_best, int64_t* pair_iters, int32_t* pair_status, double* trace,
                   double* x_best, double* ms) {
  return batch_run(b, 0, o, x0, sigma_max, pair_best, pair_iters, pair_status, trace, x_best, ms);
}

int cond_batch_run_min(cond_batch_t* b, const cond_opts_t* o, const double* x0, double* sigma_min,
                       double* pair_best, int64_t* pair_iters, int32_t* pair_status, double* trace,
                       double* x_best, double* ms) {
  return batch_run(b, 1, o, x0, sigma_min, pair_best, pair_iters, pair_status, trace, x_best, ms);
}

int cond_batch_fill(const cond_batch_t* b, int64_t* nnz_l, int64_t* nnz_u, double* lu_ms) {
  if (!b) return fail(COND_EINVAL, "null batch");
  if (!b->want_min) return fail(COND_EINVAL, "the batch has no sigma_min route");
  if (nnz_l) *nnz_l = b->nnz_l;
  if (nnz_u) *nnz_u = b->nnz_u;
  if (lu_ms) *lu_ms = b->lu_ms;
  return COND_OK;
}

int cond_batch_solve_replay(const cond_batch_t* b, const double* x, double* r, double* s) {
  if (!b || !x || !r || !s) return fail(COND_EINVAL, "null argument");
  if (!b->want_min) return fail(COND_EINVAL, "the batch has no sigma_min route");
  const int64_t n = b->nrows;
  try {
    std::vector<double> xk(n), c(n), z(n), h(n), wv(n);
    for (int k = 0; k < kBatchK; ++k) {
      for (int64_t i = 0; i < n; ++i) xk[i] = x[i * kBatchK + k];
      const bool ok = replay_solve(b->pL, b->row_perm.data(), xk.data(), c.data()) &&
                      replay_solve(b->pU, b->rev.data(), c.data(), z.data()) &&
                      replay_solve(b->pUt, b->rev.data(), z.data(), h.data()) &&
                      replay_solve(b->pLt, b->rev.data(), h.data(), wv.data());
      if (!ok) return fail(COND_ESTATE, "solve schedule reads a value before its ticket is solved");
      for (int64_t i = 0; i < n; ++i) r[static_cast<int64_t>(b->scat_r[i]) * kBatchK + k] = z[i];
      for (int64_t i = 0; i < n; ++i) s[static_cast<int64_t>(b->scat_s[i]) * kBatchK + k] = wv[i];
    }
  } catch (const std::bad_alloc&) {
    return fail(COND_ENOMEM, "host memory exhausted");
  }
  return COND_OK;
}

int cond_estimate_batched(const cond_csr_t* As, int32_t count, const cond_opts_t* o,
                          const double* x0_max, const double* x0_min, void* stream,
                          cond_result_t* outs) {
  if (!As || count <= 0 || !o || !x0_max || !outs) return fail(COND_EINVAL, "null argument");
  if (!x0_min) x0_min = x0_max;
  cond_opts_t oo = *o;
  oo.sigma_min_method = COND_MIN_LU;
  cond_batch_t* b = nullptr;
  int st = cond_batch_create(As, count, &oo, &b);
  if (st) return st;
  std::unique_ptr<cond_batch, void (*)(cond_batch*)> guard(b, cond_batch_destroy);
  if ((st = cond_batch_bind(b, nullptr, 0, stream, 0, 0))) return st;
  const size_t npairs = static_cast<size_t>(count) * kBatchK;
  std::vector<double> smax(count), smin(count), pbest(npairs);
  std::vector<int64_t> it_max(npairs), it_min(npairs);
  std::vector<int32_t> pst_max(npairs), pst_min(npairs);
  double ms_max = 0.0, ms_min = 0.0;
  const int st_max = batch_run(b, 0, &oo, x0_max, smax.data(), pbest.data(), it_max.data(),
                               pst_max.data(), nullptr, nullptr, &ms_max);
  if (st_max && st_max != COND_ENUMERIC && st_max != COND_ETIMEOUT) return st_max;
  const int st_min = batch_run(b, 1, &oo, x0_min, smin.data(), pbest.data(), it_min.data(),
                               pst_min.data(), nullptr, nullptr, &ms_min);
  if (st_min && st_min != COND_ENUMERIC && st_min != COND_ETIMEOUT) return st_min;
  for (int32_t m = 0; m < count; ++m) {
    cond_result_t& r = outs[m];
    std::memset(&r, 0, sizeof(r));
    r.sigma_max = smax[m];
    r.sigma_min = smin[m];
    r.kappa = smax[m] / smin[m];
    for (int k = 0; k < kBatchK; ++k) {
      const size_t q = static_cast<size_t>(m) * kBatchK + k;
      r.iters_max = std::max<int64_t>(r.iters_max, it_max[q]);
      r.iters_min = std::max<int64_t>(r.iters_min, it_min[q]);
      if (pst_max[q] && !r.status_max) r.status_max = pst_max[q];
      if (pst_min[q] && !r.status_min) r.status_min = pst_min[q];
    }
    if (r.kappa >= 1.0 / 2.220446049250313e-16) r.flags |= COND_F_NUMSING;
    r.ms_max = ms_max;
    r.ms_min = ms_min;
    r.setup_ms = b->setup_ms;
  }
  if (st_max) return fail(st_max, "sigma_max run of a (matrix, start) pair failed");
  if (st_min) return fail(st_min, "sigma_min run of a (matrix, start) pair failed");
  return COND_OK;
}

}  // extern "C"
