// Batch plan: block-diagonal concatenation of many matrices, K = 8 starts
// each, tile schedule chosen by a small autotuner, iterations captured in
// HIP graphs and replayed until every (matrix, start) pair has stopped.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "batch.hpp"
#include "condest.h"
#include "internal.hpp"

using namespace condest;

#define BCHK(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(COND_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

namespace {

constexpr size_t kAl = 256;
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
  struct {
    size_t a_rp, a_col, a_val, at_rp, at_col, at_val, tiles, tile_mat, mat_tile0, live_mat,
        live_pref;
    size_t vec[7], parts[4], pairs, g;
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

extern "C" {

int cond_batch_create(const cond_csr_t* As, int32_t count, const cond_opts_t* o,
                      cond_batch_t** out) {
  if (!out || !As || count <= 0 || !o) return fail(COND_EINVAL, "invalid batch arguments");
  *out = nullptr;
  auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<cond_batch> b(new (std::nothrow) cond_batch());
  if (!b) return fail(COND_ENOMEM, "allocation failed");
  try {
    b->nmat = count;
    b->row0.assign(1, 0);
    b->a_rp.assign(1, 0);
    b->at_rp.assign(1, 0);
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
  for (int k = 0; k < 7; ++k) b->o.vec[k] = take(off, n * K * 8);
  for (int k = 0; k < 4; ++k) b->o.parts[k] = take(off, b->max_tiles * K * 8);
  b->o.pairs = take(off, static_cast<size_t>(count) * K * sizeof(BatchPair));
  b->o.g = take(off, sizeof(BatchGlobal));
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
  if (b->own && b->ws) hipFree(b->ws);
  if (b->h_pairs) hipHostFree(b->h_pairs);
  for (hipEvent_t e : {b->ev0, b->ev1, b->eva, b->evb})
    if (e) hipEventDestroy(e);
  if (b->stream) hipStreamDestroy(b->stream);
  delete b;
}

int cond_batch_run(cond_batch_t* b, const cond_opts_t* o, const double* x0, double* sigma_max,
                   double* pair_best, int64_t* pair_iters, int32_t* pair_status, double* trace,
                   double* x_best, double* ms_out) {
  if (!b || !o || !x0) return fail(COND_EINVAL, "null argument");
  if (!b->bound) return fail(COND_ESTATE, "batch not bound");
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
  if (!b->exec || !(b->key == k)) {
    if (b->exec) {
      BCHK(hipGraphExecDestroy(b->exec));
      b->exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    BCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    for (int it = 0; it < chunk; ++it) enqueue_batch_iteration(b, a, p);
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (e != hipSuccess) return fail(COND_EHIP, std::string("capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(COND_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
    b->key = k;
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
    BCHK(hipGraphLaunch(b->exec, b->stream));
    launched += chunk;
    BCHK(hipMemcpyAsync(slot[s], a.pairs, npairs * sizeof(BatchPair), hipMemcpyDeviceToHost,
                        b->stream));
    BCHK(hipEventRecord(ev[s], b->stream));
    return COND_OK;
  };
  int st;
  if ((st = launch_chunk(0))) return st;
  for (;;) {
    const bool more = launched < total;
    if (more && (st = launch_chunk(cur ^ 1))) return st;
    BCHK(hipEventSynchronize(ev[cur]));
    bool all = true;
    for (int q = 0; q < npairs && all; ++q) all = slot[cur][q].stopped != 0;
    if (all || !more) break;
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
      if (s.status == COND_OK) best = std::max(best, s.best);
    }
    if (sigma_max) sigma_max[m] = best;  // every start is a lower bound: keep the largest
  }
  if (status) return fail(status, "a (matrix, start) pair failed");
  return COND_OK;
}

}  // extern "C"
