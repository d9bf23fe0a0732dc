// Device plan: host set-up, workspace layout, and the driver loop that
// replays captured iterations of Algorithm 1 until the run stops.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <future>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "condest.h"
#include "internal.hpp"
#include "bounds.hpp"
#include "kernels.hpp"
#include "panels.hpp"
#include "panels_upload.hpp"

using namespace condest;

#define CHK(expr)                                                                    \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(COND_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

namespace {


struct GraphKey {
  int route = -1;
  int scaled = 0;
  int chunk = 0;
  const void* trace = nullptr;
  const void* xbest = nullptr;
  AdamParams p{};
  bool operator==(const GraphKey& o) const {
    return route == o.route && scaled == o.scaled && chunk == o.chunk && trace == o.trace &&
           xbest == o.xbest &&
           std::memcmp(&p, &o.p, sizeof(p)) == 0;
  }
};

// Row tiles for the streaming SpMV: consecutive rows, at most kTileRowsHost
// rows and kTileEntriesHost entries per tile; a longer row is a tile alone.
std::vector<int32_t> make_tiles(const HostCsr& a) {
  std::vector<int32_t> t{0};
  int32_t s = 0;
  for (int32_t i = 0; i < a.n; ++i)
    if (i > s && (i + 1 - s > kTileRowsHost || a.rowptr[i + 1] - a.rowptr[s] > kTileEntriesHost)) {
      t.push_back(i);
      s = i;
    }
  t.push_back(a.n);
  return t;
}

}  // namespace

struct cond_plan {
  int32_t n = 0;
  cond_opts_t opts{};
  HostCsr a, at;
  std::vector<int32_t> tiles_a, tiles_at;  // row tiles of the streaming SpMV
  std::unique_ptr<cond_lu> lu;
  bool want_min = false;
  double setup_ms = 0.0;
  // device
  bool bound = false;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_a = nullptr, ev_b = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  DevCsr dA, dAt;
  // the four solves of Algorithm 2, each a forward substitution in its own
  // order: L (pivot order), U reversed, U^T (pivot order), L^T reversed
  PanelCsr pL, pU, pUt, pLt;
  std::vector<double> udiag_rev;
  std::vector<int32_t> rev, scat_s, scat_r;
  DevTri dL, dU, dUt, dLt;
  int* d_row_perm = nullptr;  // L rhs gather: x[row_perm[k]]
  int* d_rev = nullptr;       // n-1-k
  int* d_scat_s = nullptr;    // s[row_perm[n-1-k]] = result of the reversed L^T solve
  int* d_scat_r = nullptr;    // r[col_perm[n-1-k]] = result of the reversed U solve
  double *x = nullptr, *m = nullptr, *v = nullptr, *d = nullptr, *y = nullptr, *w = nullptr;
  double *c = nullptr, *z = nullptr, *h = nullptr, *wv = nullptr;
  // column scaling: D_col (column norms), its inverse, and D_col in the
  // solves' reversed pivot order (dz[k] = d[col_perm[n-1-k]])
  double *dcol = nullptr, *dinv = nullptr, *dz = nullptr;
  bool has_zero_col = false;
  bool scale_ready = false;
  // after a timed-out wait a slice may publish into a slot its finish step
  // already re-armed: every slot is re-armed before the next solve
  bool rearm_slots = false;
  bool inject_timeout = false;  // test hook: the next solve starts timed out
  double *parts_x = nullptr, *parts_y = nullptr, *parts_xd = nullptr, *parts_xx = nullptr;
  RunState* st = nullptr;
  RunState* st_free = nullptr;
  unsigned* tickets = nullptr;
  RunState* h_state = nullptr;  // pinned, two slots
  int grid = 8;
  GraphKey key[3];
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
  // eager profiling (opts.profile): event pairs around every launch
  std::vector<hipEvent_t> evpool;
  struct Rec {
    int k;
    double bytes;
  };
  std::vector<Rec> recs;
  double kms[COND_K_COUNT] = {};
  long long kcnt[COND_K_COUNT] = {};
  double kbytes[COND_K_COUNT] = {};
  bool profiling = false;
  size_t need_bytes = 0;
  // offsets into the workspace
  struct {
    size_t a_rp, a_col, a_val, at_rp, at_col, at_val, a_tiles, at_tiles;
    size_t tri[4][kTriSlots];
    size_t row_perm, rev, scat_s, scat_r;
    size_t vec[10];
    size_t scal[3];
    size_t parts[4];
    size_t st, st_free, tickets;
  } o{};
};

namespace {

bool idx64_needed(const HostCsr& a) { return a.nnz() >= (1LL << 31) - 1; }

void plan_layout(cond_plan* p) {
  Layout L;
  const size_t n = p->n;
  const bool a64 = idx64_needed(p->a);
  const size_t ri = a64 ? 8 : 4;
  p->o.a_rp = L.take((n + 1) * ri);
  p->o.a_col = L.take(p->a.nnz() * 4);
  p->o.a_val = L.take(p->a.nnz() * 8);
  p->o.at_rp = L.take((n + 1) * ri);
  p->o.at_col = L.take(p->at.nnz() * 4);
  p->o.at_val = L.take(p->at.nnz() * 8);
  p->o.a_tiles = L.take(p->tiles_a.size() * 4);
  p->o.at_tiles = L.take(p->tiles_at.size() * 4);
  if (p->want_min) {
    const PanelCsr* tris[4] = {&p->pL, &p->pU, &p->pUt, &p->pLt};
    for (int f = 0; f < 4; ++f) tri_layout(*tris[f], 1, L, p->o.tri[f]);
    p->o.row_perm = L.take(n * 4);
    p->o.rev = L.take(n * 4);
    p->o.scat_s = L.take(n * 4);
    p->o.scat_r = L.take(n * 4);
  }
  const int nvec = p->want_min ? 10 : 6;
  for (int k = 0; k < nvec; ++k) p->o.vec[k] = L.take(n * 8);
  for (int k = 0; k < 3; ++k) p->o.scal[k] = L.take(n * 8);
  for (int k = 0; k < 4; ++k) p->o.parts[k] = L.take(kMaxParts * 8);
  p->o.st = L.take(sizeof(RunState));
  p->o.st_free = L.take(sizeof(RunState));
  p->o.tickets = L.take(4 * kSolveTickets * sizeof(unsigned));  // four solves' counters
  p->need_bytes = L.off;
}

template <typename T>
T* at_off(cond_plan* p, size_t off) {
  return reinterpret_cast<T*>(p->ws + off);
}

int upload(cond_plan* p, size_t off, const void* src, size_t bytes) {
  if (!bytes) return COND_OK;
  CHK(hipMemcpyAsync(p->ws + off, src, bytes, hipMemcpyHostToDevice, p->stream));
  return COND_OK;
}

int upload_csr(cond_plan* p, const HostCsr& a, size_t rp, size_t col, size_t val, bool idx64,
               const std::vector<int32_t>& tiles, size_t tiles_off, DevCsr& out) {
  const size_t n = a.n;
  int st;
  if (idx64) {
    st = upload(p, rp, a.rowptr.data(), (n + 1) * 8);
  } else {
    std::vector<int32_t> r32(a.rowptr.begin(), a.rowptr.end());
    st = upload(p, rp, r32.data(), (n + 1) * 4);
    if (!st) CHK(hipStreamSynchronize(p->stream));  // r32 is a temporary
  }
  if (st) return st;
  if ((st = upload(p, col, a.col.data(), a.nnz() * 4))) return st;
  if ((st = upload(p, val, a.val.data(), a.nnz() * 8))) return st;
  out.n = a.n;
  out.nnz = a.nnz();
  out.rowptr = p->ws + rp;
  out.idx64 = idx64 ? 1 : 0;
  out.col = at_off<int>(p, col);
  out.val = at_off<double>(p, val);
  if ((st = upload(p, tiles_off, tiles.data(), tiles.size() * 4))) return st;
  out.tiles = at_off<int>(p, tiles_off);
  out.ntiles = static_cast<int>(tiles.size()) - 1;
  return COND_OK;
}

int upload_tri(cond_plan* p, const PanelCsr& t, const size_t* off, DevTri& out) {
  return tri_upload(p->ws, off, t, 1, p->stream, out);
}

AdamParams params_of(const cond_opts_t& o) {
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
  p.minimise = 0;
  return p;
}

int check_opts(const cond_opts_t* o) {
  if (!o) return fail(COND_EINVAL, "null options");
  if (!(o->alpha > 0) || !(o->beta1 >= 0 && o->beta1 < 1) || !(o->beta2 >= 0 && o->beta2 < 1) ||
      !(o->eps >= 0) || o->max_iter < 1 || o->stop_window < 0 || !(o->stop_rtol >= 0) ||
      o->chunk < 0)
    return fail(COND_EINVAL, "invalid Projected Adam options");
  if (!(o->alpha_min >= 0) || o->alpha_min > o->alpha ||
      (o->alpha_min > 0 && !(o->alpha_decay > 0 && o->alpha_decay < 1)))
    return fail(COND_EINVAL, "invalid step-size floor or decay");
  if (o->scaling != COND_SCALE_NONE && o->scaling != COND_SCALE_COL)
    return fail(COND_EINVAL, "unknown scaling");
  if (o->sigma_min_method != COND_MIN_LU && o->sigma_min_method != COND_MIN_SPMV &&
      o->sigma_min_method != COND_MIN_NONE)
    return fail(COND_EINVAL, "unknown sigma_min method");
  return COND_OK;
}

// Algorithmic bytes of one launch: matrix entries 12 B, row pointers, and
// every vector read or written once (gathers counted as one pass).
double spmv_bytes(const DevCsr& a) {
  return 12.0 * a.nnz + (a.idx64 ? 8.0 : 4.0) * (a.n + 1) + 16.0 * a.n;
}
// Scope guard of one launch in profiling mode: records an event before and
// after it on the plan stream (event pair r is evpool[2r], evpool[2r+1]).
struct Prof {
  cond_plan* p;
  int k;
  double bytes;
  Prof(cond_plan* pp, int kk, double by) : p(pp), k(kk), bytes(by) {
    if (p->profiling) mark(2 * p->recs.size());
  }
  ~Prof() {
    if (p->profiling) {
      mark(2 * p->recs.size() + 1);
      p->recs.push_back({k, bytes});
    }
  }
  void mark(size_t idx) {
    while (p->evpool.size() <= idx) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return;
      p->evpool.push_back(e);
    }
    hipEventRecord(p->evpool[idx], p->stream);
  }
};

// One iteration of the chosen route, enqueued on the plan stream: 0 the
// sigma_max run (M = A), 1 the sigma_min run of Algorithm 2 (M = A^-1), 2 the
// SpMV-only sigma_min ablation (M = A, minimising; ap.minimise is set).
// With `scaled` the matrix is A D^-1 (column scaling): the products take the
// factor 1/d on the fly, and the sigma_min run multiplies the solve's output
// by D twice (see scale_sumsq_k), so A's own LU serves.
void enqueue_iteration(cond_plan* p, int route, bool scaled, double* trace, double* xbest,
                       const AdamParams& ap) {
  hipStream_t s = p->stream;
  const int n = p->n, g = p->grid;
  const double dn = n;
  const double scale_bytes = scaled ? 8.0 * dn : 0.0;
  if (route != 1) {
    { Prof pr(p, COND_K_NORMALISE, 16.0 * dn);
      launch_normalise(n, p->x, p->parts_xx, g, p->parts_x, p->st, nullptr, 0, nullptr, 0, s); }
    { Prof pr(p, COND_K_SPMV_A, spmv_bytes(p->dA) + scale_bytes);
      launch_spmv(p->dA, p->x, p->y, p->parts_y, g, p->st, s, scaled ? p->dinv : nullptr,
                  nullptr); }
    { Prof pr(p, COND_K_SPMV_AT, spmv_bytes(p->dAt) + scale_bytes);
      launch_spmv(p->dAt, p->y, p->w, nullptr, g, p->st, s, nullptr,
                  scaled ? p->dinv : nullptr); }
  } else {
    const double nl = static_cast<double>(p->lu->l_rows.nnz());
    const double nu = static_cast<double>(p->lu->u_rows.nnz());
    const double rp = 8.0 * (dn + 1);
    double* resets[4] = {p->c, p->z, p->h, p->wv};
    { Prof pr(p, COND_K_NORMALISE, 48.0 * dn);
      launch_normalise(n, p->x, p->parts_xx, g, p->parts_x, p->st, resets, 4, p->tickets, 4, s); }
    // r = A^-1 x: L c = P x, U z = c (r = Q z; ||r|| = ||z||); z is kept reversed
    { Prof pr(p, COND_K_TRSV_L, 12.0 * nl + rp + 28.0 * dn);
      launch_trsv(p->dL, p->x, p->d_row_perm, p->c, nullptr, nullptr, p->tickets, p->st, s); }
    { Prof pr(p, COND_K_TRSV_U, 12.0 * nu + rp + 36.0 * dn);
      launch_trsv(p->dU, p->c, p->d_rev, p->z, nullptr, nullptr, tix(p->tickets, 1), p->st, s); }
    // scaled: z <- D z (= D r) and c <- D z (the transposed solves' input;
    // c, the L solve's output, is free once the U solve has run)
    { Prof pr(p, COND_K_SUMSQ, scaled ? 32.0 * dn : 8.0 * dn);
      if (scaled)
        launch_scale_sumsq(n, p->z, p->dz, p->c, p->parts_y, g, p->st, s);
      else
        launch_sumsq(n, p->z, p->parts_y, g, p->st, s); }
    // s = A^-T r: U^T h = Q^T r = z, L^T wv = h, s = P^T wv (wv kept reversed)
    { Prof pr(p, COND_K_TRSV_UT, 12.0 * nu + rp + 36.0 * dn);
      launch_trsv(p->dUt, scaled ? p->c : p->z, p->d_rev, p->h, nullptr, nullptr,
                  tix(p->tickets, 2), p->st, s); }
    { Prof pr(p, COND_K_TRSV_LT, 12.0 * nl + rp + 40.0 * dn);
      launch_trsv(p->dLt, p->h, p->d_rev, p->wv, p->w, p->d_scat_s, tix(p->tickets, 3), p->st, s); }
  }
  { Prof pr(p, COND_K_ADAM1, 56.0 * dn);
    launch_pass1(n, p->x, p->w, p->m, p->v, p->d, xbest, p->parts_x, p->parts_y, g, p->parts_xd,
                 p->st, trace, ap, s); }
  { Prof pr(p, COND_K_ADAM2, 24.0 * dn);
    launch_pass2(n, p->x, p->d, p->parts_xd, g, p->parts_xx, p->st, ap, s); }
}

// Fold the recorded event pairs into the per-kernel totals (stream synchronised).
int collect_profile(cond_plan* p) {
  for (size_t r = 0; r < p->recs.size(); ++r) {
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, p->evpool[2 * r], p->evpool[2 * r + 1]));
    const int k = p->recs[r].k;
    p->kms[k] += ms;
    p->kcnt[k] += 1;
    p->kbytes[k] += p->recs[r].bytes;
  }
  p->recs.clear();
  return COND_OK;
}

int get_graph(cond_plan* p, int route, bool scaled, int chunk, double* trace, double* xbest,
              const AdamParams& ap, hipGraphExec_t* out) {
  GraphKey k;
  k.route = route;
  k.scaled = scaled ? 1 : 0;
  k.chunk = chunk;
  k.trace = trace;
  k.xbest = xbest;
  k.p = ap;
  if (p->exec[route] && p->key[route] == k) {
    *out = p->exec[route];
    return COND_OK;
  }
  if (p->exec[route]) {
    CHK(hipGraphExecDestroy(p->exec[route]));
    p->exec[route] = nullptr;
  }
  hipGraph_t graph = nullptr;
  CHK(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  for (int it = 0; it < chunk; ++it) enqueue_iteration(p, route, scaled, trace, xbest, ap);
  hipError_t e = hipStreamEndCapture(p->stream, &graph);
  if (e != hipSuccess) return fail(COND_EHIP, std::string("capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&p->exec[route], graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(COND_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
  p->key[route] = k;
  *out = p->exec[route];
  return COND_OK;
}

// Replays the captured chunk until the device state says the run stopped,
// launching one chunk ahead of the poll so the device never waits on the host.
int replay_until_stop(cond_plan* p, hipGraphExec_t exec, int chunk, long long total) {
  long long launched = 0;
  RunState* slot[2] = {p->h_state, p->h_state + 1};
  hipEvent_t ev[2] = {p->ev_a, p->ev_b};
  int cur = 0;
  CHK(hipGraphLaunch(exec, p->stream));
  launched += chunk;
  CHK(hipMemcpyAsync(slot[0], p->st, sizeof(RunState), hipMemcpyDeviceToHost, p->stream));
  CHK(hipEventRecord(ev[0], p->stream));
  bool pending_next = false;
  for (;;) {
    if (launched < total) {
      CHK(hipGraphLaunch(exec, p->stream));
      launched += chunk;
      CHK(hipMemcpyAsync(slot[cur ^ 1], p->st, sizeof(RunState), hipMemcpyDeviceToHost,
                         p->stream));
      CHK(hipEventRecord(ev[cur ^ 1], p->stream));
      pending_next = true;
    } else {
      pending_next = false;
    }
    CHK(hipEventSynchronize(ev[cur]));
    if (slot[cur]->done || slot[cur]->stop_req) break;
    if (!pending_next) break;  // should not happen: the last chunk always stops
    cur ^= 1;
  }
  return COND_OK;
}

// Orders the plan stream after the work the caller queued on its stream.
int join_user_stream(cond_plan* p) {
  if (!p->user_stream) return COND_OK;
  hipEvent_t e;
  CHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  CHK(hipEventRecord(e, p->user_stream));
  CHK(hipStreamWaitEvent(p->stream, e, 0));
  CHK(hipEventDestroy(e));
  return COND_OK;
}

// Column norms and the factors of the column-scaled matrix, computed once
// per bind on the first call that needs them.
int ensure_scaling(cond_plan* p) {
  if (p->has_zero_col) return fail(COND_EINVAL, "A has a zero column: no column scaling");
  if (p->scale_ready) return COND_OK;
  launch_row_norms(p->dAt, p->dcol, p->stream);
  launch_scale_prep(p->n, p->dcol, p->dinv, p->want_min ? p->d_scat_r : nullptr, p->dz, p->stream);
  CHK(hipGetLastError());
  p->scale_ready = true;
  return COND_OK;
}

// Re-arms every slice partial slot of the four solves (kPending) when the
// previous solve on this plan timed out.
void rearm_after_timeout(cond_plan* p) {
  if (!p->rearm_slots || !p->want_min) return;
  const PanelCsr* tris[4] = {&p->pL, &p->pU, &p->pUt, &p->pLt};
  const DevTri* devs[4] = {&p->dL, &p->dU, &p->dUt, &p->dLt};
  for (int f = 0; f < 4; ++f)
    if (tris[f]->nslots > 0) launch_fill(static_cast<long long>(tris[f]->nslots) * tris[f]->prows, devs[f]->partials, kPending, p->stream);
  p->rearm_slots = false;
}

struct RouteResult {
  double sigma = 0.0;
  long long iters = 0;
  int status = 0;
  int flags = 0;
  double ms = 0.0;
};

int run_route(cond_plan* p, int route, const cond_opts_t& o, const double* x0, double* trace,
              double* xbest, RouteResult& rr) {
  AdamParams ap = params_of(o);
  ap.minimise = route == 2 ? 1 : 0;
  const bool scaled = o.scaling == COND_SCALE_COL;
  const bool inject = route == 1 && p->inject_timeout;
  if (route == 1) {
    rearm_after_timeout(p);
    p->inject_timeout = false;
  }
  const long long total = o.max_iter + 1;  // the last pass only evaluates x_T
  if (o.profile) {
    // eager launches with an event pair around each kernel; poll every iteration
    CHK(hipEventRecord(p->ev_start, p->stream));
    launch_init(p->n, x0, p->x, p->m, p->v, p->parts_xx, p->grid, p->st, o.alpha, ap.minimise,
                p->stream);
    if (inject) launch_set_int(&p->st->abort_wait, 1, p->stream);
    CHK(hipGetLastError());
    p->profiling = true;
    int st = COND_OK;
    for (long long it = 0; it < total && st == COND_OK; ++it) {
      enqueue_iteration(p, route, scaled, trace, xbest, ap);
      if (hipMemcpyAsync(p->h_state, p->st, sizeof(RunState), hipMemcpyDeviceToHost,
                         p->stream) != hipSuccess ||
          hipStreamSynchronize(p->stream) != hipSuccess) {
        st = fail(COND_EHIP, "profiled iteration failed");
        break;
      }
      st = collect_profile(p);
      if (p->h_state->stop_req) break;
    }
    p->profiling = false;
    if (st) return st;
  } else {
    const int chunk = o.chunk > 0 ? o.chunk : (route == 1 ? 4 : 32);
    hipGraphExec_t exec = nullptr;
    int st = get_graph(p, route, scaled, chunk, trace, xbest, ap, &exec);
    if (st) return st;
    CHK(hipEventRecord(p->ev_start, p->stream));
    launch_init(p->n, x0, p->x, p->m, p->v, p->parts_xx, p->grid, p->st, o.alpha, ap.minimise,
                p->stream);
    if (inject) launch_set_int(&p->st->abort_wait, 1, p->stream);
    CHK(hipGetLastError());
    if ((st = replay_until_stop(p, exec, chunk, total))) return st;
  }
  CHK(hipEventRecord(p->ev_stop, p->stream));
  CHK(hipMemcpyAsync(p->h_state, p->st, sizeof(RunState), hipMemcpyDeviceToHost, p->stream));
  CHK(hipStreamSynchronize(p->stream));
  float ms = 0.f;
  CHK(hipEventElapsedTime(&ms, p->ev_start, p->ev_stop));
  const RunState& s = *p->h_state;
  if (!s.stop_req) return fail(COND_EHIP, "run did not reach its stopping iteration");
  rr.sigma = s.stop_req && s.done ? s.best : s.best_next;
  rr.iters = s.iters;
  rr.status = s.abort_wait ? COND_ETIMEOUT : s.status;
  if (s.abort_wait) p->rearm_slots = true;
  rr.flags = s.flags;
  rr.ms = ms;
  return COND_OK;
}

}  // namespace

extern "C" {

int cond_plan_create(const cond_csr_t* A, const cond_opts_t* o, cond_plan_t** out) {
  if (!out) return fail(COND_EINVAL, "null output");
  *out = nullptr;
  int st = check_opts(o);
  if (st) return st;
  auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<cond_plan> p(new (std::nothrow) cond_plan());
  if (!p) return fail(COND_ENOMEM, "allocation failed");
  try {
    if ((st = canonical_copy(A, p->a))) return st;
    transpose(p->a, p->at);
    p->tiles_a = make_tiles(p->a);
    p->tiles_at = make_tiles(p->at);
    for (int32_t j = 0; j < p->at.n && !p->has_zero_col; ++j) {
      bool nz = false;
      for (int64_t e = p->at.rowptr[j]; e < p->at.rowptr[j + 1] && !nz; ++e) nz = p->at.val[e] != 0.0;
      p->has_zero_col = !nz;
    }
    p->n = p->a.n;
    p->opts = *o;
    p->opts.col_perm = nullptr;
    p->want_min = (o->sigma_min_method == COND_MIN_LU);
    if (p->want_min) {
      p->lu.reset(new cond_lu());
      st = lu_factor(p->a, p->at, o->col_perm, o->pivot_tol, *p->lu);
      if (st) return st;
      const cond_lu& f = *p->lu;
      const int32_t n = f.n;
      p->udiag_rev.resize(n);
      p->rev.resize(n);
      p->scat_s.resize(n);
      p->scat_r.resize(n);
      for (int32_t k = 0; k < n; ++k) {
        p->udiag_rev[k] = f.u_diag[n - 1 - k];
        p->rev[k] = n - 1 - k;
        p->scat_s[k] = f.row_perm[n - 1 - k];
        p->scat_r[k] = f.col_perm[n - 1 - k];
      }
      // the four schedules are independent host work, one thread each; each
      // is the same computation as on one thread
      auto sched = [](const HostCsr& t, const double* diag) {
        PanelCsr s = split_panels(t, kMaxPanelRows);
        invert_panels(s, diag);
        return s;
      };
      std::future<PanelCsr> fut[4] = {
          std::async(std::launch::async, [&] { return sched(f.l_rows, nullptr); }),
          std::async(std::launch::async,
                     [&] { return sched(reverse_order(f.u_rows), p->udiag_rev.data()); }),
          std::async(std::launch::async, [&] { return sched(f.u_cols, f.u_diag.data()); }),
          std::async(std::launch::async, [&] { return sched(reverse_order(f.l_cols), nullptr); })};
      p->pL = fut[0].get();  // get() rethrows a thread's exception
      p->pU = fut[1].get();
      p->pUt = fut[2].get();
      p->pLt = fut[3].get();
      // a diagonal block whose inverse overflows float64 would turn every
      // solve into NaN: refuse the plan instead
      for (const PanelCsr* t : {&p->pL, &p->pU, &p->pUt, &p->pLt})
        for (double w : t->winv)
          if (!std::isfinite(w))
            return fail(COND_ENUMERIC, "a diagonal block of the LU factors has no finite float64 inverse");
    }
  } catch (const std::bad_alloc&) {
    return fail(COND_ENOMEM, "host memory exhausted in set-up");
  }
  p->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  p->grid = grid_for(p->n);
  plan_layout(p.get());
  *out = p.release();
  return COND_OK;
}

int cond_plan_workspace_bytes(const cond_plan_t* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(COND_EINVAL, "null argument");
  *bytes = plan->need_bytes;
  return COND_OK;
}

int cond_plan_bind(cond_plan_t* p, void* workspace, size_t bytes, void* stream) {
  if (!p) return fail(COND_EINVAL, "null plan");
  if (p->bound) return fail(COND_ESTATE, "plan already bound");
  if (workspace && bytes < p->need_bytes) return fail(COND_ENOMEM, "workspace too small");
  if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign))
    return fail(COND_EINVAL, "workspace must be 256-byte aligned");
  p->user_stream = static_cast<hipStream_t>(stream);
  CHK(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
  CHK(hipEventCreate(&p->ev_start));
  CHK(hipEventCreate(&p->ev_stop));
  CHK(hipEventCreateWithFlags(&p->ev_a, hipEventDisableTiming));
  CHK(hipEventCreateWithFlags(&p->ev_b, hipEventDisableTiming));
  CHK(hipHostMalloc(reinterpret_cast<void**>(&p->h_state), 2 * sizeof(RunState), hipHostMallocDefault));
  if (workspace) {
    p->ws = static_cast<char*>(workspace);
    p->ws_bytes = bytes;
    p->own_ws = false;
  } else {
    CHK(hipMalloc(reinterpret_cast<void**>(&p->ws), p->need_bytes));
    p->ws_bytes = p->need_bytes;
    p->own_ws = true;
  }
  // order the uploads after whatever the caller queued on its stream
  int st;
  if ((st = join_user_stream(p))) return st;
  const bool a64 = idx64_needed(p->a);
  if ((st = upload_csr(p, p->a, p->o.a_rp, p->o.a_col, p->o.a_val, a64, p->tiles_a,
                       p->o.a_tiles, p->dA)))
    return st;
  if ((st = upload_csr(p, p->at, p->o.at_rp, p->o.at_col, p->o.at_val, a64, p->tiles_at,
                       p->o.at_tiles, p->dAt)))
    return st;
  if (p->want_min) {
    const cond_lu& f = *p->lu;
    if ((st = upload(p, p->o.row_perm, f.row_perm.data(), p->n * 4))) return st;
    if ((st = upload(p, p->o.rev, p->rev.data(), p->n * 4))) return st;
    if ((st = upload(p, p->o.scat_s, p->scat_s.data(), p->n * 4))) return st;
    if ((st = upload(p, p->o.scat_r, p->scat_r.data(), p->n * 4))) return st;
    if ((st = upload_tri(p, p->pL, p->o.tri[0], p->dL))) return st;
    if ((st = upload_tri(p, p->pU, p->o.tri[1], p->dU))) return st;
    if ((st = upload_tri(p, p->pUt, p->o.tri[2], p->dUt))) return st;
    if ((st = upload_tri(p, p->pLt, p->o.tri[3], p->dLt))) return st;
    p->d_row_perm = at_off<int>(p, p->o.row_perm);
    p->d_rev = at_off<int>(p, p->o.rev);
    p->d_scat_s = at_off<int>(p, p->o.scat_s);
    p->d_scat_r = at_off<int>(p, p->o.scat_r);
  }
  double** vecs[10] = {&p->x, &p->m, &p->v, &p->d, &p->y, &p->w, &p->c, &p->z, &p->h, &p->wv};
  const int nvec = p->want_min ? 10 : 6;
  for (int k = 0; k < nvec; ++k) *vecs[k] = at_off<double>(p, p->o.vec[k]);
  p->dcol = at_off<double>(p, p->o.scal[0]);
  p->dinv = at_off<double>(p, p->o.scal[1]);
  p->dz = at_off<double>(p, p->o.scal[2]);
  p->scale_ready = false;
  p->parts_x = at_off<double>(p, p->o.parts[0]);
  p->parts_y = at_off<double>(p, p->o.parts[1]);
  p->parts_xd = at_off<double>(p, p->o.parts[2]);
  p->parts_xx = at_off<double>(p, p->o.parts[3]);
  p->st = at_off<RunState>(p, p->o.st);
  p->st_free = at_off<RunState>(p, p->o.st_free);
  p->tickets = at_off<unsigned>(p, p->o.tickets);
  CHK(hipMemsetAsync(p->st, 0, sizeof(RunState), p->stream));
  CHK(hipMemsetAsync(p->st_free, 0, sizeof(RunState), p->stream));
  CHK(hipMemsetAsync(p->tickets, 0, 4 * kSolveTickets * sizeof(unsigned), p->stream));
  CHK(hipStreamSynchronize(p->stream));
  p->bound = true;
  return COND_OK;
}

void cond_plan_destroy(cond_plan_t* p) {
  if (!p) return;
  if (p->stream) hipStreamSynchronize(p->stream);
  for (auto& e : p->exec)
    if (e) hipGraphExecDestroy(e);
  if (p->own_ws && p->ws) hipFree(p->ws);
  if (p->h_state) hipHostFree(p->h_state);
  if (p->ev_start) hipEventDestroy(p->ev_start);
  if (p->ev_stop) hipEventDestroy(p->ev_stop);
  if (p->ev_a) hipEventDestroy(p->ev_a);
  if (p->ev_b) hipEventDestroy(p->ev_b);
  if (p->stream) hipStreamDestroy(p->stream);
  delete p;
}

int cond_plan_run(cond_plan_t* p, const cond_opts_t* o, const double* x0_max, const double* x0_min,
                  cond_result_t* out, double* trace_max, double* trace_min, double* x_best_max,
                  double* x_best_min) {
  if (!p || !out) return fail(COND_EINVAL, "null argument");
  if (!p->bound) return fail(COND_ESTATE, "plan not bound");
  const cond_opts_t& oo = o ? *o : p->opts;
  int st = check_opts(&oo);
  if (st) return st;
  if (!x0_max && !x0_min) return fail(COND_EINVAL, "null start vector");
  const bool run_max = x0_max != nullptr;
  if (!x0_min) x0_min = x0_max;
  std::memset(out, 0, sizeof(*out));
  out->setup_ms = p->setup_ms;
  if (p->want_min) {
    out->nnz_l = p->lu->l_rows.nnz();
    out->nnz_u = p->lu->u_rows.nnz() + p->n;
  }
  if ((st = join_user_stream(p))) return st;
  if (oo.profile) {
    std::fill(p->kms, p->kms + COND_K_COUNT, 0.0);
    std::fill(p->kcnt, p->kcnt + COND_K_COUNT, 0LL);
    std::fill(p->kbytes, p->kbytes + COND_K_COUNT, 0.0);
  }
  if (oo.scaling == COND_SCALE_COL) {
    if ((st = ensure_scaling(p))) return st;
    out->flags |= COND_F_COLSCALED;
  }
  // the sigma_min route: Algorithm 2 when the plan holds the LU, or the
  // SpMV-only ablation, which any plan can run
  const bool lu_route = p->want_min && oo.sigma_min_method == COND_MIN_LU;
  const bool spmv_route = oo.sigma_min_method == COND_MIN_SPMV;
  RouteResult rmax, rmin;
  if (run_max) {
    if ((st = run_route(p, 0, oo, x0_max, trace_max, x_best_max, rmax))) return st;
    out->sigma_max = rmax.sigma;
    out->iters_max = rmax.iters;
    out->status_max = rmax.status;
    out->ms_max = rmax.ms;
    if (rmax.flags & COND_F_MAXITER) out->flags |= COND_F_MAXITER;
  } else if (!lu_route && !spmv_route) {
    return fail(COND_EINVAL, "null sigma_max start and no sigma_min run");
  }
  if (lu_route || spmv_route) {
    if ((st = run_route(p, lu_route ? 1 : 2, oo, x0_min, trace_min, x_best_min, rmin))) return st;
    // the LU run maximises ||A^-1 x|| / ||x||; the ablation minimises ||A x|| / ||x||
    out->sigma_min = lu_route ? 1.0 / rmin.sigma : rmin.sigma;
    out->iters_min = rmin.iters;
    out->status_min = rmin.status;
    out->ms_min = rmin.ms;
    if (rmin.flags & COND_F_MAXITER) out->flags |= COND_F_MAXITER;
    if (run_max) {
      out->kappa = out->sigma_max / out->sigma_min;
      if (out->kappa >= 1.0 / 2.220446049250313e-16) out->flags |= COND_F_NUMSING;
    }
  }
  if (out->status_max) return fail(out->status_max, "sigma_max run failed");
  if (out->status_min) return fail(out->status_min, "sigma_min run failed");
  return COND_OK;
}

int cond_plan_kernel_stats(const cond_plan_t* p, double* ms, int64_t* launches, double* bytes) {
  if (!p || !ms || !launches) return fail(COND_EINVAL, "null argument");
  for (int k = 0; k < COND_K_COUNT; ++k) {
    ms[k] = p->kms[k];
    launches[k] = p->kcnt[k];
    if (bytes) bytes[k] = p->kcnt[k] ? p->kbytes[k] / static_cast<double>(p->kcnt[k]) : 0.0;
  }
  return COND_OK;
}

int cond_plan_solve_info(const cond_plan_t* p, int32_t* levels, int64_t* tasks, int64_t* panels) {
  if (!p || !levels || !tasks || !panels) return fail(COND_EINVAL, "null argument");
  if (!p->want_min) return fail(COND_EINVAL, "the plan has no sigma_min route");
  const PanelCsr* tris[4] = {&p->pL, &p->pU, &p->pUt, &p->pLt};
  for (int k = 0; k < 4; ++k) {
    levels[k] = tris[k]->levels;
    tasks[k] = static_cast<int64_t>(tris[k]->task_panel.size());
    panels[k] = static_cast<int64_t>(tris[k]->pstart.size()) - 1;
  }
  return COND_OK;
}

int cond_plan_solve_replay(const cond_plan_t* p, const double* x, double* r, double* s) {
  if (!p || !x || !r || !s) return fail(COND_EINVAL, "null argument");
  if (!p->want_min) return fail(COND_EINVAL, "the plan has no sigma_min route");
  try {
    const int32_t n = p->n;
    std::vector<double> c(n), z(n), h(n), wv(n);
    const bool ok = replay_solve(p->pL, p->lu->row_perm.data(), x, c.data()) &&
                    replay_solve(p->pU, p->rev.data(), c.data(), z.data()) &&
                    replay_solve(p->pUt, p->rev.data(), z.data(), h.data()) &&
                    replay_solve(p->pLt, p->rev.data(), h.data(), wv.data());
    if (!ok) return fail(COND_ESTATE, "solve schedule reads a value before its ticket is solved");
    for (int32_t k = 0; k < n; ++k) r[p->scat_r[k]] = z[k];
    for (int32_t k = 0; k < n; ++k) s[p->scat_s[k]] = wv[k];
  } catch (const std::bad_alloc&) {
    return fail(COND_ENOMEM, "host memory exhausted");
  }
  return COND_OK;
}

int cond_plan_spmv(cond_plan_t* p, int transpose, const double* x, double* y) {
  if (!p || !x || !y) return fail(COND_EINVAL, "null argument");
  if (!p->bound) return fail(COND_ESTATE, "plan not bound");
  int st0 = join_user_stream(p);
  if (st0) return st0;
  if (transpose & ~(COND_SPMV_T | COND_SPMV_COLSCALED)) return fail(COND_EINVAL, "unknown spmv flags");
  const bool tr = transpose & COND_SPMV_T;
  const bool scaled = transpose & COND_SPMV_COLSCALED;
  if (scaled && (st0 = ensure_scaling(p))) return st0;
  const double* cs = scaled && !tr ? p->dinv : nullptr;
  const double* rs = scaled && tr ? p->dinv : nullptr;
  launch_spmv(tr ? p->dAt : p->dA, x, y, nullptr, p->grid, nullptr, p->stream, cs, rs);
  CHK(hipGetLastError());
  CHK(hipStreamSynchronize(p->stream));
  return COND_OK;
}

int cond_plan_column_norms(cond_plan_t* p, double* d) {
  if (!p || !d) return fail(COND_EINVAL, "null argument");
  if (!p->bound) return fail(COND_ESTATE, "plan not bound");
  int st = join_user_stream(p);
  if (st) return st;
  if (p->has_zero_col) {
    launch_row_norms(p->dAt, p->dcol, p->stream);  // the norms exist, the scaling does not
    CHK(hipGetLastError());
  } else if ((st = ensure_scaling(p))) {
    return st;
  }
  CHK(hipMemcpyAsync(d, p->dcol, static_cast<size_t>(p->n) * 8, hipMemcpyDeviceToDevice, p->stream));
  CHK(hipStreamSynchronize(p->stream));
  return COND_OK;
}

int cond_plan_inverse_apply(cond_plan_t* p, const double* x, double* r, double* s) {
  if (!p || !x || !r || !s) return fail(COND_EINVAL, "null argument");
  if (!p->bound) return fail(COND_ESTATE, "plan not bound");
  if (!p->want_min) return fail(COND_ESTATE, "plan has no LU (sigma_min_method = NONE)");
  int st0 = join_user_stream(p);
  if (st0) return st0;
  hipStream_t st = p->stream;
  rearm_after_timeout(p);
  CHK(hipMemsetAsync(p->st_free, 0, sizeof(RunState), st));
  if (p->inject_timeout) launch_set_int(&p->st_free->abort_wait, 1, st);
  p->inject_timeout = false;
  launch_zero_u32(p->tickets, 4 * kSolveTickets, st);
  launch_fill(p->n, p->c, kPending, st);
  launch_fill(p->n, p->z, kPending, st);
  launch_fill(p->n, p->h, kPending, st);
  launch_fill(p->n, p->wv, kPending, st);
  launch_trsv(p->dL, x, p->d_row_perm, p->c, nullptr, nullptr, p->tickets, p->st_free, st);
  launch_trsv(p->dU, p->c, p->d_rev, p->z, r, p->d_scat_r, tix(p->tickets, 1), p->st_free, st);
  launch_trsv(p->dUt, p->z, p->d_rev, p->h, nullptr, nullptr, tix(p->tickets, 2), p->st_free, st);
  launch_trsv(p->dLt, p->h, p->d_rev, p->wv, s, p->d_scat_s, tix(p->tickets, 3), p->st_free, st);
  CHK(hipGetLastError());
  RunState hs;
  CHK(hipMemcpyAsync(&hs, p->st_free, sizeof(RunState), hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  if (hs.abort_wait) {
    p->rearm_slots = true;
    return fail(COND_ETIMEOUT, "triangular-solve wait timed out");
  }
  return COND_OK;
}

int cond_plan_inject_timeout(cond_plan_t* p) {
  if (!p) return fail(COND_EINVAL, "null plan");
  if (!p->want_min) return fail(COND_EINVAL, "the plan has no sigma_min route");
  p->inject_timeout = true;
  return COND_OK;
}

int cond_stream_triad(int64_t n, double* a, const double* b, const double* c, double scale,
                      int32_t grid, int32_t reps, void* stream, double* ms) {
  if (!a || !b || !c || !ms || n < 1 || grid < 1 || reps < 1)
    return fail(COND_EINVAL, "invalid triad arguments");
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
       reinterpret_cast<uintptr_t>(c)) % 16)
    return fail(COND_EINVAL, "triad arrays must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CHK(hipEventCreate(&e0));
  CHK(hipEventCreate(&e1));
  launch_triad(n, a, b, c, scale, grid, s);  // warm-up
  hipError_t e = hipEventRecord(e0, s);
  for (int32_t r = 0; r < reps && e == hipSuccess; ++r) {
    launch_triad(n, a, b, c, scale, grid, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return fail(COND_EHIP, std::string("triad: ") + hipGetErrorString(e));
  *ms = static_cast<double>(t) / reps;
  return COND_OK;
}

int cond_plan_error_bounds(cond_plan_t* p, const double* x_hat, const double* b, double kappa,
                           double norm_a, cond_bounds_t* out) {
  if (!p || !x_hat || !b || !out) return fail(COND_EINVAL, "null argument");
  if (!p->bound) return fail(COND_ESTATE, "plan not bound");
  if (!(kappa >= 1.0) || !std::isfinite(kappa) || !(norm_a > 0.0) || !std::isfinite(norm_a))
    return fail(COND_EINVAL, "kappa must be >= 1 and norm_a > 0, both finite");
  int st;
  if ((st = join_user_stream(p))) return st;
  // the partials go to three of the run's partial arrays, the sums to the fourth
  static_assert(kMaxParts * 8 % kAlign == 0, "partial arrays are contiguous");
  double* parts = p->parts_x;
  if (p->parts_y != parts + kMaxParts || p->parts_xd != parts + 2 * kMaxParts)
    return fail(COND_ESTATE, "partial arrays are not contiguous");
  launch_residual(p->n, p->dA.rowptr, p->dA.idx64, p->dA.col, p->dA.val, x_hat, b, parts,
                  p->parts_xx, p->grid, p->stream);
  CHK(hipGetLastError());
  double sums[3];
  CHK(hipMemcpyAsync(sums, p->parts_xx, sizeof(sums), hipMemcpyDeviceToHost, p->stream));
  CHK(hipStreamSynchronize(p->stream));
  if ((st = fill_bounds(sums, kappa, norm_a, out))) return fail(st, "zero or non-finite norm");
  return COND_OK;
}

int cond_estimate(const cond_csr_t* A, const cond_opts_t* o, const double* x0_max,
                  const double* x0_min, void* stream, cond_result_t* out) {
  cond_plan_t* p = nullptr;
  int st = cond_plan_create(A, o, &p);
  if (st) return st;
  st = cond_plan_bind(p, nullptr, 0, stream);
  if (!st) st = cond_plan_run(p, o, x0_max, x0_min, out, nullptr, nullptr, nullptr, nullptr);
  cond_plan_destroy(p);
  return st;
}

}  // extern "C"
