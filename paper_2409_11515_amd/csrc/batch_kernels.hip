// Batched, multi-start Projected Adam (sigma_max run) for gfx950.
//
// A batch is many matrices of uneven size, each with K starts. The matrices
// are concatenated block-diagonally (matrix m owns rows [row0[m], row0[m+1]))
// and the K starts of a row are interleaved: x[i*K + k]. One launch per phase
// then covers every matrix and every start, and one read of a matrix entry
// serves all K starts. The arithmetic of every (matrix, start) pair is the
// plain method's Algorithm 1; only the order of additions inside the global
// sums differs.
//
// Rows are cut into tiles that never cross a matrix boundary. Each tile
// writes K partial sums into its own slots; a per-matrix reduction kernel
// (one block per matrix) adds a matrix's tile partials in tile order, so the
// scalars are deterministic. The same kernel runs the per-pair bookkeeping of
// Algorithm 1: evaluation of the previous iterate, best tracking, the stop
// rule, retirement of a finished pair.

#include "batch.hpp"
#include "condest.h"

namespace condest {

namespace {

constexpr int kB = 256;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double bsum(double v) {
  __shared__ double red[kB / 64];
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int k = 1; k < kB / 64; ++k) r += red[k];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void tile_range(int ntiles, long long& t0, long long& t1) {
  const int b = blockIdx.x, g = gridDim.x;
  const int lb = (g % 8 == 0) ? (b % 8) * (g / 8) + b / 8 : b;
  t0 = static_cast<long long>(ntiles) * lb / g;
  t1 = static_cast<long long>(ntiles) * (lb + 1) / g;
}

// The tiles of the matrices that still have a running start ("live" tiles),
// numbered u = 0..nlive-1 in matrix order, are split over the XCDs in
// contiguous eighths, and inside an XCD dealt to its blocks round-robin
// (block j of the XCD takes live tiles j, j + g/8, ...), so the blocks of one
// XCD sweep neighbouring rows together and share the gathered vector entries
// in that XCD's L2; live tile u maps to tile mat_tile0[live_mat[j]] +
// (u - live_pref[j]) for the j with live_pref[j] <= u < live_pref[j+1].
// Once every start of a matrix has stopped, no element kernel visits its
// tiles again.
struct LiveTiles {
  long long u, u1;
  int j, step;
  __device__ __forceinline__ void begin(const BatchArgs& a) {
    const long long n = a.g->nlive;
    const int b = blockIdx.x, g = gridDim.x;
    if (g % 8 == 0) {
      const int x = b % 8;
      u = n * x / 8 + b / 8;
      u1 = n * (x + 1) / 8;
      step = g / 8;
    } else {
      u = b;
      u1 = n;
      step = g;
    }
    j = 0;
  }
  __device__ __forceinline__ void next() { u += step; }
  // the tile of live index u (advancing j), or -1 past the block's share
  __device__ __forceinline__ long long tile(const BatchArgs& a) {
    if (u >= u1) return -1;
    while (u >= a.live_pref[j + 1]) ++j;
    return a.mat_tile0[a.live_mat[j]] + (u - a.live_pref[j]);
  }
};

// Per-tile partial sums of K values, lane k of each 8-lane group owning start
// k (K == 8). The lanes of one start inside a wave are added by a fixed
// butterfly, then the block's waves in wave order: the same order on every
// run.
template <int K>
__device__ __forceinline__ void tile_partials(double acc, int tile, double* parts) {
  static_assert(K == 8, "one start per lane of an 8-lane group");
  __shared__ double red[(kB / 64) * K];
#pragma unroll
  for (int off = K; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
  const int lane = threadIdx.x & 63;
  if (lane < K) red[(threadIdx.x >> 6) * K + lane] = acc;
  __syncthreads();
  if (threadIdx.x < K) {
    double s = red[threadIdx.x];
#pragma unroll
    for (int w = 1; w < kB / 64; ++w) s += red[w * K + threadIdx.x];
    parts[static_cast<long long>(tile) * K + threadIdx.x] = s;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ init
template <int K>
__global__ __launch_bounds__(kB) void b_init_k(BatchArgs a, const double* __restrict__ x0) {
  long long t0, t1;
  tile_range(a.ntiles, t0, t1);
  const int k = threadIdx.x % K;
  for (long long t = t0; t < t1; ++t) {
    const long long r0 = a.tiles[t], r1 = a.tiles[t + 1];
    double acc = 0.0;
    for (long long e = r0 * K + threadIdx.x; e < r1 * K; e += kB) {
      const double xi = x0[e];
      a.x[e] = xi;
      a.m[e] = 0.0;
      a.v[e] = 0.0;
      acc += xi * xi;
    }
    tile_partials<K>(acc, static_cast<int>(t), a.parts_xx);
  }
  // no update of this run has seen the running matrices: the first one
  // finds them changed (and cuts the solves' lists down if some have stopped)
  if (blockIdx.x == 0 && a.mat_live)
    for (int m = threadIdx.x; m < a.nmat; m += kB) a.mat_live[m] = -1;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.g->t_done = 0;
    a.g->b1t = 1.0;
    a.g->b2t = 1.0;
    a.g->stop_all = 0;
    a.g->abort_wait = 0;
  }
}

// ------------------------------------------------------------ live tiles
// One block: matrices with a running start, and the prefix of their tile counts.
template <int K>
__global__ __launch_bounds__(kB) void b_live_k(BatchArgs a) {
  __shared__ int run_sh[kB / K];
  __shared__ int j_sh, u_sh, changed_sh;
  if (threadIdx.x == 0) j_sh = u_sh = changed_sh = 0;
  // matrices in rounds of kB / K: one thread per pair reads its state, then
  // thread 0 appends the running matrices of the round in order
  for (int m0 = 0; m0 < a.nmat; m0 += kB / K) {
    if (threadIdx.x < kB / K) run_sh[threadIdx.x] = 0;
    __syncthreads();
    const int m = m0 + static_cast<int>(threadIdx.x) / K;
    if (m < a.nmat && !a.pairs[static_cast<long long>(m) * K + threadIdx.x % K].stopped)
      run_sh[threadIdx.x / K] = 1;  // benign: every writer stores 1
    __syncthreads();
    if (a.mat_live && threadIdx.x < kB / K && m0 + static_cast<int>(threadIdx.x) < a.nmat) {
      if (a.mat_live[m0 + threadIdx.x] != run_sh[threadIdx.x]) changed_sh = 1;  // benign
      a.mat_live[m0 + threadIdx.x] = run_sh[threadIdx.x];
    }
    if (threadIdx.x == 0) {
      int j = j_sh, u = u_sh;
      for (int q = 0; q < kB / K && m0 + q < a.nmat; ++q)
        if (run_sh[q]) {
          a.live_mat[j] = m0 + q;
          a.live_pref[j] = u;
          u += a.mat_tile0[m0 + q + 1] - a.mat_tile0[m0 + q];
          ++j;
        }
      j_sh = j;
      u_sh = u;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.live_pref[j_sh] = u_sh;
    a.g->nlive = u_sh;
    a.g->stop_all = u_sh == 0 ? 1 : 0;
    a.g->live_changed = changed_sh;
    a.g->compact = j_sh < a.nmat ? 1 : 0;
  }
}

// ---------------------------------------------------------------- compaction
// Block (f, l) cuts list l of solve f down to the slots of the running
// matrices, keeping their order: 1024 slots at a time, each wave counts its
// running slots by a ballot, the waves' counts are added in wave order, and
// every running slot is written at its rank. Only when the running matrices
// changed this update and some matrix has stopped; the solves then take the
// compacted lists (each a subsequence of a list in dependency order, with
// every task of the running matrices: the waits still end).
constexpr int kCompactBlock = 1024;

__global__ __launch_bounds__(kCompactBlock) void b_compact_k(BatchArgs a, BatchLists lists) {
  if (!a.g->live_changed || !a.g->compact) return;
  const int f = blockIdx.x / kTaskLists, l = blockIdx.x % kTaskLists;
  const int q0 = lists.list_off[f][l], q1 = lists.list_off[f][l + 1];
  const int* group = lists.slot_group[f];
  int* out = lists.cl_slots[f];
  __shared__ int wave_sh[kCompactBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int base = 0;
  for (int c = q0; c < q1; c += kCompactBlock) {
    const int q = c + static_cast<int>(threadIdx.x);
    const bool run = q < q1 && a.mat_live[group[q]];
    const unsigned long long mask = __ballot(run);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wave_sh[wave] = __popcll(mask);
    __syncthreads();
    int wbase = 0, total = 0;
    for (int w = 0; w < kCompactBlock / 64; ++w) {
      if (w < wave) wbase += wave_sh[w];
      total += wave_sh[w];
    }
    if (run) out[q0 + base + wbase + before] = q;
    base += total;
    __syncthreads();  // wave_sh is reused
  }
  if (threadIdx.x == 0) lists.cl_cnt[f * kTaskLists + l] = base;
}

// --------------------------------------------------------- per-matrix reduce
// mode 0: after pass 2 (or init): nrm[p] = sqrt(sum ||x||^2)
// mode 1: after spmv(A): evaluation, best tracking, stop rule (needs x.x, y.y)
// mode 2: after pass 1: xd[p] = sum x.dx
template <int K>
__global__ __launch_bounds__(kB) void b_reduce_k(BatchArgs a, int mode, AdamParams p) {
  const int mat = blockIdx.x;
  const int t0 = a.mat_tile0[mat], t1 = a.mat_tile0[mat + 1];
  __shared__ double sh[K][3];
  const double* src0 = mode == 0 ? a.parts_xx : (mode == 1 ? a.parts_x : a.parts_xd);
  for (int src = 0; src < (mode == 1 ? 2 : 1); ++src) {
    const double* parts = src == 0 ? src0 : a.parts_y;
    // thread layout: K starts x (kB / K) strided tiles, then a fixed-order combine
    // (eight loads issued before their eight additions, in the same order)
    constexpr int S = kB / K;
    const int k = threadIdx.x % K, lane_t = threadIdx.x / K;
    double acc = 0.0;
    int t = t0 + lane_t;
    for (; t + 7 * S < t1; t += 8 * S) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = parts[static_cast<long long>(t + u * S) * K + k];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; t < t1; t += S) acc += parts[static_cast<long long>(t) * K + k];
    __shared__ double red[kB];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < K) {
      double s = 0.0;
      for (int u = threadIdx.x; u < kB; u += K) s += red[u];
      sh[threadIdx.x][src] = s;
    }
    __syncthreads();
  }
  if (threadIdx.x >= K) return;
  const int k = threadIdx.x;
  const long long pr = static_cast<long long>(mat) * K + k;  // pair index
  BatchPair& q = a.pairs[pr];
  if (mode == 0) {
    q.nrm = sqrt(sh[k][0]);
    return;
  }
  if (mode == 2) {
    q.xd = sh[k][0];
    return;
  }
  // mode 1: the evaluation and bookkeeping of Algorithm 1 for this pair
  if (q.stopped) {
    q.improved = 0;
    return;
  }
  const long long t = a.g->t_done + 1;
  const double nx2 = sh[k][0], ny2 = sh[k][1];
  q.nx2 = nx2;
  q.ny2 = ny2;
  q.improved = 0;
  if (a.g->abort_wait) {
    q.stopped = 1;
    q.status = COND_ETIMEOUT;
    q.iters = t - 1;
    return;
  }
  if (!(nx2 > 0.0) || !(ny2 > 0.0) || !isfinite(nx2) || !isfinite(ny2)) {
    q.stopped = 1;
    q.status = COND_ENUMERIC;
    q.iters = t - 1;
    return;
  }
  if (t >= 2) {
    const double sigma = sqrt(ny2 / nx2);
    if (sigma > q.best) {
      q.best = sigma;
      q.improved = 1;
    }
    const long long T = t - 1;
    if (a.trace) a.trace[pr * p.max_iter + (T - 1)] = q.best;
    if (T >= p.max_iter) {
      q.stopped = 1;
      q.iters = T;
      q.flags |= static_cast<int>(COND_F_MAXITER);
    } else if (p.stop_window > 0 && p.stop_rtol > 0.0 && T % p.stop_window == 0) {
      if (T >= 2 * p.stop_window && q.best - q.ckpt <= p.stop_rtol * q.best) {
        if (p.alpha_min > 0.0 && q.alpha > p.alpha_min) {
          q.alpha = fmax(q.alpha * p.alpha_decay, p.alpha_min);  // plateau: smaller step
        } else {
          q.stopped = 1;
          q.iters = T;
        }
      }
      q.ckpt = q.best;
    }
  }
}

// --------------------------------------------------------------- normalise
template <int K>
__global__ __launch_bounds__(kB) void b_normalise_k(BatchArgs a) {
#pragma clang fp contract(off)
  LiveTiles lt;
  lt.begin(a);
  const int k = threadIdx.x % K;
  for (long long t = lt.tile(a); t >= 0; lt.next(), t = lt.tile(a)) {
    const int mat = a.tile_mat[t];
    const BatchPair& q = a.pairs[static_cast<long long>(mat) * K + k];
    const long long r0 = a.tiles[t], r1 = a.tiles[t + 1];
    double acc = 0.0;
    if (!q.stopped) {
      const double nrm = q.nrm;
      for (long long e = r0 * K + threadIdx.x; e < r1 * K; e += kB) {
        const double xi = a.x[e] / nrm;
        a.x[e] = xi;
        acc += xi * xi;
      }
    }
    tile_partials<K>(acc, static_cast<int>(t), a.parts_x);
  }
}

// -------------------------------------------------------------------- spmm
// Y = M X for K interleaved starts. A tile's column indices, values and row
// pointers are first copied into LDS by coalesced streaming loads (when the
// tile has at most kSpmmStage entries; a larger tile reads them from memory
// row by row). Thread t then takes row t / K of a 32-row chunk and start
// t % K and walks that row: the K threads of a row read the same staged
// index and value and K contiguous entries of X (64 bytes), so one read of
// the matrix serves all starts. Starts that have stopped are skipped, and a
// tile whose matrix has no running start is skipped entirely. Y is written
// with streaming stores (nothing reads it before the next kernel).
constexpr int kChunkRowsB = kB / 8;  // 32 rows x 8 starts
constexpr int kSpmmStage = 1536;     // entries staged per tile (18 KB of LDS)
constexpr int kTileMaxRows = 256;    // the largest row tile the autotuner tries

template <int K>
__global__ __launch_bounds__(kB) void b_spmm_k(BatchArgs a, const int* __restrict__ rowptr,
                                               const int* __restrict__ col,
                                               const double* __restrict__ val,
                                               const double* __restrict__ x, double* __restrict__ y,
                                               double* __restrict__ parts) {
#pragma clang fp contract(off)  // products rounded, then added in entry order, as in the plain SpMV
  __shared__ int c_sh[kSpmmStage];
  __shared__ double v_sh[kSpmmStage];
  __shared__ int rp_sh[kTileMaxRows + 1];
  LiveTiles lt;
  lt.begin(a);
  const int k = threadIdx.x % K;
  const int rl = threadIdx.x / K;  // row of this thread inside a chunk
  for (long long t = lt.tile(a); t >= 0; lt.next(), t = lt.tile(a)) {
    const int mat = a.tile_mat[t];
    const bool mine = !a.pairs[static_cast<long long>(mat) * K + k].stopped;
    const long long r0 = a.tiles[t], r1 = a.tiles[t + 1];
    const int e0 = rowptr[r0];
    const int ne = rowptr[r1] - e0;
    const bool staged = ne <= kSpmmStage && r1 - r0 <= kTileMaxRows;
    if (staged) {
      for (int e = threadIdx.x; e < ne; e += kB) {
        c_sh[e] = __builtin_nontemporal_load(col + e0 + e);
        v_sh[e] = __builtin_nontemporal_load(val + e0 + e);
      }
      for (int i = threadIdx.x; i <= r1 - r0; i += kB) rp_sh[i] = rowptr[r0 + i] - e0;
    }
    __syncthreads();
    double sq = 0.0;
    if (mine) {
      for (long long r = r0 + rl; r < r1; r += kChunkRowsB) {
        double acc = 0.0;
        if (staged) {
          const int p0 = rp_sh[r - r0], p1 = rp_sh[r - r0 + 1];
          int q = p0;
          for (; q + 4 <= p1; q += 4) {
            const double x0 = x[static_cast<long long>(c_sh[q]) * K + k];
            const double x1 = x[static_cast<long long>(c_sh[q + 1]) * K + k];
            const double x2 = x[static_cast<long long>(c_sh[q + 2]) * K + k];
            const double x3 = x[static_cast<long long>(c_sh[q + 3]) * K + k];
            acc += v_sh[q] * x0;
            acc += v_sh[q + 1] * x1;
            acc += v_sh[q + 2] * x2;
            acc += v_sh[q + 3] * x3;
          }
          for (; q < p1; ++q) acc += v_sh[q] * x[static_cast<long long>(c_sh[q]) * K + k];
        } else {
          const int p0 = rowptr[r], p1 = rowptr[r + 1];
          for (int q = p0; q < p1; ++q) acc += val[q] * x[static_cast<long long>(col[q]) * K + k];
        }
        __builtin_nontemporal_store(acc, y + r * K + k);
        sq += acc * acc;
      }
    }
    __syncthreads();  // the staged tile is replaced next
    if (parts) tile_partials<K>(sq, static_cast<int>(t), parts);
  }
}

// ----------------------------------------------------------------- pass 1
template <int K>
__global__ __launch_bounds__(kB) void b_pass1_k(BatchArgs a, AdamParams p) {
#pragma clang fp contract(off)
  LiveTiles lt;
  lt.begin(a);
  const int k = threadIdx.x % K;
  const double b1 = p.beta1, b2 = p.beta2;
  const double b1t = a.g->b1t * b1, b2t = a.g->b2t * b2;
  for (long long t = lt.tile(a); t >= 0; lt.next(), t = lt.tile(a)) {
    const int mat = a.tile_mat[t];
    const BatchPair& q = a.pairs[static_cast<long long>(mat) * K + k];
    const long long r0 = a.tiles[t], r1 = a.tiles[t + 1];
    double acc = 0.0;
    if (q.improved && a.xbest)
      for (long long e = r0 * K + threadIdx.x; e < r1 * K; e += kB) a.xbest[e] = a.x[e];
    if (!q.stopped) {
      const double nx2 = q.nx2, ny2 = q.ny2;
      for (long long e = r0 * K + threadIdx.x; e < r1 * K; e += kB) {
        const double xi = a.x[e];
        const double g = xi / nx2 - a.w[e] / ny2;
        const double mi = b1 * a.m[e] + (1.0 - b1) * g;
        const double vi = b2 * a.v[e] + (1.0 - b2) * (g * g);
        const double mh = mi / (1.0 - b1t);
        const double vh = vi / (1.0 - b2t);
        const double di = q.alpha * mh / (sqrt(vh) + p.eps);
        a.m[e] = mi;
        a.v[e] = vi;
        a.d[e] = di;
        acc += xi * di;
      }
    }
    tile_partials<K>(acc, static_cast<int>(t), a.parts_xd);
  }
}

// ----------------------------------------------------------------- pass 2
template <int K>
__global__ __launch_bounds__(kB) void b_pass2_k(BatchArgs a, AdamParams p) {
#pragma clang fp contract(off)
  LiveTiles lt;
  lt.begin(a);
  const int k = threadIdx.x % K;
  for (long long t = lt.tile(a); t >= 0; lt.next(), t = lt.tile(a)) {
    const int mat = a.tile_mat[t];
    const BatchPair& q = a.pairs[static_cast<long long>(mat) * K + k];
    const long long r0 = a.tiles[t], r1 = a.tiles[t + 1];
    double acc = 0.0;
    if (!q.stopped) {
      const double xd = q.xd;
      for (long long e = r0 * K + threadIdx.x; e < r1 * K; e += kB) {
        const double xi = a.x[e];
        const double dd = a.d[e] - xd * xi;
        const double xn = xi - dd;
        a.x[e] = xn;
        acc += xn * xn;
      }
    }
    tile_partials<K>(acc, static_cast<int>(t), a.parts_xx);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.g->t_done = a.g->t_done + 1;
    a.g->b1t = a.g->b1t * p.beta1;
    a.g->b2t = a.g->b2t * p.beta2;
  }
}

// ------------------------------------------------------- sigma_min route
// Re-arm the solves' vectors with the not-yet-solved pattern and reset their
// ticket counters before the four solves of an update.
// Only the rows of matrices with a running start: the solves skip the rest.
// c and h are in pivot order (tile t's rows), z and wv reversed (its mirror).
__global__ __launch_bounds__(kB) void b_rearm_k(BatchArgs a) {
  if (blockIdx.x == 0)
    for (int c = threadIdx.x; c < 4 * kTaskLists; c += kB) a.tickets[c * kTicketStride] = 0u;
  if (a.g->stop_all) return;
  unsigned long long* c = reinterpret_cast<unsigned long long*>(a.c);
  unsigned long long* z = reinterpret_cast<unsigned long long*>(a.z);
  unsigned long long* h = reinterpret_cast<unsigned long long*>(a.h);
  unsigned long long* wv = reinterpret_cast<unsigned long long*>(a.wv);
  LiveTiles lt;
  lt.begin(a);
  for (long long t = lt.tile(a); t >= 0; lt.next(), t = lt.tile(a)) {
    const long long r0 = a.tiles[t], r1 = a.tiles[t + 1];
    const long long m0 = a.nrows - r1;  // the mirrored rows
    for (long long e = threadIdx.x; e < (r1 - r0) * kBatchK; e += kB) {
      c[r0 * kBatchK + e] = kPending;
      h[r0 * kBatchK + e] = kPending;
      z[m0 * kBatchK + e] = kPending;
      wv[m0 * kBatchK + e] = kPending;
    }
  }
}

// ||A^-1 x||^2 per (tile, start): z is the U solve's output in reversed pivot
// order, and the merged factors keep each matrix's pivot rows together, so
// tile t's mirrored rows belong to the same matrix.
template <int K>
__global__ __launch_bounds__(kB) void b_sumsq_rev_k(BatchArgs a) {
  LiveTiles lt;
  lt.begin(a);
  const int k = threadIdx.x % K;
  for (long long t = lt.tile(a); t >= 0; lt.next(), t = lt.tile(a)) {
    const int mat = a.tile_mat[t];
    const BatchPair& q = a.pairs[static_cast<long long>(mat) * K + k];
    const long long r0 = a.nrows - a.tiles[t + 1], r1 = a.nrows - a.tiles[t];
    double acc = 0.0;
    if (!q.stopped)
      for (long long e = r0 * K + threadIdx.x; e < r1 * K; e += kB) {
        const double zi = a.z[e];
        acc += zi * zi;
      }
    tile_partials<K>(acc, static_cast<int>(t), a.parts_y);
  }
}

}  // namespace

void batch_launch_init(const BatchArgs& a, const double* x0, int grid, hipStream_t s) {
  b_init_k<kBatchK><<<grid, kB, 0, s>>>(a, x0);
}
void batch_launch_live(const BatchArgs& a, hipStream_t s) {
  b_live_k<kBatchK><<<1, kB, 0, s>>>(a);
}
void batch_launch_reduce(const BatchArgs& a, int mode, const AdamParams& p, hipStream_t s) {
  b_reduce_k<kBatchK><<<a.nmat, kB, 0, s>>>(a, mode, p);
}
void batch_launch_normalise(const BatchArgs& a, int grid, hipStream_t s) {
  b_normalise_k<kBatchK><<<grid, kB, 0, s>>>(a);
}
void batch_launch_spmm(const BatchArgs& a, int transpose, int grid, hipStream_t s) {
  if (transpose)
    b_spmm_k<kBatchK><<<grid, kB, 0, s>>>(a, a.at_rowptr, a.at_col, a.at_val, a.y, a.w, nullptr);
  else
    b_spmm_k<kBatchK><<<grid, kB, 0, s>>>(a, a.a_rowptr, a.a_col, a.a_val, a.x, a.y, a.parts_y);
}
void batch_launch_pass1(const BatchArgs& a, const AdamParams& p, int grid, hipStream_t s) {
  b_pass1_k<kBatchK><<<grid, kB, 0, s>>>(a, p);
}
void batch_launch_pass2(const BatchArgs& a, const AdamParams& p, int grid, hipStream_t s) {
  b_pass2_k<kBatchK><<<grid, kB, 0, s>>>(a, p);
}

void batch_launch_rearm(const BatchArgs& a, int grid, hipStream_t s) {
  b_rearm_k<<<grid, kB, 0, s>>>(a);
}
void batch_launch_compact(const BatchArgs& a, const BatchLists& l, hipStream_t s) {
  b_compact_k<<<4 * kTaskLists, kCompactBlock, 0, s>>>(a, l);
}
void batch_launch_sumsq_rev(const BatchArgs& a, int grid, hipStream_t s) {
  b_sumsq_rev_k<kBatchK><<<grid, kB, 0, s>>>(a);
}

}  // namespace condest
