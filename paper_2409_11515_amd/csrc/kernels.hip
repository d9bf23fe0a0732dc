// HIP kernels for gfx950 (iteration layout and conventions in kernels.hpp).
//
// Row ranges: every fixed-grid kernel gives block b the contiguous row range
// of logical block lb = (b % 8) * (grid / 8) + b / 8 (grid a multiple of 8).
// The hardware hands consecutive block ids to the 8 XCDs in turn, so the
// logical ranges of one XCD are adjacent and the gathers of a banded matrix
// stay inside that XCD's L2.

#include "condest.h"
#include "kernels.hpp"

namespace condest {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
  // xor butterfly: every lane ends with the same, order-fixed sum
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block; every thread gets the same value. Fixed order.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / 64];
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int k = 1; k < kBlock / 64; ++k) r += red[k];
  __syncthreads();
  return r;
}

// Sum of the `count` partial slots; identical in every block.
__device__ __forceinline__ double sum_parts(const double* parts, int count) {
  double acc = 0.0;
  for (int k = threadIdx.x; k < count; k += kBlock) acc += parts[k];
  return block_sum(acc);
}

__device__ __forceinline__ int logical_block() {
  const int b = blockIdx.x, g = gridDim.x;
  return (g % 8 == 0) ? (b % 8) * (g / 8) + b / 8 : b;
}

__device__ __forceinline__ void block_range(long long n, int lb, long long& r0, long long& r1) {
  r0 = n * lb / gridDim.x;
  r1 = n * (lb + 1) / gridDim.x;
}

// ------------------------------------------------------------------ init
__global__ __launch_bounds__(kBlock) void init_k(int n, const double* __restrict__ x0,
                                                 double* __restrict__ x, double* __restrict__ m,
                                                 double* __restrict__ v, double* __restrict__ parts_xx,
                                                 RunState* st, double alpha0, int minimise) {
  const int lb = logical_block();
  long long r0, r1;
  block_range(n, lb, r0, r1);
  double acc = 0.0;
  for (long long i = r0 + threadIdx.x; i < r1; i += kBlock) {
    const double xi = x0[i];
    x[i] = xi;
    m[i] = 0.0;
    v[i] = 0.0;
    acc += xi * xi;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) parts_xx[lb] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // below (above, when minimising) any norm ratio: the first evaluation
    // always improves
    const double start = minimise ? __longlong_as_double(0x7FF0000000000000ll) : -1.0;
    st->best = start;
    st->best_next = start;
    st->b1t = 1.0;
    st->b2t = 1.0;
    st->t_done = 0;
    st->iters = 0;
    st->stop_req = 0;
    st->done = 0;
    st->status = 0;
    st->flags = 0;
    st->abort_wait = 0;
    st->ckpt = start;
    st->ckpt_next = start;
    st->alpha = alpha0;
    st->alpha_next = alpha0;
  }
}

// ------------------------------------------------------------ normalise
// x <- x / ||x|| (the last step of Algorithm 1's update), partials of x.x for
// the next gradient; optionally re-arms the triangular-solve vectors.
struct Resets {
  double* p[4];
  int count;
};

__global__ __launch_bounds__(kBlock) void normalise_k(int n, double* __restrict__ x,
                                                      const double* __restrict__ parts_xx, int np,
                                                      double* __restrict__ parts_x, RunState* st,
                                                      Resets resets, unsigned* tickets, int ntickets) {
#pragma clang fp contract(off)
  if (st->stop_req) return;
  const double nrm = sqrt(sum_parts(parts_xx, np));
  const int lb = logical_block();
  long long r0, r1;
  block_range(n, lb, r0, r1);
  double acc = 0.0;
  for (long long i = r0 + threadIdx.x; i < r1; i += kBlock) {
    const double xi = x[i] / nrm;
    x[i] = xi;
    acc += xi * xi;
  }
  for (int k = 0; k < resets.count; ++k) {
    unsigned long long* p = reinterpret_cast<unsigned long long*>(resets.p[k]);
    for (long long i = r0 + threadIdx.x; i < r1; i += kBlock) p[i] = kPending;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) parts_x[lb] = s;
  // the solves' ticket counters: kTaskLists per solve, kTicketStride apart
  if (blockIdx.x == 0)
    for (int c = threadIdx.x; c < ntickets * kTaskLists; c += kBlock) tickets[c * kTicketStride] = 0u;
}

// ---------------------------------------------------------- spmv (stream)
// y = A x by row tiles: the host cuts the rows into tiles of at most 256 rows
// and kStreamCap entries (a longer row is a tile of its own). A block streams
// a tile's entries with fully coalesced loads of col/val, gathers x and
// parks the products in LDS, then thread t adds up the products of row t.
// A tile holding one long row is summed by the whole block. Each block owns
// a contiguous range of tiles; partial sums of y.y are written per block.
constexpr int kStreamCap = 2048;
constexpr int kTileRows = 256;

//
// Column scaling (SC): y = R A C x with C = diag(cs) applied to the gathered
// x (cs may be null: no column factor) and R = diag(rs) to each row's sum (rs
// may be null). A D^-1 is then cs = 1/d on A, and (A D^-1)^T = D^-1 A^T is
// rs = 1/d on the stored A^T.
template <typename IT, bool SC>
__global__ __launch_bounds__(kBlock) void spmv_stream_k(
    int ntiles, const int* __restrict__ tiles, const IT* __restrict__ rowptr,
    const int* __restrict__ col, const double* __restrict__ val, const double* __restrict__ x,
    double* __restrict__ y, double* __restrict__ parts, const RunState* st,
    const double* __restrict__ cs, const double* __restrict__ rs) {
  if (st && st->stop_req) return;
  __shared__ double prod[kStreamCap];
  __shared__ IT rp_sh[kTileRows + 1];
  const int lb = logical_block();
  long long t0, t1;
  block_range(ntiles, lb, t0, t1);
  double sq = 0.0;
  for (long long t = t0; t < t1; ++t) {
    const int ra = tiles[t], rb = tiles[t + 1];
    const int cnt = rb - ra;
    for (int k = threadIdx.x; k <= cnt; k += kBlock) rp_sh[k] = rowptr[ra + k];
    __syncthreads();
    const IT e0 = rp_sh[0];
    const IT ne = rp_sh[cnt] - e0;
    if (ne <= kStreamCap) {
#pragma unroll 4
      for (int e = threadIdx.x; e < static_cast<int>(ne); e += kBlock) {
        const int c = col[e0 + e];
        prod[e] = val[e0 + e] * ((SC && cs) ? x[c] * cs[c] : x[c]);
      }
      __syncthreads();
      if (threadIdx.x < cnt) {
        const int a = static_cast<int>(rp_sh[threadIdx.x] - e0);
        const int b = static_cast<int>(rp_sh[threadIdx.x + 1] - e0);
        double s = 0.0;
        for (int e = a; e < b; ++e) s += prod[e];
        if (SC && rs) s *= rs[ra + threadIdx.x];
        y[ra + threadIdx.x] = s;
        sq += s * s;
      }
    } else {
      // one long row: every thread takes a strided share, then a block sum
      double acc = 0.0;
      for (IT e = e0 + threadIdx.x; e < e0 + ne; e += kBlock) {
        const int c = col[e];
        acc += val[e] * ((SC && cs) ? x[c] * cs[c] : x[c]);
      }
      acc = block_sum(acc);
      if (SC && rs) acc *= rs[ra];
      if (threadIdx.x == 0) {
        y[ra] = acc;
        sq += acc * acc;
      }
    }
    __syncthreads();  // rp_sh and prod are reused by the next tile
  }
  if (parts) {
    const double s = block_sum(sq);
    if (threadIdx.x == 0) parts[lb] = s;
  }
}

// ------------------------------------------------------------ row norms
// out[i] = ||row i||_2 (16 lanes per row); on the stored A^T these are the
// column norms of A, the D_col of column scaling.
template <typename IT>
__global__ __launch_bounds__(kBlock) void row_norms_k(int n, const IT* __restrict__ rowptr,
                                                      const double* __restrict__ val,
                                                      double* __restrict__ out) {
  constexpr int kRowLanes = 16;
  const int sub = threadIdx.x & (kRowLanes - 1);
  const long long stride = static_cast<long long>(gridDim.x) * (kBlock / kRowLanes);
  for (long long i = blockIdx.x * static_cast<long long>(kBlock / kRowLanes) + threadIdx.x / kRowLanes;
       i < n; i += stride) {
    double acc = 0.0;
    for (IT e = rowptr[i] + sub; e < rowptr[i + 1]; e += kRowLanes) acc += val[e] * val[e];
#pragma unroll
    for (int off = kRowLanes / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kRowLanes);
    if (sub == 0) out[i] = sqrt(acc);
  }
}

// dinv = 1/d; dz[k] = d[perm[k]] (perm may be null: no dz), the factor of
// the solves' reversed-order vector.
__global__ __launch_bounds__(kBlock) void scale_prep_k(int n, const double* __restrict__ d,
                                                       double* __restrict__ dinv,
                                                       const int* __restrict__ perm,
                                                       double* __restrict__ dz) {
  for (long long i = blockIdx.x * static_cast<long long>(kBlock) + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * kBlock) {
    dinv[i] = 1.0 / d[i];
    if (perm) dz[i] = d[perm[i]];
  }
}

// The sigma_min run of the column-scaled matrix: (A D^-1)^-1 = D A^-1. The
// solve's output z (r = A^-1 x in reversed pivot order) becomes z <- dz z,
// i.e. D r, whose squared norm goes to the partials; zz = dz z (= D D r) is
// the right-hand side of the transposed solves, since (D A^-1)^T = A^-T D.
__global__ __launch_bounds__(kBlock) void scale_sumsq_k(int n, double* __restrict__ z,
                                                        const double* __restrict__ dz,
                                                        double* __restrict__ zz,
                                                        double* __restrict__ parts,
                                                        const RunState* st) {
#pragma clang fp contract(off)
  if (st->stop_req) return;
  const int lb = logical_block();
  long long r0, r1;
  block_range(n, lb, r0, r1);
  double acc = 0.0;
  for (long long i = r0 + threadIdx.x; i < r1; i += kBlock) {
    const double f = dz[i];
    const double zi = z[i] * f;
    z[i] = zi;
    zz[i] = zi * f;
    acc += zi * zi;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) parts[lb] = s;
}

// ---------------------------------------------------------------- sumsq
__global__ __launch_bounds__(kBlock) void sumsq_k(int n, const double* __restrict__ z,
                                                  double* __restrict__ parts, const RunState* st) {
  if (st->stop_req) return;
  const int lb = logical_block();
  long long r0, r1;
  block_range(n, lb, r0, r1);
  double acc = 0.0;
  for (long long i = r0 + threadIdx.x; i < r1; i += kBlock) {
    const double zi = z[i];
    acc += zi * zi;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) parts[lb] = s;
}

// ----------------------------------------------------------------- trsv
// Sparse lower-triangular solve in solve order (upper factors arrive
// reversed). Work items ("tasks") come in the order the host prepared, by
// dependency level of their panel (at most 128 consecutive rows for the
// single-side solve, 64 for the several-sides one). A task is a
// whole panel, or -- for a panel with many entries left of it -- one slice
// of those entries, or the finish step of such a panel; it only waits on
// tasks earlier in that order (panels of lower level, or the slices of its
// own panel).
//
// The tasks are dealt round-robin into kTaskLists lists, each keeping that
// order, and each list has its own ticket counter: one counter taking every
// block's atomic would hand out a ticket only every ~12 ns, which for
// 10^4 tasks is a large part of the whole solve. Every wait ends: of the
// tasks held by blocks, the earliest in the order waits only on earlier
// tasks, and each of those is finished or still untaken in its list -- and
// an untaken one is next in line for that list's blocks, which hold nothing
// earlier, so they are free to take it (each list has a resident block:
// the grid is a multiple of kTaskLists and the lowest block ids start
// first).
//
// Off-panel sums: each row by its 1024 / R lanes (8 for 128-row panels, 16
// for 64-row ones), loads unrolled for memory-level parallelism. A slice
// task stores its partial sums into fixed slots; the finish task adds the
// slices in slice order, so the result does not depend on timing. In-panel
// part: the inverse of the panel's triangle, formed on the host, is copied
// into LDS before the first wait, and once the sums are in the panel's
// values are one product with it, each row by its lanes, instead of a
// substitution whose dependent steps (one per row) sat on the critical path
// of every level.
//
// Solved values and slice partials are published by one 64-bit atomic store
// each; until then a slot holds the kPending pattern, so the value is its
// own ready flag. Waits back off exponentially and give up after a bounded
// number of sleeps, marking the run aborted (NaN results) instead of hanging.
constexpr unsigned kSleepLimit = 1u << 26;  // sleep units (64 clocks each) per wait
constexpr int kTrsvBlock = 1024;
constexpr int kUnroll = 8;
constexpr int kLanesPerRow = 16;

constexpr unsigned kMaxBackoff = 4u;        // sleep units between polls, at most

// Resolves the still-pending values among the U x S gathered slots of one
// lane (value u * S + k at out[j[u] * S + k], for j[u] >= 0; S > 1 for
// interleaved sides) together: every pass re-reads all of the
// pending ones at the coherent level at once, so values that were published
// at about the same time (the rows of one panel) cost one round trip, not
// one each. Between passes the lane sleeps, backing off exponentially; after
// kSleepLimit sleep units it gives up and sets *abort, and a wait that finds
// *abort set gives up too: its still-pending values read as NaN.
template <int U, int S = 1>
__device__ __forceinline__ void resolve_pending(const double* out, const int (&j)[U],
                                                unsigned long long (&bits)[U * S], int* abort) {
  unsigned slept = 0, backoff = 1, polls = 0;
  for (;;) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < S; ++k)
        if (j[u] >= 0 && bits[u * S + k] == kPending)
          bits[u * S + k] = __hip_atomic_load(
              reinterpret_cast<const unsigned long long*>(out + static_cast<long long>(j[u]) * S + k),
              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool pend = false;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < S; ++k) pend = pend || (j[u] >= 0 && bits[u * S + k] == kPending);
    if (!pend) return;
    if ((++polls & 63u) == 0u) {
      bool give_up = __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
      if (!give_up && slept >= kSleepLimit) {
        __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        give_up = true;
      }
      if (give_up) {
#pragma unroll
        for (int e = 0; e < U * S; ++e)
          if (j[e / S] >= 0 && bits[e] == kPending) bits[e] = 0x7FF8000000000000ull;
        return;
      }
    }
    for (unsigned k = 0; k < backoff; ++k) __builtin_amdgcn_s_sleep(1);
    slept += backoff;
    if (backoff < kMaxBackoff) backoff <<= 1;
  }
}

__device__ __forceinline__ void publish(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     static_cast<unsigned long long>(__double_as_longlong(v)), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of off-panel entries [p0, p1) of one row against the solved values,
// by the LPR lanes of a row group (sub = 0..LPR-1); every lane of the group
// gets it.
template <int LPR = kLanesPerRow>
__device__ __forceinline__ double row_sum(long long p0, long long p1, int sub,
                                          const int* __restrict__ col,
                                          const double* __restrict__ val, const double* out,
                                          RunState* st) {
  double acc = 0.0;
  for (long long base = p0; base < p1; base += LPR * kUnroll) {
    int j[kUnroll];
    double a[kUnroll];
    unsigned long long bits[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const long long p = base + u * LPR + sub;
      const bool act = p < p1;
      j[u] = act ? col[p] : -1;
      a[u] = act ? val[p] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      bits[u] = j[u] >= 0 ? __hip_atomic_load(reinterpret_cast<const unsigned long long*>(out + j[u]),
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                          : 0ull;
    bool pend = false;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) pend = pend || (j[u] >= 0 && bits[u] == kPending);
    if (pend) resolve_pending<kUnroll>(out, j, bits, &st->abort_wait);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (j[u] >= 0) acc += a[u] * __longlong_as_double(static_cast<long long>(bits[u]));
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
  return acc;
}

// 16 bytes from src (16-byte aligned) into LDS at dst + 16 * (lane in its
// wave) bytes, without passing through registers (dst: the same for every
// lane of the wave).
__device__ __forceinline__ void copy16_to_lds(const double* src, double* dst) {
  __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}

// Waits until every memory access this wave issued has completed (the
// copies into LDS among them).
__device__ __forceinline__ void wait_all_memory() { __builtin_amdgcn_s_waitcnt(0); }

// A panel of up to R rows (R = kPanel or kMaxPanelRows) is solved by one
// block: row r by the LPR = 1024 / R lanes of row group r (16 lanes for
// 64-row panels, 8 for 128-row ones). Everything that does not depend on
// solved values -- the right-hand side (into registers) and the panel's
// triangle's inverse (copied from memory straight into LDS, 16 bytes per
// lane, without passing through registers) -- is requested before the first
// wait, so that once the panel's inputs are published only the off-panel
// sums and one product with the inverse remain.

template <int R>
__global__ __launch_bounds__(kTrsvBlock) void trsv_k(TrsvArgs t, const double* __restrict__ rhs,
                                                     const int* __restrict__ rhs_perm, double* out,
                                                     double* __restrict__ scatter,
                                                     const int* __restrict__ scatter_perm,
                                                     unsigned* ticket, RunState* st) {
  constexpr int LPR = kTrsvBlock / R;  // lanes per row
  constexpr int CPL = R / LPR;         // inverse columns per lane
  constexpr int kW = R * (R + 1) / 2;  // values of a packed R-row triangle (even)
  static_assert(LPR == 8 || LPR == 16, "64- or 128-row panels");
  static_assert(kW % 2 == 0, "whole 16-byte chunks");
  __shared__ double w_sh[kW];  // the panel's inverse, rows packed: (r, c) at r (r + 1) / 2 + c
  __shared__ double t_sh[R];   // off-panel sums
  __shared__ double b_sh[R];   // right-hand side of the panel's rows
  __shared__ unsigned task_sh;
  __shared__ int quit_sh;
  // one read for the whole block: abort_wait may change while blocks start
  if (threadIdx.x == 0)
    quit_sh = st->stop_req ||
              __hip_atomic_load(&st->abort_wait, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (quit_sh) return;
  const int wave = threadIdx.x >> 6;
  const int sub = threadIdx.x & (LPR - 1);
  const int r = threadIdx.x / LPR;  // this group's row, 0..R-1
  // this block's task list (block b serves list b mod kTaskLists: on the
  // usual round-robin dispatch, one list per XCD) and its ticket counter
  const int lst = static_cast<int>(blockIdx.x % kTaskLists);
  const int l0 = t.list_off[lst];
  const unsigned lcount = static_cast<unsigned>(t.list_off[lst + 1] - l0);
  unsigned* const ctr = ticket + lst * kTicketStride;
  for (;;) {
    if (threadIdx.x == 0) task_sh = atomicAdd(ctr, 1u);
    __syncthreads();
    if (task_sh >= lcount) break;
    const long long T = l0 + static_cast<long long>(task_sh);  // the task's slot
    // the task's record: one round trip instead of the task list and then
    // the panel's own arrays
    const int4 ra = reinterpret_cast<const int4*>(t.task_rec)[2 * T];
    const int4 rb = reinterpret_cast<const int4*>(t.task_rec)[2 * T + 1];
    const int kind = ra.y;  // -1 whole panel, 0..S-1 slice, S finish
    const long long lo = ra.z;
    const int cnt = ra.w;
    const int S = rb.x;
    double* slots = t.partials + static_cast<long long>(rb.y) * R;
    const long long woff = static_cast<long long>(static_cast<unsigned>(rb.z)) |
                           (static_cast<long long>(rb.w) << 32);
    // the task's row pointers and split points, loaded by slot alone (in
    // flight together with the record, not after it)
    const long long* trp = t.task_rp + T * (R + 1);
    const long long* tsp = t.task_sp + T * R;
    const bool live = r < cnt;
    const long long a0 = trp[r], a1 = trp[r + 1];
    long long q0 = live ? a0 : 0, q1 = live ? a1 : 0;  // the row's off-panel range
    if (kind >= 0 && kind < S) {
      // ---- slice task: partial off-panel sums over one slice of the row's
      // older entries (the ones on rows before off_split; the finish step
      // adds the newest ones itself)
      if (live) q1 = tsp[r];
      const long long len = q1 - q0;
      const long long s1 = q0 + len * (kind + 1) / S, s0 = q0 + len * kind / S;
      const double part = row_sum<LPR>(s0, s1, sub, t.off_col, t.off_val, out, st);
      if (live && sub == 0) publish(slots + static_cast<long long>(kind) * R + r, part);
      __syncthreads();  // task_sh is reused
      continue;
    }
    // ---- everything that needs no solved value: the inverse, 16-byte chunk
    // ch of the packed triangle by thread ch mod kTrsvBlock into the same
    // place in LDS (the triangle starts 16-byte aligned; the last chunk may
    // take one value past its end, still inside winv), and the right-hand
    // side into registers
    {
      const double* w = t.winv + woff;
      const int nch = (cnt * (cnt + 1) / 2 + 1) / 2;
      for (int c0 = 0; c0 < nch; c0 += kTrsvBlock)
        if (c0 + static_cast<int>(threadIdx.x) < nch)
          copy16_to_lds(w + 2 * (c0 + threadIdx.x), w_sh + 2 * (c0 + wave * 64));
    }
    const double bval = (live && sub == 0) ? (rhs_perm ? rhs[rhs_perm[lo + r]] : rhs[lo + r]) : 0.0;
    // ---- off-panel sums of the row (these wait for the panel's inputs)
    double sum;
    if (kind < 0) {
      sum = row_sum<LPR>(q0, q1, sub, t.off_col, t.off_val, out, st);
    } else {
      // finish: the LPR lanes of a row read its slice partials together
      // (lane sub takes slices sub, sub + LPR, ...), add them in that fixed
      // order, then re-arm the slots they read for the next solve
      double acc = 0.0;
      if (live) {
        constexpr int kSlotsPerLane = kMaxSlicesDev / LPR;
        unsigned long long bits[kSlotsPerLane];
        int so[kSlotsPerLane];  // slot offsets from the row's first slot
        unsigned long long* sp = reinterpret_cast<unsigned long long*>(slots) + r;
#pragma unroll
        for (int u = 0; u < kSlotsPerLane; ++u) {
          const int k = sub + u * LPR;
          so[u] = k < S ? k * R : -1;
          bits[u] = k < S ? __hip_atomic_load(sp + so[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                          : 0ull;
        }
        resolve_pending<kSlotsPerLane>(slots + r, so, bits, &st->abort_wait);
#pragma unroll
        for (int u = 0; u < kSlotsPerLane; ++u)
          if (so[u] >= 0) {
            acc += __longlong_as_double(static_cast<long long>(bits[u]));
            __hip_atomic_store(sp + so[u], kPending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
      }
#pragma unroll
      for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
      // the row's newest entries (on the panel just before this one): the
      // finish step waits for them itself, one hop fewer on a chain
      const double recent = live ? row_sum<LPR>(tsp[r], trp[r + 1], sub, t.off_col, t.off_val, out, st)
                                 : 0.0;
      sum = acc + recent;
    }
    if (live && sub == 0) {
      t_sh[r] = sum;
      b_sh[r] = bval;
    }
    wait_all_memory();  // the inverse's copies into LDS have landed
    __syncthreads();
    // ---- x = W (b - sums), row r by its LPR lanes
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int c = sub + u * LPR;
      if (c <= r && c < cnt) acc += w_sh[r * (r + 1) / 2 + c] * (b_sh[c] - t_sh[c]);
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
    if (live && sub == 0) {
      const long long i = lo + r;
      publish(out + i, acc);
      if (scatter) scatter[scatter_perm[i]] = acc;
    }
    __syncthreads();  // LDS and task_sh are reused
  }
}

// ------------------------------------------------- trsv, several sides
// The same solve for K interleaved right-hand sides (row i, side k at index
// i * K + k), on the same kind of tasks, records, packed panel inverses and
// waits as trsv_k, with panels of at most kPanel = 64 rows (the host plans
// these schedules with that height). Each row has 16 lanes. In the
// off-panel sums every lane takes a share of the row's entries for all K
// sides at once: it reads an entry's column and value once and its K
// contiguous solved values, so one pass over the factor, and one wait per
// dependency, serve all K sides. In the finish step and the product the 16
// lanes are EL = 16 / K entry lanes times K side lanes. Slice partials are
// K per row. The run is skipped when *stop is non-zero (every start of the
// run has stopped); a wait that times out sets *abort.

// Off-panel sums of one row over entries [p0, p1) for all K sides at once:
// lane sub of the row's 16 takes entries sub, sub + 16, ... (the single-side
// solve's order, so each side's sum is rounded exactly as there), reads the
// entry's column and value once and the K solved values of that column as
// K/2 16-byte loads, and keeps K sums; a 16-lane butterfly then gives every
// lane all K sums, and the lane returns side kk's.
template <int K>
__device__ __forceinline__ double row_sum_multi(long long p0, long long p1, int sub, int kk,
                                                const int* __restrict__ col,
                                                const double* __restrict__ val, const double* out,
                                                int* abort) {
  constexpr int U = 2;  // entries in flight per lane
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (long long base = p0; base < p1; base += kLanesPerRow * U) {
    int j[U];
    double a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long p = base + u * kLanesPerRow + sub;
      const bool act = p < p1;
      j[u] = act ? col[p] : -1;
      a[u] = act ? val[p] : 0.0;
    }
    double2 v[U][K / 2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double2* src = reinterpret_cast<const double2*>(out + static_cast<long long>(j[u] < 0 ? 0 : j[u]) * K);
#pragma unroll
      for (int h = 0; h < K / 2; ++h) v[u][h] = j[u] >= 0 ? src[h] : make_double2(0.0, 0.0);
    }
    // the values still pending, re-read together (see resolve_pending)
    unsigned long long bits[U * K];
    bool pend = false;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int h = 0; h < K / 2; ++h) {
        bits[u * K + 2 * h] = static_cast<unsigned long long>(__double_as_longlong(v[u][h].x));
        bits[u * K + 2 * h + 1] = static_cast<unsigned long long>(__double_as_longlong(v[u][h].y));
      }
#pragma unroll
    for (int e = 0; e < U * K; ++e) pend = pend || (j[e / K] >= 0 && bits[e] == kPending);
    if (pend) resolve_pending<U, K>(out, j, bits, abort);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j[u] < 0) continue;
#pragma unroll
      for (int k = 0; k < K; ++k)
        acc[k] += a[u] * __longlong_as_double(static_cast<long long>(bits[u * K + k]));
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int off = kLanesPerRow / 2; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, kLanesPerRow);
  double r = acc[0];
#pragma unroll
  for (int k = 1; k < K; ++k) r = kk == k ? acc[k] : r;
  return r;
}

template <int K>
__global__ __launch_bounds__(kTrsvBlock) void trsv_multi_k(TrsvArgs t, const double* __restrict__ rhs,
                                                           const int* __restrict__ rhs_perm,
                                                           double* out, double* __restrict__ scatter,
                                                           const int* __restrict__ scatter_perm,
                                                           unsigned* ticket, const int* stop,
                                                           int* abort, const int* compact) {
  constexpr int EL = kLanesPerRow / K;
  static_assert(EL >= 1 && EL * K == kLanesPerRow, "K divides the 16 lanes of a row");
  constexpr int kW = kPanel * (kPanel + 1) / 2;  // values of a packed 64-row triangle (even)
  __shared__ double w_sh[kW];  // the panel's inverse, rows packed: (r, c) at r (r + 1) / 2 + c
  __shared__ double t_sh[kPanel * K];     // off-panel sums, row r side k at r * K + k
  __shared__ double b_sh[kPanel * K];     // right-hand sides
  __shared__ unsigned task_sh;
  __shared__ int quit_sh, compact_sh;
  if (threadIdx.x == 0) {
    quit_sh = (stop && *stop) ||
              __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    compact_sh = compact && *compact;
  }
  __syncthreads();
  if (quit_sh) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int sub = lane & (kLanesPerRow - 1);
  const int es = sub / K, kk = sub % K;
  const int g = wave * (64 / kLanesPerRow) + lane / kLanesPerRow;  // this group's row, 0..63
  // as in trsv_k; while the batch compacts its lists, list lst holds only
  // the slots of the blocks (matrices) that still run, in the same order
  const int lst = static_cast<int>(blockIdx.x % kTaskLists);
  const int l0 = t.list_off[lst];
  const bool cmp = compact_sh != 0;
  const unsigned lcount = static_cast<unsigned>(cmp ? t.cl_cnt[lst] : t.list_off[lst + 1] - l0);
  unsigned* const ctr = ticket + lst * kTicketStride;
  for (;;) {
    if (threadIdx.x == 0) task_sh = atomicAdd(ctr, 1u);
    __syncthreads();
    if (task_sh >= lcount) break;
    const long long T = cmp ? t.cl_slots[l0 + task_sh] : l0 + static_cast<long long>(task_sh);
    const int4 ra = reinterpret_cast<const int4*>(t.task_rec)[2 * T];
    const int4 rb = reinterpret_cast<const int4*>(t.task_rec)[2 * T + 1];
    const int kind = ra.y;  // -1 whole panel, 0..S-1 slice, S finish
    const long long lo = ra.z;
    const int cnt = ra.w;
    const int S = rb.x;
    double* slots = t.partials + static_cast<long long>(rb.y) * kPanel * K;
    const long long woff = static_cast<long long>(static_cast<unsigned>(rb.z)) |
                           (static_cast<long long>(rb.w) << 32);
    const long long* trp = t.task_rp + T * (kPanel + 1);
    const long long* tsp = t.task_sp + T * kPanel;
    const bool row = g < cnt;
    const long long a0 = trp[g], a1 = trp[g + 1], sp = tsp[g];
    long long q0 = row ? a0 : 0, q1 = row ? a1 : 0;
    if (kind >= 0 && kind < S) {
      // slice task: partial sums over one slice of the row's older entries
      if (row) q1 = sp;
      const long long len = q1 - q0;
      const long long s1 = q0 + len * (kind + 1) / S;
      const long long s0 = q0 + len * kind / S;
      const double part = row_sum_multi<K>(s0, s1, sub, kk, t.off_col, t.off_val, out, abort);
      if (row && es == 0)
        publish(slots + (static_cast<long long>(kind) * kPanel + g) * K + kk, part);
      __syncthreads();  // task_sh is reused
      continue;
    }
    // everything that needs no solved value: right-hand sides and the
    // inverse, copied from memory straight into LDS as in trsv_k (no
    // registers, and no wait before the sums' loads are issued)
    if (row && es == 0)
      b_sh[g * K + kk] = rhs_perm ? rhs[static_cast<long long>(rhs_perm[lo + g]) * K + kk]
                                  : rhs[(lo + g) * K + kk];
    {
      const double* w = t.winv + woff;
      const int nch = (cnt * (cnt + 1) / 2 + 1) / 2;
      for (int c0 = 0; c0 < nch; c0 += kTrsvBlock)
        if (c0 + static_cast<int>(threadIdx.x) < nch)
          copy16_to_lds(w + 2 * (c0 + threadIdx.x), w_sh + 2 * (c0 + wave * 64));
    }
    double sum;
    if (kind < 0) {
      sum = row_sum_multi<K>(q0, q1, sub, kk, t.off_col, t.off_val, out, abort);
    } else {
      // finish: entry lane es adds slices es, es + EL, ... of side kk in that
      // fixed order (4 loads in flight), re-arming each slot it read
      double acc = 0.0;
      if (row) {
        unsigned long long* sp = reinterpret_cast<unsigned long long*>(slots);
        for (int k0 = es; k0 < S; k0 += EL * 4) {
          unsigned long long bits[4];
          int so[4];  // slot offsets
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * EL;
            so[u] = k < S ? (k * kPanel + g) * K + kk : -1;
            bits[u] = k < S ? __hip_atomic_load(sp + so[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                            : 0ull;
          }
          resolve_pending<4>(slots, so, bits, abort);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (so[u] >= 0) {
              acc += __longlong_as_double(static_cast<long long>(bits[u]));
              __hip_atomic_store(sp + so[u], kPending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
      }
#pragma unroll
      for (int off = kLanesPerRow / 2; off >= K; off >>= 1) acc += __shfl_xor(acc, off, kLanesPerRow);
      const double recent = row ? row_sum_multi<K>(sp, q1, sub, kk, t.off_col, t.off_val, out, abort)
                                : 0.0;
      sum = acc + recent;
    }
    if (row && es == 0) t_sh[g * K + kk] = sum;
    wait_all_memory();  // the inverse's copies into LDS have landed
    __syncthreads();
    // x = W (b - sums) for side kk: entry lane es takes columns es, es + EL, ...
    double acc = 0.0;
#pragma unroll 8
    for (int u = 0; u < kPanel / EL; ++u) {
      const int c = es + u * EL;
      if (c <= g && c < cnt) acc += w_sh[g * (g + 1) / 2 + c] * (b_sh[c * K + kk] - t_sh[c * K + kk]);
    }
#pragma unroll
    for (int off = kLanesPerRow / 2; off >= K; off >>= 1) acc += __shfl_xor(acc, off, kLanesPerRow);
    if (row && es == 0) {
      const long long i = lo + g;
      publish(out + i * K + kk, acc);
      if (scatter) scatter[static_cast<long long>(scatter_perm[i]) * K + kk] = acc;
    }
    __syncthreads();  // LDS and task_sh are reused
  }
}

// ---------------------------------------------------------- adam pass 1
// Evaluation of the previous iterate, best-iterate tracking, stop rule, and
// the moment update with bias correction (Algorithm 1), partials of x.dx.
__global__ __launch_bounds__(kBlock) void pass1_k(int n, const double* __restrict__ x,
                                                  const double* __restrict__ w,
                                                  double* __restrict__ m, double* __restrict__ v,
                                                  double* __restrict__ d, double* __restrict__ xbest,
                                                  const double* __restrict__ parts_x,
                                                  const double* __restrict__ parts_y, int np,
                                                  double* __restrict__ parts_xd, RunState* st,
                                                  double* __restrict__ trace, AdamParams p) {
#pragma clang fp contract(off)
  if (st->done) return;
  const long long t = st->t_done + 1;  // index of the update this pass prepares
  const double nx2 = sum_parts(parts_x, np);
  const double ny2 = sum_parts(parts_y, np);
  const double best = st->best;
  double best_next = best;
  double ckpt_next = st->ckpt;
  bool improved = false;
  int stop = 0, status = COND_OK, flags = 0;
  long long iters = t - 1;
  double alpha = st->alpha;
  if (st->abort_wait) {
    stop = 1;
    status = COND_ETIMEOUT;
  } else if (!(nx2 > 0.0) || !(ny2 > 0.0) || !isfinite(nx2) || !isfinite(ny2)) {
    stop = 1;
    status = COND_ENUMERIC;
  } else if (t >= 2) {
    // sigma(x_{t-1}) = ||M x|| / ||x||; a strict comparison keeps the earliest best
    const double sigma = sqrt(ny2 / nx2);
    if (p.minimise ? sigma < best : sigma > best) {
      improved = true;
      best_next = sigma;
    }
    const long long T = t - 1;
    if (T >= p.max_iter) {
      stop = 1;
      flags |= static_cast<int>(COND_F_MAXITER);
    } else if (p.stop_window > 0 && p.stop_rtol > 0.0 && T % p.stop_window == 0) {
      const double gain = p.minimise ? st->ckpt - best_next : best_next - st->ckpt;
      if (T >= 2 * p.stop_window && gain <= p.stop_rtol * best_next) {
        // plateau: with a step-size floor, continue with a smaller step until it is reached
        if (p.alpha_min > 0.0 && alpha > p.alpha_min)
          alpha = fmax(alpha * p.alpha_decay, p.alpha_min);
        else
          stop = 1;
      }
      ckpt_next = best_next;
    }
  }
  const int lb = logical_block();
  long long r0, r1;
  block_range(n, lb, r0, r1);
  if (improved && xbest)
    for (long long i = r0 + threadIdx.x; i < r1; i += kBlock) xbest[i] = x[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->best_next = best_next;
    st->ckpt_next = ckpt_next;
    st->alpha_next = alpha;
    if (t >= 2 && trace && status == COND_OK) trace[t - 2] = best_next;
    if (stop) {
      st->iters = iters;
      st->status = status;
      st->flags = flags;
      st->stop_req = 1;
    }
  }
  if (stop) return;
  const double b1 = p.beta1, b2 = p.beta2;
  const double b1t = st->b1t * b1, b2t = st->b2t * b2;
  double acc = 0.0;
  for (long long i = r0 + threadIdx.x; i < r1; i += kBlock) {
    const double xi = x[i];
    // equation nabla_loss (negated when minimising)
    const double g = p.minimise ? w[i] / ny2 - xi / nx2 : xi / nx2 - w[i] / ny2;
    const double mi = b1 * m[i] + (1.0 - b1) * g;
    const double vi = b2 * v[i] + (1.0 - b2) * (g * g);
    const double mh = mi / (1.0 - b1t);
    const double vh = vi / (1.0 - b2t);
    const double di = alpha * mh / (sqrt(vh) + p.eps);
    m[i] = mi;
    v[i] = vi;
    d[i] = di;
    acc += xi * di;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) parts_xd[lb] = s;
}

// ---------------------------------------------------------- adam pass 2
// Tangent projection dx <- dx - (x.dx) x and the update x <- x - dx; partials
// of ||x||^2 for the normalisation that opens the next iteration.
__global__ __launch_bounds__(kBlock) void pass2_k(int n, double* __restrict__ x,
                                                  const double* __restrict__ d,
                                                  const double* __restrict__ parts_xd, int np,
                                                  double* __restrict__ parts_xx, RunState* st,
                                                  AdamParams p) {
#pragma clang fp contract(off)
  if (st->done) return;
  if (st->stop_req) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->best = st->best_next;
      st->done = 1;
    }
    return;
  }
  const double xd = sum_parts(parts_xd, np);
  const int lb = logical_block();
  long long r0, r1;
  block_range(n, lb, r0, r1);
  double acc = 0.0;
  for (long long i = r0 + threadIdx.x; i < r1; i += kBlock) {
    const double xi = x[i];
    const double dd = d[i] - xd * xi;
    const double xn = xi - dd;
    x[i] = xn;
    acc += xn * xn;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) parts_xx[lb] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->t_done = st->t_done + 1;
    st->b1t = st->b1t * p.beta1;
    st->b2t = st->b2t * p.beta2;
    st->best = st->best_next;
    st->ckpt = st->ckpt_next;
    st->alpha = st->alpha_next;
  }
}

// ------------------------------------------------------------- residual
// Error bounds of an approximate solution: r = A x_hat - b row by row (16
// lanes per row, a block's rows a contiguous range), with block partials of
// r.r, x_hat.x_hat and b.b in fixed slots; reduce3_k adds each set of
// partials in slot order (one block), so the three sums do not depend on
// timing.
template <typename IT>
__global__ __launch_bounds__(kBlock) void residual_k(int n, const IT* __restrict__ rowptr,
                                                     const int* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ parts) {
#pragma clang fp contract(off)
  constexpr int kRowLanes = 16;
  const int lb = logical_block();
  long long r0, r1;
  block_range(n, lb, r0, r1);
  const int sub = threadIdx.x & (kRowLanes - 1);
  const int grp = threadIdx.x / kRowLanes;
  double ar = 0.0, ax = 0.0, ab = 0.0;
  for (long long i = r0 + grp; i < r1; i += kBlock / kRowLanes) {
    const IT p0 = rowptr[i], p1 = rowptr[i + 1];
    double acc = 0.0;
    for (IT e = p0 + sub; e < p1; e += kRowLanes) acc += val[e] * x[col[e]];
#pragma unroll
    for (int off = kRowLanes / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kRowLanes);
    if (sub == 0) {
      const double bi = b[i], xi = x[i];
      const double ri = acc - bi;
      ar += ri * ri;
      ax += xi * xi;
      ab += bi * bi;
    }
  }
  const double sr = block_sum(ar);
  const double sx = block_sum(ax);
  const double sb = block_sum(ab);
  if (threadIdx.x == 0) {
    parts[lb] = sr;
    parts[kMaxParts + lb] = sx;
    parts[2 * kMaxParts + lb] = sb;
  }
}

__global__ __launch_bounds__(kBlock) void reduce3_k(const double* __restrict__ parts, int np,
                                                    double* __restrict__ out) {
  for (int k = 0; k < 3; ++k) {
    const double v = sum_parts(parts + static_cast<long long>(k) * kMaxParts, np);
    if (threadIdx.x == 0) out[k] = v;
  }
}

// ---------------------------------------------------------------- triad
// a = b + s c over n doubles: the streaming reference every HBM-bound kernel
// is quoted against (24 bytes per element). Each thread moves two elements
// per chunk as 16-byte loads and stores, four chunks in flight; consecutive
// threads take consecutive 16-byte chunks.
__global__ __launch_bounds__(kBlock) void triad_k(long long n, double* __restrict__ a,
                                                  const double* __restrict__ b,
                                                  const double* __restrict__ c, double s) {
  const long long n2 = n / 2;
  const double2* b2 = reinterpret_cast<const double2*>(b);
  const double2* c2 = reinterpret_cast<const double2*>(c);
  double2* a2 = reinterpret_cast<double2*>(a);
  const long long stride = static_cast<long long>(gridDim.x) * kBlock;
  long long i = blockIdx.x * static_cast<long long>(kBlock) + threadIdx.x;
  // four chunks in flight per thread, then the remainder one at a time
  for (; i + 3 * stride < n2; i += 4 * stride) {
    double2 x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = b2[i + u * stride];
      y[u] = c2[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) a2[i + u * stride] = make_double2(x[u].x + s * y[u].x, x[u].y + s * y[u].y);
  }
  for (; i < n2; i += stride) {
    const double2 x = b2[i], y = c2[i];
    a2[i] = make_double2(x.x + s * y.x, x.y + s * y.y);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) a[n - 1] = b[n - 1] + s * c[n - 1];
}

__global__ void fill_k(long long n, unsigned long long* p, unsigned long long bits) {
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    p[i] = bits;
}

__global__ void set_int_k(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void zero_u32_k(unsigned* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

}  // namespace

int grid_for(int n) {
  // about 256 rows per block, at most kMaxParts blocks, a multiple of 8
  long long g = (static_cast<long long>(n) + 255) / 256;
  if (g < 8) g = 8;
  if (g > kMaxParts) g = kMaxParts;
  return static_cast<int>((g + 7) / 8 * 8);
}

void launch_init(int n, const double* x0, double* x, double* m, double* v, double* parts_xx,
                 int grid, RunState* st, double alpha0, int minimise, hipStream_t s) {
  init_k<<<grid, kBlock, 0, s>>>(n, x0, x, m, v, parts_xx, st, alpha0, minimise);
}

void launch_normalise(int n, double* x, const double* parts_xx, int grid, double* parts_x,
                      RunState* st, double* const* resets, int nresets, unsigned* tickets,
                      int ntickets, hipStream_t s) {
  Resets r{};
  r.count = nresets;
  for (int k = 0; k < nresets && k < 4; ++k) r.p[k] = resets[k];
  normalise_k<<<grid, kBlock, 0, s>>>(n, x, parts_xx, grid, parts_x, st, r, tickets, ntickets);
}

void launch_spmv(const DevCsr& a, const double* x, double* y, double* parts_y, int grid,
                 const RunState* st, hipStream_t s, const double* cs, const double* rs) {
  const bool sc = cs || rs;
  const long long* rp64 = static_cast<const long long*>(a.rowptr);
  const int* rp32 = static_cast<const int*>(a.rowptr);
  if (a.idx64 && sc)
    spmv_stream_k<long long, true><<<grid, kBlock, 0, s>>>(a.ntiles, a.tiles, rp64, a.col, a.val,
                                                           x, y, parts_y, st, cs, rs);
  else if (a.idx64)
    spmv_stream_k<long long, false><<<grid, kBlock, 0, s>>>(a.ntiles, a.tiles, rp64, a.col, a.val,
                                                            x, y, parts_y, st, nullptr, nullptr);
  else if (sc)
    spmv_stream_k<int, true><<<grid, kBlock, 0, s>>>(a.ntiles, a.tiles, rp32, a.col, a.val, x, y,
                                                     parts_y, st, cs, rs);
  else
    spmv_stream_k<int, false><<<grid, kBlock, 0, s>>>(a.ntiles, a.tiles, rp32, a.col, a.val, x, y,
                                                      parts_y, st, nullptr, nullptr);
}

void launch_row_norms(const DevCsr& a, double* out, hipStream_t s) {
  long long blocks = (static_cast<long long>(a.n) + kBlock / 16 - 1) / (kBlock / 16);
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (a.idx64)
    row_norms_k<long long><<<static_cast<int>(blocks), kBlock, 0, s>>>(
        a.n, static_cast<const long long*>(a.rowptr), a.val, out);
  else
    row_norms_k<int><<<static_cast<int>(blocks), kBlock, 0, s>>>(
        a.n, static_cast<const int*>(a.rowptr), a.val, out);
}

void launch_scale_prep(int n, const double* d, double* dinv, const int* perm, double* dz,
                       hipStream_t s) {
  long long blocks = (static_cast<long long>(n) + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  scale_prep_k<<<static_cast<int>(blocks), kBlock, 0, s>>>(n, d, dinv, perm, dz);
}

void launch_scale_sumsq(int n, double* z, const double* dz, double* zz, double* parts, int grid,
                        const RunState* st, hipStream_t s) {
  scale_sumsq_k<<<grid, kBlock, 0, s>>>(n, z, dz, zz, parts, st);
}

void launch_sumsq(int n, const double* z, double* parts, int grid, const RunState* st,
                  hipStream_t s) {
  sumsq_k<<<grid, kBlock, 0, s>>>(n, z, parts, st);
}

// Blocks of a solve: a multiple of kTaskLists, so every list has its blocks
// (block b serves list b mod kTaskLists), at most 512.
static int trsv_grid(int ntasks) {
  long long blocks = ntasks < 512 ? ntasks : 512;
  blocks = (blocks + kTaskLists - 1) / kTaskLists * kTaskLists;
  return static_cast<int>(blocks < kTaskLists ? kTaskLists : blocks);
}

void launch_trsv(const DevTri& t, const double* rhs, const int* rhs_perm, double* out,
                 double* scatter, const int* scatter_perm, unsigned* ticket, RunState* st,
                 hipStream_t s) {
  const int g = trsv_grid(t.ntasks);
  if (t.prows == kMaxPanelRows)
    trsv_k<kMaxPanelRows><<<g, kTrsvBlock, 0, s>>>(t, rhs, rhs_perm, out, scatter, scatter_perm, ticket, st);
  else
    trsv_k<kPanel><<<g, kTrsvBlock, 0, s>>>(t, rhs, rhs_perm, out, scatter, scatter_perm, ticket, st);
}

void launch_trsv_multi(int K, const DevTri& t, const double* rhs, const int* rhs_perm, double* out,
                       double* scatter, const int* scatter_perm, unsigned* ticket, const int* stop,
                       int* abort, const int* compact, hipStream_t s) {
  const int g = trsv_grid(t.ntasks);
  switch (K) {
    case 2:
      trsv_multi_k<2><<<g, kTrsvBlock, 0, s>>>(t, rhs, rhs_perm, out, scatter, scatter_perm, ticket,
                                               stop, abort, compact);
      break;
    case 4:
      trsv_multi_k<4><<<g, kTrsvBlock, 0, s>>>(t, rhs, rhs_perm, out, scatter, scatter_perm, ticket,
                                               stop, abort, compact);
      break;
    default:
      trsv_multi_k<8><<<g, kTrsvBlock, 0, s>>>(t, rhs, rhs_perm, out, scatter, scatter_perm, ticket,
                                               stop, abort, compact);
      break;
  }
}

void launch_pass1(int n, const double* x, const double* w, double* m, double* v, double* d,
                  double* xbest, const double* parts_x, const double* parts_y, int grid,
                  double* parts_xd, RunState* st, double* trace, const AdamParams& p,
                  hipStream_t s) {
  pass1_k<<<grid, kBlock, 0, s>>>(n, x, w, m, v, d, xbest, parts_x, parts_y, grid, parts_xd, st,
                                  trace, p);
}

void launch_pass2(int n, double* x, const double* d, const double* parts_xd, int grid,
                  double* parts_xx, RunState* st, const AdamParams& p, hipStream_t s) {
  pass2_k<<<grid, kBlock, 0, s>>>(n, x, d, parts_xd, grid, parts_xx, st, p);
}

void launch_residual(int n, const void* rowptr, int idx64, const int* col, const double* val,
                     const double* x, const double* b, double* parts, double* sums, int grid,
                     hipStream_t s) {
  if (idx64)
    residual_k<long long><<<grid, kBlock, 0, s>>>(n, static_cast<const long long*>(rowptr), col,
                                                  val, x, b, parts);
  else
    residual_k<int><<<grid, kBlock, 0, s>>>(n, static_cast<const int*>(rowptr), col, val, x, b,
                                            parts);
  reduce3_k<<<1, kBlock, 0, s>>>(parts, grid, sums);
}

void launch_triad(long long n, double* a, const double* b, const double* c, double scale, int grid,
                  hipStream_t s) {
  triad_k<<<grid, kBlock, 0, s>>>(n, a, b, c, scale);
}

void launch_fill(long long n, double* p, unsigned long long bits, hipStream_t s) {
  long long blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  fill_k<<<static_cast<int>(blocks), kBlock, 0, s>>>(n, reinterpret_cast<unsigned long long*>(p), bits);
}

void launch_set_int(int* p, int v, hipStream_t s) { set_int_k<<<1, 64, 0, s>>>(p, v); }

void launch_zero_u32(unsigned* p, int count, hipStream_t s) {
  zero_u32_k<<<(count + 63) / 64, 64, 0, s>>>(p, count);
}

}  // namespace condest
