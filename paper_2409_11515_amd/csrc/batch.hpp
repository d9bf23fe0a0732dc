// Batched multi-start Projected Adam: device structures shared by the
// batch kernels and the batch plan.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace condest {

constexpr int kBatchK = 8;  // starts per matrix, interleaved x[i*K + k]

// Per (matrix, start) state of Algorithm 1. Written only by the per-matrix
// reduction kernel (one thread per pair) and read by the element kernels.
struct BatchPair {
  double best;      // best sigma over evaluated iterates
  double ckpt;      // best at the last stop-window boundary
  double nrm;       // ||x|| before normalisation
  double nx2, ny2;  // x.x and ||M x||^2 of the current iterate
  double xd;        // x . dx
  double alpha;     // step size of the coming update
  long long iters;  // final T once stopped
  int improved;     // the current iterate is the new best
  int stopped;
  int status;
  int flags;
};

struct BatchGlobal {
  long long t_done;
  double b1t, b2t;
  int nlive;         // tiles of the matrices that still have a running start
  int stop_all;      // 1 once every pair has stopped (the solves then skip)
  int abort_wait;    // 1 when a triangular-solve wait timed out
  int live_changed;  // 1 when this update's running matrices differ from the last's
  int compact;       // 1 while some matrix has stopped: the solves take compacted lists
  int pad_;
};

struct BatchArgs {
  int nmat = 0;
  int ntiles = 0;
  const long long* tiles = nullptr;  // tile t = rows [tiles[t], tiles[t+1]) of one matrix
  const int* tile_mat = nullptr;     // matrix of tile t
  const int* mat_tile0 = nullptr;    // tiles of matrix m: [mat_tile0[m], mat_tile0[m+1])
  int* live_mat = nullptr;           // matrices with a running start, in order
  int* live_pref = nullptr;          // their tiles: live index u in [live_pref[j], live_pref[j+1])
  int* mat_live = nullptr;           // per matrix: 1 while one of its starts runs
  const int* a_rowptr = nullptr;     // block-diagonal A (global row and column indices)
  const int* a_col = nullptr;
  const double* a_val = nullptr;
  const int* at_rowptr = nullptr;  // block-diagonal A^T
  const int* at_col = nullptr;
  const double* at_val = nullptr;
  double *x = nullptr, *m = nullptr, *v = nullptr, *d = nullptr, *y = nullptr, *w = nullptr;
  double* xbest = nullptr;
  double *parts_x = nullptr, *parts_y = nullptr, *parts_xd = nullptr, *parts_xx = nullptr;
  BatchPair* pairs = nullptr;
  BatchGlobal* g = nullptr;
  double* trace = nullptr;  // [pair][max_iter] or nullptr
  // sigma_min route (Algorithm 2 over the block-diagonal factors): the
  // solves' vectors (K interleaved sides), re-armed every update, and their
  // ticket counters; z is in reversed pivot order, so tile t's rows
  // [r0, r1) sit at [nrows - r1, nrows - r0) of z
  long long nrows = 0;
  double *c = nullptr, *z = nullptr, *h = nullptr, *wv = nullptr;
  unsigned* tickets = nullptr;
};

// The four solves' task lists for the compaction: solve f's slots of list l
// are [list_off[f][l], list_off[f][l+1]), slot_group[f] the matrix of each
// slot; the compacted list l goes to cl_slots[f] from list_off[f][l] on, its
// length to cl_cnt[f * kTaskLists + l].
struct BatchLists {
  const int* slot_group[4] = {};
  int list_off[4][kTaskLists + 1] = {};
  int* cl_slots[4] = {};
  int* cl_cnt = nullptr;
};

void batch_launch_init(const BatchArgs& a, const double* x0, int grid, hipStream_t s);
void batch_launch_live(const BatchArgs& a, hipStream_t s);
void batch_launch_reduce(const BatchArgs& a, int mode, const AdamParams& p, hipStream_t s);
void batch_launch_normalise(const BatchArgs& a, int grid, hipStream_t s);
void batch_launch_spmm(const BatchArgs& a, int transpose, int grid, hipStream_t s);
void batch_launch_pass1(const BatchArgs& a, const AdamParams& p, int grid, hipStream_t s);
void batch_launch_pass2(const BatchArgs& a, const AdamParams& p, int grid, hipStream_t s);
// sigma_min route: re-arm c, z, h, wv and the tickets; squared norms of z per
// (tile, start) from the mirrored tiles
void batch_launch_rearm(const BatchArgs& a, int grid, hipStream_t s);
void batch_launch_sumsq_rev(const BatchArgs& a, int grid, hipStream_t s);
// When the running matrices changed and some matrix has stopped: cut each
// list of each solve down to the slots of the running matrices, in order.
void batch_launch_compact(const BatchArgs& a, const BatchLists& l, hipStream_t s);

}  // namespace condest
