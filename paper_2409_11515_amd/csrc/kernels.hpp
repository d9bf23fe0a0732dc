// Device kernels of the Projected Adam estimator (gfx950, wave64, FP64).
//
// One iteration of Algorithm 1 is a fixed sequence of launches on one stream:
//
//   sigma_max (M = A):      normalise -> spmv(A) -> spmv(A^T) -> adam_pass1 -> adam_pass2
//   sigma_min (M = A^-1):   normalise -> trsv(L) -> trsv(U) -> sumsq -> trsv(U^T)
//                           -> trsv(L^T) -> adam_pass1 -> adam_pass2
//
// Global sums (||x||^2, ||M x||^2, x.dx) are deterministic: every producer
// block writes one partial into a fixed slot, and every consumer block adds
// the same slots in the same order, so all blocks see bit-identical scalars
// and two runs give bit-identical results. No floating-point atomics are used.
//
// All per-run scalars live in a device-resident RunState so that a whole
// chunk of iterations can be captured in one HIP graph and replayed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "solve_consts.hpp"

namespace condest {

constexpr int kBlock = 256;      // threads per block (4 waves of 64)
constexpr int kMaxParts = 2048;  // max blocks (and partial slots) of a fixed-grid kernel
// A signalling-NaN bit pattern marks "not solved yet" in the triangular
// solves; arithmetic never produces a signalling NaN, so a solved entry,
// even a NaN one, can never be mistaken for it.
constexpr unsigned long long kPending = 0x7FF0DEAD0000BEEFull;

// Device-resident state of one Projected Adam run. Each field has one
// writer kernel (noted) so that no kernel reads a field it may be changing.
struct RunState {
  double best;       // best sigma over evaluated iterates (adam_pass2, block 0)
  double best_next;  // best after this iteration's evaluation (adam_pass1, block 0)
  double ckpt;       // best at the last stop-window boundary (adam_pass2, block 0)
  double ckpt_next;  // (adam_pass1, block 0)
  double b1t, b2t;   // beta1^t, beta2^t for t = updates done (adam_pass2, block 0)
  long long t_done;  // Adam updates done (adam_pass2, block 0)
  long long iters;   // final T (adam_pass1, block 0, when stopping)
  int stop_req;      // 1 once the run has decided to stop (adam_pass1, block 0)
  int done;          // 1 after the stopping iteration has drained (adam_pass2, block 0)
  int status;        // COND_OK or an error code (adam_pass1, block 0)
  int flags;         // COND_F_* bits of this run (adam_pass1, block 0)
  int abort_wait;    // 1 when a triangular-solve wait timed out (trsv)
  int pad_;
  double alpha;       // step size of the coming update (adam_pass2, block 0)
  double alpha_next;  // after this iteration's stop check (adam_pass1, block 0)
};

struct AdamParams {
  double alpha, beta1, beta2, eps;
  double stop_rtol;
  long long stop_window;
  long long max_iter;
  double alpha_min;    // > 0: on a stop-rule plateau shrink alpha instead of stopping
  double alpha_decay;  // factor of each shrink
  // 1: descend on log||M v|| - log||v|| (the gradient of equation nabla_loss
  // negated) and keep the smallest sigma -- the SpMV-only sigma_min ablation
  int minimise;
  int pad_;
};

// CSR on the device. rowptr is int32 when idx64 == 0, else int64.
struct DevCsr {
  int n = 0;
  long long nnz = 0;
  const void* rowptr = nullptr;
  int idx64 = 0;
  const int* col = nullptr;
  const double* val = nullptr;
  // row tiles of the streaming SpMV: tile t holds rows [tiles[t],
  // tiles[t+1]), at most 256 rows and 2048 entries unless one row
  const int* tiles = nullptr;
  int ntiles = 0;
};

// Row tiles for the streaming SpMV (see DevCsr::tiles).
constexpr int kTileRowsHost = 256;
constexpr long long kTileEntriesHost = 2048;

// A lower-triangular factor in solve order (upper factors are reversed on the
// host, row i -> n-1-i, so every solve is a forward substitution), cut into
// panels of at most prows consecutive rows. Per row, the entries with a column
// before the row's panel ("off") and inside it ("in", column relative to the
// panel start). The solve is a list of tasks in dependency-level order:
// task t works on panel task_panel[t]; task_kind[t] = -1 for the whole panel,
// 0..S-1 for slice k of its off-panel entries, S for the step that adds the
// slices and finishes the panel (S = panel_split[panel]).
struct DevTri {
  int n = 0;
  const long long* off_rp = nullptr;
  const int* off_col = nullptr;
  const double* off_val = nullptr;
  const long long* off_split = nullptr;  // per row of a sliced panel: first entry the finish adds
  // inverse of each panel's triangle (its in-panel entries and the
  // diagonal, unit for L), lower rows packed: (r, c) at r (r + 1) / 2 + c;
  // panel p's at winv + woff[p]
  const double* winv = nullptr;
  const long long* woff = nullptr;
  double* partials = nullptr;  // slice partial sums, prows doubles per slot (times the sides); kPending when idle
  int prows = kPanel;          // most rows of a panel
  int ntasks = 0;
  // the tasks in kTaskLists lists, each in dependency order and handed out
  // by its own ticket counter: list l is the slots [list_off[l],
  // list_off[l+1]); the per-task arrays below are indexed by slot
  int list_off[kTaskLists + 1] = {};
  // per slot, 8 ints (two 16-byte loads): panel, kind (-1 whole panel,
  // 0..S-1 slice, S finish), first row, rows, slices S, first partial-sum
  // slot, offset of the panel's inverse in winv (low and high 32 bits)
  const int* task_rec = nullptr;
  // per slot: off-panel row pointers of its rows (prows + 1 values,
  // padded) and their split points (prows values)
  const long long* task_rp = nullptr;
  const long long* task_sp = nullptr;
  // joined schedules (a batch): the block (matrix) of each slot, and the
  // lists cut down to the slots of the blocks that still run (list l's at
  // cl_slots[list_off[l] ..], cl_cnt[l] of them), used while the batch's
  // compaction flag is set; or null
  const int* slot_group = nullptr;
  const int* cl_slots = nullptr;
  const int* cl_cnt = nullptr;
};
using TrsvArgs = DevTri;

int grid_for(int n);  // fixed grid size of the reduction kernels for length n

void launch_init(int n, const double* x0, double* x, double* m, double* v, double* parts_xx,
                 int grid, RunState* st, double alpha0, int minimise, hipStream_t s);
// The ticket counters of solve k in an area of kSolveTickets per solve.
inline unsigned* tix(unsigned* base, int k) { return base + k * kSolveTickets; }
// x <- x / ||x||, partials of x.x; re-arms the `nresets` solve vectors and
// the ticket counters of `ntickets` solves (an area as above).
void launch_normalise(int n, double* x, const double* parts_xx, int grid, double* parts_x,
                      RunState* st, double* const* resets, int nresets, unsigned* tickets,
                      int ntickets, hipStream_t s);
// y = R A C x with C = diag(cs), R = diag(rs) when given (null: identity).
void launch_spmv(const DevCsr& a, const double* x, double* y, double* parts_y, int grid,
                 const RunState* st, hipStream_t s, const double* cs = nullptr,
                 const double* rs = nullptr);
// out[i] = 2-norm of row i (column norms of A when a is the stored A^T).
void launch_row_norms(const DevCsr& a, double* out, hipStream_t s);
// dinv = 1/d and, when perm is given, dz[k] = d[perm[k]].
void launch_scale_prep(int n, const double* d, double* dinv, const int* perm, double* dz,
                       hipStream_t s);
// z <- dz z with partials of its squared norm, and zz = dz z (after the scaling).
void launch_scale_sumsq(int n, double* z, const double* dz, double* zz, double* parts, int grid,
                        const RunState* st, hipStream_t s);
void launch_sumsq(int n, const double* z, double* parts, int grid, const RunState* st,
                  hipStream_t s);
void launch_trsv(const DevTri& t, const double* rhs, const int* rhs_perm, double* out,
                 double* scatter, const int* scatter_perm, unsigned* ticket, RunState* st,
                 hipStream_t s);
// The same solve for K in {2, 4, 8} interleaved right-hand sides (row i,
// side k at i * K + k; rhs, out and scatter in that layout, the permutations
// over rows). t.partials must hold K values per slot row. Skipped when *stop
// (may be null) is non-zero; a timed-out wait sets *abort. While *compact
// (may be null) is non-zero the tasks come from t's compacted lists (the
// blocks of a joined schedule that still run; they never read the others'
// values).
void launch_trsv_multi(int K, const DevTri& t, const double* rhs, const int* rhs_perm, double* out,
                       double* scatter, const int* scatter_perm, unsigned* ticket, const int* stop,
                       int* abort, const int* compact, hipStream_t s);
void launch_pass1(int n, const double* x, const double* w, double* m, double* v, double* d,
                  double* xbest, const double* parts_x, const double* parts_y, int grid,
                  double* parts_xd, RunState* st, double* trace, const AdamParams& p,
                  hipStream_t s);
void launch_pass2(int n, double* x, const double* d, const double* parts_xd, int grid,
                  double* parts_xx, RunState* st, const AdamParams& p, hipStream_t s);
// r = A x - b: parts (3 * kMaxParts doubles) receives the block partials of
// r.r, x.x and b.b; sums (3 doubles) their totals, added in slot order.
void launch_residual(int n, const void* rowptr, int idx64, const int* col, const double* val,
                     const double* x, const double* b, double* parts, double* sums, int grid,
                     hipStream_t s);
// a = b + scale c (n doubles; a, b, c 16-byte aligned): the streaming ceiling.
void launch_triad(long long n, double* a, const double* b, const double* c, double scale, int grid,
                  hipStream_t s);
void launch_fill(long long n, double* p, unsigned long long bits, hipStream_t s);
void launch_zero_u32(unsigned* p, int count, hipStream_t s);
void launch_set_int(int* p, int v, hipStream_t s);

}  // namespace condest
