/*
 * condest.h -- C ABI of the MI355X Projected Adam condition-number estimator.
 *
 * The library computes kappa_2(A) = sigma_max(A) / sigma_min(A) of a square
 * sparse matrix without singular values, by the method of Ferrari,
 * "A Comparison of Sparse Solvers for Severely Ill-Conditioned Linear Systems
 * in Geophysical Marker-In-Cell Simulations" (arXiv 2409.11515):
 *
 *   - sigma_max = ||A||_2 as the maximum of ||A v|| / ||v|| (Theorem
 *     "Equivalent definitions of the L2 matrix norm"), reached by Projected
 *     Adam (Algorithm 1) on the loss L(v) = log||v|| - log||A v|| whose
 *     gradient is v/||v||^2 - A^T A v/||A v||^2 (equation nabla_loss);
 *   - 1/sigma_min = ||A^-1||_2 by the same iteration applied to A^-1, with the
 *     gradient from one LU factorisation and triangular solves (Algorithm 2,
 *     "Compute Gradient for A^-1");
 *   - kappa_2 = ||A||_2 ||A^-1||_2 (equation kappa and its singular-value form
 *     in section "Computing the condition number of a matrix").
 *
 * Conventions for every entry point:
 *   - return 0 (COND_OK) on success or a negative COND_E* status; the text of
 *     the last error on the calling thread is available from
 *     cond_last_error();
 *   - the caller owns every array it passes in; the library never frees or
 *     keeps a caller pointer beyond the call, except the device workspace
 *     handed to cond_plan_bind (kept until cond_plan_destroy);
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the current device;
 *   - all floating point is IEEE double; indices are int32 except row
 *     pointers, which are int64;
 *   - one plan is used by one thread and one stream at a time.
 */
#ifndef CONDEST_H
#define CONDEST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define COND_OK 0
#define COND_EINVAL (-1)    /* malformed CSR (non-square, bad rowptr, column out of
                               range), non-finite entry, zero matrix, bad option */
#define COND_ESINGULAR (-2) /* the LU met an exactly zero pivot column: A is singular;
                               sigma_min = 0 and kappa = +inf are reported */
#define COND_ENOMEM (-3)    /* host allocation failed or the workspace is too small */
#define COND_EHIP (-4)      /* a HIP runtime call failed */
#define COND_ENUMERIC (-5)  /* a norm became zero or non-finite during the iteration, or
                               (cond_plan_create) a diagonal block of the LU factors
                               has no finite float64 inverse */
#define COND_ESTATE (-6)    /* entry points called out of order (e.g. run before bind) */
#define COND_ETIMEOUT (-7)  /* a triangular-solve wait exceeded its spin limit */

/* sigma_min route */
#define COND_MIN_LU 0   /* the paper's route: Algorithm 2, one LU + triangular solves */
#define COND_MIN_SPMV 1 /* ablation, not the paper's method: sigma_min as the smallest
                           ||A x|| / ||x|| reached by the same Projected Adam iteration
                           descending on log||A v|| - log||v|| (the gradient of equation
                           nabla_loss negated), with products by A and A^T only. Every
                           value is an upper bound of sigma_min; at large kappa it does
                           not converge in practice, which is why the paper factors A.
                           Needs no LU: any plan can run it */
#define COND_MIN_NONE 2 /* skip the sigma_min run */

/* result flags */
#define COND_F_NUMSING 1u  /* kappa >= 1/eps_mach: numerically singular (Theorem on
                              numerical singularity) */
#define COND_F_MAXITER 2u  /* a run ended at max_iter rather than by the stop rule */
#define COND_F_SINGULAR 4u /* exactly singular (zero pivot) */
#define COND_F_COLSCALED 8u /* the estimate is of A D_col^-1 (opts.scaling) */

/* ------------------------------------------------------------------- types */

/* A square n x n CSR matrix in host memory. Column indices need not be
 * sorted; duplicates are summed. rowptr[0] = 0, rowptr[n] = nnz. */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int64_t* rowptr; /* host, n+1 */
  const int32_t* col;    /* host, nnz */
  const double* val;     /* host, nnz */
} cond_csr_t;

/* Options of Algorithm 1. The paper fixes none of alpha, beta1, beta2, eps or
 * max_iter (they are inputs of the algorithm); cond_opts_default() gives
 * alpha = 1e-2, beta1 = 0.9, beta2 = 0.999, eps = 1e-8, max_iter = 20000,
 * no early stop, no step-size floor (alpha_min = 0, alpha_decay = 0.5). */
typedef struct {
  double alpha, beta1, beta2, eps;
  int64_t max_iter;    /* Adam updates per run (>= 1) */
  double stop_rtol;    /* early stop: after T updates, T a multiple of stop_window,
                          T >= 2*stop_window, stop when
                          best_T - best_{T-W} <= stop_rtol * best_T; 0 = off */
  int64_t stop_window; /* W; 0 = off */
  int32_t sigma_min_method; /* COND_MIN_LU, COND_MIN_SPMV or COND_MIN_NONE; chosen at
                               create (COND_MIN_LU factors A there) and may change at run
                               to COND_MIN_SPMV or COND_MIN_NONE */
  int32_t chunk;       /* iterations per captured HIP graph launch (0 = automatic) */
  const int32_t* col_perm; /* optional fill-reducing column order for the LU (host,
                              n entries, a permutation); NULL = built-in nested
                              dissection */
  double pivot_tol;    /* threshold partial pivoting: keep the diagonal candidate
                          when |a_jj| >= pivot_tol * max |a_ij| (0 < tol <= 1;
                          0 = default 1e-6). A small threshold keeps the
                          nested-dissection structure (few off-diagonal pivots):
                          less fill and far shorter dependency chains in the
                          triangular solves */
  int32_t profile;     /* 1: launch eagerly (no graph) with a HIP event pair around
                          every kernel; per-kernel times via cond_plan_kernel_stats */
  double alpha_min;    /* step-size floor. 0 (default) = Algorithm 1 as written:
                          alpha is constant and the stop rule ends the run. > 0:
                          when the stop rule fires and alpha > alpha_min, the run
                          continues with alpha = max(alpha * alpha_decay,
                          alpha_min) (moments kept) and stops at the first
                          plateau at the floor. A constant alpha leaves the
                          estimate short of the optimum by an amount that
                          shrinks about as alpha^2; the floor sets that bias.
                          0 <= alpha_min <= alpha */
  double alpha_decay;  /* factor of each decrease, 0 < alpha_decay < 1 (default
                          0.5); used only when alpha_min > 0 */
  int32_t scaling;     /* COND_SCALE_NONE (default): estimate kappa_2(A).
                          COND_SCALE_COL: estimate kappa_2(A D_col^-1), the
                          column-scaled matrix of section "Row and Column Scaling"
                          (D_col = diag of the column 2-norms of A), from the same
                          plan: the products scale on the fly and the sigma_min
                          run reuses A's LU, since (A D^-1)^-1 = D A^-1. A plan
                          with a zero column refuses it (COND_EINVAL). May change
                          from run to run */
} cond_opts_t;

/* cond_opts_t.scaling */
#define COND_SCALE_NONE 0
#define COND_SCALE_COL 1

typedef struct {
  double sigma_max, sigma_min, kappa;
  int64_t iters_max, iters_min; /* Adam updates performed by each run */
  uint32_t flags;               /* COND_F_* */
  int32_t status_max, status_min;
  double ms_max, ms_min;        /* device time of each run (HIP events) */
  double setup_ms;              /* host setup: validation, transpose, ordering, LU */
  int64_t nnz_l, nnz_u;         /* LU fill (strictly lower L, upper U incl. diagonal) */
} cond_result_t;

typedef struct cond_plan cond_plan_t;
typedef struct cond_lu cond_lu_t;

/* ------------------------------------------------------------------ basics */
const char* cond_strerror(int status);
const char* cond_last_error(void);
void cond_opts_default(cond_opts_t* o);
int cond_version(void);

/* -------------------------------------------------- host steps (no device)
 * These run on the CPU only and are what the plan does at set-up; they are
 * exported so each step can be checked on its own. */

/* Validate a CSR matrix: square, monotone rowptr starting at 0, columns in
 * [0, n), finite values, not all zero. Returns COND_OK or COND_EINVAL. */
int cond_csr_check(const cond_csr_t* A);

/* Explicit transpose A^T in CSR (the gradient of equation nabla_loss needs
 * A^T A v). Output arrays are caller-allocated: t_rowptr[n+1], t_col[nnz],
 * t_val[nnz]. Stable: within a row of A^T, entries appear in increasing row
 * order of A. */
int cond_csr_transpose(const cond_csr_t* A, int64_t* t_rowptr, int32_t* t_col, double* t_val);

/* Fill-reducing order of the symmetric pattern of A + A^T by recursive
 * level-structure bisection (nested dissection). perm[k] = the column of A
 * placed at position k. */
int cond_order_nd(const cond_csr_t* A, int32_t* perm);

/* Sparse LU with threshold partial pivoting, P A Q = L U (Algorithm 2 writes
 * A = L U; the permutations are this library's choice). L is unit lower
 * triangular, U upper triangular. col_perm may be NULL (nested dissection).
 * pivot_tol as in cond_opts_t. Fails with COND_ESINGULAR on a zero pivot
 * column. */
int cond_lu_factor(const cond_csr_t* A, const int32_t* col_perm, double pivot_tol, cond_lu_t** lu);
void cond_lu_destroy(cond_lu_t* lu);
/* nnz of strictly-lower L and of U (diagonal included). */
int cond_lu_info(const cond_lu_t* lu, int32_t* n, int64_t* nnz_l, int64_t* nnz_u);
/* Copy out the factors as CSR in pivot order plus the permutations:
 * row_perm[k] = row of A that is row k of P A; col_perm[k] = column of A that
 * is column k of A Q. Any output pointer may be NULL to skip it. l_* hold the
 * strictly lower part of L; u_* the strictly upper part of U; u_diag the
 * diagonal of U. */
int cond_lu_export(const cond_lu_t* lu, int64_t* l_rowptr, int32_t* l_col, double* l_val,
                   int64_t* u_rowptr, int32_t* u_col, double* u_val, double* u_diag,
                   int32_t* row_perm, int32_t* col_perm);
/* Host reference solve with the factors: trans = 0 gives r = A^-1 x,
 * trans = 1 gives r = A^-T x. */
int cond_lu_solve_host(const cond_lu_t* lu, int trans, const double* x, double* r);

/* ------------------------------------------------------------ device plan
 * cond_plan_create does the host set-up (validation, A^T, and for the
 * sigma_min route the ordering and the LU); cond_plan_workspace_bytes says
 * how much device memory the plan needs; cond_plan_bind takes that memory
 * (workspace != NULL: caller-owned, e.g. allocated by PyTorch; NULL: the
 * library allocates it with hipMalloc and frees it in destroy) and uploads
 * the matrices on the given stream (hipStream_t; NULL = default stream).
 * Every later device call of this plan is enqueued on that stream. */
int cond_plan_create(const cond_csr_t* A, const cond_opts_t* o, cond_plan_t** plan);
int cond_plan_workspace_bytes(const cond_plan_t* plan, size_t* bytes);
int cond_plan_bind(cond_plan_t* plan, void* workspace, size_t bytes, void* stream);
void cond_plan_destroy(cond_plan_t* plan);

/* Run both Projected Adam passes and assemble kappa. x0_max, x0_min: device
 * start vectors of length n (any non-zero scale; normalised inside; x0_min
 * may equal x0_max; x0_min = NULL uses x0_max). x0_max = NULL with x0_min
 * given runs the sigma_min pass alone (sigma_max, iters_max and kappa are
 * then 0); both NULL is COND_EINVAL. trace_max / trace_min: optional device arrays of length
 * o->max_iter receiving best-sigma after each evaluated iterate (trace[t-1] =
 * best over x_1..x_t; for the sigma_min run the values are ||A^-1 x||, i.e.
 * 1/sigma_min estimates). x_best_max / x_best_min: optional device outputs
 * (length n) of the maximising iterates. o may differ from the create-time
 * options only in alpha, beta1, beta2, eps, max_iter, stop_*, chunk.
 * Returns after the result is on the host. */
int cond_plan_run(cond_plan_t* plan, const cond_opts_t* o, const double* x0_max,
                  const double* x0_min, cond_result_t* out, double* trace_max,
                  double* trace_min, double* x_best_max, double* x_best_min);

/* Kernel ids of cond_plan_kernel_stats. */
#define COND_K_NORMALISE 0
#define COND_K_SPMV_A 1
#define COND_K_SPMV_AT 2
#define COND_K_SUMSQ 3
#define COND_K_TRSV_L 4
#define COND_K_TRSV_U 5
#define COND_K_TRSV_UT 6
#define COND_K_TRSV_LT 7
#define COND_K_ADAM1 8
#define COND_K_ADAM2 9
#define COND_K_COUNT 10

/* Per-kernel device time of the last cond_plan_run with opts.profile = 1:
 * ms[k] = total milliseconds and launches[k] = number of launches of kernel
 * k (arrays of COND_K_COUNT entries, caller-allocated). Also reports the
 * algorithmic bytes one launch of each kernel must move (bytes[k], may be
 * NULL): matrix/factor entries 12 B each plus row pointers and every vector
 * read or written once. */
int cond_plan_kernel_stats(const cond_plan_t* plan, double* ms, int64_t* launches, double* bytes);

/* Schedule of the four triangular solves of Algorithm 2 (order L, U, U^T,
 * L^T; caller-allocated arrays of 4): dependency levels of the panel graph
 * (its longest chain), tasks handed out per solve (whole panels, slices and
 * finish steps) and panels. Host data, available after cond_plan_create;
 * COND_EINVAL for a plan without the sigma_min route. */
int cond_plan_solve_info(const cond_plan_t* plan, int32_t* levels, int64_t* tasks, int64_t* panels);

/* Algorithm 2's r = A^-1 x and s = A^-T r (x, r, s: host arrays of length
 * n, caller-owned) computed on the host from the same device-ready data the
 * four solves run on -- task records, slices and their partial-sum slots,
 * packed inverses of the panel triangles, right-hand-side gathers and
 * output scatters -- taking the tasks in ticket order. For checking the
 * solve schedule without a device; available after cond_plan_create.
 * COND_ESTATE if a task would read a value that only a later ticket solves,
 * or a slot no slice wrote (the device would then wait on work handed out
 * after it); COND_EINVAL for a plan without the sigma_min route; COND_ENOMEM
 * if host scratch cannot be allocated. */
int cond_plan_solve_replay(const cond_plan_t* plan, const double* x, double* r, double* s);

/* One step of the path at a time, on device vectors of length n (for checks
 * against the oracle): y = A x; y = A^T x; r = A^-1 x and s = A^-T r
 * (Algorithm 2). Asynchronous on the plan's stream. */
/* Test hook for the failure path: the next sigma_min run or inverse apply
 * of this plan starts as if one of its triangular-solve waits had already
 * timed out, so every solve kernel exits at once and the call reports
 * COND_ETIMEOUT, with no kernel waiting on anything. The call after that
 * re-arms the solves' slice slots and runs normally, as after a real
 * time-out. COND_EINVAL for a plan without the sigma_min route. */
int cond_plan_inject_timeout(cond_plan_t* plan);
int cond_plan_spmv(cond_plan_t* plan, int transpose, const double* x, double* y);
/* flags of cond_plan_spmv's `transpose` argument: bit 0 = A^T; bit 1 = the
 * column-scaled matrix, y = (A D^-1) x or (A D^-1)^T x */
#define COND_SPMV_T 1
#define COND_SPMV_COLSCALED 2

/* The column norms of A, d_j = ||A[:, j]||_2 (section "Row and Column
 * Scaling", D_col), computed on the device as row norms of the stored A^T,
 * into the device array d (n doubles, caller-owned). Returns after d is
 * written. */
int cond_plan_column_norms(cond_plan_t* plan, double* d);
int cond_plan_inverse_apply(cond_plan_t* plan, const double* x, double* r, double* s);

/* ---------------------------------------------------- batched multi-start
 * Many matrices of uneven size, 8 starts each, in one launch per phase of
 * the sigma_max run (Algorithm 1 with M = A for every (matrix, start) pair;
 * the arithmetic of each pair is the plain method's, only the order of the
 * additions inside its global sums differs). The matrices are concatenated
 * block-diagonally: matrix m owns global rows [row0[m], row0[m+1]), and the
 * 8 starts of a row are interleaved, element (i, k) at index 8*i + k.
 *
 * cond_batch_create: host set-up (validation, A^T of every matrix, the
 * concatenation). cond_batch_info: row0 (count+1 entries, host), workspace
 * size, and after bind the tile schedule in use. cond_batch_bind: takes the
 * workspace as cond_plan_bind does, uploads, and picks the row-tile size and
 * grid by timing the A-product for each candidate on this batch (an
 * autotuner), unless tile_rows and grid are both given (> 0), which fixes the
 * schedule and makes runs reproducible bit for bit across processes.
 * cond_batch_run: x0 is a device array of (row0[count]) * 8 doubles; results
 * on the host: sigma_max[count] = the largest best over a matrix's starts
 * (each start gives a lower bound), pair_best / pair_iters / pair_status
 * [count * 8] per (matrix, start) (any of them may be NULL); trace (device,
 * count * 8 * max_iter, optional) receives each pair's running best per
 * update; x_best (device, optional) the best iterates; ms the device time. */
typedef struct cond_batch cond_batch_t;
int cond_batch_create(const cond_csr_t* As, int32_t count, const cond_opts_t* o, cond_batch_t** b);
int cond_batch_info(const cond_batch_t* b, int64_t* row0, size_t* workspace_bytes,
                    int32_t* tile_rows, int32_t* grid);
int cond_batch_bind(cond_batch_t* b, void* workspace, size_t bytes, void* stream,
                    int32_t tile_rows, int32_t grid);
int cond_batch_run(cond_batch_t* b, const cond_opts_t* o, const double* x0, double* sigma_max,
                   double* pair_best, int64_t* pair_iters, int32_t* pair_status, double* trace,
                   double* x_best, double* ms);
void cond_batch_destroy(cond_batch_t* b);

/* The batched sigma_min run (Algorithm 2 for every (matrix, start) pair).
 * Needs a batch created with o->sigma_min_method = COND_MIN_LU: create then
 * factors every matrix on the host (P_m A_m Q_m = L_m U_m, in parallel
 * threads, one matrix per thread) and merges the factors block-diagonally,
 * each matrix's pivot rows kept together; each update's four triangular
 * solves then take every matrix and all 8 starts in one launch each (one
 * read of a factor entry serves the 8 starts, and the matrices' dependency
 * levels overlap). Arguments as cond_batch_run; pair_best receives each
 * pair's largest ||A^-1 x|| / ||x|| and sigma_min[count] = 1 / the largest
 * over a matrix's starts (each start gives an upper bound of sigma_min).
 * COND_ESTATE for a batch created without the route. */
int cond_batch_run_min(cond_batch_t* b, const cond_opts_t* o, const double* x0, double* sigma_min,
                       double* pair_best, int64_t* pair_iters, int32_t* pair_status, double* trace,
                       double* x_best, double* ms);
/* Algorithm 2's r = A_m^-1 x and s = A_m^-T r for every (matrix, start) on
 * the host, from the same merged factors and solve schedules the device
 * runs (tasks in ticket order); x, r, s: host arrays in the batch layout
 * (row0[count] * 8). For checking the batched solves without a device.
 * COND_ESTATE if a task would read a value solved by a later ticket;
 * COND_EINVAL for a batch without the sigma_min route. */
int cond_batch_solve_replay(const cond_batch_t* b, const double* x, double* r, double* s);
/* Fill of the merged factors (strictly lower L; U with its diagonal) and the
 * host time of the per-matrix LUs, of a batch with the sigma_min route. */
int cond_batch_fill(const cond_batch_t* b, int64_t* nnz_l, int64_t* nnz_u, double* lu_ms);

/* kappa_2 of every matrix of a batch: create (with the LUs) + bind (library
 * memory, autotuned schedule) + the sigma_max and sigma_min runs + destroy.
 * x0_max, x0_min: device start vectors in the batch layout (8 starts per
 * row, rows of the matrices concatenated; x0_min = NULL uses x0_max).
 * outs[count]: per matrix sigma_max, sigma_min and kappa from its best
 * starts, iters_max / iters_min = the most updates any of its starts took,
 * status of its first failed start (if any), flags (COND_F_NUMSING), the
 * device time of each whole batched run and the set-up time. */
int cond_estimate_batched(const cond_csr_t* As, int32_t count, const cond_opts_t* o,
                          const double* x0_max, const double* x0_min, void* stream,
                          cond_result_t* outs);

/* ------------------------------------------------------ learned warm start
 * A start vector for the sigma_min run (Algorithm 2) predicted from the two
 * coefficient fields of a hydro-mechanical grid by a small CNN: four 3x3
 * zero-padded convolutions, 2 -> 64 -> 64 -> 64 -> 6 channels, ReLU after the
 * first three. bfloat16 weights and activations, float32 accumulation on the
 * matrix cores; float32 master weights trained by Adam on the loss
 * l = 1 - (p.u)^2 / ((p.p)(u.u)) against minimisers u found by plain runs.
 * The paper has no such network; a start only changes how many updates the
 * run needs, never what it computes, and callers keep a random start beside
 * it (the larger lower bound wins).
 *
 * Parameters: one float32 vector of cond_cnn_param_count() values, layer by
 * layer, W[ky][kx][ci][co] then b[co]. Fields: device float64 array
 * [batch][2][side-1][side-1] of per-cell log10 viscosity and log10
 * permeability. Start vectors: device float64 [batch][6 side^2] in the
 * matrix's node-major order 6 (i side + j) + f. Labels: device float32 in the
 * same layout. Every sample of a call has the same side.
 *
 * cond_cnn_create: device buffers for up to max_batch samples of side up to
 * max_side, with the training buffers if train != 0; all work goes on
 * `stream` (0 = the null stream) and every call returns after its work has
 * finished. cond_cnn_set_params uploads parameters (host) and resets Adam.
 * cond_cnn_predict writes x0. cond_cnn_gradients writes the gradient of the
 * batch's mean loss (host float32, param_count values, may be NULL) and the
 * per-sample losses (host, batch values, may be NULL). cond_cnn_train_step
 * does the same forward and backward, then one Adam step (beta1 0.9, beta2
 * 0.999, eps 1e-8) with rate lr; mean_loss (host, may be NULL) receives the
 * batch's mean loss before the step. cond_cnn_activation copies layer
 * `layer`'s stored activation of the last call (0 = input, 1..3 = hidden
 * outputs, channels padded to 8, 64, 64, 64, as float32 [batch][side][side]
 * [channels]; 4 = the float32 output padded to 16 channels) to host memory.
 * Errors: COND_EINVAL for sizes beyond those given at create or NULL
 * required pointers, COND_ESTATE for training calls on a network created
 * without training buffers, COND_EHIP for runtime failures. */
typedef struct cond_cnn cond_cnn_t;
int cond_cnn_param_count(void);
int cond_cnn_create(int32_t max_batch, int32_t max_side, int32_t train, void* stream,
                    cond_cnn_t** out);
int cond_cnn_set_params(cond_cnn_t* net, const float* params);
int cond_cnn_get_params(const cond_cnn_t* net, float* params);
int cond_cnn_predict(cond_cnn_t* net, const double* fields, int32_t batch, int32_t side, double* x0);
int cond_cnn_gradients(cond_cnn_t* net, const double* fields, const float* labels, int32_t batch,
                       int32_t side, float* grad, float* losses);
int cond_cnn_train_step(cond_cnn_t* net, const double* fields, const float* labels, int32_t batch,
                        int32_t side, float lr, float* mean_loss);
int cond_cnn_activation(const cond_cnn_t* net, int32_t layer, int32_t batch, int32_t side,
                        float* host);
void cond_cnn_destroy(cond_cnn_t* net);

/* Measurement: the streaming ceiling of the device. a = b + scale c over n
 * doubles (device arrays, 16-byte aligned, caller-owned; 24 n bytes move per
 * launch), `grid` blocks of 256 threads, timed over `reps` launches after one
 * warm-up on `stream`; *ms = average milliseconds per launch. The HBM-bound
 * kernels of the estimator are quoted against this as well as against the
 * vendor peak. */
int cond_stream_triad(int64_t n, double* a, const double* b, const double* c, double scale,
                      int32_t grid, int32_t reps, void* stream, double* ms);

/* ------------------------------------------------------------ error bounds
 * What the paper computes kappa for (section "Error estimates and
 * conditioning"): bounds on the error of an approximate solution x_hat of
 * A x = b from its residual b_hat - b = A x_hat - b, kappa = kappa_2(A) and
 * ||A||_2 = sigma_max (both from cond_plan_run). All norms are 2-norms. */
typedef struct {
  double res_norm;          /* ||A x_hat - b|| */
  double b_norm, x_norm;    /* ||b||, ||x_hat|| */
  double rel_residual;      /* ||A x_hat - b|| / ||b|| */
  double err_x_lower;       /* Theorem "Bounds on the relative error ||x_hat - x|| / ||x||": */
  double err_x_upper;       /*   rel_residual / kappa <= . <= kappa rel_residual */
  double err_xhat_lower;    /* Theorem "Bounds on the relative error ||x_hat - x|| / ||x_hat||": */
  double err_xhat_upper;    /*   ||r|| / (||A|| ||x_hat||) <= . <= kappa ||r|| / (||A|| ||x_hat||) =: epsilon */
  double err_x_tight;       /* Theorem "Tight upper bound of the error": epsilon / (1 - epsilon)
                               bounds ||x_hat - x|| / ||x||; +inf when epsilon >= 1 */
  double roundoff_floor;    /* Theorem "Numerical singularity of a matrix": 2 eps kappa /
                               (1 - kappa eps), eps = 2^-52; +inf when kappa eps >= 1 */
} cond_bounds_t;

/* Bounds for x_hat and b (device arrays of length n, on the plan's device;
 * ordered after the work the caller queued on the plan's stream) with the
 * plan's A. kappa >= 1 and norm_a > 0, both finite, else COND_EINVAL;
 * COND_ENUMERIC when b or x_hat is zero or a norm is not finite. The
 * residual's partial sums use the plan's workspace; returns after the result
 * is on the host. */
int cond_plan_error_bounds(cond_plan_t* plan, const double* x_hat, const double* b, double kappa,
                           double norm_a, cond_bounds_t* out);

/* The same bounds for callers that cannot allocate device memory (code that
 * must not call hipMalloc, e.g. inside a serving loop): A is given on the
 * device as CSR (rowptr int64 [n+1], col int32 [nnz], val [nnz]; caller-owned,
 * columns in [0, n)), x_hat and b as device arrays of length n, all on the
 * current device; work is enqueued on `stream` (hipStream_t, NULL = the null
 * stream) and the call returns after the result is on the host. The
 * residual's block partials and sums live in a fixed scratch array inside
 * the library, 4 x 2048 doubles (64 KiB) per device, held until the process
 * ends; a launch uses at most 2048 blocks, so no n exceeds it, and every
 * call writes every slot it reads (nothing carries over between calls).
 * Calls that overlap on one device share that array and race: serialise
 * them. Same arguments and results as cond_plan_error_bounds (which it
 * matches bit for bit on the same data); COND_EINVAL also for n < 1,
 * nnz < 0 or a null pointer. */
int cond_error_bounds_noalloc(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
                              const double* val, const double* x_hat, const double* b,
                              double kappa, double norm_a, void* stream, cond_bounds_t* out);

/* create + bind (library-owned memory) + run + destroy. */
int cond_estimate(const cond_csr_t* A, const cond_opts_t* o, const double* x0_max,
                  const double* x0_min, void* stream, cond_result_t* out);

#ifdef __cplusplus
}
#endif

#endif /* CONDEST_H */
