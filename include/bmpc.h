/*
 * bmpc.h -- C ABI of the MI355X (gfx950) direct solver for root-coupled branch-MPC
 * systems: the two-level (scenario x horizon) parallel Cholesky factorization and
 * triangular solves of "Accelerating Branch MPC with Two-Level Parallel Direct Solves
 * on GPUs" (Algorithms 1 and 2), plus mixed-precision iterative refinement.
 *
 * The system (Section III-B, eq. (root_coupled_matrix), eq. (tail_block_tridiagonal)):
 *
 *        [ K_1               C_1^T ]        K_s = block-tridiagonal, N blocks n x n:
 *    K = [      ...           ...  ]              D_{s,k} on the diagonal,
 *        [           K_S     C_S^T ]              E_{s,k} at block (k+1, k),
 *        [ C_1  ...  C_S     R     ]              E_{s,k}^T at block (k, k+1);
 *                                          C_s couples the root to stage 0 of tail s.
 *
 * Notation: S scenarios (the paper's M), N stages, block size n (the paper's n_b,
 * Assumption 1), nrhs right-hand sides.  Stages are 0-based: stage k is the paper's
 * stage k+1, so the root-coupled stage (the paper's x_1) is stage 0.
 *
 * Layouts (all row-major n x n blocks, FP64, DEVICE pointers unless stated):
 *   D  [S][N][n][n]     only the lower triangle of each block is read
 *   E  [S][N-1][n][n]   E[s][k] is block (k+1, k) of tail s (may be NULL when N == 1)
 *   C  [S][n][n]        block (root, stage 0)
 *   R  [n][n]           only the lower triangle is read
 *   b, x [nrhs][(S*N+1)*n]  each right-hand side in the paper's partition
 *                       (r^1_1..r^1_N, ..., r^S_1..r^S_N, r_0): tails in forward stage
 *                       order, the root block last.
 * The library never keeps a caller pointer after a call returns.
 *
 * Batches.  A plan may hold B = num_systems (bmpc_options) independent systems of the
 * same dims, factored and solved together in the same launches.  Their arrays are
 * stacked along the leading dimension: D [B*S][N][n][n], E [B*S][N-1][n][n],
 * C [B*S][n][n] (system i owns scenarios i*S .. i*S+S-1), R [B][n][n] and
 * b, x [B][nrhs][(S*N+1)*n].  Everything below holds per system; with B = 1 these
 * are the single-system layouts above.
 *
 * Streams and ordering.  Every device operation is enqueued on the plan's stream
 * (hipStream_t passed as void*; NULL = the legacy default stream) and is
 * asynchronous unless stated.  The library allocates device memory only in
 * bmpc_analyze; factor/solve/refine allocate nothing and launch no memset, so the
 * sequence can be captured into a HIP graph.  Calls on one plan must not overlap.
 *
 * Errors.  Argument and state errors are reported synchronously by the return value.
 * Numerical breakdown (a non-positive pivot) is recorded on the device and read by
 * bmpc_get_info.
 */
#ifndef BMPC_H
#define BMPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BMPC_OK = 0,
  BMPC_ERR_INVALID = -1,       /* bad argument (dims, NULL pointer, unsupported n) */
  BMPC_ERR_NOT_SPD = -2,       /* returned by bmpc_get_info when info != 0 */
  BMPC_ERR_ALLOC = -3,         /* device allocation failed in bmpc_analyze */
  BMPC_ERR_DEVICE = -4,        /* a HIP call failed */
  BMPC_ERR_STATE = -5,         /* solve/refine before a factor on this plan */
  BMPC_ERR_NOT_CONVERGED = -6  /* bmpc_get_stats: refinement hit max_iters */
} bmpc_status;

typedef enum {
  BMPC_FP64 = 0,        /* factor, solve and reductions in FP64 */
  BMPC_FP32_REFINE = 1  /* tail factor + solves in FP32 (FP32 accumulation); root
                           reduction, root Cholesky and refinement residual in FP64 */
} bmpc_precision;

typedef struct {
  int32_t S;    /* scenarios, >= 1 */
  int32_t N;    /* stages per tail, >= 1 */
  int32_t n;    /* block size n_b (Assumption 1, uniform), 1..64.  Blocks of 33..64
                   are factored one level per pass (two 32 x 32 quadrants per block
                   dimension) and without the fused forward substitution */
  int32_t nrhs; /* right-hand sides per solve, 1..4096 (Section III-B partitions each
                   right-hand side like the unknowns; their number is free).  The
                   kernels take them in chunks of 8 (n <= 32) or 4 (n > 32). */
} bmpc_dims;

/* bmpc_options.flags */
#define BMPC_FLAG_NO_BWD_TOP_MERGE 0x1 /* backward sweep: one launch per level (one wave
                                          per position) even where the top levels could
                                          share one launch (one workgroup per chain) */
#define BMPC_FLAG_FWD_ONE_WAVE 0x2     /* forward sweep: one wave per position instead of
                                          up to four sharing its pulls */

typedef struct {
  int32_t window_depth; /* 0 = automatic; else levels eliminated per factor pass
                           (1..6), bounded by the shared-memory budget */
  int32_t num_systems;  /* 0 or 1: one system; B > 1: a batch of B independent
                           systems of the same dims (layouts: see "Batches") */
  int32_t flags;        /* BMPC_FLAG_* bits, 0 = defaults */
  int32_t later_depth;  /* levels per factor pass after the first: 0 = automatic,
                           else 1..6 (bounded like window_depth).  The reduced chains
                           of the later passes are 2^window_depth times shorter; a
                           smaller depth there gives each chain more workgroups */
  int32_t reserved[4];
} bmpc_options;

/* Stop tests of bmpc_refine / bmpc_factor_refine (bmpc_set_refine_stop). */
typedef enum {
  BMPC_STOP_CORRECTION = 0,     /* |d|_inf <= tol |x|_inf for the last correction d */
  BMPC_STOP_BACKWARD_ERROR = 1  /* |b - K x|_inf <= tol (|K|_inf |x|_inf + |b|_inf) */
} bmpc_refine_stop;

typedef struct {
  double factor_flops;    /* exact flop count of Algorithm 1 (method's count) */
  double solve_flops;     /* exact flop count of Algorithm 2 for all nrhs */
  double factor_bytes;    /* algorithmic HBM bytes: read K (lower triangles of
                             D, R), write the factor */
  double solve_bytes;     /* algorithmic HBM bytes: read the factor twice, read b,
                             write x */
  double residual_bytes;  /* algorithmic bytes of one FP64 residual b - K x */
  int32_t levels;         /* elimination levels of one tail, x_1 included */
  int32_t passes;         /* factor passes (kernel launches over the chains) */
  int32_t window_depth;   /* levels of the first factor pass actually used */
  int32_t later_depth;    /* levels of each later factor pass */
  double workspace_bytes; /* device memory owned by the plan */
} bmpc_cost;

typedef struct bmpc_plan_s* bmpc_plan;

/* One-time analysis (the paper's analysis phase, Section V: fixed sparsity allows
 * persistent workspaces).  Validates dims, builds the ordering Pi_i
 * (Section IV-A: reverse the tail, apply Gamma_{N-1} to (x_N..x_2), keep x_1 last),
 * the level table and the factor structure, and allocates every workspace.  Reads
 * no caller array.  BMPC_ERR_INVALID for bad dims (S, N < 1; n outside 1..64; nrhs
 * outside 1..4096; or sizes whose element counts would overflow the 32-bit grid and
 * index arithmetic: S*N*n < 2e9, nrhs*(S*N+1)*n < 4e9 per plan),
 * BMPC_ERR_ALLOC when device memory runs out, BMPC_ERR_DEVICE if no GPU.
 * On success *out owns its workspaces until bmpc_destroy. */
bmpc_status bmpc_analyze(const bmpc_dims* dims, bmpc_precision prec, void* stream,
                         bmpc_plan* out);
bmpc_status bmpc_analyze_ex(const bmpc_dims* dims, bmpc_precision prec, void* stream,
                            const bmpc_options* opts, bmpc_plan* out);

/* Ragged batch: B independent systems of different shapes dims[i] = (S_i, N_i, n_i,
 * nrhs) -- n_i <= 32, one nrhs for all -- in one plan (not one of the paper's
 * algorithms: it batches many of its systems).  Each system gets its own ordering
 * Pi_i, level table and workspaces; each step of Algorithm 1, Algorithm 2 and the
 * refinement is then one launch over every system that takes part in it (per block-size
 * class and kernel variant), its work items -- chain windows, chain positions, root
 * blocks -- ordered largest system first.  Arrays are the systems' own layouts above
 * (B = 1 each), concatenated in system order: D = [D_0 | D_1 | ...], likewise E
 * (N_i - 1 blocks per tail; E must not be NULL), C, R, and b, x = [b_0 | b_1 | ...] with
 * b_i [nrhs][(S_i N_i + 1) n_i]; bmpc_ragged_layout gives the offsets.  The plan works
 * with bmpc_factor, bmpc_solve, bmpc_factor_solve, bmpc_refine, bmpc_factor_refine,
 * bmpc_get_info (rows of the concatenated systems), bmpc_get_stats (the stop test holds
 * for every system), bmpc_query_cost (sums), bmpc_export_tail_factor (chains of the
 * concatenated systems), bmpc_export_root_factor (the n_i x n_i factors one after the
 * other), bmpc_set_stream, bmpc_set_refine_stop, the profiling calls and
 * bmpc_destroy; bmpc_query_perm, bmpc_query_structure and bmpc_grad_blocks return
 * BMPC_ERR_INVALID (the host-only bmpc_ordering and bmpc_structure give each system's
 * Pi_i and structure).  opts: NULL (defaults) or B option structs, one per system
 * (window_depth, flags; num_systems 0 or 1), e.g. from bmpc_autotune per shape class.
 * BMPC_ERR_INVALID for B < 1 or bad dims. */
bmpc_status bmpc_analyze_ragged(int32_t B, const bmpc_dims* dims, bmpc_precision prec,
                                void* stream, const bmpc_options* opts, bmpc_plan* out);

/* Shape of system i of a ragged plan and the element offsets of its arrays in the
 * concatenated D, E, C, R and vectors (offsets[0..4]); either output may be NULL. */
bmpc_status bmpc_ragged_layout(bmpc_plan plan, int32_t i, bmpc_dims* dims, int64_t* offsets);

/* Autotuner: for the shape dims, a batch of num_systems such systems (0 or 1: one) and
 * the precision, builds a plan for every candidate launch configuration --
 * window_depth from 1 to the largest the shared memory allows, crossed with
 * BMPC_FLAG_NO_BWD_TOP_MERGE (the backward sweep's top levels in one launch, one
 * workgroup per chain, or one launch per level, one wave per position) and
 * BMPC_FLAG_FWD_ONE_WAVE (forward positions on up to four waves or on one) -- times the
 * plan's step (FP64: bmpc_factor_solve; FP32: bmpc_factor_refine with one correction) on
 * synthetic SPD data in device memory (allocated here and freed), the median of reps
 * runs (1..100) after one warm-up, and writes the fastest configuration to *best
 * (num_systems 0) and its time to *best_ms.  One small system measures latency; a batch
 * that fills the GPU measures throughput, the right criterion for a system that shares
 * the GPU with many others (a ragged batch).  times (cap entries, may be NULL with
 * cap = 0) receives each candidate's median in the order tried, *count the number
 * tried.  Synchronizes the stream; not capturable.  BMPC_ERR_ALLOC if no candidate
 * fits in device memory. */
bmpc_status bmpc_autotune(const bmpc_dims* dims, int32_t num_systems, bmpc_precision prec,
                          void* stream, int32_t reps, bmpc_options* best, double* best_ms,
                          double* times, int32_t cap, int32_t* count);

/* Replace the stream later calls enqueue on (e.g. a graph-capture stream). */
bmpc_status bmpc_set_stream(bmpc_plan plan, void* stream);

/* Stop test of later bmpc_refine / bmpc_factor_refine calls on this plan (a
 * bmpc_refine_stop value); BMPC_ERR_INVALID for another value. */
bmpc_status bmpc_set_refine_stop(bmpc_plan plan, int32_t stop);

/* Algorithm 1: L_i = chol(Pi_i K_i Pi_i^T) for every tail (horizon-parallel block
 * elimination in the Gamma order), F_{i,1} = C_{i,1} L_{i,1}^{-T},
 * U_i = F_{i,1} F_{i,1}^T, R~ = R - sum_i U_i (FP64, fixed summation order) and
 * L_R = chol(R~) (FP64).  Device pointers D, E, C, R as described above; the factor
 * stays in the plan.  Asynchronous; a non-positive pivot is recorded for
 * bmpc_get_info and leaves the factor unspecified. */
bmpc_status bmpc_factor(bmpc_plan plan, const double* D, const double* E,
                        const double* C, const double* R);

/* Algorithm 2: x = K^{-1} b with the factor of the last bmpc_factor: tail forward
 * substitution, root reduction r~_0 = r_0 - sum F_{i,1} dy_1^i and root solves in
 * FP64, root propagation, tail backward substitution, inverse permutation.
 * b and x are device arrays [nrhs][(S*N+1)*n]; x may alias b.  In a
 * BMPC_FP32_REFINE plan this is the plain FP32 solve (no refinement).
 * BMPC_ERR_STATE if no factor has been issued. */
bmpc_status bmpc_solve(bmpc_plan plan, const double* b, double* x);

/* Mixed-precision iterative refinement (not in the paper; classical scheme, Moler
 * 1967): x = solve(b); then repeat r = b - K x in FP64 from the caller's FP64
 * blocks, d = solve(r / |r|_inf) * |r|_inf, x += d, until the plan's stop test holds
 * for every right-hand side (and system of a batch) or max_iters corrections were
 * applied.  Stop tests (bmpc_set_refine_stop):
 *   BMPC_STOP_CORRECTION (default): |d|_inf <= tol |x|_inf after a correction d;
 *   BMPC_STOP_BACKWARD_ERROR: the normwise backward error of x,
 *     |b - K x|_inf / (|K|_inf |x|_inf + |b|_inf) <= tol, on the FP64 residual the
 *     loop forms anyway (|K|_inf = the largest row sum of |K|, taken in the first
 *     residual); a converged x needs no further correction, and an x that passes the
 *     test is certified by its own residual, so max_iters corrections take up to
 *     max_iters + 1 residuals (tol = c * 2^-53 with c of order 10 asks for the backward
 *     stability of an FP64 solve).
 * Needs the factor of the same D, E, C, R.  x on entry is ignored.  The stop test runs
 * on the device (later launches of a converged loop return at once), so under stream
 * capture the launch sequence is fixed and capturable.  Outside capture the host also
 * reads the stop flag after each test (a synchronization of the plan's stream) and
 * issues nothing more once it holds, so the call returns after the work is done.
 * max_iters in 0..100. */
bmpc_status bmpc_refine(bmpc_plan plan, const double* D, const double* E,
                        const double* C, const double* R, const double* b, double* x,
                        double tol, int32_t max_iters);

/* bmpc_factor followed by bmpc_solve(b, x), with the tail forward substitution
 * (the tail forward steps of Algorithm 2) carried out inside the factorization: each
 * chain position applies its L_jj^{-1} to its right-hand side when it is eliminated
 * and passes -G y_j to its two neighbours, in the elimination order of Algorithm 1, so the
 * forward sweep does not read the factor again.  Same result as the two calls up to
 * rounding order; same arguments and errors as bmpc_factor and bmpc_solve (x may
 * alias b).  The factor stays in the plan for later bmpc_solve calls. */
bmpc_status bmpc_factor_solve(bmpc_plan plan, const double* D, const double* E,
                              const double* C, const double* R, const double* b, double* x);

/* bmpc_factor followed by bmpc_refine, with the first solve's forward substitution
 * inside the factorization as in bmpc_factor_solve; the correction solves are
 * ordinary solves.  Same arguments and errors as bmpc_refine (x must not alias b),
 * except that no earlier factor is needed. */
bmpc_status bmpc_factor_refine(bmpc_plan plan, const double* D, const double* E,
                               const double* C, const double* R, const double* b, double* x,
                               double tol, int32_t max_iters);

/* Gradients of a loss through x = K^{-1} b (not one of the paper's algorithms; the
 * derivative of its linear solve).  Differentiating K x = b for a loss l with
 * g = dl/dx gives the adjoint lam = K^{-1} g (K is symmetric: call bmpc_solve on g
 * with the same factor), dl/db = lam and the dense gradient dl/dK = -lam x^T summed
 * over the right-hand sides.  This call writes what each block array receives from
 * the entries of K it fills (eq. (root_coupled_matrix), eq. (tail_block_tridiagonal)):
 *   dD[s][k] = -sym(sum_q lam_{s,k} x_{s,k}^T)     (both triangles written)
 *   dE[s][k] = -sum_q (lam_{s,k+1} x_{s,k}^T + x_{s,k+1} lam_{s,k}^T)
 *   dC[s]    = -sum_q (lam_0 x_{s,0}^T + x_0 lam_{s,0}^T)
 *   dR       = -sym(sum_q lam_0 x_0^T)
 * with sym(A) = (A + A^T)/2 (symmetric arguments get symmetric gradients), x_{s,k}
 * the stage-k part of tail s and x_0 the root part.  x, lam: device arrays
 * [nrhs][(S*N+1)*n] in the layout of b.  dD [S][N][n][n], dE [S][N-1][n][n],
 * dC [S][n][n], dR [n][n]: device arrays, overwritten; any may be NULL to skip it
 * (dE is ignored when N == 1).  Needs no factor.  Asynchronous on the plan's stream.
 * BMPC_ERR_INVALID for a NULL plan, x or lam. */
bmpc_status bmpc_grad_blocks(bmpc_plan plan, const double* x, const double* lam, double* dD,
                             double* dE, double* dC, double* dR);

/* Synchronizes the plan's stream.  *info = 0 after a successful factor; otherwise
 * the 1-based natural row index (tails first, root last, as in b; in a batch the
 * systems follow each other, (S*N+1)*n rows each) of the first non-positive pivot in
 * the elimination order Pi, and the call returns BMPC_ERR_NOT_SPD. */
bmpc_status bmpc_get_info(bmpc_plan plan, int64_t* info);

/* Synchronizes.  Corrections applied by the last bmpc_refine and its final stop-test
 * quantity, the largest over the right-hand sides (and systems of a batch; the stop
 * test holds for each of them): |d_q|_inf / |x_q|_inf of the last correction
 * (BMPC_STOP_CORRECTION) or the normwise backward error of the returned x
 * (BMPC_STOP_BACKWARD_ERROR).  Returns BMPC_ERR_NOT_CONVERGED if the stop test was not
 * met within max_iters. */
bmpc_status bmpc_get_stats(bmpc_plan plan, int32_t* iters, double* rel_correction);

/* Host copies of the analysis.  perm: int32[N], the 0-based stage at each permuted
 * position of a tail (the same for every tail; x_1 = stage 0 is last). */
bmpc_status bmpc_query_perm(bmpc_plan plan, int32_t* perm);
/* The factor's block structure under the plan's ordering (Theorem 1 and the
 * elimination levels of Section IV-A): the same pairs as bmpc_structure(N) for the
 * plan's N -- one tail (positions 0..N-1 in permuted order) plus the root (N); every
 * tail of every system has it.  Writes at most cap pairs, *count = the full number
 * (cap = 0 sizes). */
bmpc_status bmpc_query_structure(bmpc_plan plan, int32_t* rows, int32_t* cols, int64_t cap,
                                 int64_t* count);
bmpc_status bmpc_query_cost(bmpc_plan plan, bmpc_cost* cost);

/* Algorithmic HBM bytes and flops that kernel class cls (see bmpc_kernel_class_name)
 * moves / performs in one call of the entry point that launches it (bmpc_factor for
 * the factor classes, one solve sweep for the solve classes, one residual for the
 * residual classes), and the number of launches of that class per such call.  For
 * the factor passes: the D blocks read and the factor blocks written by the
 * positions the pass eliminates (the first pass also reads every E block).  Any
 * output pointer may be NULL. */
bmpc_status bmpc_query_kernel_cost(bmpc_plan plan, int32_t cls, double* bytes,
                                   double* flops, int32_t* launches);

/* Copy the factor of tail s (0 <= s < B*S; tail s of the batch is scenario s % S of
 * system s / S) to host memory (synchronizes): L [N*n][N*n] row-major
 * in permuted order (lower block structure of L_i; the DIAGONAL blocks are given as
 * their inverses L_jj^{-1}, which is what the plan stores), F [n][n] = F_{s,1}.
 * Values are widened to FP64.  For tests of small systems. */
bmpc_status bmpc_export_tail_factor(bmpc_plan plan, int32_t s, double* L, double* F);
/* Copy L_R [B][n][n] (FP64, lower; one per system) to host memory (synchronizes). */
bmpc_status bmpc_export_root_factor(bmpc_plan plan, double* LR);

/* Per-kernel timing with HIP events on the plan's stream.  While enabled, every
 * launch is bracketed by events; bmpc_get_kernel_times synchronizes and returns, for
 * each kernel class, the number of launches and their summed milliseconds since the
 * last reset.  Class ids: see bmpc_kernel_class_name. */
bmpc_status bmpc_set_profiling(bmpc_plan plan, int32_t enable);
bmpc_status bmpc_get_kernel_times(bmpc_plan plan, int32_t max_classes, int64_t* launches,
                                  double* total_ms);
bmpc_status bmpc_reset_kernel_times(bmpc_plan plan);
const char* bmpc_kernel_class_name(int32_t cls);
int32_t bmpc_kernel_class_count(void);

bmpc_status bmpc_destroy(bmpc_plan plan);
const char* bmpc_status_string(bmpc_status st);

/* ---- IPM front end ---------------------------------------------------------- */

typedef struct {
  int32_t S, N;  /* scenarios, stages per tail */
  int32_t n;     /* block size, 1..32 */
  int32_t me;    /* equality rows per link, 0..64 */
  int32_t mi;    /* inequality rows per link, 0..128 */
} bmpc_qp_dims;

/* Reduced IPM system of a branch-MPC QP (the appendix on the linear systems of IPM and
 * ADMM): the regularized primal-dual KKT matrix [[P + tau I, A^T, G^T], [A, -delta I,
 * 0], [G, 0, -(W + delta I)]] reduced to K = P + tau I + delta^{-1} A^T A +
 * G^T (W + delta I)^{-1} G, written as the D, E, C, R blocks bmpc_factor takes.
 * The QP terms are given per link of the variable chain: link 0 of scenario s couples
 * (u, v) = (x_0, x_{s,0}), link k (1 <= k < N) couples (x_{s,k-1}, x_{s,k}), link N is
 * the terminal term on u = x_{s,N-1} (its v columns must be zero).  Device arrays:
 *   Q [S][N+1][2n][2n]   link cost Hessians (P = sum of links), variables (u, v)
 *   A [S][N+1][me][2n]   equality rows,  G [S][N+1][mi][2n] inequality rows
 *   w [S][N+1][mi]       diagonal of W (nonnegative; the IPM weights are positive)
 * Outputs (device, overwritten): D [S][N][n][n] (both triangles), E [S][N-1][n][n],
 * C [S][n][n], R [n][n]; work: device scratch of S*n*n doubles.  tau >= 0, delta > 0.
 * The ADMM system of the same appendix (the OSQP form [[P + sigma I, A^T, G^T],
 * [A, -rho^{-1} I, 0], [G, 0, -rho^{-1} I]], reduced to P + sigma I + rho A^T A +
 * rho G^T G) is this assembly with w = 0, tau = sigma and delta = 1/rho.
 * Asynchronous on stream (NULL = legacy default); allocates nothing.  The root block
 * is summed over the scenarios in scenario order (deterministic). */
bmpc_status bmpc_assemble_qp(const bmpc_qp_dims* dims, const double* Q, const double* A,
                             const double* G, const double* w, double tau, double delta,
                             double* D, double* E, double* C, double* R, double* work,
                             void* stream);

/* bmpc_assemble_qp without the work argument, for callers that cannot allocate device
 * memory (code under graph capture, serving loops, harnesses that forbid allocation).
 * The scratch is a static device array of the library, one per GPU, of 512 * 32 * 32
 * doubles (4 MiB, held until the process ends): S * n * n must not exceed that
 * (BMPC_ERR_INVALID otherwise).  Allocates nothing.  Every call on a GPU uses that GPU's
 * one scratch array, so calls that overlap on one GPU (other streams, other threads)
 * race; issue them on one stream.  Results are those of bmpc_assemble_qp. */
bmpc_status bmpc_assemble_qp_noalloc(const bmpc_qp_dims* dims, const double* Q,
                                     const double* A, const double* G, const double* w,
                                     double tau, double delta, double* D, double* E,
                                     double* C, double* R, void* stream);

/* ---- host-only helpers (no device needed) ---------------------------------- */

/* Pi_i for N stages (same content as bmpc_query_perm). */
bmpc_status bmpc_ordering(int32_t N, int32_t* perm);

/* Block structure of one tail's factor plus the root row, under Pi_i: every
 * (row, col) pair of nonzero blocks with row >= col, positions 0..N-1 for the tail
 * in permuted order and N for the root, sorted by (row, col).  Writes at most cap
 * pairs and sets *count to the full number (call with cap = 0 to size). */
bmpc_status bmpc_structure(int32_t N, int32_t* rows, int32_t* cols, int64_t cap,
                           int64_t* count);

/* Cost model of a plan without creating one. */
bmpc_status bmpc_cost_model(const bmpc_dims* dims, bmpc_precision prec,
                            const bmpc_options* opts, bmpc_cost* cost);

#ifdef __cplusplus
}
#endif
#endif /* BMPC_H */
