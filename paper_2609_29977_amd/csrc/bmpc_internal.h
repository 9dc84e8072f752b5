// Internal declarations of the bmpc HIP library (gfx950).
//
// Chain notation used by every kernel (Section IV-A).  Tail s is reversed
// (Omega_i) so that chain position j = 1..m, m = N-1, holds stage N-j; the
// root-coupled stage 0 (the paper's x_1) is kept last and is called X below
// (position N).  The coupling from chain position j to its successor is
// K[pos j+1, pos j] = E[s][N-1-j]^T (for j = m the successor is X).  Under
// Gamma_{N-1} position j is eliminated at level tz(j)+1 (tz = trailing zeros):
// level 1 takes the odd positions, level 2 the positions 2*odd, ... (the groups of
// the recursion in Section II), and X comes last.  When position j (level t+1) is
// eliminated, its current neighbours are j-2^t (left, if >= 1) and j+2^t (right,
// or X when j+2^t > m).
//
// Factor storage (plan-owned, precision T of the tail factor):
//   Linv[S][N][n][n]  L_jj^{-1} of position j at index j-1, X at index N-1, each
//                     block packed by rows (element (r, c), c <= r, at r(r+1)/2 + c)
//   Gl  [S][m][n][n]  factor block of the left neighbour's row, G_l = K[left,j] L_jj^{-T}
//   Gr  [S][m][n][n]  factor block of the right neighbour's row (or X's row)
//   F   [S][n][n]     F_{s,1} = C_s L_X^{-T} (the only block of the root row, Thm 1)
//   U   [S][n][n]     F F^T in FP64;  LR[n][n] = chol(R - sum U) in FP64
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmpc {

constexpr int kFactorThreads = 256;
constexpr int kSolveThreads = 64;
// Right-hand sides per kernel launch: the solve, the fused forward substitution and the
// residual take them in chunks of at most kMaxRhs (kMaxRhs64 at n > 32, where the
// residual's LDS holds fewer vectors); a plan's nrhs has no such limit.
constexpr int kMaxRhs = 8;
constexpr int kMaxRhs64 = 4;
constexpr __host__ __device__ int rhs_chunk(int nmax) { return nmax > 32 ? kMaxRhs64 : kMaxRhs; }

// Blocks per chain in the G_l and G_r arrays: the N-1 blocks of the positions 1..N-1,
// padded to N so that every factor array (L^{-1} has N) shares one chain stride; the
// solve streams read the three arrays at the same offsets, which HBM serves faster than
// offsets that drift apart by one block per chain.
inline __host__ __device__ size_t g_chain_blocks(int N) { return (size_t)N; }
constexpr int kMaxWindowDepth = 6;

// Kernel classes for per-kernel event timing.
enum KernelClass : int {
  KC_FACTOR_INIT = 0,
  KC_FACTOR_FIRST,   // first factor pass when it is not also the last
  KC_FACTOR_MID,     // intermediate factor passes
  KC_FACTOR_FINAL,   // last factor pass + the x_1 step (F, U)
  KC_ROOT_REDUCE,    // partial sums of U over scenario groups
  KC_ROOT_POTRF,     // R~ = R - sum U, L_R = chol(R~)
  KC_SOLVE_FWD,      // tail forward substitution, one launch per level
  KC_SOLVE_X_FWD,    // x_1 forward step + F y products
  KC_SOLVE_ROOT,     // root reduction and root triangular solves
  KC_SOLVE_X_BWD,    // root propagation and x_1 backward step
  KC_SOLVE_BWD,      // tail backward substitution, one launch per level
  KC_RESIDUAL,       // FP64 tail residual b - K x
  KC_RESIDUAL_ROOT,  // FP64 root residual
  KC_REFINE_MISC,    // refinement bookkeeping (norm reset, stop test)
  KC_GRAD_BLOCKS,    // block gradients through the solve
  KC_FACTOR_L1INV,   // level-1 diagonal inverses before the first factor pass
  KC_COUNT
};

// Batches: B independent systems of one shape are factored and solved together.
// The tail kernels run over the B*S chains (chain g is scenario g % S of system
// g / S); the root steps run once per system.  Vectors b, x, r are [B][nrhs][len]
// with len = (S*N+1)*n.
struct FactorPassArgs {
  int S, N, n, m;       // S = chains of the batch (B * scenarios); m = N - 1
  int Ssys;             // scenarios per system (for natural row numbers)
  int Tw;               // window depth (levels per pass)
  int pass, npass;      // index of this pass and total passes
  int mk, shift;        // reduced chain length, position stride log2
  int windows;          // windows per chain
  int is_final;
  const double* D;
  const double* E;
  const double* C;
  // reduced-chain inputs written by the previous pass (null for pass 0)
  const void* accR_in;  // [S][stride] : update of a node from the window on its left
  const void* accL_in;  // [S][stride] : update of a node from the window on its right
  const void* fill_in;  // [S][stride] : coupling from node q to its successor
  void* accR_out;
  void* accL_out;
  void* fill_out;
  int stride;           // blocks per chain in the reduced-chain buffers
  void* accX;           // [S][npass] : X updates of each pass
  void* Linv;
  void* Gl;
  void* Gr;
  void* F;
  double* U;
  const int* permpos;   // [N] permuted position of chain position j at j-1 (X at N-1)
  unsigned long long* info;
  // Forward substitution fused into the elimination (null b: factor only).  b is the
  // FP64 right-hand side in the vector layout of the solve ([B][nrhs][len]); y
  // receives L^{-1} Pi b per chain position ([S][N][nrhs][n], precision T) and w the
  // FP64 products F_s y_X ([S][nrhs][n]).  The vector accumulators mirror accR /
  // accL / accX per right-hand side ([S][stride][nrhs][n] and [S][npass][nrhs][n]).
  const double* b;       // right-hand side q = 0 of this chunk (b + q0 * len)
  int nrhs;              // right-hand sides of this chunk
  size_t vsys;           // vector elements per system (all right-hand sides)
  void* y;
  double* w;
  const void* vaccR_in;
  const void* vaccL_in;
  void* vaccR_out;
  void* vaccL_out;
  void* vaccX;
};

// Vectors b, x, r are [B][nrhs][len]; a launch takes a chunk of the right-hand sides:
// its pointers are those of the chunk's first right-hand side in system 0 (offset by
// q0 * len), nrhs counts the chunk, vsys = (all right-hand sides) * len is the stride
// between systems and seg_sys the stride of the per-(system, right-hand side) norms.
struct SolveArgs {
  int S, N, n, m, nrhs;  // S = scenarios per system, nrhs of this chunk
  int B;                 // systems in the batch
  size_t vsys;           // vector elements per system
  int seg_sys;           // norm entries per system
  const void* Linv;
  const void* Gl;
  const void* Gr;
  const void* F;
  const double* LR;
  const double* b;       // [nrhs][len] FP64 input
  double* x;             // [nrhs][len] FP64 output
  void* y;               // [S][N][nrhs][n] scratch, precision T
  double* w;             // [S][nrhs][n] FP64 products F_s y_X
  double* x0;            // [nrhs][n]
  const double* rnorm;   // refinement: input scale 1/rnorm, output x += rnorm * d
  double* dstore;        // refinement: rnorm * d stored here ([nrhs][len], may alias b)
  const int* done;       // refinement stop flag (null outside refinement)
  int accumulate;        // 0: x = d ; 1: x += rnorm * d (refinement update)
  int fwd_waves;         // forward level positions: at most this many waves (0: 4)
};

struct ResidualArgs {
  int S, N, n, nrhs;     // S = scenarios per system, nrhs of this chunk
  int B;                 // systems in the batch
  size_t vsys;           // vector elements per system (all right-hand sides)
  int chunk;             // stages per work item of the tail residual
  const double* D;
  const double* E;
  const double* C;
  const double* R;       // [B][n][n]
  const double* b;
  const double* x;
  double* r;             // [B][nrhs][len]
  double* w;             // [S][nrhs][n] products C_s x_{s,0}
  const int* done;
  // Row sums of |K| (backward-error stop): per workgroup of the tail residual the
  // maximum over its rows (knorm_part[blockIdx]), per system the maximum over the
  // root rows (knorm_root[sys]) and the per-chain |C_s| row sums (crow [B*S][n]).
  // Null: not computed.
  double* knorm_part;
  double* knorm_root;
  double* crow;
};

struct GradArgs {
  int S, N, n, nrhs;     // S = scenarios per system, all right-hand sides
  int B;                 // systems in the batch
  const double* x;       // [nrhs][len] solution
  const double* lam;     // [nrhs][len] adjoint K^{-1} g
  double* dD;            // [S][N][n][n] or null
  double* dE;            // [S][N-1][n][n] or null
  double* dC;            // [S][n][n] or null
  double* dR;            // [n][n] or null
};

// launchers (defined next to their kernels)
template <typename T>
void launch_factor_pass(const FactorPassArgs& a, int nmax, hipStream_t st);
// L^{-1} of the odd chain positions' diagonal blocks (D only), before the first pass
// (whose arguments a are).
template <typename T>
void launch_level1_inverse(const FactorPassArgs& a, int nmax, hipStream_t st);
// block sizes 33..64: window depth 1, no fused forward substitution (factor64.hip)
template <typename T>
void launch_factor_pass64(const FactorPassArgs& a, hipStream_t st);
size_t factor64_lds_bytes(bool fp64);
void launch_factor_init(unsigned long long* info, hipStream_t st);
// part[sys][g] = sum of U over the scenarios of group g of system sys (B systems of S)
void launch_root_reduce(const double* U, double* part, int B, int S, int n, int groups,
                        hipStream_t st);
// LR[sys] = chol(R[sys] - sum_g part[sys][g]) for every system; row numbers of system
// sys start at sys * sys_rows, its root rows at root_row within it
void launch_root_potrf(const double* R, const double* part, int B, int groups, int n,
                       double* LR, int64_t sys_rows, int64_t root_row,
                       unsigned long long* info, hipStream_t st);

template <typename T>
void launch_solve_fwd_level(const SolveArgs& a, int level, int nmax, hipStream_t st);
template <typename T>
void launch_solve_x_fwd(const SolveArgs& a, int nmax, hipStream_t st);
void launch_solve_root(const SolveArgs& a, hipStream_t st);
template <typename T>
void launch_solve_x_bwd(const SolveArgs& a, int nmax, hipStream_t st);
template <typename T>
void launch_solve_bwd_level(const SolveArgs& a, int level, int nmax, hipStream_t st);
// The backward levels from level_lo up to the top, in one launch (one workgroup per
// chain, one wave per position, top level first); only where bwd_top_level says so.
template <typename T>
void launch_solve_bwd_top(const SolveArgs& a, int level_lo, hipStream_t st);

// block sizes 33..64 (solve64.hip): one level of either sweep, the x_1 forward step
// (fwd) or root propagation + x_1 backward step
template <typename T>
void launch_solve64_level(const SolveArgs& a, int level, bool fwd, hipStream_t st);
template <typename T>
void launch_solve64_x(const SolveArgs& a, bool fwd, hipStream_t st);

void launch_residual(const ResidualArgs& a, int nmax, hipStream_t st);
void launch_grad_blocks(const GradArgs& a, hipStream_t st);
void launch_residual_root(const ResidualArgs& a, hipStream_t st);
void launch_refine_reset(int* flags, hipStream_t st);
// Infinity norms by a two-stage maximum (kNormBlocks block partials, then one wave),
// deterministic and NaN-propagating; skipped when *done is set.
constexpr int kNormBlocks = 1024;
// out[q] = max_i |v[q][i]|, through partial[nrhs][kNormBlocks]
void launch_maxabs(const double* v, int nrhs, size_t len, double* partial, double* out,
                   const int* done, hipStream_t st);
// dnorm[q] = |d_q|_inf, xnorm[q] = |x_q|_inf (partials in partial[2][nrhs][kNormBlocks]),
// then the stop test: flags[0] = 1 if dnorm <= tol * xnorm for every q; flags[1] counts
// the corrections; relcorr = max_q dnorm / xnorm.
void launch_refine_check(const double* d, const double* x, int nrhs, size_t len,
                         double* partial, double tol, int* flags, double* relcorr,
                         double* dnorm, double* xnorm, hipStream_t st);

// Backward-error stop test after a residual r = b - K x of B systems with nrhs
// right-hand sides each (see refine_be_check_kernel): |r| and |x| by block partials,
// |K| per system reduced from the residual's row-sum partials when kpart is not null
// (kper partials per system), |b| from bnorm.  Sets flags[0] when every normwise
// backward error is <= tol, else counts a correction (flags[1]) if count; |r| into rnorm.
void launch_refine_be_check(const double* r, const double* x, int B, int nrhs, size_t len,
                            double* partial, const double* kpart, int kper,
                            const double* kroot, double* knorm, const double* bnorm,
                            double tol, int count, int* flags, double* relcorr, double* rnorm,
                            hipStream_t st);

// number of chain positions eliminated at level l (1-based) of a chain of length m
__host__ __device__ inline int level_count(int m, int l) {
  int ml = m >> (l - 1);
  return (ml + 1) >> 1;
}
__host__ __device__ inline int chain_levels(int m) {
  int L = 0;
  while ((m >> L) > 0) ++L;
  return L;  // floor(log2 m) + 1 for m >= 1, 0 for m = 0
}

// Positions per chain up to which backward levels share one launch.
constexpr int kBwdTopWaves = 8;
// Lowest backward level walked by launch_solve_bwd_top: the levels with at most
// kBwdTopWaves positions per chain, when the plan's backward levels use the one-vector
// kernels (one right-hand side, n = 8, 16 or 32, S and B within the grid's y and z
// limits); otherwise chain_levels(m) + 1, i.e. no level.
inline int bwd_top_level(int m, int n, int nrhs, int S, int B) {
  const int L = chain_levels(m);
  if ((n != 8 && n != 16 && n != 32) || nrhs != 1 || S > 65535 || B > 65535) return L + 1;
  int l = L + 1;
  while (l > 1 && level_count(m, l - 1) <= kBwdTopWaves) --l;
  return l;
}

}  // namespace bmpc
