// Block gradients of a loss through the solve x = K^{-1} b (gfx950).
//
// Differentiating K x = b: with lam = K^{-1} g (g = dloss/dx, one more solve with the
// same factor) the dense gradient is dK = -lam x^T, summed over the right-hand sides.
// Each block array collects the entries of K it fills (eq. (root_coupled_matrix),
// eq. (tail_block_tridiagonal)): D and R symmetrically (sym(A) = (A + A^T) / 2),
// E[s][k] at (k+1, k) and transposed at (k, k+1), C[s] at (root, stage 0) and
// transposed at (stage 0, root).  One workgroup per tail stage writes dD and dE of
// that stage (and dC for stage 0); one more workgroup per system writes its dR.  The vectors are
// staged in LDS; every output element is written once, coalesced.  HBM-bound on the
// writes: 8 n^2 bytes per D, E and C block.
#include "bmpc_internal.h"

namespace bmpc {

namespace {

constexpr int GT = 256;
constexpr int GQ = 8;                // right-hand sides staged per round
constexpr int GN = 64;               // largest block size
constexpr int EPT = GN * GN / GT;    // output elements per thread

__global__ void __launch_bounds__(GT) grad_blocks_kernel(GradArgs a) {
  __shared__ double xs[GQ][3][GN];  // x of stage k, stage k+1, root
  __shared__ double ls[GQ][3][GN];  // lam of the same
  const int n = a.n, N = a.N, S = a.S, nrhs = a.nrhs;
  const size_t nn = (size_t)n * n;
  const size_t len = ((size_t)S * N + 1) * n;
  const int chains = a.B * S;
  // workgroups [0, chains*N): stage k of chain s; then one per system for dR
  const bool is_root = blockIdx.x >= (unsigned)(chains * N);
  const int s = is_root ? 0 : blockIdx.x / N;
  const int k = is_root ? 0 : blockIdx.x - s * N;
  const int sys = is_root ? (int)blockIdx.x - chains * N : s / S;
  const int sl = s - (s / S) * S;
  const size_t vbase = (size_t)sys * nrhs * len;
  const size_t root = vbase + (size_t)S * N * n;
  // sums over the right-hand sides, GQ of them staged at a time: d0 (dD or dR),
  // dE, dC for this thread's elements e = threadIdx.x + t * GT
  double d0[EPT], dE[EPT], dC[EPT];
#pragma unroll
  for (int t = 0; t < EPT; ++t) d0[t] = dE[t] = dC[t] = 0.0;
  for (int q0 = 0; q0 < nrhs; q0 += GQ) {
    const int nq = min(GQ, nrhs - q0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nq * 3 * n; idx += GT) {
      const int q = idx / (3 * n), rem = idx - q * 3 * n, w = rem / n, i = rem - w * n;
      size_t off;
      bool ok = true;
      if (w == 2) {
        off = root + i;
      } else {
        const int st = k + w;
        ok = !is_root && st < N;
        off = vbase + ((size_t)sl * N + (ok ? st : 0)) * n + i;
      }
      const size_t qo = (size_t)(q0 + q) * len + off;
      xs[q][w][i] = ok ? a.x[qo] : 0.0;
      ls[q][w][i] = ok ? a.lam[qo] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
      const int e = threadIdx.x + t * GT;
      if (e >= n * n) continue;
      const int r = e / n, c = e - r * n;
      if (is_root) {
        for (int q = 0; q < nq; ++q) d0[t] += ls[q][2][r] * xs[q][2][c] + ls[q][2][c] * xs[q][2][r];
      } else {
        for (int q = 0; q < nq; ++q) {
          d0[t] += ls[q][0][r] * xs[q][0][c] + ls[q][0][c] * xs[q][0][r];
          dE[t] += ls[q][1][r] * xs[q][0][c] + xs[q][1][r] * ls[q][0][c];
          dC[t] += ls[q][2][r] * xs[q][0][c] + xs[q][2][r] * ls[q][0][c];
        }
      }
    }
  }
  const size_t blk = (size_t)s * N + k;
#pragma unroll
  for (int t = 0; t < EPT; ++t) {
    const int e = threadIdx.x + t * GT;
    if (e >= n * n) continue;
    if (is_root) {
      if (a.dR) a.dR[(size_t)sys * nn + e] = -0.5 * d0[t];
      continue;
    }
    if (a.dD) a.dD[blk * nn + e] = -0.5 * d0[t];
    if (a.dE && k + 1 < N) a.dE[((size_t)s * (N - 1) + k) * nn + e] = -dE[t];
    if (a.dC && k == 0) a.dC[(size_t)s * nn + e] = -dC[t];
  }
}

}  // namespace

void launch_grad_blocks(const GradArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(grad_blocks_kernel, dim3((unsigned)(a.B * a.S * a.N + a.B)), dim3(GT), 0,
                     st, a);
}

}  // namespace bmpc
