// Block gradients of a loss through the solve x = K^{-1} b (gfx950).
//
// Differentiating K x = b: with lam = K^{-1} g (g = dloss/dx, one more solve with the
// same factor) the dense gradient is dK = -lam x^T, summed over the right-hand sides.
// Each block array collects the entries of K it fills (eq. (root_coupled_matrix),
// eq. (tail_block_tridiagonal)): D and R symmetrically (sym(A) = (A + A^T) / 2),
// E[s][k] at (k+1, k) and transposed at (k, k+1), C[s] at (root, stage 0) and
// transposed at (stage 0, root).
//
// One workgroup takes SPW consecutive stages of one tail (SPW chosen so that a
// workgroup writes about 2048 entries of each array) and writes dD and dE of those
// stages (and dC for stage 0); one more workgroup per system writes its dR.  The
// vectors of the stages (and of the next stage and the root) are staged in LDS for up
// to GQ right-hand sides at a time; with more, later rounds add to what the first round
// wrote (the sum over the right-hand sides stays in order).  Every output element is
// written by one thread, coalesced.  HBM-bound on the writes: 8 n^2 bytes per D, E and
// C block.
#include <algorithm>

#include "bmpc_internal.h"

namespace bmpc {

namespace {

constexpr int GT = 256;
constexpr int GQ = 8;  // right-hand sides staged per round

// Stages per workgroup: about 2048 block entries, at most 16 stages.
inline int grad_spw(int n) { return std::max(1, std::min(16, 2048 / (n * n))); }

__global__ void __launch_bounds__(GT) grad_blocks_kernel(GradArgs a, int spw, int wpc) {
  extern __shared__ double gsm[];
  const int n = a.n, N = a.N, S = a.S, nrhs = a.nrhs;
  const int nn = n * n;
  const size_t len = ((size_t)S * N + 1) * n;
  const int chains = a.B * S;
  const int qs = min(GQ, nrhs);       // right-hand sides per round
  const int V = spw + 2;              // staged vectors: spw + 1 stages, the root
  double* xs = gsm;                   // [qs][V][n]
  double* ls = gsm + (size_t)qs * V * n;
  // workgroups [0, chains * wpc): stages k0 .. k0 + spw - 1 of chain s; then one per
  // system for dR
  const bool is_root = blockIdx.x >= (unsigned)(chains * wpc);
  const int s = is_root ? 0 : (int)blockIdx.x / wpc;
  const int k0 = is_root ? 0 : ((int)blockIdx.x - s * wpc) * spw;
  const int sys = is_root ? (int)blockIdx.x - chains * wpc : s / S;
  const int sl = s - (s / S) * S;
  const size_t vbase = (size_t)sys * nrhs * len;
  const size_t root = vbase + (size_t)S * N * n;
  const int ne = is_root ? nn : spw * nn;
  for (int q0 = 0; q0 < nrhs; q0 += GQ) {
    const int nq = min(GQ, nrhs - q0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nq * V * n; idx += GT) {
      const int q = idx / (V * n), rem = idx - q * V * n, w = rem / n, i = rem - w * n;
      size_t off;
      bool ok = true;
      if (w == V - 1) {
        off = root + i;
      } else {
        const int st = k0 + w;
        ok = !is_root && st < N;
        off = vbase + ((size_t)sl * N + (ok ? st : 0)) * n + i;
      }
      const size_t qo = (size_t)(q0 + q) * len + off;
      xs[(q * V + w) * n + i] = ok ? a.x[qo] : 0.0;
      ls[(q * V + w) * n + i] = ok ? a.lam[qo] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ne; e += GT) {
      const int j = e / nn, rem = e - j * nn, r = rem / n, c = rem - r * n;
      const int k = k0 + j;
      if (!is_root && k >= N) continue;
      double d0 = 0.0, dE = 0.0, dC = 0.0;
      if (is_root) {
        const int w = V - 1;
        for (int q = 0; q < nq; ++q) {
          const double* xq = xs + (q * V + w) * n;
          const double* lq = ls + (q * V + w) * n;
          d0 += lq[r] * xq[c] + lq[c] * xq[r];
        }
        if (a.dR) {
          double* o = a.dR + (size_t)sys * nn + rem;
          *o = q0 == 0 ? -0.5 * d0 : *o - 0.5 * d0;
        }
        continue;
      }
      for (int q = 0; q < nq; ++q) {
        const double* x0 = xs + (q * V + j) * n;  // stage k
        const double* l0 = ls + (q * V + j) * n;
        const double* x1 = x0 + n;                // stage k + 1 (zero past the tail)
        const double* l1 = l0 + n;
        d0 += l0[r] * x0[c] + l0[c] * x0[r];
        dE += l1[r] * x0[c] + x1[r] * l0[c];
        if (k == 0) {
          const double* xr = xs + (q * V + V - 1) * n;
          const double* lr = ls + (q * V + V - 1) * n;
          dC += lr[r] * x0[c] + xr[r] * l0[c];
        }
      }
      const size_t blk = (size_t)s * N + k;
      if (a.dD) {
        double* o = a.dD + blk * nn + rem;
        *o = q0 == 0 ? -0.5 * d0 : *o - 0.5 * d0;
      }
      if (a.dE && k + 1 < N) {
        double* o = a.dE + ((size_t)s * (N - 1) + k) * nn + rem;
        *o = q0 == 0 ? -dE : *o - dE;
      }
      if (a.dC && k == 0) {
        double* o = a.dC + (size_t)s * nn + rem;
        *o = q0 == 0 ? -dC : *o - dC;
      }
    }
  }
}

}  // namespace

void launch_grad_blocks(const GradArgs& a, hipStream_t st) {
  const int spw = grad_spw(a.n);
  const int wpc = (a.N + spw - 1) / spw;  // workgroups per chain
  const size_t lds = 2 * (size_t)std::min(GQ, a.nrhs) * (spw + 2) * a.n * sizeof(double);
  hipLaunchKernelGGL(grad_blocks_kernel, dim3((unsigned)(a.B * a.S * wpc + a.B)), dim3(GT), lds,
                     st, a, spw, wpc);
}

}  // namespace bmpc
