// Mixed-precision iterative refinement support (FP64 residual r = b - K x).
//
// The residual is formed from the caller's FP64 blocks exactly as K is defined in
// eq. (root_coupled_matrix) / eq. (tail_block_tridiagonal): row block (s,k) of a
// tail is D_{s,k} x_{s,k} + E_{s,k-1} x_{s,k-1} + E_{s,k}^T x_{s,k+1} (+ C_s^T x_0
// for k = 0); the root row block is R x_0 + sum_s C_s x_{s,0}, with the sum over s
// taken in scenario order.  The infinity norms needed by the refinement loop are
// maxima, which are order independent, so device atomics keep them deterministic.
#include "bmpc_internal.h"
#include "blockops.h"

namespace bmpc {

namespace {

constexpr int NT = 64;

__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

__device__ inline void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            static_cast<unsigned long long>(__double_as_longlong(v)));
}

template <int NMAX>
struct ResSmem {
  double blk[Lay<NMAX>::SZ];
  double xv[3][kMaxRhs][NMAX];  // x_{k-1}, x_k, x_{k+1}
  double acc[kMaxRhs][NMAX];
};

// acc[q][row] -= op(B) xin[q]; B is a global n x n FP64 block (sym: lower triangle)
template <int NMAX>
__device__ inline void sub_block_product(ResSmem<NMAX>& sm, const double* __restrict__ B,
                                         int mode, double (*xin)[NMAX], int n, int nrhs) {
  constexpr int LD = Lay<NMAX>::LD;
  // mode 0: B (general), 1: B^T, 2: symmetric from lower triangle
  if (mode == 2)
    lds_load_sym_lower<double, NMAX, NT>(sm.blk, B, n);
  else
    lds_load<double, NMAX, NT>(sm.blk, B, n, false);
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += NT) {
    const int q = idx / n, row = idx - (idx / n) * n;
    double t = 0.0;
    if (mode == 1) {
      for (int k = 0; k < n; ++k) t += sm.blk[k * LD + row] * xin[q][k];
    } else {
      for (int k = 0; k < n; ++k) t += sm.blk[row * LD + k] * xin[q][k];
    }
    sm.acc[q][row] -= t;
  }
  __syncthreads();
}

template <int NMAX>
__global__ void __launch_bounds__(NT) residual_kernel(ResidualArgs a) {
  if (a.done && *a.done) return;
  __shared__ ResSmem<NMAX> sm;
  const int n = a.n, N = a.N, S = a.S, nrhs = a.nrhs;
  const size_t nn = (size_t)n * n;
  const size_t len = ((size_t)S * N + 1) * n;
  const int s = blockIdx.x / N;
  const int k = blockIdx.x - s * N;
  const size_t off = ((size_t)s * N + k) * n;
  for (int idx = threadIdx.x; idx < n * nrhs; idx += NT) {
    const int q = idx / n, i = idx - (idx / n) * n;
    sm.acc[q][i] = a.b[(size_t)q * len + off + i];
    sm.xv[1][q][i] = a.x[(size_t)q * len + off + i];
    if (k >= 1) sm.xv[0][q][i] = a.x[(size_t)q * len + off - n + i];
    if (k + 1 < N) sm.xv[2][q][i] = a.x[(size_t)q * len + off + n + i];
    if (k == 0) sm.xv[0][q][i] = a.x[(size_t)q * len + (size_t)S * N * n + i];  // x_0
  }
  sub_block_product<NMAX>(sm, a.D + ((size_t)s * N + k) * nn, 2, sm.xv[1], n, nrhs);
  if (k >= 1)
    sub_block_product<NMAX>(sm, a.E + ((size_t)s * (N - 1) + (k - 1)) * nn, 0, sm.xv[0], n,
                            nrhs);
  if (k + 1 < N)
    sub_block_product<NMAX>(sm, a.E + ((size_t)s * (N - 1) + k) * nn, 1, sm.xv[2], n, nrhs);
  if (k == 0) {
    sub_block_product<NMAX>(sm, a.C + (size_t)s * nn, 1, sm.xv[0], n, nrhs);
    // w_s = C_s x_{s,0} for the root row
    constexpr int LD = Lay<NMAX>::LD;
    lds_load<double, NMAX, NT>(sm.blk, a.C + (size_t)s * nn, n, false);
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * nrhs; idx += NT) {
      const int q = idx / n, row = idx - (idx / n) * n;
      double t = 0.0;
      for (int c = 0; c < n; ++c) t += sm.blk[row * LD + c] * sm.xv[1][q][c];
      a.w[((size_t)s * nrhs + q) * n + row] = t;
    }
  }
  for (int q = 0; q < nrhs; ++q) {
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) {
      const double v = sm.acc[q][i];
      a.r[(size_t)q * len + off + i] = v;
      mx = fmax(mx, fabs(v));
    }
    mx = wave_max(mx);
    if (threadIdx.x == 0) atomic_max_nonneg(&a.rnorm[q], mx);
  }
}

__global__ void __launch_bounds__(256) residual_root_kernel(ResidualArgs a) {
  if (a.done && *a.done) return;
  __shared__ double part[256];
  const int n = a.n, N = a.N, S = a.S, nrhs = a.nrhs;
  const size_t len = ((size_t)S * N + 1) * n;
  const size_t root = (size_t)S * N * n;
  const int tpe = 8;
  for (int q = 0; q < nrhs; ++q) {
    const int i = threadIdx.x / tpe, g = threadIdx.x - (threadIdx.x / tpe) * tpe;
    double acc = 0.0;
    if (i < n)
      for (int s = g; s < S; s += tpe) acc += a.w[((size_t)s * nrhs + q) * n + i];
    part[threadIdx.x] = acc;
    __syncthreads();
    double mx = 0.0;
    if (threadIdx.x < n) {
      const int row = threadIdx.x;
      double sum = 0.0;
      for (int gg = 0; gg < tpe; ++gg) sum += part[row * tpe + gg];
      double rx = 0.0;
      for (int c = 0; c < n; ++c) {
        const double rv = (row >= c) ? a.R[row * n + c] : a.R[c * n + row];
        rx += rv * a.x[(size_t)q * len + root + c];
      }
      const double v = a.b[(size_t)q * len + root + row] - rx - sum;
      a.r[(size_t)q * len + root + row] = v;
      mx = fabs(v);
    }
    if (threadIdx.x < 64) {
      mx = wave_max(mx);
      if (threadIdx.x == 0) atomic_max_nonneg(&a.rnorm[q], mx);
    }
    __syncthreads();
  }
}

// flags[0] = done, flags[1] = corrections applied
__global__ void refine_reset_kernel(double* norms, int count, int* flags, int reset_iters) {
  if (reset_iters) {
    if (threadIdx.x == 0) {
      flags[0] = 0;
      flags[1] = 0;
    }
    return;
  }
  if (flags[0]) return;
  for (int i = threadIdx.x; i < count; i += blockDim.x) norms[i] = 0.0;
}

__global__ void refine_check_kernel(const double* dnorm, const double* xnorm, int nrhs,
                                    double tol, int* flags, double* relcorr) {
  if (threadIdx.x != 0 || flags[0]) return;
  flags[1] += 1;
  bool ok = true;
  double worst = 0.0;
  for (int q = 0; q < nrhs; ++q) {
    const double rel = xnorm[q] > 0.0 ? dnorm[q] / xnorm[q] : dnorm[q];
    worst = fmax(worst, rel);
    if (!(dnorm[q] <= tol * xnorm[q])) ok = false;
  }
  *relcorr = worst;
  if (ok) flags[0] = 1;
}

}  // namespace

void launch_residual(const ResidualArgs& a, int nmax, hipStream_t st) {
  const dim3 grid((unsigned)a.S * (unsigned)a.N);
  if (nmax <= 8)
    hipLaunchKernelGGL(residual_kernel<8>, grid, dim3(NT), 0, st, a);
  else if (nmax <= 16)
    hipLaunchKernelGGL(residual_kernel<16>, grid, dim3(NT), 0, st, a);
  else
    hipLaunchKernelGGL(residual_kernel<32>, grid, dim3(NT), 0, st, a);
}

void launch_residual_root(const ResidualArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(residual_root_kernel, dim3(1), dim3(256), 0, st, a);
}

void launch_refine_reset(double* norms, int count, int* flags, int reset_iters,
                         hipStream_t st) {
  hipLaunchKernelGGL(refine_reset_kernel, dim3(1), dim3(64), 0, st, norms, count, flags,
                     reset_iters);
}

void launch_refine_check(const double* dnorm, const double* xnorm, int nrhs, double tol,
                         int* flags, double* relcorr, hipStream_t st) {
  hipLaunchKernelGGL(refine_check_kernel, dim3(1), dim3(64), 0, st, dnorm, xnorm, nrhs, tol,
                     flags, relcorr);
}

}  // namespace bmpc
