// Mixed-precision iterative refinement support (FP64 residual r = b - K x).
//
// The residual is formed from the caller's FP64 blocks exactly as K is defined in
// eq. (root_coupled_matrix) / eq. (tail_block_tridiagonal): row block (s,k) of a
// tail is D_{s,k} x_{s,k} + E_{s,k-1} x_{s,k-1} + E_{s,k}^T x_{s,k+1} (+ C_s^T x_0
// for k = 0); the root row block is R x_0 + sum_s C_s x_{s,0}, with the sum over s
// taken in scenario order.  One wave walks a chunk of consecutive stages of one tail,
// so each E block is fetched from HBM once and used for both rows it touches; the
// blocks of the next stage are loaded while the current one is applied.  Infinity
// norms are maxima taken by a two-stage reduction (per-block partial maxima, then
// one block), so they are deterministic and need no atomics.
#include "bmpc_internal.h"
#include "regblock.h"

namespace bmpc {

namespace {

// Waves per tail work item: the rows of each block are split over WAVES waves so that
// the three blocks of a stage and their prefetched successors take at most 12 doubles
// per lane each (about 128 VGPRs at n = 32, four waves per SIMD for this HBM-bound
// kernel).
template <int NMAX>
struct ResCfg {
  static constexpr int WAVES = NMAX == 32 ? 4 : (NMAX == 16 ? 2 : 1);
  static constexpr int NT = 64 * WAVES;
  typedef RegBlock<double, NMAX, WAVES> RB;
};

// Register block of a symmetric matrix stored by its lower triangle, normal mapping:
// lane holds row o, columns base..base+EPL of sym(D).
template <int NMAX>
__device__ inline void load_sym(typename ResCfg<NMAX>::RB& rb, const double* __restrict__ g,
                                int n) {
  typedef typename ResCfg<NMAX>::RB RB;
  const int o = RB::out_index(), b = RB::base();
  const auto rs = block_rsrc(g, (unsigned)(n * n) * sizeof(double));
  // element (o, c) is read from whichever triangle holds it; padding reads as zero
#pragma unroll
  for (int e = 0; e < RB::EPL; ++e) {
    const int c = b + e;
    const int idx = c <= o ? o * n + c : c * n + o;
    const unsigned off = (o < n && c < n) ? (unsigned)idx * sizeof(double) : kOutOfRange;
    rb.v[e] = buf_load_f64(rs, off);
  }
}

template <int NMAX>
struct StageBlocks {
  typename ResCfg<NMAX>::RB d, en, et;  // D_k (sym), E_k (normal), E_k (transposed)
  __device__ void load(const ResidualArgs& a, int s, int k) {
    const int n = a.n, N = a.N;
    const size_t nn = (size_t)n * n;
    load_sym<NMAX>(d, a.D + ((size_t)s * N + k) * nn, n);
    if (k + 1 < N) {
      const auto rs = block_rsrc(a.E + ((size_t)s * (N - 1) + k) * nn,
                                 (unsigned)nn * sizeof(double));
      en.template load_buf<false>(rs, n);
      et.template load_buf<true>(rs, n);
    }
  }
};

template <int NMAX>
__global__ void __launch_bounds__(ResCfg<NMAX>::NT) residual_kernel(ResidualArgs a, int chunks) {
  if (a.done && *a.done) return;
  typedef typename ResCfg<NMAX>::RB RB;
  constexpr int NT = ResCfg<NMAX>::NT;
  __shared__ double xs[3][kMaxRhs][NMAX];  // x_{k-1}, x_k, x_{k+1} (rotating)
  __shared__ double x0s[kMaxRhs][NMAX];
  const int n = a.n, N = a.N, S = a.S, nrhs = a.nrhs;
  const size_t nn = (size_t)n * n;
  const size_t len = ((size_t)S * N + 1) * n;
  const int s = blockIdx.x / chunks;  // chain of the batch
  const int ch = blockIdx.x - s * chunks;
  const int sys = s / S, sl = s - sys * S;
  const size_t vbase = (size_t)sys * nrhs * len;  // this system's vectors
  const int k0 = ch * a.chunk, k1 = min(N, k0 + a.chunk);
  const int o = RB::out_index(), b = RB::base();

  auto load_x = [&](double (*dst)[NMAX], int k) {
    for (int idx = threadIdx.x; idx < nrhs * NMAX; idx += NT) {
      const int q = idx / NMAX, i = idx % NMAX;
      dst[q][i] = (k >= 0 && k < N && i < n)
                      ? a.x[vbase + (size_t)q * len + ((size_t)sl * N + k) * n + i]
                      : 0.0;
    }
  };
  int ip = 0, ic = 1, in = 2;  // rotating indices of x_{k-1}, x_k, x_{k+1}
  load_x(xs[ip], k0 - 1);
  load_x(xs[ic], k0);
  if (k0 == 0)
    for (int idx = threadIdx.x; idx < nrhs * NMAX; idx += NT) {
      const int q = idx / NMAX, i = idx % NMAX;
      x0s[q][i] = i < n ? a.x[vbase + (size_t)q * len + (size_t)S * N * n + i] : 0.0;
    }
  // carry: this lane's partial of E_{k0-1} x_{k0-1} for row k0, one slot per
  // right-hand side (LDS, so the loop over right-hand sides need not be unrolled)
  __shared__ double carry[kMaxRhs][NT];
  double* my = &carry[0][threadIdx.x];
  for (int q = 0; q < nrhs; ++q) my[q * NT] = 0.0;
  StageBlocks<NMAX> cur;
  cur.load(a, s, k0);
  if (k0 > 0) {
    RB ep;
    ep.template load<false>(a.E + ((size_t)s * (N - 1) + (k0 - 1)) * nn, n);
    __syncthreads();
    for (int q = 0; q < nrhs; ++q) my[q * NT] = ep.dot(xs[ip][q]);
  }
  for (int k = k0; k < k1; ++k) {
    load_x(xs[in], k + 1);
    StageBlocks<NMAX> nxt;
    if (k + 1 < k1) nxt.load(a, s, k + 1);
    __syncthreads();
    const size_t off = vbase + ((size_t)sl * N + k) * n;
#pragma unroll 1
    for (int q = 0; q < nrhs; ++q) {
      double p = cur.d.dot(xs[ic][q]) + my[q * NT];
      if (k + 1 < N) {
        p += cur.et.dot(xs[in][q]);
        my[q * NT] = cur.en.dot(xs[ic][q]);
      }
      p = lane_group_sum<RB::LPR>(p);
      if (b == 0 && o < n) a.r[(size_t)q * len + off + o] = a.b[(size_t)q * len + off + o] - p;
    }
    if (k == 0) {
      // C_s^T x_0 enters row 0; w_s = C_s x_{s,0} feeds the root row
      RB ct, cn;
      ct.template load<true>(a.C + (size_t)s * nn, n);
      cn.template load<false>(a.C + (size_t)s * nn, n);
#pragma unroll 1
      for (int q = 0; q < nrhs; ++q) {
        const double pc = lane_group_sum<RB::LPR>(ct.dot(x0s[q]));
        const double pw = lane_group_sum<RB::LPR>(cn.dot(xs[ic][q]));
        if (b == 0 && o < n) {
          a.r[(size_t)q * len + off + o] -= pc;
          a.w[((size_t)s * nrhs + q) * n + o] = pw;
        }
      }
    }
    __syncthreads();
    cur = nxt;
    const int t = ip;
    ip = ic;
    ic = in;
    in = t;
  }
}

__global__ void __launch_bounds__(1024) residual_root_kernel(ResidualArgs a) {
  if (a.done && *a.done) return;
  __shared__ double part[32][33];
  const int n = a.n, N = a.N, S = a.S, nrhs = a.nrhs;
  const int sys = blockIdx.x;  // one workgroup per system
  const size_t len = ((size_t)S * N + 1) * n;
  const size_t root = (size_t)sys * nrhs * len + (size_t)S * N * n;
  const double* w = a.w + (size_t)sys * S * nrhs * n;
  const double* R = a.R + (size_t)sys * n * n;
  const int t = threadIdx.x, i = t & 31, g = t >> 5;
  for (int q = 0; q < nrhs; ++q) {
    double acc = 0.0;
    if (i < n) {
      constexpr int B = 8;
      for (int s0 = g; s0 < S; s0 += 32 * B) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const int sc = s0 + 32 * u;
          v[u] = sc < S ? w[((size_t)sc * nrhs + q) * n + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) acc += v[u];
      }
    }
    part[g][i] = acc;
    __syncthreads();
    if (t < n) {
      const int row = t;
      double sum = 0.0;
      for (int gg = 0; gg < 32; ++gg) sum += part[gg][row];
      double rx = 0.0;
      for (int c = 0; c < n; ++c) {
        const double rv = (row >= c) ? R[row * n + c] : R[c * n + row];
        rx += rv * a.x[(size_t)q * len + root + c];
      }
      a.r[(size_t)q * len + root + row] = a.b[(size_t)q * len + root + row] - rx - sum;
    }
    __syncthreads();
  }
}

// Maximum that propagates NaN (so a NaN residual or correction fails the stop test).
__device__ inline double nan_max(double a, double b) { return (a != a || a > b) ? a : b; }

__device__ inline double block_max(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_xor(v, off));
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wv] = v;
  __syncthreads();
  double m = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = nan_max(m, sh[i]);
  __syncthreads();
  return m;
}

// partial[t][q][blk] = max over this block's slice of |v_t[q][.]| (t = 0: v, 1: v2).
// Each thread keeps four independent loads in flight per iteration.
__global__ void __launch_bounds__(256) maxabs_partial_kernel(const double* v, const double* v2,
                                                             int nrhs, size_t len,
                                                             double* partial, const int* done) {
  if (done && *done) return;
  __shared__ double sh[4];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int t = 0; t < (v2 ? 2 : 1); ++t) {
    const double* src = t == 0 ? v : v2;
    for (int q = 0; q < nrhs; ++q) {
      const double* p = src + (size_t)q * len;
      double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
      size_t i = t0;
      for (; i + 3 * stride < len; i += 4 * stride) {
        const double a0 = p[i], a1 = p[i + stride], a2 = p[i + 2 * stride], a3 = p[i + 3 * stride];
        m0 = nan_max(fabs(a0), m0);
        m1 = nan_max(fabs(a1), m1);
        m2 = nan_max(fabs(a2), m2);
        m3 = nan_max(fabs(a3), m3);
      }
      for (; i < len; i += stride) m0 = nan_max(fabs(p[i]), m0);
      double mx = block_max(nan_max(nan_max(m0, m1), nan_max(m2, m3)), sh);
      if (threadIdx.x == 0) partial[((size_t)t * nrhs + q) * gridDim.x + blockIdx.x] = mx;
    }
  }
}

// max over the block partials of one vector and right-hand side, on one wave
__device__ inline double wave_reduce_partials(const double* part, int blocks) {
  double mx = 0.0;
  for (int i = threadIdx.x; i < blocks; i += 64) mx = nan_max(part[i], mx);
  for (int off = 32; off > 0; off >>= 1) mx = nan_max(mx, __shfl_xor(mx, off));
  return mx;
}

__global__ void __launch_bounds__(64) maxabs_final_kernel(const double* partial, int blocks,
                                                          int nrhs, double* out,
                                                          const int* done) {
  if (done && *done) return;
  for (int q = 0; q < nrhs; ++q) {
    const double mx = wave_reduce_partials(partial + (size_t)q * blocks, blocks);
    if (threadIdx.x == 0) out[q] = mx;
  }
}

// flags[0] = done, flags[1] = corrections applied
__global__ void refine_reset_kernel(int* flags) {
  if (threadIdx.x == 0) {
    flags[0] = 0;
    flags[1] = 0;
  }
}

// |d|_inf and |x|_inf from the block partials, then the stop test
// |d_q|_inf <= tol |x_q|_inf for every right-hand side.
__global__ void __launch_bounds__(64) refine_check_kernel(const double* partial, int blocks,
                                                          int nrhs, double tol, int* flags,
                                                          double* relcorr, double* dnorm,
                                                          double* xnorm) {
  if (flags[0]) return;
  bool ok = true;
  double worst = 0.0;
  for (int q = 0; q < nrhs; ++q) {
    const double d = wave_reduce_partials(partial + (size_t)q * blocks, blocks);
    const double xv = wave_reduce_partials(partial + ((size_t)nrhs + q) * blocks, blocks);
    const double rel = xv > 0.0 ? d / xv : d;
    worst = nan_max(worst, rel);
    if (!(d <= tol * xv)) ok = false;
    if (threadIdx.x == 0) {
      dnorm[q] = d;
      xnorm[q] = xv;
    }
  }
  if (threadIdx.x == 0) {
    flags[1] += 1;
    *relcorr = worst;
    if (ok) flags[0] = 1;
  }
}

}  // namespace

void launch_residual(const ResidualArgs& a, int nmax, hipStream_t st) {
  const int chunks = (a.N + a.chunk - 1) / a.chunk;
  const dim3 grid((unsigned)(a.B * a.S) * (unsigned)chunks);
  if (nmax <= 8)
    hipLaunchKernelGGL(residual_kernel<8>, grid, dim3(ResCfg<8>::NT), 0, st, a, chunks);
  else if (nmax <= 16)
    hipLaunchKernelGGL(residual_kernel<16>, grid, dim3(ResCfg<16>::NT), 0, st, a, chunks);
  else
    hipLaunchKernelGGL(residual_kernel<32>, grid, dim3(ResCfg<32>::NT), 0, st, a, chunks);
}

void launch_residual_root(const ResidualArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(residual_root_kernel, dim3(a.B), dim3(1024), 0, st, a);
}

void launch_maxabs(const double* v, int nrhs, size_t len, double* partial, double* out,
                   const int* done, hipStream_t st) {
  hipLaunchKernelGGL(maxabs_partial_kernel, dim3(kNormBlocks), dim3(256), 0, st, v,
                     (const double*)nullptr, nrhs, len, partial, done);
  hipLaunchKernelGGL(maxabs_final_kernel, dim3(1), dim3(64), 0, st, partial, kNormBlocks, nrhs,
                     out, done);
}

void launch_refine_reset(int* flags, hipStream_t st) {
  hipLaunchKernelGGL(refine_reset_kernel, dim3(1), dim3(64), 0, st, flags);
}

void launch_refine_check(const double* d, const double* x, int nrhs, size_t len,
                         double* partial, double tol, int* flags, double* relcorr,
                         double* dnorm, double* xnorm, hipStream_t st) {
  hipLaunchKernelGGL(maxabs_partial_kernel, dim3(kNormBlocks), dim3(256), 0, st, d, x, nrhs, len,
                     partial, (const int*)flags);
  hipLaunchKernelGGL(refine_check_kernel, dim3(1), dim3(64), 0, st, (const double*)partial,
                     kNormBlocks, nrhs, tol, flags, relcorr, dnorm, xnorm);
}

}  // namespace bmpc
