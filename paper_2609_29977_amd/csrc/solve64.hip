// Two-level triangular solves (Algorithm 2) for block sizes 33..64 (gfx950).
//
// The same sweeps as solve.hip -- forward substitution one Gamma level per launch, the
// x_1 step, and after the root step the backward substitution in reverse level order,
// with the permutation applied as an index map -- for blocks that are too large for one
// wave's registers: a 64 x 64 block is held by the four waves of a workgroup
// (RegBlock<T, 64, 4>: sixteen output indices per wave, four lanes per output index,
// sixteen elements per lane).  One workgroup per chain position.  A position pulls its
// factor blocks one at a time; each block's neighbour vector is staged in LDS and the
// partial sums stay in registers until the pulls are done.
#include "bmpc_internal.h"
#include "regblock.h"
#include "solve_common.h"

namespace bmpc {

namespace {

constexpr int W64 = 4;
constexpr int T64 = 64 * W64;

// Right-hand side of a position in LDS: FWD, the gathered b scaled by 1/rnorm; else y.
template <typename T, bool FWD>
__device__ inline void stage_rhs64(const SolveArgs& a, T (*rhs)[64], size_t off, int seg0,
                                   const T* yj) {
  const size_t len = vec_len(a);
  for (int idx = threadIdx.x; idx < a.nrhs * 64; idx += T64) {
    const int q = idx >> 6, i = idx & 63;
    T v = T(0);
    if (i < a.n) {
      if constexpr (FWD) {
        double bv = a.b[(size_t)q * len + off + i];
        if (a.rnorm) {
          const double rn = a.rnorm[seg0 + q];
          bv = rn > 0.0 ? bv / rn : 0.0;
        }
        v = static_cast<T>(bv);
      } else {
        v = yj[q * a.n + i];
      }
    }
    rhs[q][i] = v;
  }
}

template <typename T>
__device__ inline void stage_vec64(T (*dst)[64], const T* src, int n, int nrhs) {
  for (int idx = threadIdx.x; idx < nrhs * 64; idx += T64) {
    const int q = idx >> 6, i = idx & 63;
    dst[q][i] = i < n ? src[q * n + i] : T(0);
  }
}

// One position of a level: rhs -= sum over the pulls of op(G) v, then L_jj^{-1} (FWD) or
// L_jj^{-T} applied.  Forward pulls: G_r of the left neighbours j - 2^t and G_l of the
// right neighbours j + 2^t (t < level - 1); backward: G_l^T with x of the left
// neighbour and G_r^T with x of the right one (or of X).
template <typename T, bool FWD>
__global__ void __launch_bounds__(T64) solve64_level_kernel(SolveArgs a, int level, int count) {
  if (a.done && *a.done) return;
  typedef RegBlock<T, 64, W64> RB;
  __shared__ T vec[kMaxRhs64][64];
  __shared__ T rhs[kMaxRhs64][64];
  const int n = a.n, N = a.N, nrhs = a.nrhs, m = a.m;
  const size_t nn = (size_t)n * n;
  const int s = blockIdx.x / count;
  const int i = blockIdx.x - s * count;
  const int j = (2 * i + 1) << (level - 1);
  const size_t gstride = g_chain_blocks(N);
  const T* Gl = reinterpret_cast<const T*>(a.Gl) + (size_t)s * gstride * nn;
  const T* Gr = reinterpret_cast<const T*>(a.Gr) + (size_t)s * gstride * nn;
  const T* Linv = reinterpret_cast<const T*>(a.Linv) + (size_t)s * N * nn;
  T* y = reinterpret_cast<T*>(a.y) + (size_t)s * N * nrhs * n;
  T* yj = y + (size_t)(j - 1) * nrhs * n;
  const int half = 1 << (level - 1);
  const int npull = FWD ? 2 * (level - 1) : 2;
  const size_t off = vec_off(a, s, N - j);
  const int seg0 = seg_of(a, s);
  stage_rhs64<T, FWD>(a, rhs, off, seg0, yj);
  __syncthreads();  // rhs is complete before any lane updates it (also with no pulls)
  T part[kMaxRhs64];
#pragma unroll
  for (int q = 0; q < kMaxRhs64; ++q) part[q] = T(0);
  for (int p = 0; p < npull; ++p) {
    const T* blk;
    const T* vp;
    if constexpr (FWD) {
      const int t = p >> 1;
      const int c = (p & 1) ? j + (1 << t) : j - (1 << t);
      if (c > m) continue;
      blk = ((p & 1) ? Gl : Gr) + (size_t)(c - 1) * nn;
      vp = y + (size_t)(c - 1) * nrhs * n;
    } else {
      if (p == 0) {
        if (j - half < 1) continue;
        blk = Gl + (size_t)(j - 1) * nn;
        vp = y + (size_t)(j - half - 1) * nrhs * n;
      } else {
        const int ir = j + half <= m ? j + half - 1 : N - 1;
        blk = Gr + (size_t)(j - 1) * nn;
        vp = y + (size_t)ir * nrhs * n;
      }
    }
    RB b;
    b.template load<!FWD>(blk, n);
    __syncthreads();  // the previous pull's vector is consumed
    stage_vec64<T>(vec, vp, n, nrhs);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxRhs64; ++q)
      if (q < nrhs) part[q] += b.dot(vec[q]);
  }
  const int o = RB::out_index();
#pragma unroll
  for (int q = 0; q < kMaxRhs64; ++q) {
    if (q < nrhs) {
      const T t = lane_group_sum<RB::LPR>(part[q]);
      if (RB::base() == 0) rhs[q][o] -= t;
    }
  }
  __syncthreads();
  RB lin;
  lin.template load_packed<!FWD>(Linv + (size_t)(j - 1) * nn, n);
#pragma unroll
  for (int q = 0; q < kMaxRhs64; ++q) {
    if (q < nrhs) {
      const T v = lane_group_sum<RB::LPR>(lin.dot(rhs[q]));
      if (RB::base() == 0 && o < n) {
        yj[q * n + o] = v;
        if constexpr (!FWD) scatter_value(a, q, off + o, seg0, static_cast<double>(v));
      }
    }
  }
}

// x_1 forward step: its row holds G_r of the last position of every level with an odd
// chain length; y_X = L_X^{-1} (r_X - those products), w_s = F_s y_X in FP64.
template <typename T>
__global__ void __launch_bounds__(T64) solve64_x_fwd_kernel(SolveArgs a) {
  if (a.done && *a.done) return;
  typedef RegBlock<T, 64, W64> RB;
  __shared__ T vec[kMaxRhs64][64];
  __shared__ T rhs[kMaxRhs64][64];
  const int n = a.n, N = a.N, nrhs = a.nrhs, m = a.m;
  const size_t nn = (size_t)n * n;
  const int s = blockIdx.x;
  const T* Gr = reinterpret_cast<const T*>(a.Gr) + (size_t)s * g_chain_blocks(N) * nn;
  const T* Linv = reinterpret_cast<const T*>(a.Linv) + (size_t)s * N * nn;
  T* y = reinterpret_cast<T*>(a.y) + (size_t)s * N * nrhs * n;
  stage_rhs64<T, true>(a, rhs, vec_off(a, s, 0), seg_of(a, s), nullptr);
  __syncthreads();  // rhs is complete before any lane updates it (also with no pulls)
  T part[kMaxRhs64];
#pragma unroll
  for (int q = 0; q < kMaxRhs64; ++q) part[q] = T(0);
  for (int t = 0; t < chain_levels(m); ++t) {
    if (((m >> t) & 1) == 0) continue;
    const int c = (m >> t) << t;
    RB b;
    b.template load<false>(Gr + (size_t)(c - 1) * nn, n);
    __syncthreads();
    stage_vec64<T>(vec, y + (size_t)(c - 1) * nrhs * n, n, nrhs);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxRhs64; ++q)
      if (q < nrhs) part[q] += b.dot(vec[q]);
  }
  const int o = RB::out_index(), bs = RB::base();
#pragma unroll
  for (int q = 0; q < kMaxRhs64; ++q) {
    if (q < nrhs) {
      const T t = lane_group_sum<RB::LPR>(part[q]);
      if (bs == 0) rhs[q][o] -= t;
    }
  }
  __syncthreads();
  RB lin, fb;
  lin.template load_packed<false>(Linv + (size_t)(N - 1) * nn, n);
  fb.template load<false>(reinterpret_cast<const T*>(a.F) + (size_t)s * nn, n);
  T* yx = y + (size_t)(N - 1) * nrhs * n;
#pragma unroll
  for (int q = 0; q < kMaxRhs64; ++q) {
    if (q < nrhs) {
      const T v = lane_group_sum<RB::LPR>(lin.dot(rhs[q]));
      if (bs == 0) {
        vec[q][o] = o < n ? v : T(0);
        if (o < n) yx[q * n + o] = v;
      }
    }
  }
  __syncthreads();
  // w_s = F_s y_X in FP64 (the root reduction input)
#pragma unroll
  for (int q = 0; q < kMaxRhs64; ++q) {
    if (q < nrhs) {
      double p = 0.0;
#pragma unroll
      for (int e = 0; e < RB::EPL; ++e)
        p += static_cast<double>(fb.v[e]) * static_cast<double>(vec[q][bs + e]);
      p = lane_group_sum<RB::LPR>(p);
      if (bs == 0 && o < n) a.w[((size_t)s * nrhs + q) * n + o] = p;
    }
  }
}

// Root propagation and x_1 backward step: dy_X -= F^T x_0 (FP64), x_X = L_X^{-T} dy_X.
template <typename T>
__global__ void __launch_bounds__(T64) solve64_x_bwd_kernel(SolveArgs a) {
  if (a.done && *a.done) return;
  typedef RegBlock<T, 64, W64> RB;
  __shared__ T rhs[kMaxRhs64][64];
  __shared__ double x0s[kMaxRhs64][64];
  const int n = a.n, N = a.N, nrhs = a.nrhs;
  const size_t nn = (size_t)n * n;
  const int s = blockIdx.x;
  const T* Linv = reinterpret_cast<const T*>(a.Linv) + (size_t)s * N * nn;
  T* yx = reinterpret_cast<T*>(a.y) + ((size_t)s * N + (N - 1)) * nrhs * n;
  for (int idx = threadIdx.x; idx < nrhs * 64; idx += T64) {
    const int q = idx >> 6, i = idx & 63;
    x0s[q][i] = i < n ? a.x0[((size_t)(s / a.S) * nrhs + q) * n + i] : 0.0;
    rhs[q][i] = i < n ? yx[q * n + i] : T(0);
  }
  RB lin, fb;
  lin.template load_packed<true>(Linv + (size_t)(N - 1) * nn, n);
  fb.template load<true>(reinterpret_cast<const T*>(a.F) + (size_t)s * nn, n);
  __syncthreads();
  const int o = RB::out_index(), bs = RB::base();
#pragma unroll
  for (int q = 0; q < kMaxRhs64; ++q) {
    if (q < nrhs) {
      double p = 0.0;
#pragma unroll
      for (int e = 0; e < RB::EPL; ++e) p += static_cast<double>(fb.v[e]) * x0s[q][bs + e];
      p = lane_group_sum<RB::LPR>(p);
      if (bs == 0) rhs[q][o] = static_cast<T>(static_cast<double>(rhs[q][o]) - p);
    }
  }
  __syncthreads();
  const size_t off = vec_off(a, s, 0);
  const int seg0 = seg_of(a, s);
#pragma unroll
  for (int q = 0; q < kMaxRhs64; ++q) {
    if (q < nrhs) {
      const T v = lane_group_sum<RB::LPR>(lin.dot(rhs[q]));
      if (bs == 0 && o < n) {
        yx[q * n + o] = v;
        scatter_value(a, q, off + o, seg0, static_cast<double>(v));
      }
    }
  }
}

}  // namespace

template <typename T>
void launch_solve64_level(const SolveArgs& a, int level, bool fwd, hipStream_t st) {
  const int count = level_count(a.m, level);
  if (count <= 0) return;
  const dim3 grid((unsigned)(a.B * a.S) * (unsigned)count);
  if (fwd)
    hipLaunchKernelGGL((solve64_level_kernel<T, true>), grid, dim3(T64), 0, st, a, level, count);
  else
    hipLaunchKernelGGL((solve64_level_kernel<T, false>), grid, dim3(T64), 0, st, a, level, count);
}
template <typename T>
void launch_solve64_x(const SolveArgs& a, bool fwd, hipStream_t st) {
  const dim3 grid((unsigned)(a.B * a.S));
  if (fwd)
    hipLaunchKernelGGL((solve64_x_fwd_kernel<T>), grid, dim3(T64), 0, st, a);
  else
    hipLaunchKernelGGL((solve64_x_bwd_kernel<T>), grid, dim3(T64), 0, st, a);
}
template void launch_solve64_level<double>(const SolveArgs&, int, bool, hipStream_t);
template void launch_solve64_level<float>(const SolveArgs&, int, bool, hipStream_t);
template void launch_solve64_x<double>(const SolveArgs&, bool, hipStream_t);
template void launch_solve64_x<float>(const SolveArgs&, bool, hipStream_t);

}  // namespace bmpc
