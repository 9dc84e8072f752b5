// Two-level triangular solves (Algorithm 2) for gfx950.
//
// Forward substitution L dy = Pi r, one launch per Gamma level: a position j of
// level l pulls the contributions of the positions that precede it in the factor's
// row j -- the left neighbours j-2^t and right neighbours j+2^t of levels t+1 < l --
// so every factor block is read exactly once per sweep and no two work items write
// the same vector (no atomics, fixed summation order).  Then X (x_1), whose row holds
// the G_r blocks of the last position of every level with an odd chain length, and
// the FP64 root step (Algorithm 2, lines 5-7).  Backward substitution walks the
// levels in reverse; position j reads the already known x of its two neighbours.
// The permutation Pi_i (Algorithm 2, lines 2 and 11) is applied as an index map:
// chain position j reads and writes stage N-j of the natural-order vectors.
#include "bmpc_internal.h"
#include "blockops.h"

namespace bmpc {

namespace {

constexpr int NT = kSolveThreads;

template <typename T, int NMAX>
struct SolveSmem {
  T M[Lay<NMAX>::SZ];
  T v[kMaxRhs][NMAX];
  T r[kMaxRhs][NMAX];
};

__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

__device__ inline void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            static_cast<unsigned long long>(__double_as_longlong(v)));
}

// out[q][row] (+)= alpha * op(M) vin[q] with M an n x n block in global memory.
template <typename T, int NMAX>
__device__ inline void gemv(SolveSmem<T, NMAX>& sm, const T* __restrict__ gM, bool trans,
                            T (*vin)[NMAX], T (*out)[NMAX], T alpha, bool accumulate, int n,
                            int nrhs) {
  constexpr int LD = Lay<NMAX>::LD;
  lds_load<T, NMAX, NT>(sm.M, gM, n, false);
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += NT) {
    const int q = idx / n, row = idx - (idx / n) * n;
    T acc = T(0);
    if (trans) {
      for (int k = 0; k < n; ++k) acc += sm.M[k * LD + row] * vin[q][k];
    } else {
      for (int k = 0; k < n; ++k) acc += sm.M[row * LD + k] * vin[q][k];
    }
    out[q][row] = accumulate ? out[q][row] + alpha * acc : alpha * acc;
  }
  __syncthreads();
}

template <typename T, int NMAX>
__device__ inline void load_vec(T (*dst)[NMAX], const T* __restrict__ src, int n, int nrhs) {
  for (int idx = threadIdx.x; idx < n * nrhs; idx += NT) {
    const int q = idx / n, i = idx - (idx / n) * n;
    dst[q][i] = src[idx];
  }
}

template <typename T, int NMAX>
__device__ inline void store_vec(T* __restrict__ dst, T (*src)[NMAX], int n, int nrhs) {
  for (int idx = threadIdx.x; idx < n * nrhs; idx += NT) {
    const int q = idx / n, i = idx - (idx / n) * n;
    dst[idx] = src[q][i];
  }
}

// r[q] = scale_q * b[q][off .. off+n)
template <typename T, int NMAX>
__device__ inline void gather_rhs(const SolveArgs& a, T (*dst)[NMAX], size_t off) {
  const size_t len = ((size_t)a.S * a.N + 1) * a.n;
  for (int idx = threadIdx.x; idx < a.n * a.nrhs; idx += NT) {
    const int q = idx / a.n, i = idx - (idx / a.n) * a.n;
    double v = a.b[(size_t)q * len + off + i];
    if (a.rnorm) {
      const double rn = a.rnorm[q];
      v = rn > 0.0 ? v / rn : 0.0;
    }
    dst[q][i] = static_cast<T>(v);
  }
}

template <typename T, int NMAX>
__device__ inline void scatter_x(const SolveArgs& a, T (*src)[NMAX], size_t off) {
  const size_t len = ((size_t)a.S * a.N + 1) * a.n;
  for (int q = 0; q < a.nrhs; ++q) {
    double dmax = 0.0, xmax = 0.0;
    for (int i = threadIdx.x; i < a.n; i += NT) {
      const size_t idx = (size_t)q * len + off + i;
      const double d = static_cast<double>(src[q][i]);
      if (a.accumulate) {
        const double dd = a.rnorm[q] * d;
        const double xn = a.x[idx] + dd;
        a.x[idx] = xn;
        dmax = fmax(dmax, fabs(dd));
        xmax = fmax(xmax, fabs(xn));
      } else {
        a.x[idx] = d;
      }
    }
    if (a.accumulate) {
      dmax = wave_max(dmax);
      xmax = wave_max(xmax);
      if (threadIdx.x == 0) {
        atomic_max_nonneg(&a.dnorm[q], dmax);
        atomic_max_nonneg(&a.xnorm[q], xmax);
      }
    }
  }
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(NT) solve_fwd_level_kernel(SolveArgs a, int level, int count) {
  if (a.done && *a.done) return;
  __shared__ SolveSmem<T, NMAX> sm;
  const int n = a.n, N = a.N, nrhs = a.nrhs;
  const size_t nn = (size_t)n * n;
  const int s = blockIdx.x / count;
  const int i = blockIdx.x - s * count;
  const int j = (2 * i + 1) << (level - 1);
  const size_t gstride = (size_t)(N > 1 ? N - 1 : 1);
  const T* Gl = reinterpret_cast<const T*>(a.Gl) + (size_t)s * gstride * nn;
  const T* Gr = reinterpret_cast<const T*>(a.Gr) + (size_t)s * gstride * nn;
  const T* Linv = reinterpret_cast<const T*>(a.Linv) + (size_t)s * N * nn;
  T* y = reinterpret_cast<T*>(a.y) + (size_t)s * N * nrhs * n;

  gather_rhs<T, NMAX>(a, sm.r, ((size_t)s * N + (N - j)) * n);
  for (int t = 0; t + 1 < level; ++t) {
    const int cl = j - (1 << t);  // its right neighbour at level t+1 is j
    __syncthreads();
    load_vec<T, NMAX>(sm.v, y + (size_t)(cl - 1) * nrhs * n, n, nrhs);
    gemv<T, NMAX>(sm, Gr + (size_t)(cl - 1) * nn, false, sm.v, sm.r, T(-1), true, n, nrhs);
    const int cr = j + (1 << t);  // its left neighbour at level t+1 is j
    if (cr <= a.m) {
      load_vec<T, NMAX>(sm.v, y + (size_t)(cr - 1) * nrhs * n, n, nrhs);
      gemv<T, NMAX>(sm, Gl + (size_t)(cr - 1) * nn, false, sm.v, sm.r, T(-1), true, n, nrhs);
    }
  }
  __syncthreads();
  gemv<T, NMAX>(sm, Linv + (size_t)(j - 1) * nn, false, sm.r, sm.v, T(1), false, n, nrhs);
  store_vec<T, NMAX>(y + (size_t)(j - 1) * nrhs * n, sm.v, n, nrhs);
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(NT) solve_x_fwd_kernel(SolveArgs a) {
  if (a.done && *a.done) return;
  __shared__ SolveSmem<T, NMAX> sm;
  const int n = a.n, N = a.N, nrhs = a.nrhs, m = a.m;
  const size_t nn = (size_t)n * n;
  const int s = blockIdx.x;
  const size_t gstride = (size_t)(N > 1 ? N - 1 : 1);
  const T* Gr = reinterpret_cast<const T*>(a.Gr) + (size_t)s * gstride * nn;
  const T* Linv = reinterpret_cast<const T*>(a.Linv) + (size_t)s * N * nn;
  T* y = reinterpret_cast<T*>(a.y) + (size_t)s * N * nrhs * n;

  gather_rhs<T, NMAX>(a, sm.r, ((size_t)s * N + 0) * n);
  // The last position of level t+1 has X as its right neighbour iff floor(m/2^t) is odd.
  for (int t = 0; (m >> t) > 0; ++t) {
    if ((m >> t) & 1) {
      const int c = (m >> t) << t;
      __syncthreads();
      load_vec<T, NMAX>(sm.v, y + (size_t)(c - 1) * nrhs * n, n, nrhs);
      gemv<T, NMAX>(sm, Gr + (size_t)(c - 1) * nn, false, sm.v, sm.r, T(-1), true, n, nrhs);
    }
  }
  __syncthreads();
  gemv<T, NMAX>(sm, Linv + (size_t)(N - 1) * nn, false, sm.r, sm.v, T(1), false, n, nrhs);
  store_vec<T, NMAX>(y + (size_t)(N - 1) * nrhs * n, sm.v, n, nrhs);
  // w_s = F_s y_X in FP64 (root reduction input, Algorithm 2 line 5)
  constexpr int LD = Lay<NMAX>::LD;
  lds_load<T, NMAX, NT>(sm.M, reinterpret_cast<const T*>(a.F) + (size_t)s * nn, n, false);
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += NT) {
    const int q = idx / n, row = idx - (idx / n) * n;
    double acc = 0.0;
    for (int k = 0; k < n; ++k)
      acc += static_cast<double>(sm.M[row * LD + k]) * static_cast<double>(sm.v[q][k]);
    a.w[((size_t)s * nrhs + q) * n + row] = acc;
  }
}

// Root step in FP64 (Algorithm 2, lines 5-7).  One workgroup of 256 threads.
__global__ void __launch_bounds__(256) solve_root_kernel(SolveArgs a) {
  if (a.done && *a.done) return;
  __shared__ double part[256];
  __shared__ double r0[kMaxRhs][32];
  const int n = a.n, S = a.S, nrhs = a.nrhs;
  const size_t len = ((size_t)S * a.N + 1) * n;
  const size_t root_off = (size_t)S * a.N * n;
  // sum_s w_s for every (q, i): 8 thread groups over scenario slices, then a fixed
  // combination order.
  const int tpe = 256 / 32;  // threads per element slot
  for (int q = 0; q < nrhs; ++q) {
    const int i = threadIdx.x / tpe, g = threadIdx.x - (threadIdx.x / tpe) * tpe;
    double acc = 0.0;
    if (i < n)
      for (int s = g; s < S; s += tpe) acc += a.w[((size_t)s * nrhs + q) * n + i];
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < n) {
      double t = 0.0;
      for (int gg = 0; gg < tpe; ++gg) t += part[threadIdx.x * tpe + gg];
      double bv = a.b[(size_t)q * len + root_off + threadIdx.x];
      if (a.rnorm) {
        const double rn = a.rnorm[q];
        bv = rn > 0.0 ? bv / rn : 0.0;
      }
      r0[q][threadIdx.x] = bv - t;
    }
    __syncthreads();
  }
  // triangular solves with L_R, one thread per right-hand side
  if (threadIdx.x < nrhs) {
    const int q = threadIdx.x;
    double* v = r0[q];
    for (int i = 0; i < n; ++i) {
      double t = v[i];
      for (int k = 0; k < i; ++k) t -= a.LR[i * n + k] * v[k];
      v[i] = t / a.LR[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = v[i];
      for (int k = i + 1; k < n; ++k) t -= a.LR[k * n + i] * v[k];
      v[i] = t / a.LR[i * n + i];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += 256) {
    const int q = idx / n, i = idx - (idx / n) * n;
    a.x0[idx] = r0[q][i];
  }
  for (int q = 0; q < nrhs; ++q) {
    double dmax = 0.0, xmax = 0.0;
    if (threadIdx.x < n) {
      const size_t idx = (size_t)q * len + root_off + threadIdx.x;
      const double d = r0[q][threadIdx.x];
      if (a.accumulate) {
        const double dd = a.rnorm[q] * d;
        const double xn = a.x[idx] + dd;
        a.x[idx] = xn;
        dmax = fabs(dd);
        xmax = fabs(xn);
      } else {
        a.x[idx] = d;
      }
    }
    if (a.accumulate && threadIdx.x < 64) {
      dmax = wave_max(dmax);
      xmax = wave_max(xmax);
      if (threadIdx.x == 0) {
        atomic_max_nonneg(&a.dnorm[q], dmax);
        atomic_max_nonneg(&a.xnorm[q], xmax);
      }
    }
  }
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(NT) solve_x_bwd_kernel(SolveArgs a) {
  if (a.done && *a.done) return;
  __shared__ SolveSmem<T, NMAX> sm;
  constexpr int LD = Lay<NMAX>::LD;
  const int n = a.n, N = a.N, nrhs = a.nrhs;
  const size_t nn = (size_t)n * n;
  const int s = blockIdx.x;
  const T* Linv = reinterpret_cast<const T*>(a.Linv) + (size_t)s * N * nn;
  T* y = reinterpret_cast<T*>(a.y) + (size_t)s * N * nrhs * n;
  // dy_X -= F^T x_0 (root propagation, Algorithm 2 line 9), product in FP64
  lds_load<T, NMAX, NT>(sm.M, reinterpret_cast<const T*>(a.F) + (size_t)s * nn, n, false);
  load_vec<T, NMAX>(sm.r, y + (size_t)(N - 1) * nrhs * n, n, nrhs);
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * nrhs; idx += NT) {
    const int q = idx / n, row = idx - (idx / n) * n;
    double acc = 0.0;
    for (int k = 0; k < n; ++k)
      acc += static_cast<double>(sm.M[k * LD + row]) * a.x0[q * n + k];
    sm.v[q][row] = static_cast<T>(static_cast<double>(sm.r[q][row]) - acc);
  }
  __syncthreads();
  gemv<T, NMAX>(sm, Linv + (size_t)(N - 1) * nn, true, sm.v, sm.r, T(1), false, n, nrhs);
  store_vec<T, NMAX>(y + (size_t)(N - 1) * nrhs * n, sm.r, n, nrhs);
  scatter_x<T, NMAX>(a, sm.r, ((size_t)s * N + 0) * n);
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(NT) solve_bwd_level_kernel(SolveArgs a, int level, int count) {
  if (a.done && *a.done) return;
  __shared__ SolveSmem<T, NMAX> sm;
  const int n = a.n, N = a.N, nrhs = a.nrhs;
  const size_t nn = (size_t)n * n;
  const int s = blockIdx.x / count;
  const int i = blockIdx.x - s * count;
  const int j = (2 * i + 1) << (level - 1);
  const size_t gstride = (size_t)(N > 1 ? N - 1 : 1);
  const T* Gl = reinterpret_cast<const T*>(a.Gl) + (size_t)s * gstride * nn;
  const T* Gr = reinterpret_cast<const T*>(a.Gr) + (size_t)s * gstride * nn;
  const T* Linv = reinterpret_cast<const T*>(a.Linv) + (size_t)s * N * nn;
  T* y = reinterpret_cast<T*>(a.y) + (size_t)s * N * nrhs * n;

  load_vec<T, NMAX>(sm.r, y + (size_t)(j - 1) * nrhs * n, n, nrhs);
  const int jl = j - (1 << (level - 1));
  const int jr = j + (1 << (level - 1));
  const int ir = jr <= a.m ? jr - 1 : N - 1;
  __syncthreads();
  if (jl >= 1) {
    load_vec<T, NMAX>(sm.v, y + (size_t)(jl - 1) * nrhs * n, n, nrhs);
    gemv<T, NMAX>(sm, Gl + (size_t)(j - 1) * nn, true, sm.v, sm.r, T(-1), true, n, nrhs);
  }
  load_vec<T, NMAX>(sm.v, y + (size_t)ir * nrhs * n, n, nrhs);
  gemv<T, NMAX>(sm, Gr + (size_t)(j - 1) * nn, true, sm.v, sm.r, T(-1), true, n, nrhs);
  gemv<T, NMAX>(sm, Linv + (size_t)(j - 1) * nn, true, sm.r, sm.v, T(1), false, n, nrhs);
  store_vec<T, NMAX>(y + (size_t)(j - 1) * nrhs * n, sm.v, n, nrhs);
  scatter_x<T, NMAX>(a, sm.v, ((size_t)s * N + (N - j)) * n);
}

#define BMPC_DISPATCH_NMAX(nmax, FN, ...) \
  do {                                    \
    if ((nmax) <= 8)                      \
      FN<T, 8>(__VA_ARGS__);              \
    else if ((nmax) <= 16)                \
      FN<T, 16>(__VA_ARGS__);             \
    else                                  \
      FN<T, 32>(__VA_ARGS__);             \
  } while (0)

template <typename T, int NMAX>
void fwd_level_t(const SolveArgs& a, int level, hipStream_t st) {
  const int count = level_count(a.m, level);
  if (count <= 0) return;
  hipLaunchKernelGGL((solve_fwd_level_kernel<T, NMAX>), dim3(a.S * count), dim3(NT), 0, st,
                     a, level, count);
}
template <typename T, int NMAX>
void bwd_level_t(const SolveArgs& a, int level, hipStream_t st) {
  const int count = level_count(a.m, level);
  if (count <= 0) return;
  hipLaunchKernelGGL((solve_bwd_level_kernel<T, NMAX>), dim3(a.S * count), dim3(NT), 0, st,
                     a, level, count);
}
template <typename T, int NMAX>
void x_fwd_t(const SolveArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((solve_x_fwd_kernel<T, NMAX>), dim3(a.S), dim3(NT), 0, st, a);
}
template <typename T, int NMAX>
void x_bwd_t(const SolveArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((solve_x_bwd_kernel<T, NMAX>), dim3(a.S), dim3(NT), 0, st, a);
}

}  // namespace

template <typename T>
void launch_solve_fwd_level(const SolveArgs& a, int level, int nmax, hipStream_t st) {
  BMPC_DISPATCH_NMAX(nmax, fwd_level_t, a, level, st);
}
template <typename T>
void launch_solve_bwd_level(const SolveArgs& a, int level, int nmax, hipStream_t st) {
  BMPC_DISPATCH_NMAX(nmax, bwd_level_t, a, level, st);
}
template <typename T>
void launch_solve_x_fwd(const SolveArgs& a, int nmax, hipStream_t st) {
  BMPC_DISPATCH_NMAX(nmax, x_fwd_t, a, st);
}
template <typename T>
void launch_solve_x_bwd(const SolveArgs& a, int nmax, hipStream_t st) {
  BMPC_DISPATCH_NMAX(nmax, x_bwd_t, a, st);
}
void launch_solve_root(const SolveArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(solve_root_kernel, dim3(1), dim3(256), 0, st, a);
}

template void launch_solve_fwd_level<double>(const SolveArgs&, int, int, hipStream_t);
template void launch_solve_fwd_level<float>(const SolveArgs&, int, int, hipStream_t);
template void launch_solve_bwd_level<double>(const SolveArgs&, int, int, hipStream_t);
template void launch_solve_bwd_level<float>(const SolveArgs&, int, int, hipStream_t);
template void launch_solve_x_fwd<double>(const SolveArgs&, int, hipStream_t);
template void launch_solve_x_fwd<float>(const SolveArgs&, int, hipStream_t);
template void launch_solve_x_bwd<double>(const SolveArgs&, int, hipStream_t);
template void launch_solve_x_bwd<float>(const SolveArgs&, int, hipStream_t);

}  // namespace bmpc
