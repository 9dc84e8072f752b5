// Dense n x n block operations on LDS-resident blocks (n <= NMAX <= 32), gfx950.
//
// A block lives in LDS row-major with a padded leading dimension LD = NMAX + 1 so
// that column walks hit distinct banks.  All helpers are called by every thread of
// the workgroup (NT threads) unless the name says "wave"; helpers that write LDS end
// with a workgroup barrier.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmpc {

template <int NMAX>
struct Lay {
  static constexpr int LD = NMAX + 1;
  static constexpr int SZ = NMAX * LD;
};

// ---- global <-> LDS ----------------------------------------------------------

// dst = the symmetric matrix whose lower triangle is src (row-major n x n, FP64).
// Only the lower triangle of src is read.
template <typename T, int NMAX, int NT>
__device__ inline void lds_load_sym_lower(T* dst, const double* __restrict__ src, int n) {
  constexpr int LD = Lay<NMAX>::LD;
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int r = e / n, c = e - (e / n) * n;
    if (r >= c) {
      const T v = static_cast<T>(src[e]);
      dst[r * LD + c] = v;
      dst[c * LD + r] = v;
    }
  }
}

// dst (+)= src or src^T; src is a row-major n x n block of type S.
template <typename T, int NMAX, int NT, typename S>
__device__ inline void lds_load(T* dst, const S* __restrict__ src, int n, bool transpose,
                                bool add = false) {
  constexpr int LD = Lay<NMAX>::LD;
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int r = e / n, c = e - (e / n) * n;
    const T v = static_cast<T>(src[e]);
    const int o = transpose ? c * LD + r : r * LD + c;
    dst[o] = add ? dst[o] + v : v;
  }
}

template <typename T, int NMAX, int NT>
__device__ inline void lds_zero(T* dst, int n) {
  constexpr int LD = Lay<NMAX>::LD;
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int r = e / n, c = e - (e / n) * n;
    dst[r * LD + c] = T(0);
  }
}

template <typename T, int NMAX, int NT>
__device__ inline void lds_store(T* __restrict__ dst, const T* src, int n) {
  constexpr int LD = Lay<NMAX>::LD;
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int r = e / n, c = e - (e / n) * n;
    dst[e] = src[r * LD + c];
  }
}

// ---- block products ------------------------------------------------------------

// out = alpha * op(X) * Y^T           (accumulate == false)
// out = out + alpha * op(X) * Y^T     (accumulate == true)
// with op(X)[r][k] = X[k][r] if transX else X[r][k].  out may alias X or Y: the
// products are formed in registers and written after a barrier.
template <typename T, int NMAX, int NT>
__device__ inline void lds_gemm_nt(T* out, const T* X, bool transX, const T* Y, T alpha,
                                   bool accumulate, int n) {
  constexpr int LD = Lay<NMAX>::LD;
  constexpr int OUTS = (NMAX * NMAX + NT - 1) / NT;   // outputs per thread
  constexpr int CPT = OUTS < 1 ? 1 : OUTS;            // consecutive columns per thread
  constexpr int TPR = NMAX / CPT;                     // threads per row
  const int tid = threadIdx.x;
  const int r = tid / TPR;
  const int c0 = (tid - r * TPR) * CPT;
  const bool active = (tid < NMAX * TPR) && (r < n);
  T acc[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) acc[q] = T(0);
  if (active) {
    for (int k = 0; k < n; ++k) {
      const T xv = transX ? X[k * LD + r] : X[r * LD + k];
#pragma unroll
      for (int q = 0; q < CPT; ++q) acc[q] += xv * Y[(c0 + q) * LD + k];
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int c = c0 + q;
      if (c < n) {
        T* o = &out[r * LD + c];
        *o = accumulate ? *o + alpha * acc[q] : alpha * acc[q];
      }
    }
  }
  __syncthreads();
}

// ---- Cholesky of one block (one wave, lane = row) ------------------------------

// In place: A (symmetric, lower triangle read) := L with L L^T = A, zeros above the
// diagonal.  Returns (on every lane) the 0-based row of the first non-positive
// pivot, or -1.  Must be called by all 64 lanes of one wave.
template <typename T, int NMAX>
__device__ inline int wave_potrf(T* A, int n) {
  constexpr int LD = Lay<NMAX>::LD;
  const int lane = threadIdx.x & 63;
  T a[NMAX];
#pragma unroll
  for (int c = 0; c < NMAX; ++c)
    a[c] = (lane < n && c < n && c <= lane) ? A[lane * LD + c] : T(0);
  int fail = -1;
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    if (k < n) {
      const T piv = __shfl(a[k], k);
      if (fail < 0 && !(piv > T(0))) fail = k;
      const T d = sqrt(piv);
      const T inv = T(1) / d;
      const T lik = (lane == k) ? d : a[k] * inv;
      if (lane >= k) a[k] = lik;
#pragma unroll
      for (int c = k + 1; c < NMAX; ++c) {
        if (c < n) {
          const T lck = __shfl(lik, c);
          if (lane >= c) a[c] -= lik * lck;
        }
      }
    }
  }
  if (lane < n) {
#pragma unroll
    for (int c = 0; c < NMAX; ++c)
      if (c < n) A[lane * LD + c] = (c <= lane) ? a[c] : T(0);
  }
  return fail;
}

// In place: L (lower triangular) := L^{-1}.  One wave; lane j forms column j by
// forward substitution L x = e_j with the rows of L read as LDS broadcasts.
template <typename T, int NMAX>
__device__ inline void wave_trtri(T* A, int n) {
  constexpr int LD = Lay<NMAX>::LD;
  const int lane = threadIdx.x & 63;
  T x[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (i < n) {
      T s = (i == lane) ? T(1) : T(0);
#pragma unroll
      for (int k = 0; k < i; ++k) s -= A[i * LD + k] * x[k];
      x[i] = s / A[i * LD + i];
    } else {
      x[i] = T(0);
    }
  }
  // all lanes have finished reading L (the wave runs in lockstep); write columns
  __builtin_amdgcn_wave_barrier();
  if (lane < n) {
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
      if (i < n) A[i * LD + lane] = (i >= lane) ? x[i] : T(0);
  }
}

}  // namespace bmpc
