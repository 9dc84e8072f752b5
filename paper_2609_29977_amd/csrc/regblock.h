// Register-resident n x n blocks for matrix-vector products on one wave (gfx950).
//
// A block is split over the 64 lanes of a wave: LPR = 64/NMAX lanes share one output
// index o = lane / LPR and each holds EPL = NMAX/LPR consecutive elements of the
// contraction index, starting at base = (lane % LPR) * EPL.  In the normal mapping a
// lane holds part of row o (products M v); in the transposed mapping part of column o
// (products M^T v).  Both load coalesced from a row-major block and share the same
// dot-product / reduction code.  Rows and columns >= n read as zero.
#pragma once

#include <hip/hip_runtime.h>

namespace bmpc {

template <typename T, int NMAX>
struct RegBlock {
  static_assert(NMAX == 8 || NMAX == 16 || NMAX == 32, "block size bound");
  static constexpr int LPR = 64 / NMAX;
  static constexpr int EPL = NMAX / LPR;
  T v[EPL];

  __device__ static int out_index() { return (threadIdx.x & 63) / LPR; }
  __device__ static int base() { return ((threadIdx.x & 63) % LPR) * EPL; }

  template <bool TRANS>
  __device__ void load(const T* __restrict__ g, int n) {
    const int o = out_index(), b = base();
    if (n == NMAX) {
#pragma unroll
      for (int e = 0; e < EPL; ++e) v[e] = TRANS ? g[(b + e) * NMAX + o] : g[o * NMAX + b + e];
    } else {
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int r = TRANS ? b + e : o, c = TRANS ? o : b + e;
        v[e] = (r < n && c < n) ? g[r * n + c] : T(0);
      }
    }
  }

  // partial sum of this lane's elements against vec[base .. base+EPL) (LDS, padded)
  __device__ T dot(const T* vec) const {
    const int b = base();
    T p = T(0);
#pragma unroll
    for (int e = 0; e < EPL; ++e) p += v[e] * vec[b + e];
    return p;
  }
};

// Sum over the LPR lanes that share an output index (all of them get the sum).
template <int LPR, typename T>
__device__ inline T lane_group_sum(T p) {
#pragma unroll
  for (int off = 1; off < LPR; off <<= 1) p += __shfl_xor(p, off);
  return p;
}

}  // namespace bmpc
