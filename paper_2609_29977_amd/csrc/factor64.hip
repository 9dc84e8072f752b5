// Factor passes for block sizes 33..64 (gfx950).
//
// The same elimination as factor.hip (the tail factorization of Algorithm 1 in the
// Gamma level order; Section IV-B in block form), for blocks up to 64 x 64, which are
// 33 KB each in FP64 LDS: too large for the depth-first window walk, whose live set
// holds 2 Tw + 3 blocks.  Here every pass is one level (window depth 1): window w of a
// pass holds the pass-local position q = 2w + 1 with its left neighbour lo = 2w and its
// right neighbour 2w + 2 (X beyond the reduced chain).  The live set is three LDS
// blocks -- A_q and the two couplings K[q+1, q] and K[q, lo] -- and the Schur updates
// of the two neighbours (A_r -= G_r G_r^T, A_l -= G_l G_l^T and the fill -G_r G_l^T)
// stay in the MFMA accumulators of the sixteen waves, one 16 x 16 output tile each,
// until they are written to the reduced-chain buffers that the next pass reads (the
// accumulator scheme of factor.hip: a boundary node's updates from earlier passes ride
// in its left accumulator).  The last pass (reduced chain of at most one position) also
// eliminates x_1 and forms F = C L_X^{-T} and U = F F^T in FP64.
//
// The diagonal factorization is blocked 2 x 2 into 32 x 32 blocks: the one-wave
// factorization + inverse of factor.hip on the diagonal blocks, the off-diagonal
// products on four waves' matrix cores.
#include "bmpc_internal.h"
#include "blockops.h"

namespace bmpc {

namespace {

constexpr int N64 = 64;
constexpr int LD64 = Lay<N64>::LD;
constexpr int SZ64 = Lay<N64>::SZ;
constexpr int NT64 = TileCfg<N64>::NT;  // 1024: one wave per 16 x 16 output tile

// dst = the symmetric block whose lower triangle is that of D (FP64) plus, after the
// first pass, the carried updates a1 + a2 (lower triangles), identity padded.
template <typename T>
__device__ inline void load_diag64(T* dst, const double* __restrict__ D, const T* a1, const T* a2,
                                   int n) {
  for (int e = threadIdx.x; e < N64 * N64; e += NT64) {
    const int r = e >> 6, c = e & 63;
    T v;
    if (r < n && c < n) {
      const int o = r >= c ? r * n + c : c * n + r;
      v = static_cast<T>(D[o]);
      if (a1) v = (v + a1[o]) + a2[o];
    } else {
      v = (r == c) ? T(1) : T(0);
    }
    dst[r * LD64 + c] = v;
  }
}

// dst = src (TRANS: src^T), src row-major n x n of type S, zero padded.
template <typename T, typename S>
__device__ inline void load_block64(T* dst, const S* __restrict__ src, int n, bool trans) {
  for (int e = threadIdx.x; e < N64 * N64; e += NT64) {
    const int r = e >> 6, c = e & 63;
    T v = T(0);
    if (r < n && c < n) v = static_cast<T>(trans ? src[c * n + r] : src[r * n + c]);
    dst[r * LD64 + c] = v;
  }
}

// Tile (ti, tj) of a 32 x 32 product on one wave, K = 32:
// out[r][c] = init[r][c] + sum_k (NEG ? -X[r][k] : X[r][k]) * (NT ? Y[c][k] : Y[k][c]).
template <typename T, bool NT, bool NEG>
__device__ inline typename Mfma<T>::acc_t prod32(const T* X, const T* Y, int ti, int tj,
                                                 typename Mfma<T>::acc_t acc) {
  const int l = threadIdx.x & 63, g = l >> 4, i = l & 15;
  const int r = ti * 16 + i, c = tj * 16 + i;
#pragma unroll
  for (int st = 0; st < 8; ++st) {
    const int k = 8 * g + st;
    const T a = X[r * LD64 + k];
    const T b = NT ? Y[c * LD64 + k] : Y[k * LD64 + c];
    acc = Mfma<T>::mma(NEG ? -a : a, b, acc);
  }
  return acc;
}

template <typename T>
__device__ inline typename Mfma<T>::acc_t tile32_load(const T* X, int ti, int tj) {
  const int l = threadIdx.x & 63;
  typename Mfma<T>::acc_t t;
#pragma unroll
  for (int v = 0; v < 4; ++v) t[v] = X[(ti * 16 + Mfma<T>::row(l, v)) * LD64 + tj * 16 + (l & 15)];
  return t;
}
template <typename T>
__device__ inline void tile32_store(T* X, int ti, int tj, const typename Mfma<T>::acc_t& t) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 4; ++v) X[(ti * 16 + Mfma<T>::row(l, v)) * LD64 + tj * 16 + (l & 15)] = t[v];
}

// In place: A (64 x 64 symmetric in LDS, identity padded) := L^{-1}, L L^T = A, by the
// 2 x 2 blocking of factor.hip one size up:
//   L11^{-1} (one wave);  L21 = A21 L11^{-T};  S = A22 - L21 L21^T;  L22^{-1} (one wave);
//   (L^{-1})21 = -L22^{-1} (L21 L11^{-1}),
// the products on waves 0..3 (one 16 x 16 tile of the 32 x 32 result each).  Called by
// every thread.  Returns, on wave 0, the 0-based row of the first non-positive pivot
// or -1.
template <typename T>
__device__ int potrf_inv64(T* A) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int wv = threadIdx.x >> 6;
  const int ti = wv >> 1, tj = wv & 1;
  const bool prod = wv < 4;
  T* A11 = A;
  T* A21 = A + 32 * LD64;
  T* A22 = A + 32 * LD64 + 32;
  T* A12 = A + 32;
  int f1 = -1, f2 = -1;
  if (wv == 0) f1 = wave_potrf_inv<T, 32, LD64>(A11);
  __syncthreads();
  const acc_t z = {0, 0, 0, 0};
  acc_t t = z;
  if (prod) t = prod32<T, true, false>(A21, A11, ti, tj, z);  // L21 = A21 L11^{-T}
  __syncthreads();
  if (prod) tile32_store(A21, ti, tj, t);
  __syncthreads();
  if (prod) t = prod32<T, true, true>(A21, A21, ti, tj, tile32_load(A22, ti, tj));  // S
  __syncthreads();
  if (prod) tile32_store(A22, ti, tj, t);
  __syncthreads();
  if (wv == 0) f2 = wave_potrf_inv<T, 32, LD64>(A22);
  __syncthreads();
  if (prod) t = prod32<T, false, false>(A21, A11, ti, tj, z);  // W = L21 L11^{-1}
  __syncthreads();
  if (prod) tile32_store(A21, ti, tj, t);
  __syncthreads();
  if (prod) t = prod32<T, false, true>(A22, A21, ti, tj, z);  // -L22^{-1} W
  __syncthreads();
  if (prod) {
    tile32_store(A21, ti, tj, t);
    tile32_store(A12, ti, tj, z);
  }
  __syncthreads();
  if (f1 >= 0) return f1;
  return f2 >= 0 ? 32 + f2 : -1;
}

// This wave's tile of an accumulator block, read from / written to global n x n blocks
// (elements outside n x n are skipped; reads give zero).
template <typename T>
__device__ inline void tile_read_add(typename Mfma<T>::acc_t& t, const T* src, int n) {
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int ti = wv >> 2, tj = wv & 3, c = tj * 16 + (l & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = ti * 16 + Mfma<T>::row(l, v);
    if (r < n && c < n) t[v] += src[r * n + c];
  }
}
template <typename T>
__device__ inline void tile_write(T* dst, const typename Mfma<T>::acc_t& t, int n) {
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int ti = wv >> 2, tj = wv & 3, c = tj * 16 + (l & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = ti * 16 + Mfma<T>::row(l, v);
    if (r < n && c < n) dst[r * n + c] = t[v];
  }
}
template <typename T>
__device__ inline typename Mfma<T>::acc_t tile_from_lds(const T* X) {
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int ti = wv >> 2, tj = wv & 3;
  typename Mfma<T>::acc_t t;
#pragma unroll
  for (int v = 0; v < 4; ++v) t[v] = X[(ti * 16 + Mfma<T>::row(l, v)) * LD64 + tj * 16 + (l & 15)];
  return t;
}

template <typename T>
__device__ inline void lds_store_full(T* __restrict__ dst, const T* src, int n) {
  for (int e = threadIdx.x; e < n * n; e += NT64) {
    const int r = e / n, c = e - r * n;
    dst[e] = src[r * LD64 + c];
  }
}
template <typename T>
__device__ inline void lds_store_packed(T* __restrict__ dst, const T* src, int n) {
  for (int e = threadIdx.x; e < n * n; e += NT64) {
    const int r = e / n, c = e - r * n;
    if (c <= r) dst[r * (r + 1) / 2 + c] = src[r * LD64 + c];
  }
}

template <typename T, bool FIRST, bool FINAL>
__global__ void __launch_bounds__(NT64, 1) factor64_pass_kernel(FactorPassArgs a) {
  typedef typename Mfma<T>::acc_t acc_t;
  extern __shared__ __align__(16) unsigned char smem64[];
  T* Aq = reinterpret_cast<T*>(smem64);
  T* Cr = Aq + SZ64;  // K[rb, q], then G_r
  T* Cl = Cr + SZ64;  // K[q, lo], then G_l
  const int n = a.n, N = a.N;
  const size_t nn = (size_t)n * n;
  const int s = blockIdx.x / a.windows;
  const int w = blockIdx.x - s * a.windows;
  const int lo = 2 * w, q = lo + 1;
  const bool has_q = q <= a.mk, has_left = lo >= 1;
  const bool rb_is_x = lo + 2 > a.mk;
  const int j = q << a.shift;  // chain position of q
  T* Linv = reinterpret_cast<T*>(a.Linv) + (size_t)s * N * nn;
  T* Gl = reinterpret_cast<T*>(a.Gl) + (size_t)s * g_chain_blocks(N) * nn;
  T* Gr = reinterpret_cast<T*>(a.Gr) + (size_t)s * g_chain_blocks(N) * nn;
  const int sys = s / a.Ssys;
  const unsigned long long chain_row0 =
      (unsigned long long)sys * ((unsigned long long)a.Ssys * N + 1) * n +
      (unsigned long long)(s - sys * a.Ssys) * N * n;
  const size_t base = (size_t)s * a.stride;
  const T* accR_in = reinterpret_cast<const T*>(a.accR_in);
  const T* accL_in = reinterpret_cast<const T*>(a.accL_in);
  const T* fill_in = reinterpret_cast<const T*>(a.fill_in);

  const acc_t z = {0, 0, 0, 0};
  acc_t AL = z, AR = z, FL = z;
  if (has_left && !FIRST) {
    tile_read_add<T>(AL, accR_in + (base + lo) * nn, n);
    tile_read_add<T>(AL, accL_in + (base + lo) * nn, n);
  }
  if (has_q) {
    load_diag64<T>(Aq, a.D + ((size_t)s * N + (N - j)) * nn,
                   FIRST ? nullptr : accR_in + (base + q) * nn,
                   FIRST ? nullptr : accL_in + (base + q) * nn, n);
    if constexpr (FIRST)
      load_block64<T, double>(Cr, a.E + ((size_t)s * (N - 1) + (N - 1 - q)) * nn, n, true);
    else
      load_block64<T, T>(Cr, fill_in + (base + q) * nn, n, false);
  }
  if (has_left) {
    if constexpr (FIRST)
      load_block64<T, double>(Cl, a.E + ((size_t)s * (N - 1) + (N - 1 - lo)) * nn, n, true);
    else
      load_block64<T, T>(Cl, fill_in + (base + lo) * nn, n, false);
  }
  __syncthreads();
  if (has_q) {
    const int fail = potrf_inv64<T>(Aq);
    if (threadIdx.x == 0 && fail >= 0 && fail < n)
      atomicMin(a.info, chain_row0 + (unsigned long long)a.permpos[j - 1] * n + fail + 1);
    const acc_t gr = mfma_tile_nt<T, N64, false>(Cr, Aq);  // G_r = K[rb,q] L^{-T}
    acc_t gl = z;
    if (has_left) gl = mfma_tile_nt<T, N64, true>(Cl, Aq);  // G_l = K[q,lo]^T L^{-T}
    __syncthreads();
    mfma_tile_store<T, N64, false>(Cr, gr, T(1));
    if (has_left) mfma_tile_store<T, N64, false>(Cl, gl, T(1));
    __syncthreads();
    lds_store_packed<T>(Linv + (size_t)(j - 1) * nn, Aq, n);
    lds_store_full<T>(Gr + (size_t)(j - 1) * nn, Cr, n);
    if (has_left) lds_store_full<T>(Gl + (size_t)(j - 1) * nn, Cl, n);
    const acc_t ur = mfma_tile_nt<T, N64, false>(Cr, Cr);
#pragma unroll
    for (int v = 0; v < 4; ++v) AR[v] = -ur[v];
    if (has_left) {
      const acc_t ul = mfma_tile_nt<T, N64, false>(Cl, Cl);
      const acc_t uf = mfma_tile_nt<T, N64, false>(Cr, Cl);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        AL[v] = AL[v] - ul[v];
        FL[v] = -uf[v];
      }
    }
  } else if (has_left) {
    FL = tile_from_lds(Cl);  // no position: lo keeps its coupling to X
  }

  if constexpr (!FINAL) {
    if (has_left) {
      tile_write<T>(reinterpret_cast<T*>(a.accL_out) + (base + w) * nn, AL, n);
      tile_write<T>(reinterpret_cast<T*>(a.fill_out) + (base + w) * nn, FL, n);
    }
    if (!rb_is_x)
      tile_write<T>(reinterpret_cast<T*>(a.accR_out) + (base + w + 1) * nn, AR, n);
    else
      tile_write<T>(reinterpret_cast<T*>(a.accX) + ((size_t)s * a.npass + a.pass) * nn, AR, n);
  } else {
    // ---- last pass: x_1 step (the coupling solve and local Schur update) ----
    __syncthreads();  // the position's blocks are stored; Aq and Cr are free
    const double* D0 = a.D + (size_t)s * N * nn;
    for (int e = threadIdx.x; e < N64 * N64; e += NT64) {
      const int r = e >> 6, c = e & 63;
      T v;
      if (r < n && c < n) {
        v = static_cast<T>(r >= c ? D0[r * n + c] : D0[c * n + r]);
        for (int p = 0; p < a.pass; ++p)
          v += reinterpret_cast<const T*>(a.accX)[((size_t)s * a.npass + p) * nn + r * n + c];
      } else {
        v = (r == c) ? T(1) : T(0);
      }
      Aq[r * LD64 + c] = v;
    }
    load_block64<T, double>(Cr, a.C + (size_t)s * nn, n, false);
    __syncthreads();
    {
      const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
      const int ti = wv >> 2, tj = wv & 3, c = tj * 16 + (l & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = ti * 16 + Mfma<T>::row(l, v);
        if (r < n && c < n) Aq[r * LD64 + c] += AR[v];
      }
    }
    __syncthreads();
    const int fail = potrf_inv64<T>(Aq);
    if (threadIdx.x == 0 && fail >= 0 && fail < n)
      atomicMin(a.info, chain_row0 + (unsigned long long)a.permpos[N - 1] * n + fail + 1);
    lds_store_packed<T>(Linv + (size_t)(N - 1) * nn, Aq, n);
    const acc_t f = mfma_tile_nt<T, N64, false>(Cr, Aq);  // F = C L_X^{-T}
    __syncthreads();
    mfma_tile_store<T, N64, false>(Cr, f, T(1));
    __syncthreads();
    lds_store_full<T>(reinterpret_cast<T*>(a.F) + (size_t)s * nn, Cr, n);
    double* U = a.U + (size_t)s * nn;  // U = F F^T in FP64 from the stored F
    for (int e = threadIdx.x; e < n * n; e += NT64) {
      const int r = e / n, c = e - r * n;
      double acc = 0.0;
      for (int k = 0; k < n; ++k)
        acc += static_cast<double>(Cr[r * LD64 + k]) * static_cast<double>(Cr[c * LD64 + k]);
      U[e] = acc;
    }
  }
}

template <typename T, bool FIRST, bool FINAL>
void launch64_k(const FactorPassArgs& a, hipStream_t st) {
  const size_t lds = 3 * (size_t)SZ64 * sizeof(T);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(
        reinterpret_cast<const void*>(&factor64_pass_kernel<T, FIRST, FINAL>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr_set = true;
  }
  hipLaunchKernelGGL((factor64_pass_kernel<T, FIRST, FINAL>),
                     dim3((unsigned)a.S * (unsigned)a.windows), dim3(NT64), lds, st, a);
}

}  // namespace

size_t factor64_lds_bytes(bool fp64) { return 3 * (size_t)SZ64 * (fp64 ? 8 : 4); }

template <typename T>
void launch_factor_pass64(const FactorPassArgs& a, hipStream_t st) {
  const bool first = a.pass == 0;
  if (first && a.is_final)
    launch64_k<T, true, true>(a, st);
  else if (first)
    launch64_k<T, true, false>(a, st);
  else if (a.is_final)
    launch64_k<T, false, true>(a, st);
  else
    launch64_k<T, false, false>(a, st);
}
template void launch_factor_pass64<double>(const FactorPassArgs&, hipStream_t);
template void launch_factor_pass64<float>(const FactorPassArgs&, hipStream_t);

}  // namespace bmpc
