// Dense n x n block operations on LDS-resident blocks (n <= NMAX <= 32), gfx950.
//
// A block lives in LDS row-major with a padded leading dimension LD = NMAX + 1 so
// that column walks hit distinct banks.  All helpers are called by every thread of
// the workgroup (NT threads) unless the name says "wave"; helpers that write LDS end
// with a workgroup barrier.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

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

// ---- wave-uniform broadcast and reciprocal square root ---------------------------

// This wave's index in the workgroup, in a scalar register (the compiler cannot tell
// that threadIdx.x / 64 is the same on every lane, and would branch on it per lane).
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ inline float wave_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ inline double wave_bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// v with lane LANE's value replaced by the wave-uniform x (v_writelane with an
// immediate lane select, so that x is the instruction's one scalar operand).
template <int LANE>
__device__ inline int wave_set_lane_b32(int v, int x) {
  asm("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(x), "n"(LANE));
  return v;
}
template <int LANE>
__device__ inline float wave_set_lane(float v, float x) {
  return __int_as_float(wave_set_lane_b32<LANE>(__float_as_int(v), __float_as_int(x)));
}
template <int LANE>
__device__ inline double wave_set_lane(double v, double x) {
  const int lo = wave_set_lane_b32<LANE>(__double2loint(v), __double2loint(x));
  const int hi = wave_set_lane_b32<LANE>(__double2hiint(v), __double2hiint(x));
  return __hiloint2double(hi, lo);
}

// v -= yb[SRC of v's 16-lane row] * m: the row broadcast (DPP row_newbcast) is an
// operand of the multiply-add, and so is the negation (a source modifier), so neither
// costs an instruction of its own.  WAIT
// puts in front the two wait states that a DPP read needs after a vector write of its
// source (the read is inside the asm, where the compiler cannot see it); the
// statements are volatile so that they keep their order and the first one of a group
// is the one that waits.
template <int SRC, bool WAIT>
__device__ __attribute__((always_inline)) inline void row_bcast_fms(float& v, float yb,
                                                                    float m) {
  if constexpr (WAIT)
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(v) : "v"(yb), "v"(m), "n"(SRC));
  else
    asm volatile("v_fmac_f32_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(v) : "v"(yb), "v"(m), "n"(SRC));
}
template <int SRC, bool WAIT>
__device__ __attribute__((always_inline)) inline void row_bcast_fms(double& v, double yb,
                                                                    double m) {
  if constexpr (WAIT)
    asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(v) : "v"(yb), "v"(m), "n"(SRC));
  else
    asm volatile("v_fmac_f64_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(v) : "v"(yb), "v"(m), "n"(SRC));
}

// Lanes 0-15 of y copied into lanes 16-31 (and 32-47 into 48-63): the odd 16-lane rows
// of one copy swapped with the even rows of another (v_permlane16_swap).
__device__ inline float rows_even_to_odd(float y) {
  const unsigned u = __float_as_uint(y);
  return __uint_as_float(__builtin_amdgcn_permlane16_swap(u, u, false, false)[0]);
}
__device__ inline double rows_even_to_odd(double y) {
  const unsigned lo = __double2loint(y), hi = __double2hiint(y);
  const unsigned l2 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false)[0];
  const unsigned h2 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false)[0];
  return __hiloint2double((int)h2, (int)l2);
}

// The first two 16-lane rows of y each copied into both rows: lo = rows (0, 0, 2, 2),
// hi = rows (1, 1, 3, 3) of y (both outputs of one v_permlane16_swap per 32 bits).
__device__ inline void rows_both(float y, float& lo, float& hi) {
  const unsigned u = __float_as_uint(y);
  const auto pr = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  lo = __uint_as_float(pr[0]);
  hi = __uint_as_float(pr[1]);
}
__device__ inline void rows_both(double y, double& lo, double& hi) {
  const unsigned l = __double2loint(y), h = __double2hiint(y);
  const auto pl = __builtin_amdgcn_permlane16_swap(l, l, false, false);
  const auto ph = __builtin_amdgcn_permlane16_swap(h, h, false, false);
  lo = __hiloint2double((int)ph[0], (int)pl[0]);
  hi = __hiloint2double((int)ph[1], (int)pl[1]);
}

// Lane K of rows 0 and 2 to every lane of rows 0-1 and 2-3: a row broadcast (DPP
// row_newbcast) and the even-to-odd row copy.  The pivot broadcast of a leaf that
// factors one block in each 32-lane half of the wave.
template <int K>
__device__ inline float half_bcast(float x) {
  const int b = __builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x150 + K, 0xf, 0xf, false);
  return rows_even_to_odd(__int_as_float(b));
}
template <int K>
__device__ inline double half_bcast(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x150 + K, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x150 + K, 0xf, 0xf, false);
  return rows_even_to_odd(__hiloint2double(hi, lo));
}

// f(std::integral_constant<int, K>{}) for K = 0 .. N-1 in order (a loop whose index is
// a constant expression in the body).
template <typename F, int... Ks>
__device__ __attribute__((always_inline)) inline void static_for_impl(
    F&& f, std::integer_sequence<int, Ks...>) {
  (f(std::integral_constant<int, Ks>{}), ...);
}
template <int N, typename F>
__device__ __attribute__((always_inline)) inline void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// 1/sqrt(x).  FP32: the hardware reciprocal square root, accurate to about one unit in
// the last place, which is the rounding level of the FP32 factor anyway (and the
// refinement around the FP32 path removes it); a Newton step would only lengthen the
// dependency chain of every column of a factorization.  FP64: the hardware estimate
// (relative error below 2^-24 on gfx950) refined by one Halley step: with
// e = 1 - x y^2, the series 1/sqrt(1 - e) = 1 + e/2 + 3e^2/8 + O(e^3) gives
// y <- y + y e (1/2 + 3e/8), whose error is cubic in the estimate's (below 2^-70).
// Four dependent operations, where two Newton steps (quadratic each) take six.
__device__ inline float pivot_rsqrt(float x) {
  return __builtin_amdgcn_rsqf(x);
}
__device__ inline double pivot_rsqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-(x * y), y, 1.0);
  return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}

// ---- Cholesky of one block (one wave, lane = row) ------------------------------

// In place: A (symmetric NMAX x NMAX, lower triangle read; pad smaller blocks with an
// identity block) := L with L L^T = A, zeros above the diagonal.  One wave, lane i
// keeps row i; column k of L is broadcast to the other rows: up to 32 rows as a DPP
// row-broadcast operand of each multiply-add (as in the inverse leaves), 64 rows with
// readlane.  Returns (on every lane) the 0-based row of the first non-positive pivot,
// or -1.
template <typename T, int NMAX>
__device__ __attribute__((always_inline)) inline int wave_potrf(T* A) {
  constexpr int LD = Lay<NMAX>::LD;
  const int lane = threadIdx.x & 63;
  const int row = lane < NMAX ? lane : NMAX - 1;
  T a[NMAX];
#pragma unroll
  for (int c = 0; c < NMAX; ++c) a[c] = A[row * LD + c];
  int fail = -1;
  if constexpr (NMAX <= 32) {
    static_for<NMAX>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const T piv = wave_bcast(a[k], k);
      if (fail < 0 && !(piv > T(0))) fail = k;
      const T inv = pivot_rsqrt(piv);
      const T lik = (lane == k) ? piv * inv : a[k] * inv;
      a[k] = lik;
      if constexpr (k + 1 < NMAX) {
        // L[c][k] is lik on lane c.  With 32 rows both 16-lane rows get a copy of rows
        // 0-15 (lo) and of rows 16-31 (hi); entry c of every lane then takes one
        // multiply-add whose first factor is lane c % 16 of the copy holding row c.
        T lo = lik, hi = lik;
        if constexpr (NMAX == 32) rows_both(lik, lo, hi);
        static_for<NMAX - 1 - k>([&](auto uc) {
          constexpr int u = decltype(uc)::value, c = k + 1 + u;
          // the first use of each copy waits for its write
          if constexpr (c < 16)
            row_bcast_fms<c, u == 0>(a[c], lo, lik);
          else
            row_bcast_fms<c - 16, u == 0 || c == 16>(a[c], hi, lik);
        });
      }
    });
    if (lane < NMAX) {
#pragma unroll
      for (int c = 0; c < NMAX; ++c) A[lane * LD + c] = (c <= lane) ? a[c] : T(0);
    }
    return fail;
  }
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    const T piv = wave_bcast(a[k], k);
    if (fail < 0 && !(piv > T(0))) fail = k;
    // L[k][k] = piv * piv^{-1/2} and L[i][k] = a[i][k] * piv^{-1/2}: one refined
    // reciprocal square root instead of a square root and a division per column
    const T inv = pivot_rsqrt(piv);
    const T lik = (lane == k) ? piv * inv : a[k] * inv;
    a[k] = lik;
#pragma unroll
    for (int c = k + 1; c < NMAX; ++c) a[c] -= lik * wave_bcast(lik, c);
  }
  if (lane < NMAX) {
#pragma unroll
    for (int c = 0; c < NMAX; ++c) A[lane * LD + c] = (c <= lane) ? a[c] : T(0);
  }
  return fail;
}

// Where entry (r, c) of a block lives in LDS.  RowMajor: rows of LD entries (the padded
// slots).  PackedLower: only the lower triangle of a 32 x 32 block, packed by rows
// ((r, c), c <= r, at r (r + 1) / 2 + c); R0 selects the diagonal sub-block starting at
// (R0, R0).  Entries above the diagonal do not exist there: reads of them are replaced by
// zero and writes dropped.
template <int LD>
struct RowMajor {
  static constexpr bool kLowerOnly = false;
  __device__ static int at(int r, int c) { return r * LD + c; }
};
template <int R0>
struct PackedLower {
  static constexpr bool kLowerOnly = true;
  __device__ static int at(int r, int c) { return (R0 + r) * (R0 + r + 1) / 2 + R0 + c; }
};
constexpr int kPacked32 = 32 * 33 / 2;  // entries of a packed 32 x 32 lower triangle

// In place: A (symmetric NMAX x NMAX, lower triangle read) := L^{-1} with L L^T = A.
// One wave, two lane groups.  Lane i < NMAX keeps row i of A and runs the
// right-looking Cholesky sweep: step k forms column k of L (L[i][k] on lane i).
// Lane NMAX + j keeps column j of Z, the inverse being built by the same elimination
// applied to the identity with unscaled rows: row c of Z loses (L[c][k] / L[k][k])
// times row k, and row k is divided by L[k][k] once step k has used it.  Both updates
// of step k are "entry c -= L[c][k] * y" with y = entry k / L[k][k] on every lane
// (L[i][k] on a row lane, Z[k][j] / L[k][k] on a column lane), so one FMA per column
// c > k, with L[c][k] broadcast inside it, serves the factor and the inverse together,
// and entry k keeps y (the finished entry of L^{-1} on a column lane).  No
// per-lane branches: row lanes also update entries above the diagonal, which are
// never read.  Blocks smaller than NMAX must be padded with an identity block.
// Returns (on every lane) the 0-based row of the first non-positive pivot, or -1.
// PAIR: two independent blocks, one per 32-lane half of the wave (A is the lane's own
// block; lanes 32-63 repeat the layout of lanes 0-31), each half's pivot broadcast to
// its half only; the return value is per half.  The instructions are the same as for
// one block, so the pair costs one block's issue slots.
template <typename T, int NMAX, typename Ix = RowMajor<Lay<NMAX>::LD>, bool PAIR = false>
__device__ __attribute__((always_inline)) inline int wave_potrf_inv_leaf(T* A) {
  static_assert(NMAX == 8 || NMAX == 16, "row and column lanes in the first 32 lanes");
  const int lane = threadIdx.x & (PAIR ? 31 : 63);
  const bool rowl = lane < NMAX;
  const int j = lane - NMAX;
  const int idx = rowl ? lane : (j < NMAX ? j : NMAX - 1);
  // Every lane reads a row (column lanes a row they then discard): loads under a lane
  // condition become a branch per element, each waiting for its own read.  (In packed
  // storage the places above the diagonal hold later rows' entries, in range.)
  T v[NMAX];
#pragma unroll
  for (int c = 0; c < NMAX; ++c) v[c] = A[Ix::at(idx, c)];
#pragma unroll
  for (int c = 0; c < NMAX; ++c) v[c] = (rowl && (!Ix::kLowerOnly || c <= idx)) ? v[c] : T(0);
  int fail = -1;
  static_for<NMAX>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    // Column lane k's identity entry.  Set here rather than at the start: until step k
    // it would not change (the entries above a column's diagonal stay zero, so every
    // earlier step subtracts zero from it), and a per-lane constant per column would
    // otherwise be kept in a register across the caller's loop.
    v[k] = wave_set_lane<NMAX + k>(v[k], T(1));
    if constexpr (PAIR) v[k] = wave_set_lane<32 + NMAX + k>(v[k], T(1));
    T piv;
    if constexpr (PAIR)
      piv = half_bcast<k>(v[k]);
    else
      piv = wave_bcast(v[k], k);
    if (fail < 0 && !(piv > T(0))) fail = k;
    const T inv = pivot_rsqrt(piv);
    const T y = v[k] * inv;  // L[i][k] on row lane i (>= k); Z[k][j] / L[k][k] on column lane j
    v[k] = y;
    if constexpr (k + 1 < NMAX) {
      // L[c][k] is y on row lane c.  The row lanes and the column lanes share one 16-lane
      // row at NMAX = 8; at NMAX = 16 the column lanes are the next row, which gets a copy
      // of the row lanes' y.  Then entry c of every lane is updated by one multiply-add
      // whose first factor is lane c of its row.
      const T yb = NMAX == 16 ? rows_even_to_odd(y) : y;
      static_for<NMAX - 1 - k>([&](auto uc) {
        constexpr int u = decltype(uc)::value;
        row_bcast_fms<k + 1 + u, u == 0>(v[k + 1 + u], yb, y);
      });
    }
  });
  // Column lane j's entries above the diagonal (i < j) are exact zeros: they start at
  // zero, and each update subtracts a multiple of y = Z[k][j] / L[k][k] with k < i < j,
  // itself zero.  So in row-major storage the whole column is stored without a mask
  // (packed storage has no places above the diagonal).
  if (!rowl && j < NMAX) {
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
      if (!Ix::kLowerOnly || i >= j) A[Ix::at(i, j)] = v[i];
  }
  return fail;
}

// ---- MFMA block products (16x16x4 tiles) ------------------------------------------

typedef float mf32x4 __attribute__((ext_vector_type(4)));
typedef double mf64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef mf32x4 acc_t;
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of accumulator element v held by lane l (column is l % 16)
  __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <>
struct Mfma<double> {
  typedef mf64x4 acc_t;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int v) { return 4 * v + (l >> 4); }
};

// Threads per workgroup of the blocked kernels: one wave per 16x16 output tile.
template <int NMAX>
struct TileCfg {
  static constexpr int TILES = (NMAX + 15) / 16;     // tiles per dimension
  static constexpr int NT = 64 * TILES * TILES;      // one wave per output tile
  static constexpr int KSTEPS = NMAX / 4;            // MFMA k-steps (4 k per step)
};

// This wave's 16x16 tile of op(X) Y^T (NMAX x NMAX blocks in LDS, zero padded beyond
// the used size) in MFMA accumulator layout, op(X)[r][k] = X[k][r] if transX.  The
// contraction index is distributed as k = KSTEPS*(lane/16) + s over the MFMA steps s,
// identically for both operands.  Blocks smaller than a tile (NMAX = 8) are masked.
// 8 x 8 blocks: one product per wave on the vector ALU, lane l forming element
// (l / 8, l % 8) in acc[0].  A 16 x 16 MFMA tile leaves three quarters of its lanes idle
// here; measured on n = 8 systems the vector path makes the first factor pass 8-10%
// faster in both precisions.
constexpr bool kValu8 = true;

template <typename T, int NMAX, bool TRANSX>
__device__ __attribute__((always_inline)) inline typename Mfma<T>::acc_t mfma_tile_nt(
    const T* X, const T* Y) {
  constexpr int LD = Lay<NMAX>::LD;
  if constexpr (NMAX == 8 && kValu8) {
    const int l = threadIdx.x & 63, r = l >> 3, c = l & 7;
    T a = T(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) a += (TRANSX ? X[k * LD + r] : X[r * LD + k]) * Y[c * LD + k];
    return {a, T(0), T(0), T(0)};
  }
  constexpr int KS = TileCfg<NMAX>::KSTEPS;
  const int w = wave_id() % (TileCfg<NMAX>::TILES * TileCfg<NMAX>::TILES);
  const int l = threadIdx.x & 63;
  const int ti = w / TileCfg<NMAX>::TILES, tj = w % TileCfg<NMAX>::TILES;
  const int g = l >> 4, i = l & 15;
  const int r = ti * 16 + i, c = tj * 16 + i;
  const bool rin = NMAX >= 16 || r < NMAX, cin = NMAX >= 16 || c < NMAX;
  const int rr = rin ? r : 0, cc = cin ? c : 0;
  typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = KS * g + s;
    T a = TRANSX ? X[k * LD + rr] : X[rr * LD + k];
    T b = Y[cc * LD + k];
    if (!rin) a = T(0);
    if (!cin) b = T(0);
    acc = Mfma<T>::mma(a, b, acc);
  }
  return acc;
}

// Row tile ti of op(X) L^T for a lower triangular L (32 x 32 blocks in LDS, L's upper
// triangle zero): t0 = columns 0..15, which only meet k < 16 (four MFMA steps), t1 =
// columns 16..31 (eight).  The contraction index of step s is
// k = 16 (s / 4) + 4 (lane / 16) + s % 4, the same for both tiles, so the first four
// steps' X operands serve both.  op(X)[r][k] = X[k][r] if TRANSX.  One wave.
template <typename T, bool TRANSX>
__device__ __attribute__((always_inline)) inline void mfma_rowtile_lower(
    const T* X, const T* L, int ti, typename Mfma<T>::acc_t& t0, typename Mfma<T>::acc_t& t1) {
  constexpr int LD = Lay<32>::LD;
  const int l = threadIdx.x & 63;
  const int g = l >> 4, i = l & 15;
  const int r = ti * 16 + i;
  t0 = {0, 0, 0, 0};
  t1 = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int k = 16 * (s >> 2) + 4 * g + (s & 3);
    const T a = TRANSX ? X[k * LD + r] : X[r * LD + k];
    if (s < 4) t0 = Mfma<T>::mma(a, L[i * LD + k], t0);
    t1 = Mfma<T>::mma(a, L[(16 + i) * LD + k], t1);
  }
}

// out[tile (ti, tj)] = alpha * acc or += alpha * acc for a 32 x 32 block, the tile given.
template <typename T, bool ACCUMULATE>
__device__ __attribute__((always_inline)) inline void mfma_tile_store_at(
    T* out, const typename Mfma<T>::acc_t& acc, T alpha, int ti, int tj) {
  constexpr int LD = Lay<32>::LD;
  const int l = threadIdx.x & 63;
  const int c = tj * 16 + (l & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T* o = &out[(ti * 16 + Mfma<T>::row(l, v)) * LD + c];
    *o = ACCUMULATE ? *o + alpha * acc[v] : alpha * acc[v];
  }
}

// out[tile] = alpha * acc  or  out[tile] += alpha * acc (NMAX x NMAX blocks)
template <typename T, int NMAX, bool ACCUMULATE>
__device__ __attribute__((always_inline)) inline void mfma_tile_store(
    T* out, const typename Mfma<T>::acc_t& acc, T alpha) {
  constexpr int LD = Lay<NMAX>::LD;
  if constexpr (NMAX == 8 && kValu8) {
    const int l = threadIdx.x & 63;
    T* o = &out[(l >> 3) * LD + (l & 7)];
    *o = ACCUMULATE ? *o + alpha * acc[0] : alpha * acc[0];
    return;
  }
  const int w = wave_id() % (TileCfg<NMAX>::TILES * TileCfg<NMAX>::TILES);
  const int l = threadIdx.x & 63;
  const int ti = w / TileCfg<NMAX>::TILES, tj = w % TileCfg<NMAX>::TILES;
  const int c = tj * 16 + (l & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = ti * 16 + Mfma<T>::row(l, v);
    if (NMAX >= 16 || (r < NMAX && c < NMAX)) {
      T* o = &out[r * LD + c];
      *o = ACCUMULATE ? *o + alpha * acc[v] : alpha * acc[v];
    }
  }
}

// ---- blocked potrf + inverse ------------------------------------------------------

__device__ __attribute__((always_inline)) inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// In place: A (NMAX x NMAX symmetric in LDS, padded with an identity block if smaller)
// := L^{-1}.  For NMAX = 32 the block is split 2 x 2 into 16 x 16 blocks:
//   L11^{-1} by the lane-per-row leaf;  L21 = A21 L11^{-T} (MFMA);
//   S = A22 - L21 L21^T (MFMA);  L22^{-1} by the leaf on S;
//   (L^{-1})21 = -L22^{-1} (L21 L11^{-1}) (two MFMA products).
// The leaves do two 16-row factorizations instead of one 32-row one, which halves
// their per-lane state and cuts the scalar broadcasts; the rest runs on the matrix
// cores.  One wave.  Returns the 0-based row of the first non-positive pivot, or -1.
template <typename T, int NMAX, int LD = Lay<NMAX>::LD>
__device__ __attribute__((always_inline)) inline int wave_potrf_inv(T* A) {
  static_assert(NMAX <= 32, "one wave per block up to 32 x 32");
  if constexpr (NMAX < 32) {
    return wave_potrf_inv_leaf<T, NMAX, RowMajor<LD>>(A);
  } else {
    typedef typename Mfma<T>::acc_t acc_t;
    const int l = threadIdx.x & 63, g = l >> 4, i = l & 15;
    T* A21 = A + 16 * LD;
    T* A22 = A + 16 * LD + 16;
    int fail = wave_potrf_inv_leaf<T, 16, RowMajor<LD>>(A);  // A11 := L11^{-1}
    wave_lds_fence();
    // L21 = A21 L11^{-T}: out[r][c] = sum_k A21[r][k] Linv11[c][k]
    acc_t t = {0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * g + st;
      t = Mfma<T>::mma(A21[i * LD + k], A[i * LD + k], t);
    }
    wave_lds_fence();
#pragma unroll
    for (int v = 0; v < 4; ++v) A21[Mfma<T>::row(l, v) * LD + i] = t[v];
    wave_lds_fence();
    // S = A22 - L21 L21^T
    acc_t sacc;
#pragma unroll
    for (int v = 0; v < 4; ++v) sacc[v] = A22[Mfma<T>::row(l, v) * LD + i];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * g + st;
      sacc = Mfma<T>::mma(-A21[i * LD + k], A21[i * LD + k], sacc);
    }
    wave_lds_fence();
#pragma unroll
    for (int v = 0; v < 4; ++v) A22[Mfma<T>::row(l, v) * LD + i] = sacc[v];
    wave_lds_fence();
    const int fail2 = wave_potrf_inv_leaf<T, 16, RowMajor<LD>>(A22);  // A22 := L22^{-1}
    wave_lds_fence();
    // W = L21 L11^{-1}: out[r][c] = sum_k L21[r][k] Linv11[k][c]
    acc_t w = {0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * g + st;
      w = Mfma<T>::mma(A21[i * LD + k], A[k * LD + i], w);
    }
    wave_lds_fence();
#pragma unroll
    for (int v = 0; v < 4; ++v) A21[Mfma<T>::row(l, v) * LD + i] = w[v];
    wave_lds_fence();
    // (L^{-1})21 = -L22^{-1} W: out[r][c] = sum_k Linv22[r][k] W[k][c]
    acc_t x = {0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * g + st;
      x = Mfma<T>::mma(-A22[i * LD + k], A21[k * LD + i], x);
    }
    wave_lds_fence();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      A21[Mfma<T>::row(l, v) * LD + i] = x[v];
      A[Mfma<T>::row(l, v) * LD + 16 + i] = T(0);  // upper right block
    }
    wave_lds_fence();
    if (fail >= 0) return fail;
    return fail2 >= 0 ? 16 + fail2 : -1;
  }
}

// wave_potrf_inv for a 32 x 32 block held as its packed lower triangle (kPacked32
// entries): the same 2 x 2 blocked steps, reading only entries on or below the diagonal
// (the operands' upper entries are zeros of the triangular factors) and leaving L^{-1}'s
// lower triangle in place.  Half the LDS of a padded slot.  One wave.
template <typename T>
__device__ __attribute__((always_inline)) inline int wave_potrf_inv_packed(T* A) {
  typedef typename Mfma<T>::acc_t acc_t;
  typedef PackedLower<0> P;
  const int l = threadIdx.x & 63, g = l >> 4, i = l & 15;
  int fail = wave_potrf_inv_leaf<T, 16, PackedLower<0>>(A);  // A11 := L11^{-1}
  wave_lds_fence();
  // L21 = A21 L11^{-T}: out[r][c] = sum_k A21[r][k] Linv11[c][k]
  acc_t t = {0, 0, 0, 0};
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int k = 4 * g + st;
    const T li = A[P::at(i, k)];  // in range for k > i too; replaced by zero there
    t = Mfma<T>::mma(A[P::at(16 + i, k)], k <= i ? li : T(0), t);
  }
  wave_lds_fence();
#pragma unroll
  for (int v = 0; v < 4; ++v) A[P::at(16 + Mfma<T>::row(l, v), i)] = t[v];
  wave_lds_fence();
  // S = A22 - L21 L21^T, lower triangle
  acc_t sacc;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = Mfma<T>::row(l, v);
    const T a22 = A[P::at(16 + r, 16 + i)];
    sacc[v] = i <= r ? a22 : T(0);
  }
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int k = 4 * g + st;
    const T l21 = A[P::at(16 + i, k)];
    sacc = Mfma<T>::mma(-l21, l21, sacc);
  }
  wave_lds_fence();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = Mfma<T>::row(l, v);
    if (i <= r) A[P::at(16 + r, 16 + i)] = sacc[v];
  }
  wave_lds_fence();
  const int fail2 = wave_potrf_inv_leaf<T, 16, PackedLower<16>>(A);  // A22 := L22^{-1}
  wave_lds_fence();
  // W = L21 L11^{-1}: out[r][c] = sum_k L21[r][k] Linv11[k][c]
  acc_t w = {0, 0, 0, 0};
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int k = 4 * g + st;
    const T li = A[P::at(k, i)];  // in range for i > k too; replaced by zero there
    w = Mfma<T>::mma(A[P::at(16 + i, k)], i <= k ? li : T(0), w);
  }
  wave_lds_fence();
#pragma unroll
  for (int v = 0; v < 4; ++v) A[P::at(16 + Mfma<T>::row(l, v), i)] = w[v];
  wave_lds_fence();
  // (L^{-1})21 = -L22^{-1} W: out[r][c] = sum_k Linv22[r][k] W[k][c]
  acc_t x = {0, 0, 0, 0};
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int k = 4 * g + st;
    const T l22 = A[P::at(16 + i, 16 + k)];
    x = Mfma<T>::mma(k <= i ? -l22 : T(0), A[P::at(16 + k, i)], x);
  }
  wave_lds_fence();
#pragma unroll
  for (int v = 0; v < 4; ++v) A[P::at(16 + Mfma<T>::row(l, v), i)] = x[v];
  wave_lds_fence();
  if (fail >= 0) return fail;
  return fail2 >= 0 ? 16 + fail2 : -1;
}

// wave_potrf_inv_packed for two blocks (A0 and A1) in one wave: the leaves factor both
// at once, one per 32-lane half, and each MFMA step is taken for A0 and then A1 between
// the same LDS fences.  Returns, on lanes 0-31, the row of A0's first non-positive pivot
// (or -1), on lanes 32-63 that of A1.
template <typename T>
__device__ __attribute__((always_inline)) inline int wave_potrf_inv_packed_pair(T* A0, T* A1) {
  typedef typename Mfma<T>::acc_t acc_t;
  typedef PackedLower<0> P;
  const int l = threadIdx.x & 63, g = l >> 4, i = l & 15;
  T* const Ab[2] = {A0, A1};
  T* const Ah = (l & 32) ? A1 : A0;
  int fail = wave_potrf_inv_leaf<T, 16, PackedLower<0>, true>(Ah);  // A11 := L11^{-1}
  wave_lds_fence();
  // L21 = A21 L11^{-T}: out[r][c] = sum_k A21[r][k] Linv11[c][k]
  acc_t t[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    T* A = Ab[b];
    t[b] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * g + st;
      const T li = A[P::at(i, k)];  // in range for k > i too; replaced by zero there
      t[b] = Mfma<T>::mma(A[P::at(16 + i, k)], k <= i ? li : T(0), t[b]);
    }
  }
  wave_lds_fence();
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) Ab[b][P::at(16 + Mfma<T>::row(l, v), i)] = t[b][v];
  wave_lds_fence();
  // S = A22 - L21 L21^T, lower triangle
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    T* A = Ab[b];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = Mfma<T>::row(l, v);
      const T a22 = A[P::at(16 + r, 16 + i)];
      t[b][v] = i <= r ? a22 : T(0);
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * g + st;
      const T l21 = A[P::at(16 + i, k)];
      t[b] = Mfma<T>::mma(-l21, l21, t[b]);
    }
  }
  wave_lds_fence();
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = Mfma<T>::row(l, v);
      if (i <= r) Ab[b][P::at(16 + r, 16 + i)] = t[b][v];
    }
  wave_lds_fence();
  const int fail2 = wave_potrf_inv_leaf<T, 16, PackedLower<16>, true>(Ah);  // A22 := L22^{-1}
  wave_lds_fence();
  // W = L21 L11^{-1}: out[r][c] = sum_k L21[r][k] Linv11[k][c]
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    T* A = Ab[b];
    t[b] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * g + st;
      const T li = A[P::at(k, i)];  // in range for i > k too; replaced by zero there
      t[b] = Mfma<T>::mma(A[P::at(16 + i, k)], i <= k ? li : T(0), t[b]);
    }
  }
  wave_lds_fence();
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) Ab[b][P::at(16 + Mfma<T>::row(l, v), i)] = t[b][v];
  wave_lds_fence();
  // (L^{-1})21 = -L22^{-1} W: out[r][c] = sum_k Linv22[r][k] W[k][c]
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    T* A = Ab[b];
    t[b] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * g + st;
      const T l22 = A[P::at(16 + i, 16 + k)];
      t[b] = Mfma<T>::mma(k <= i ? -l22 : T(0), A[P::at(16 + k, i)], t[b]);
    }
  }
  wave_lds_fence();
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) Ab[b][P::at(16 + Mfma<T>::row(l, v), i)] = t[b][v];
  wave_lds_fence();
  if (fail >= 0) return fail;
  return fail2 >= 0 ? 16 + fail2 : -1;
}

}  // namespace bmpc
