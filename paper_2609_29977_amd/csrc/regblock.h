// Register-resident n x n blocks for matrix-vector products on one or more waves
// (gfx950).
//
// A block is split over the lanes of WAVES waves: wave w owns the RPW = NMAX/WAVES
// output indices starting at w*RPW; within a wave LPR = 64/RPW lanes share one output
// index o and each holds EPL = NMAX/LPR consecutive elements of the contraction index,
// starting at base = (lane % LPR) * EPL.  In the normal mapping a
// lane holds part of row o (products M v); in the transposed mapping part of column o
// (products M^T v).  Both load coalesced from a row-major block and share the same
// dot-product / reduction code.  Rows and columns >= n read as zero.
#pragma once

#include <hip/hip_runtime.h>

namespace bmpc {

// Raw buffer resource over `bytes` bytes at `base` (wave-uniform).  Loads through it
// take a 32-bit byte offset; an offset at or past `bytes` reads as zero.
__device__ inline __amdgpu_buffer_rsrc_t block_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
constexpr unsigned kOutOfRange = 0x80000000u;

__device__ inline double buf_load_f64(__amdgpu_buffer_rsrc_t r, unsigned off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  double d;
  __builtin_memcpy(&d, &v, sizeof(d));
  return d;
}
__device__ inline float buf_load_f32(__amdgpu_buffer_rsrc_t r, unsigned off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  float f;
  __builtin_memcpy(&f, &v, sizeof(f));
  return f;
}

template <typename T, int NMAX, int WAVES = 1>
struct RegBlock {
  static_assert(NMAX == 8 || NMAX == 16 || NMAX == 32 || NMAX == 64, "block size bound");
  static_assert(WAVES == 1 || WAVES == 2 || WAVES == 4, "waves per block");
  static constexpr int RPW = NMAX / WAVES;
  static constexpr int LPR = 64 / RPW;
  static constexpr int EPL = NMAX / LPR;
  T v[EPL];

  __device__ static int out_index() {
    return (WAVES > 1 ? (int)(threadIdx.x >> 6) * RPW : 0) + (threadIdx.x & 63) / LPR;
  }
  __device__ static int base() { return ((threadIdx.x & 63) % LPR) * EPL; }

  template <bool TRANS>
  __device__ void load(const T* __restrict__ g, int n) {
    const int o = out_index(), b = base();
    if (n == NMAX) {
#pragma unroll
      for (int e = 0; e < EPL; ++e) v[e] = TRANS ? g[(b + e) * NMAX + o] : g[o * NMAX + b + e];
    } else {
      // branch-free: out-of-range elements load element 0 and are replaced by zero
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int r = TRANS ? b + e : o, c = TRANS ? o : b + e;
        const bool ok = r < n && c < n;
        const T t = g[ok ? r * n + c : 0];
        v[e] = ok ? t : T(0);
      }
    }
  }

  // FULL (n == NMAX known at compile time): every element of the lane sits at a fixed
  // offset from one lane base address.  Otherwise the block is read through a buffer
  // resource and out-of-range elements read as zero.
  template <bool TRANS, bool FULL>
  __device__ void load_fixed(const T* __restrict__ g, int n) {
    const int o = out_index(), b = base();
    if constexpr (FULL) {
      const T* p = TRANS ? g + b * NMAX + o : g + o * NMAX + b;
#pragma unroll
      for (int e = 0; e < EPL; ++e) v[e] = TRANS ? p[e * NMAX] : p[e];
    } else {
      load_buf<TRANS>(block_rsrc(g, (unsigned)(n * n) * sizeof(T)), n);
    }
  }

  // Same as load, through a buffer resource covering the n x n block (out-of-range
  // elements read as zero without a branch or a select).
  template <bool TRANS>
  __device__ void load_buf(__amdgpu_buffer_rsrc_t rs, int n) {
    const int o = out_index(), b = base();
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int r = TRANS ? b + e : o, c = TRANS ? o : b + e;
      const unsigned off = (r < n && c < n) ? (unsigned)(r * n + c) * sizeof(T) : kOutOfRange;
      if constexpr (sizeof(T) == 8)
        v[e] = buf_load_f64(rs, off);
      else
        v[e] = buf_load_f32(rs, off);
    }
  }

  // Lower-triangular block stored packed by rows (element (r, c), c <= r, at
  // r (r + 1) / 2 + c); entries above the diagonal and padding read as zero.
  template <bool TRANS>
  __device__ void load_packed(const T* __restrict__ g, int n) {
    const int o = out_index(), b = base();
    const auto rs = block_rsrc(g, (unsigned)(n * (n + 1) / 2) * sizeof(T));
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int r = TRANS ? b + e : o, c = TRANS ? o : b + e;
      const bool ok = c <= r && r < n;
      const unsigned off = ok ? (unsigned)(r * (r + 1) / 2 + c) * sizeof(T) : kOutOfRange;
      if constexpr (sizeof(T) == 8)
        v[e] = buf_load_f64(rs, off);
      else
        v[e] = buf_load_f32(rs, off);
    }
  }

  // load_packed for n == NMAX without control flow, in two steps so that the loads can
  // be in flight while other loads are issued: load_packed_raw reads every element at
  // its packed offset (above the diagonal: an in-range offset of another element), and
  // mask_packed zeroes the entries above the diagonal.  In the transposed mapping the
  // offset of row b+e is (b(b+1)/2 + o) + e*b + e(e+1)/2: one lane-varying add and an
  // immediate per element.
  template <bool TRANS>
  __device__ void load_packed_raw(const T* __restrict__ g) {
    constexpr unsigned SZ = sizeof(T);
    const int o = out_index(), b = base();
    const auto rs = block_rsrc(g, (unsigned)(NMAX * (NMAX + 1) / 2) * SZ);
    const unsigned v0 = TRANS ? (unsigned)(b * (b + 1) / 2 + o) * SZ
                              : (unsigned)(o * (o + 1) / 2 + b) * SZ;
    const unsigned st = TRANS ? (unsigned)b * SZ : SZ;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const unsigned off = v0 + e * st + (TRANS ? (unsigned)(e * (e + 1) / 2) * SZ : 0u);
      if constexpr (sizeof(T) == 8)
        v[e] = buf_load_f64(rs, off);
      else
        v[e] = buf_load_f32(rs, off);
    }
  }
  template <bool TRANS>
  __device__ void mask_packed() {
    const int o = out_index(), b = base();
#pragma unroll
    for (int e = 0; e < EPL; ++e)
      if (!(TRANS ? b + e >= o : b + e <= o)) v[e] = T(0);
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

// The same sum through DPP lane permutations (xor 1 and xor 2 within quads, then the
// mirrored quad and the mirrored half row, which pair each partial sum with one that
// does not overlap it).  Additions are commutative, so all lanes of a group end up with
// bit-identical sums, in the same pairwise order as lane_group_sum.
template <int CTRL>
__device__ inline float dpp_perm(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_perm(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int LPR, typename T>
__device__ inline T lane_group_sum_dpp(T p) {
  static_assert(LPR >= 1 && LPR <= 16, "groups within a DPP row");
  if constexpr (LPR >= 2) p += dpp_perm<0xB1>(p);   // quad_perm [1,0,3,2]: lane ^ 1
  if constexpr (LPR >= 4) p += dpp_perm<0x4E>(p);   // quad_perm [2,3,0,1]: lane ^ 2
  if constexpr (LPR >= 8) p += dpp_perm<0x141>(p);  // row_half_mirror: the other quad
  if constexpr (LPR >= 16) p += dpp_perm<0x140>(p); // row_mirror: the other half row
  return p;
}

// Value of lane ^ OFF for OFF in {8, 16, 32}: DPP row rotation by 8 within a row of 16,
// ds_swizzle with xor 16 within 32 lanes, a shuffle across the halves of the wave.
template <int OFF>
__device__ inline float xor_lane(float v) {
  static_assert(OFF == 8 || OFF == 16 || OFF == 32, "lane distance");
  if constexpr (OFF == 8)
    return dpp_perm<0x128>(v);  // row_ror:8
  else if constexpr (OFF == 16)
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
  else
    return __shfl_xor(v, 32);
}
template <int OFF>
__device__ inline double xor_lane(double v) {
  const long long b = __double_as_longlong(v);
  const float lo = xor_lane<OFF>(__int_as_float((int)(b & 0xffffffffll)));
  const float hi = xor_lane<OFF>(__int_as_float((int)(b >> 32)));
  return __longlong_as_double(((long long)__float_as_int(hi) << 32) |
                              (unsigned)__float_as_int(lo));
}
// Sum over the lanes that agree in lane % QPR (QPR = 8 or 16: a column group whose rows
// are spread over the wave); every lane of a group gets the same sum.
template <int QPR, typename T>
__device__ inline T column_group_sum(T p) {
  static_assert(QPR == 8 || QPR == 16, "lanes per row");
  if constexpr (QPR == 8) p += xor_lane<8>(p);
  p += xor_lane<16>(p);
  p += xor_lane<32>(p);
  return p;
}

}  // namespace bmpc
