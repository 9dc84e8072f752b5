// Factorization kernels (Algorithm 1) for gfx950.
//
// Tail factorization, L_i = chol(Pi_i K_i Pi_i^T).  Any schedule that eliminates the
// chain positions with their Gamma levels (position j at level tz(j)+1, Section II)
// and respects the dependencies yields the same unique factor.  This kernel walks
// the chain in windows of 2^Tw positions: inside a window the positions are read in
// order and each position is eliminated as soon as its right neighbour at its level
// has been read -- a depth-first walk of the reduction tree whose live set is at most
// one block per level.  The live blocks stay in LDS, indexed by their level, so the
// only HBM traffic is reading D and E and writing the factor.  The window's
// boundary positions (multiples of 2^Tw) are not eliminated: the window hands its
// Schur updates to them and the coupling (fill) between them to the next pass, which
// runs the same walk on the reduced chain of boundary positions (levels Tw+1..2Tw),
// and so on.  A boundary node's updates from all earlier passes ride along in the
// left accumulator of the window it starts, so its A is always D + all updates.
// The last pass also eliminates x_1 (position X) and forms the coupling solve
// F = C L_X^{-T} and the local Schur update U = F F^T (Algorithm 1, coupling solve
// and local Schur update).
// FIRST (the pass reading D and E) and FINAL are template flags so that each pass
// kind is its own kernel symbol in profiles.
//
// Elimination of position j with neighbours l (left, optional) and r (right),
// Section IV-B in block form:
//   L_jj = chol(A_j);  G_l = K[l,j] L_jj^{-T};  G_r = K[r,j] L_jj^{-T}
//   A_l -= G_l G_l^T;  A_r -= G_r G_r^T;  K[r,l] = -G_r G_l^T (fill)
#include <type_traits>

#include "bmpc_internal.h"
#include "blockops.h"
#include "multi.h"
#include "regblock.h"

namespace bmpc {

namespace {

template <typename T, int NMAX>
struct Slots {
  static constexpr int SZ = Lay<NMAX>::SZ;
  T* base;
  int Tw;
  int VS;  // one right-hand-side slot: nrhs x NMAX (fused forward substitution)
  __device__ T* A(int t) const { return base + (2 * t) * SZ; }
  __device__ T* Cp(int t) const { return base + (2 * t + 1) * SZ; }
  __device__ T* AL() const { return base + (2 * Tw) * SZ; }
  __device__ T* CL() const { return base + (2 * Tw + 1) * SZ; }
  __device__ T* AR() const { return base + (2 * Tw + 2) * SZ; }
  // right-hand sides of the live nodes (by level), the boundaries, y_j and the pushes
  __device__ T* V(int t) const { return base + (2 * Tw + 3) * SZ + t * VS; }
  __device__ T* VL() const { return V(Tw); }
  __device__ T* VR() const { return V(Tw + 1); }
  __device__ T* Y() const { return V(Tw + 2); }
  __device__ T* Pr() const { return V(Tw + 3); }  // pushes of an elimination
  __device__ T* Pl() const { return V(Tw + 4); }
};

// Per-thread share of an NMAX x NMAX block: element e = threadIdx.x + j*NT.
template <int NMAX>
struct Share {
  static constexpr int NT = TileCfg<NMAX>::NT;
  static constexpr int ELEMS = (NMAX * NMAX + NT - 1) / NT;
  // (the mask tells the compiler that the index is below NT, so the loops' range tests
  // fold away)
  __device__ static int elem(int j) { return (int)(threadIdx.x & (NT - 1)) + j * NT; }
};

// Zero an NMAX x NMAX slot (padding included).
template <typename T, int NMAX>
__device__ inline void slot_zero(T* dst) {
  constexpr int LD = Lay<NMAX>::LD;
#pragma unroll
  for (int j = 0; j < Share<NMAX>::ELEMS; ++j) {
    const int e = Share<NMAX>::elem(j);
    if (e < NMAX * NMAX) dst[(e / NMAX) * LD + e % NMAX] = T(0);
  }
}

// Zero the entries of an NMAX x NMAX slot above its diagonal.
template <typename T, int NMAX>
__device__ inline void slot_zero_upper(T* dst) {
  constexpr int LD = Lay<NMAX>::LD;
#pragma unroll
  for (int j = 0; j < Share<NMAX>::ELEMS; ++j) {
    const int e = Share<NMAX>::elem(j);
    if (e < NMAX * NMAX && e % NMAX > e / NMAX) dst[(e / NMAX) * LD + e % NMAX] = T(0);
  }
}

// dst = src (n x n global, type S, optionally added to dst), zero padding.
template <typename T, int NMAX, typename S>
__device__ inline void slot_load(T* dst, const S* __restrict__ src, int n, bool add) {
  constexpr int LD = Lay<NMAX>::LD;
#pragma unroll
  for (int j = 0; j < Share<NMAX>::ELEMS; ++j) {
    const int e = Share<NMAX>::elem(j);
    if (e < NMAX * NMAX) {
      const int r = e / NMAX, c = e % NMAX;
      const T v = (r < n && c < n) ? static_cast<T>(src[r * n + c]) : T(0);
      dst[r * LD + c] = add ? dst[r * LD + c] + v : v;
    }
  }
}

// Fused forward substitution: the right-hand side of a chain node, b at its stage plus
// (after the first pass) the vector updates carried from earlier passes, in the same
// order as the diagonal block (D + accR + accL).  Lanes past the data read a clamped
// in-range element; commit() zero pads.
// Chain bases of the fused forward substitution, computed once per workgroup: b at
// stage 0 of the chain (right-hand side 0; the stage of position j is N - j), the
// vector length, and the chain's carried vector updates.
template <typename T>
struct VecChain {
  const double* b;
  size_t len;
  const T* vR;
  const T* vL;
};

template <typename T, int NMAX, bool FIRST, bool FWD>
struct VecFetch {
  static constexpr int NT = TileCfg<NMAX>::NT;
  static constexpr int VPER = FWD ? (kMaxRhs * NMAX + NT - 1) / NT : 1;
  double bv[VPER];
  T cr[VPER], cl[VPER];

  __device__ void issue(const FactorPassArgs& a, const VecChain<T>& vc, int q) {
    if constexpr (!FWD) return;
    const int n = a.n, nrhs = a.nrhs;
    const double* bj = vc.b + (size_t)(a.N - (q << a.shift)) * n;
    const int vo = q * nrhs * n;
#pragma unroll
    for (int u = 0; u < VPER; ++u) {
      if (u * NT >= nrhs * NMAX) continue;  // wave-uniform
      const int idx = threadIdx.x + u * NT;
      const int qr = min(idx / NMAX, nrhs - 1), i = min(idx % NMAX, n - 1);
      bv[u] = bj[(size_t)qr * vc.len + i];
      if constexpr (!FIRST) {
        cr[u] = vc.vR[vo + qr * n + i];
        cl[u] = vc.vL[vo + qr * n + i];
      }
    }
  }

  __device__ void commit(const FactorPassArgs& a, T* V) const {
    if constexpr (!FWD) return;
    const int n = a.n, nrhs = a.nrhs;
#pragma unroll
    for (int u = 0; u < VPER; ++u) {
      const int idx = threadIdx.x + u * NT;
      if (u * NT >= nrhs * NMAX || idx >= nrhs * NMAX) continue;
      T v = T(0);
      if (idx % NMAX < n) {
        v = static_cast<T>(bv[u]);
        if constexpr (!FIRST) v = (v + cr[u]) + cl[u];
      }
      V[idx] = v;
    }
  }
};

// Vector part of the window's left boundary: the updates it received in earlier passes
// (nothing in the first pass).  The right boundary starts from zero.
template <typename T, int NMAX, bool FIRST, bool FWD>
struct BoundaryVec {
  static constexpr int NT = TileCfg<NMAX>::NT;
  static constexpr int VPER = FWD ? (kMaxRhs * NMAX + NT - 1) / NT : 1;
  T cr[VPER] = {}, cl[VPER] = {};

  __device__ void issue(const FactorPassArgs& a, int s, int lo) {
    if constexpr (!FIRST && FWD) {
      const int n = a.n, nrhs = a.nrhs;
      const size_t vo = ((size_t)s * a.stride + lo) * nrhs * n;
#pragma unroll
      for (int u = 0; u < VPER; ++u) {
        if (u * NT >= nrhs * NMAX) continue;
        const int idx = threadIdx.x + u * NT;
        const int qr = min(idx / NMAX, nrhs - 1), i = min(idx % NMAX, n - 1);
        cr[u] = reinterpret_cast<const T*>(a.vaccR_in)[vo + qr * n + i];
        cl[u] = reinterpret_cast<const T*>(a.vaccL_in)[vo + qr * n + i];
      }
    }
  }

  __device__ void commit(const FactorPassArgs& a, T* VL, T* VR) const {
    if constexpr (!FWD) return;
    const int n = a.n, nrhs = a.nrhs;
#pragma unroll
    for (int u = 0; u < VPER; ++u) {
      const int idx = threadIdx.x + u * NT;
      if (u * NT >= nrhs * NMAX || idx >= nrhs * NMAX) continue;
      T v = T(0);
      if constexpr (!FIRST)
        if (idx % NMAX < n) v = cr[u] + cl[u];
      VL[idx] = v;
      VR[idx] = T(0);
    }
  }
};

// dst[q][i] (n-compact) = V[q][i] (NMAX-padded) for the nrhs right-hand sides.
template <typename T, int NMAX>
__device__ inline void vec_store(T* __restrict__ dst, const T* V, int n, int nrhs) {
  for (int idx = threadIdx.x; idx < nrhs * n; idx += TileCfg<NMAX>::NT)
    dst[idx] = V[(idx / n) * NMAX + idx % n];
}

// out[q][o] = sum_c M[o][c] v[q][c] for the LDS block M (rows of NMAX, stride LD) and
// the padded vectors v: row o is split over TPR = NT / NMAX threads (DPP sum); the
// thread with p == 0 calls put(q, o, value).
template <typename T, int NMAX, typename Put>
__device__ inline void block_matvec(const T* M, const T* v, int nrhs, Put put) {
  constexpr int NT = TileCfg<NMAX>::NT;
  constexpr int LD = Lay<NMAX>::LD;
  constexpr int TPR = NT / NMAX;
  constexpr int CPT = NMAX / TPR;
  const int o = threadIdx.x / TPR, p = threadIdx.x % TPR;
  for (int q = 0; q < nrhs; ++q) {
    T acc = T(0);
#pragma unroll
    for (int u = 0; u < CPT; ++u) acc += M[o * LD + p * CPT + u] * v[q * NMAX + p * CPT + u];
    acc = lane_group_sum_dpp<TPR>(acc);
    if (p == 0) put(q, o, acc);
  }
}

// Both pushes of an elimination, V_r -= G_r y and (with a left neighbour)
// V_l -= G_l y, in two steps so that each overlaps other work of the elimination:
// push_products forms the reduced sums (G and y read from LDS, same thread split as
// block_matvec) into the LDS vectors Pr, Pl; push_apply subtracts them later, one
// element per thread.
template <typename T, int NMAX>
__device__ inline void push_products(const T* Gr, const T* Gl, const T* y, T* Pr, T* Pl,
                                     int nrhs) {
  constexpr int NT = TileCfg<NMAX>::NT;
  constexpr int LD = Lay<NMAX>::LD;
  constexpr int TPR = NT / NMAX;
  constexpr int CPT = NMAX / TPR;
  const int o = threadIdx.x / TPR, p = threadIdx.x % TPR;
  T gr[CPT], gl[CPT];
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    gr[u] = Gr[o * LD + p * CPT + u];
    gl[u] = Gl ? Gl[o * LD + p * CPT + u] : T(0);
  }
  for (int q = 0; q < nrhs; ++q) {
    T r = T(0), l = T(0);
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const T yv = y[q * NMAX + p * CPT + u];
      r += gr[u] * yv;
      l += gl[u] * yv;
    }
    r = lane_group_sum_dpp<TPR>(r);
    if (Gl) l = lane_group_sum_dpp<TPR>(l);
    if (p == 0) {
      Pr[q * NMAX + o] = r;
      if (Gl) Pl[q * NMAX + o] = l;
    }
  }
}
template <typename T, int NMAX>
__device__ inline void push_apply(T* Vr, T* Vl, const T* Pr, const T* Pl, int nrhs) {
  for (int idx = threadIdx.x; idx < nrhs * NMAX; idx += TileCfg<NMAX>::NT) {
    Vr[idx] -= Pr[idx];
    if (Vl) Vl[idx] -= Pl[idx];
  }
}

// Register prefetch of chain nodes, issued a pair of positions ahead so that the
// global loads overlap the eliminations in between.  Odd pass-local positions were
// factored by the window prologue: their fetch reloads L^{-1} and the coupling to the
// successor.  Even positions fetch D plus the updates carried from earlier passes and
// the coupling.
template <typename T, int NMAX, bool FIRST, bool FWD, bool FULL>
struct FetchOdd {
  static constexpr int EL = Share<NMAX>::ELEMS;
  static constexpr int NT = Share<NMAX>::NT;
  typedef typename std::conditional<FIRST, double, T>::type CT;
  // Full 32 x 32 FP64 blocks: L^{-1} read as V consecutive packed entries per 16-byte
  // load, in R rounds of the workgroup, and placed on and below the diagonal only (the
  // level-0 slot's upper triangle is zeroed once per window and nothing else writes
  // there).  (In FP32 the commit's registers make the first pass spill.)
  static constexpr int V = 16 / (int)sizeof(T);
  static constexpr int NP = NMAX * (NMAX + 1) / 2;
  static constexpr bool PACKED = FULL && NMAX == 32 && sizeof(T) == 8;
  static constexpr int R = (NP / V + NT - 1) / NT;
  static_assert(!PACKED || (NP % V == 0 && R * V <= EL), "chunks fit the registers");
  T li[EL];
  CT cp[EL];
  VecFetch<T, NMAX, FIRST, FWD> vf;

  __device__ void issue(const FactorPassArgs& a, const VecChain<T>& vc, int s, int q) {
    const int n = a.n, N = a.N;
    const size_t nn = (size_t)n * n;
    const int j = q << a.shift;
    vf.issue(a, vc, q);
    const T* Li = reinterpret_cast<const T*>(a.Linv) + ((size_t)s * N + (j - 1)) * nn;
    const CT* cpl;
    if constexpr (FIRST)
      cpl = a.E + ((size_t)s * (N - 1) + (N - 1 - q)) * nn;  // K[q+1,q] = E[s][N-1-q]^T
    else
      cpl = reinterpret_cast<const T*>(a.fill_in) + ((size_t)s * a.stride + q) * nn;
    if constexpr (PACKED) {
      typedef T vt __attribute__((ext_vector_type(V)));
#pragma unroll
      for (int h = 0; h < R; ++h) {
        const int k = (int)(threadIdx.x & (NT - 1)) + h * NT;
        if (k < NP / V) {
          const vt w = *reinterpret_cast<const vt*>(Li + V * k);
#pragma unroll
          for (int u = 0; u < V; ++u) li[h * V + u] = w[u];
        }
      }
#pragma unroll
      for (int jj = 0; jj < EL; ++jj) {
        const int e = Share<NMAX>::elem(jj);
        cp[jj] = cpl[e];
      }
      return;
    }
#pragma unroll
    for (int jj = 0; jj < EL; ++jj) {
      const int e = Share<NMAX>::elem(jj);
      const int r = e / NMAX, c = e % NMAX;
      const bool in = e < NMAX * NMAX && r < n && c < n;
      // the places above the diagonal are buffer loads out of range (zero, no memory
      // access)
      const auto rl = block_rsrc(Li, (unsigned)(n * (n + 1) / 2) * (unsigned)sizeof(T));
      const unsigned o =
          in && c <= r ? (unsigned)(r * (r + 1) / 2 + c) * (unsigned)sizeof(T) : kOutOfRange;
      if constexpr (sizeof(T) == 8)
        li[jj] = buf_load_f64(rl, o);
      else
        li[jj] = buf_load_f32(rl, o);
      cp[jj] = in ? cpl[r * n + c] : CT(0);
    }
  }

  __device__ void commit(T* A, T* C, int n) const {
    constexpr int LD = Lay<NMAX>::LD;
    if constexpr (PACKED) {
#pragma unroll
      for (int h = 0; h < R; ++h) {
        const int k = (int)(threadIdx.x & (NT - 1)) + h * NT;
        if (k < NP / V) {
          // row of packed entry p: the r with r (r + 1) / 2 <= p < (r + 1) (r + 2) / 2
          const int p = V * k;
          int r = (int)((__fsqrt_rn(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
          r = (r * (r + 1) / 2 > p) ? r - 1 : r;
          r = ((r + 1) * (r + 2) / 2 <= p) ? r + 1 : r;
          int c = p - r * (r + 1) / 2;
#pragma unroll
          for (int u = 0; u < V; ++u) {
            A[r * LD + c] = li[h * V + u];
            const bool wrap = c == r;  // the next packed entry starts row r + 1
            r = wrap ? r + 1 : r;
            c = wrap ? 0 : c + 1;
          }
        }
      }
#pragma unroll
      for (int jj = 0; jj < EL; ++jj) {
        const int e = Share<NMAX>::elem(jj);
        const int r = e / NMAX, c = e % NMAX;
        const T cv = static_cast<T>(cp[jj]);
        if constexpr (FIRST)
          C[c * LD + r] = cv;
        else
          C[r * LD + c] = cv;
      }
      return;
    }
#pragma unroll
    for (int jj = 0; jj < EL; ++jj) {
      const int e = Share<NMAX>::elem(jj);
      if (e >= NMAX * NMAX) continue;
      const int r = e / NMAX, c = e % NMAX;
      const bool in = r < n && c < n;
      A[r * LD + c] = in ? li[jj] : ((r == c) ? T(1) : T(0));
      const T cv = static_cast<T>(cp[jj]);
      if constexpr (FIRST)
        C[c * LD + r] = cv;
      else
        C[r * LD + c] = cv;
    }
  }
};

template <typename T, int NMAX, bool FIRST, bool FWD>
struct FetchEven {
  static constexpr int EL = Share<NMAX>::ELEMS;
  typedef typename std::conditional<FIRST, double, T>::type CT;
  double d[EL];
  T ar[EL], al[EL];
  CT cp[EL];
  VecFetch<T, NMAX, FIRST, FWD> vf;

  __device__ void issue(const FactorPassArgs& a, const VecChain<T>& vc, int s, int q) {
    const int n = a.n, N = a.N;
    const size_t nn = (size_t)n * n;
    const int j = q << a.shift;
    vf.issue(a, vc, q);
    const double* D = a.D + ((size_t)s * N + (N - j)) * nn;
    const T* accR = nullptr;
    const T* accL = nullptr;
    const CT* cpl;
    if constexpr (FIRST) {
      cpl = a.E + ((size_t)s * (N - 1) + (N - 1 - q)) * nn;
    } else {
      const size_t o = ((size_t)s * a.stride + q) * nn;
      accR = reinterpret_cast<const T*>(a.accR_in) + o;
      accL = reinterpret_cast<const T*>(a.accL_in) + o;
      cpl = reinterpret_cast<const T*>(a.fill_in) + o;
    }
    // The upper half of the slot is never used before the block is factored, so it is
    // not read from the blocks: the entries above the diagonal of D and of the carried
    // updates are buffer loads out of range (zero, no memory access).  No lane mask.
#pragma unroll
    for (int jj = 0; jj < EL; ++jj) {
      const int e = Share<NMAX>::elem(jj);
      const int r = e / NMAX, c = e % NMAX;
      const bool in = e < NMAX * NMAX && r < n && c < n;
      const bool low = in && c <= r;
      const auto rd = block_rsrc(D, (unsigned)nn * 8u);
      d[jj] = buf_load_f64(rd, low ? (unsigned)(r * n + c) * 8u : kOutOfRange);
      if constexpr (!FIRST) {
        const auto rr = block_rsrc(accR, (unsigned)nn * (unsigned)sizeof(T));
        const auto rl = block_rsrc(accL, (unsigned)nn * (unsigned)sizeof(T));
        const unsigned o = low ? (unsigned)(r * n + c) * (unsigned)sizeof(T) : kOutOfRange;
        if constexpr (sizeof(T) == 8) {
          ar[jj] = buf_load_f64(rr, o);
          al[jj] = buf_load_f64(rl, o);
        } else {
          ar[jj] = buf_load_f32(rr, o);
          al[jj] = buf_load_f32(rl, o);
        }
      }
      cp[jj] = in ? cpl[r * n + c] : CT(0);
    }
  }

  __device__ void commit(T* A, T* C, int n) const {
    constexpr int LD = Lay<NMAX>::LD;
#pragma unroll
    for (int jj = 0; jj < EL; ++jj) {
      const int e = Share<NMAX>::elem(jj);
      if (e >= NMAX * NMAX) continue;
      const int r = e / NMAX, c = e % NMAX;
      const bool in = r < n && c < n;
      T v = (r == c) ? T(1) : T(0);  // identity padding of diagonal blocks
      if (in) {
        v = static_cast<T>(d[jj]);
        if constexpr (!FIRST) v = (v + ar[jj]) + al[jj];
      }
      A[r * LD + c] = v;
      const T cv = static_cast<T>(cp[jj]);
      if constexpr (FIRST)
        C[c * LD + r] = cv;
      else
        C[r * LD + c] = cv;
    }
  }
};

// The window's left boundary node: its accumulated updates from earlier passes (AL)
// and its coupling to its successor (CL: E^T in the first pass, the carried fill after).
// Fetched into registers before the prologue, placed in LDS after it.
template <typename T, int NMAX, bool FIRST>
struct BoundaryFetch {
  static constexpr int EL = Share<NMAX>::ELEMS;
  typedef typename std::conditional<FIRST, double, T>::type CT;
  CT cl[EL];
  T al[EL];

  __device__ void issue(const FactorPassArgs& a, int s, int lo) {
    const int n = a.n, N = a.N;
    const size_t nn = (size_t)n * n;
    const CT* src;
    const T* accR = nullptr;
    const T* accL = nullptr;
    if constexpr (FIRST) {
      src = a.E + ((size_t)s * (N - 1) + (N - 1 - lo)) * nn;
    } else {
      const size_t o = ((size_t)s * a.stride + lo) * nn;
      src = reinterpret_cast<const T*>(a.fill_in) + o;
      accR = reinterpret_cast<const T*>(a.accR_in) + o;
      accL = reinterpret_cast<const T*>(a.accL_in) + o;
    }
#pragma unroll
    for (int j = 0; j < EL; ++j) {
      const int e = Share<NMAX>::elem(j);
      const int r = e / NMAX, c = e % NMAX;
      const bool in = e < NMAX * NMAX && r < n && c < n;
      cl[j] = in ? src[r * n + c] : CT(0);
      if constexpr (!FIRST) al[j] = in ? accR[r * n + c] + accL[r * n + c] : T(0);
    }
  }

  __device__ void commit(T* AL, T* CL) const {
    constexpr int LD = Lay<NMAX>::LD;
#pragma unroll
    for (int j = 0; j < EL; ++j) {
      const int e = Share<NMAX>::elem(j);
      if (e >= NMAX * NMAX) continue;
      const int r = e / NMAX, c = e % NMAX;
      if constexpr (FIRST) {
        CL[c * LD + r] = static_cast<T>(cl[j]);  // K[lo+1, lo] = E^T
        AL[r * LD + c] = T(0);
      } else {
        CL[r * LD + c] = cl[j];
        AL[r * LD + c] = al[j];
      }
    }
  }
};

template <typename T, int NMAX>
__device__ inline void slot_store(T* __restrict__ dst, const T* src, int n) {
  constexpr int LD = Lay<NMAX>::LD;
  constexpr int NT = TileCfg<NMAX>::NT;
  constexpr int V = 16 / (int)sizeof(T);  // entries per 16-byte store
  if constexpr (NMAX * NMAX % (V * NT) == 0 && NMAX % V == 0) {
    if (n == NMAX) {  // full block: V consecutive row entries per store
      typedef T vt __attribute__((ext_vector_type(V)));
#pragma unroll
      for (int k = 0; k < NMAX * NMAX / (V * NT); ++k) {
        const int e = V * ((int)(threadIdx.x & (NT - 1)) + k * NT);
        const int r = e / NMAX, c = e % NMAX;
        vt w;
#pragma unroll
        for (int u = 0; u < V; ++u) w[u] = src[r * LD + c + u];
        *reinterpret_cast<vt*>(dst + e) = w;
      }
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < Share<NMAX>::ELEMS; ++j) {
    const int e = Share<NMAX>::elem(j);
    if (e < NMAX * NMAX) {
      const int r = e / NMAX, c = e % NMAX;
      if (r < n && c < n) dst[r * n + c] = src[r * LD + c];
    }
  }
}

// Lower triangle of an LDS block to global memory, packed by rows: element (r, c),
// c <= r, at r (r + 1) / 2 + c (the storage of the inverted diagonal blocks).  The
// threads walk the packed indices, so only the last round has idle lanes: the row of
// index p is the r with r (r + 1) / 2 <= p < (r + 1) (r + 2) / 2, estimated from the
// square root and corrected by one where rounding put it off.
template <typename T, int NMAX>
__device__ inline void slot_store_packed(T* __restrict__ dst, const T* src, int n) {
  constexpr int LD = Lay<NMAX>::LD;
  constexpr int NT = TileCfg<NMAX>::NT;
  const int np = n * (n + 1) / 2;
#pragma unroll
  for (int p0 = 0; p0 < NMAX * (NMAX + 1) / 2; p0 += NT) {
    const int p = p0 + (int)threadIdx.x;
    int r = (int)((__fsqrt_rn(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
    r = (r * (r + 1) / 2 > p) ? r - 1 : r;
    r = ((r + 1) * (r + 2) / 2 <= p) ? r + 1 : r;
    const int c = p - r * (r + 1) / 2;
    if (p < np) dst[p] = src[r * LD + c];
  }
}

// L_jj^{-1} of the block in Aj (in place) by one wave; which wave does it rotates
// with the workgroup index so that the latency-bound factorizations of the resident
// workgroups spread over the SIMDs.
template <typename T, int NMAX>
__device__ __attribute__((always_inline)) inline void factor_diag(T* A, unsigned long long perm_row0, int n,
                                   unsigned long long* info) {
  constexpr int NW = TileCfg<NMAX>::NT / 64;
  if (wave_id() == (int)(blockIdx.x % NW)) {
    const int fail = wave_potrf_inv<T, NMAX>(A);
    if (fail >= 0 && fail < n && (threadIdx.x & 63) == 0) atomicMin(info, perm_row0 + fail + 1);
  }
  __syncthreads();
}

// One elimination (Section IV-B in block form): Aj := L_jj^{-1};
// G_r = K[r,j] L^{-T} (into Cj), G_l = K[l,j] L^{-T} (into Cl, which holds K[j,l]);
// A_r -= G_r G_r^T; A_l -= G_l G_l^T; K[r,l] = -G_r G_l^T (into Cl).
// With a fused forward substitution (gy not null) the node's right-hand side Vj,
// complete once every lower neighbour is eliminated, gives y_j = L_jj^{-1} Vj (into
// Yt and gy), and the neighbours' right-hand sides take V_r -= G_r y_j and
// V_l -= G_l y_j (Algorithm 2's forward step in the elimination order).
template <typename T, int NMAX, bool FWD>
__device__ __attribute__((always_inline)) inline void eliminate(T* Aj, T* Cj, T* Al, T* Cl, T* Ar, int n, T* gLinv,
                                 T* gGl, T* gGr, unsigned long long perm_row0,
                                 unsigned long long* info, bool have_inverse, T* Vj,
                                 T* Vl, T* Vr, T* Yt, T* Pr, T* Pl, T* gy, int nrhs) {
  typedef typename Mfma<T>::acc_t acc_t;
  if (!have_inverse) factor_diag<T, NMAX>(Aj, perm_row0, n, info);
  const bool left = Cl != nullptr;
  if constexpr (NMAX == 32) {
    // G products: wave w forms row tile w % 2 of G_r (w < 2) or of G_l (w >= 2), both
    // column tiles, skipping the zero upper quadrant of L^{-1}: 12 MFMA steps per wave
    // instead of 16.  Without a left neighbour waves 2 and 3 have nothing to do here.
    const int w = wave_id();
    const int ti = w & 1;
    acc_t g0, g1;
    if (w < 2)
      mfma_rowtile_lower<T, false>(Cj, Aj, ti, g0, g1);
    else if (left)
      mfma_rowtile_lower<T, true>(Cl, Aj, ti, g0, g1);
    __syncthreads();
    if (w < 2 || left) {
      T* G = w < 2 ? Cj : Cl;
      mfma_tile_store_at<T, false>(G, g0, T(1), ti, 0);
      mfma_tile_store_at<T, false>(G, g1, T(1), ti, 1);
    }
  } else {
    acc_t gr = mfma_tile_nt<T, NMAX, false>(Cj, Aj);
    acc_t gl = {0, 0, 0, 0};
    if (left) gl = mfma_tile_nt<T, NMAX, true>(Cl, Aj);
    __syncthreads();
    mfma_tile_store<T, NMAX, false>(Cj, gr, T(1));
    if (left) mfma_tile_store<T, NMAX, false>(Cl, gl, T(1));
  }
  if constexpr (FWD)  // y_j = L_jj^{-1} V_j (Aj and Vj are not written in this phase)
    block_matvec<T, NMAX>(Aj, Vj, nrhs, [&](int q, int o, T v) {
      Yt[q * NMAX + o] = v;
      if (o < n) gy[q * n + o] = v;
    });
  __syncthreads();
  if (!have_inverse) slot_store_packed<T, NMAX>(gLinv, Aj, n);
  slot_store<T, NMAX>(gGr, Cj, n);
  if (left) slot_store<T, NMAX>(gGl, Cl, n);
  // The diagonal blocks' updates are symmetric and only their lower triangles are ever
  // read (the factorization, and the lower-triangle loads of the next pass), so the
  // wave of the upper-right tile skips them.
  const bool upper = TileCfg<NMAX>::TILES == 2 && wave_id() == 1;
  acc_t ur = {0, 0, 0, 0}, ul = {0, 0, 0, 0}, uf = {0, 0, 0, 0};
  if (!upper) ur = mfma_tile_nt<T, NMAX, false>(Cj, Cj);
  if (left) {
    if (!upper) ul = mfma_tile_nt<T, NMAX, false>(Cl, Cl);
    uf = mfma_tile_nt<T, NMAX, false>(Cj, Cl);
  }
  if constexpr (FWD)  // G_l is still in Cl
    push_products<T, NMAX>(Cj, left ? Cl : nullptr, Yt, Pr, Pl, nrhs);
  __syncthreads();
  if (!upper) mfma_tile_store<T, NMAX, true>(Ar, ur, T(-1));
  if (left) {
    if (!upper) mfma_tile_store<T, NMAX, true>(Al, ul, T(-1));
    mfma_tile_store<T, NMAX, false>(Cl, uf, T(-1));
  }
  if constexpr (FWD) push_apply<T, NMAX>(Vr, left ? Vl : nullptr, Pr, Pl, nrhs);
  __syncthreads();
}

// Waves per SIMD the register allocation must allow.  The last pass has one workgroup
// per chain; two per CU keep all of them resident.  The FP32 first pass of 32 x 32
// blocks fits in 128 registers without spilling, which with three levels per pass
// (39 KB of LDS) lets four workgroups share a CU instead of three: measured against
// four levels at three workgroups, the first pass is 16% and the whole factorization 5%
// faster.
template <typename T, int NMAX, bool FIRST, bool FINAL, bool FULL>
constexpr int pass_min_blocks() {
  return FINAL ? 2 : ((FIRST && FULL && NMAX == 32 && sizeof(T) == 4) ? 4 : 1);
}

// FULL: the block size is NMAX (n == NMAX), a compile-time constant here, so that the
// per-element tests against n in the loads, stores and padding fold away.
template <typename T, int NMAX, bool FIRST, bool FINAL, bool FWD, bool FULL>
__device__ __attribute__((always_inline)) inline void factor_pass_body(
    const FactorPassArgs& a_in, unsigned bx) {
  FactorPassArgs a = a_in;
  if constexpr (FULL) a.n = NMAX;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Slots<T, NMAX> sl{reinterpret_cast<T*>(smem_raw), a.Tw, FWD ? a.nrhs * NMAX : 0};
  const int n = a.n, N = a.N;
  const size_t nn = (size_t)n * n;
  const int s = bx / a.windows;
  const int w = bx - s * a.windows;
  const int lo = w << a.Tw;
  const int hi = min(lo + (1 << a.Tw) - 1, a.mk);
  const bool has_left = lo >= 1;
  const int rb = lo + (1 << a.Tw);
  const bool rb_is_x = rb > a.mk;

  T* Linv = reinterpret_cast<T*>(a.Linv) + (size_t)s * N * nn;
  T* Gl = reinterpret_cast<T*>(a.Gl) + (size_t)s * g_chain_blocks(N) * nn;
  T* Gr = reinterpret_cast<T*>(a.Gr) + (size_t)s * g_chain_blocks(N) * nn;
  // natural row of the chain's first entry: systems in order, tails before the root
  const int sys = s / a.Ssys;
  const unsigned long long chain_row0 =
      (unsigned long long)sys * ((unsigned long long)a.Ssys * N + 1) * n +
      (unsigned long long)(s - sys * a.Ssys) * N * n;

  BoundaryFetch<T, NMAX, FIRST> bf;
  if (has_left) bf.issue(a, s, lo);
  BoundaryVec<T, NMAX, FIRST, FWD> bvf;
  if (has_left) bvf.issue(a, s, lo);
  T* ych = FWD ? reinterpret_cast<T*>(a.y) + (size_t)s * N * a.nrhs * n : nullptr;
  VecChain<T> vc{};
  if constexpr (FWD) {
    vc.len = ((size_t)a.Ssys * N + 1) * n;
    vc.b = a.b + (size_t)sys * a.vsys + (size_t)(s - sys * a.Ssys) * N * n;
    if constexpr (!FIRST) {
      const size_t vo = (size_t)s * a.stride * a.nrhs * n;
      vc.vR = reinterpret_cast<const T*>(a.vaccR_in) + vo;
      vc.vL = reinterpret_cast<const T*>(a.vaccL_in) + vo;
    }
  }

  // The first even position's fetch does not depend on the prologue: in FP32 it is
  // issued before it, so that the prologue hides its latency (the odd position's fetch
  // reloads inverses the prologue writes).  In FP64 the registers it holds across the
  // prologue cost more than the wait they save.
  constexpr bool kEarlyEvenFetch = sizeof(T) == 4;
  FetchEven<T, NMAX, FIRST, FWD> fe;
  if constexpr (kEarlyEvenFetch)
    if (lo + 2 <= hi) fe.issue(a, vc, s, lo + 2);
  // Prologue (passes after the first): the pass-local level-1 positions (odd q) see no
  // update from inside the window, so their diagonal blocks (D plus updates carried from
  // earlier passes) are factored and inverted up front.  In the first pass these blocks
  // are D alone, and level1_inverse_kernel has inverted them before the pass.  Up to kBatch blocks at a time are loaded by the
  // whole workgroup into the window's still unused LDS slots (all loads in flight at
  // once), then each wave inverts its share of them, and the inverses go to the
  // factor storage; the streaming phase below reloads them.
  {
    constexpr int NW = TileCfg<NMAX>::NT / 64;
    constexpr int LD = Lay<NMAX>::LD;
    constexpr int SZ = Lay<NMAX>::SZ;
    constexpr int EL = Share<NMAX>::ELEMS;
    constexpr int kBatch = 4;
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    // the first pass's level-1 inverses come from level1_inverse_kernel
    const int nodd = FIRST ? 0 : (hi - lo + 1) / 2;
    const int cap = min(kBatch, 2 * a.Tw + 3);
    for (int i0 = 0; i0 < nodd; i0 += cap) {
      const int cnt = min(cap, nodd - i0);
      double dv[kBatch][EL];
      T av[kBatch][EL];
      // one 32-bit offset per element serves every block (buffer loads, the block
      // bases stay scalar); out-of-range elements read as zero
      unsigned off[EL];
#pragma unroll
      for (int jj = 0; jj < EL; ++jj) {
        const int e = Share<NMAX>::elem(jj);
        const int r = e / NMAX, c = e % NMAX;
        const bool in = e < NMAX * NMAX && r < n && c <= r;  // lower triangle only
        off[jj] = in ? (unsigned)(r * n + c) : kOutOfRange / 8;
      }
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        if (b < cnt) {
          const int q = lo + 1 + 2 * (i0 + b);
          const int j = q << a.shift;
          const auto rd = block_rsrc(a.D + ((size_t)s * N + (N - j)) * nn,
                                     (unsigned)nn * sizeof(double));
          [[maybe_unused]] __amdgpu_buffer_rsrc_t rr, rl;
          if constexpr (!FIRST) {
            const size_t ob = ((size_t)s * a.stride + q) * nn;
            rr = block_rsrc(reinterpret_cast<const T*>(a.accR_in) + ob, (unsigned)nn * sizeof(T));
            rl = block_rsrc(reinterpret_cast<const T*>(a.accL_in) + ob, (unsigned)nn * sizeof(T));
          }
#pragma unroll
          for (int jj = 0; jj < EL; ++jj) {
            dv[b][jj] = buf_load_f64(rd, off[jj] * 8u);
            if constexpr (!FIRST) {
              if constexpr (sizeof(T) == 8)
                av[b][jj] = buf_load_f64(rr, off[jj] * 8u) + buf_load_f64(rl, off[jj] * 8u);
              else
                av[b][jj] = buf_load_f32(rr, off[jj] * 4u) + buf_load_f32(rl, off[jj] * 4u);
            }
          }
        }
      }
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        if (b < cnt) {
          T* dst = sl.base + b * SZ;
#pragma unroll
          for (int jj = 0; jj < EL; ++jj) {
            const int e = Share<NMAX>::elem(jj);
            if (e >= NMAX * NMAX) continue;
            const int r = e / NMAX, c = e % NMAX;
            T v;
            if (r < n && c < n) {
              v = static_cast<T>(dv[b][jj]);
              if constexpr (!FIRST) v = v + av[b][jj];
            } else {
              v = (r == c) ? T(1) : T(0);
            }
            dst[r * LD + c] = v;
          }
        }
      }
      __syncthreads();
      for (int b = wv; b < cnt; b += NW) {
        const int j = (lo + 1 + 2 * (i0 + b)) << a.shift;
        const int fail = wave_potrf_inv<T, NMAX>(sl.base + b * SZ);
        if (fail >= 0 && fail < n && lane == 0)
          atomicMin(a.info, chain_row0 + (unsigned long long)a.permpos[j - 1] * n + fail + 1);
      }
      __syncthreads();
      for (int b = 0; b < cnt; ++b) {
        const int j = (lo + 1 + 2 * (i0 + b)) << a.shift;
        slot_store_packed<T, NMAX>(Linv + (size_t)(j - 1) * nn, sl.base + b * SZ, n);
      }
      __syncthreads();
    }
    __threadfence_block();
  }
  FetchOdd<T, NMAX, FIRST, FWD, FULL> fo;
  if (lo + 1 <= hi) fo.issue(a, vc, s, lo + 1);
  if constexpr (!kEarlyEvenFetch)
    if (lo + 2 <= hi) fe.issue(a, vc, s, lo + 2);

  // The left boundary node keeps the updates it received while it was a window
  // boundary in earlier passes; they travel with it in its left accumulator.
  if (has_left) bf.commit(sl.AL(), sl.CL());
  slot_zero<T, NMAX>(sl.AR());
  if constexpr (decltype(fo)::PACKED) slot_zero_upper<T, NMAX>(sl.A(0));
  bvf.commit(a, sl.VL(), sl.VR());
  __syncthreads();

  unsigned live = 0u;
  // Position q is read at step q; step hi+1 reads the right boundary.  After a read,
  // every live level below the new node's level is eliminated, lowest first, with the
  // new node as right neighbour (Gamma order: level tz(j)+1).
  for (int q = lo + 1; q <= hi + 1; ++q) {
    const bool is_rb = q > hi;
    int v = 0;
    unsigned todo;
    if (!is_rb) {
      v = __builtin_ctz((unsigned)q);
      if (q & 1) {
        // An odd step eliminates nothing, so it also places the even position q+1
        // (its slot is free: the previous node of that level is already eliminated)
        // and then fetches the next pair, which the eliminations of step q+1 hide.
        fo.commit(sl.A(0), sl.Cp(0), n);
        fo.vf.commit(a, sl.V(0));
        if (q + 1 <= hi) {
          const int v1 = __builtin_ctz((unsigned)(q + 1));
          fe.commit(sl.A(v1), sl.Cp(v1), n);
          fe.vf.commit(a, sl.V(v1));
        }
        __syncthreads();
        if (q + 2 <= hi) fo.issue(a, vc, s, q + 2);
        if (q + 3 <= hi) fe.issue(a, vc, s, q + 3);
      }
      todo = live & ((1u << v) - 1u);
    } else {
      todo = live;
    }
    T* Ar = is_rb ? sl.AR() : sl.A(v);
    T* Vr = is_rb ? sl.VR() : sl.V(v);
    while (todo) {
      const int t = __builtin_ctz(todo);
      todo &= todo - 1u;
      const unsigned above = live & ~((2u << t) - 1u);
      T* Al = nullptr;
      T* Cl = nullptr;
      T* Vl = nullptr;
      if (above) {
        const int u = __builtin_ctz(above);
        Al = sl.A(u);
        Cl = sl.Cp(u);
        Vl = sl.V(u);
      } else if (has_left) {
        Al = sl.AL();
        Cl = sl.CL();
        Vl = sl.VL();
      }
      // position of the live node of level t
      const int pos = !is_rb ? q - (1 << t) : (rb_is_x ? ((hi >> t) << t) : rb - (1 << t));
      const int j = pos << a.shift;  // original chain position
      const unsigned long long prow = chain_row0 + (unsigned long long)a.permpos[j - 1] * n;
      eliminate<T, NMAX, FWD>(sl.A(t), sl.Cp(t), Al, Cl, Ar, n, Linv + (size_t)(j - 1) * nn,
                         Gl + (size_t)(j - 1) * nn, Gr + (size_t)(j - 1) * nn, prow, a.info,
                         (pos & 1) != 0, sl.V(t), Vl, Vr, sl.Y(), sl.Pr(), sl.Pl(),
                         ych ? ych + (size_t)(j - 1) * a.nrhs * n : nullptr, a.nrhs);
      live &= ~(1u << t);
    }
    if (!is_rb) live |= (1u << v);
  }

  if constexpr (!FINAL) {
    const size_t base = (size_t)s * a.stride;
    if (has_left) {
      slot_store<T, NMAX>(reinterpret_cast<T*>(a.accL_out) + (base + w) * nn, sl.AL(), n);
      slot_store<T, NMAX>(reinterpret_cast<T*>(a.fill_out) + (base + w) * nn, sl.CL(), n);
    }
    if (!rb_is_x) {
      slot_store<T, NMAX>(reinterpret_cast<T*>(a.accR_out) + (base + w + 1) * nn, sl.AR(), n);
    } else {
      slot_store<T, NMAX>(reinterpret_cast<T*>(a.accX) + ((size_t)s * a.npass + a.pass) * nn,
                          sl.AR(), n);
    }
    if constexpr (FWD) {
      const int nr = a.nrhs;
      const size_t vs = (size_t)nr * n;
      if (has_left)
        vec_store<T, NMAX>(reinterpret_cast<T*>(a.vaccL_out) + (base + w) * vs, sl.VL(), n, nr);
      if (!rb_is_x)
        vec_store<T, NMAX>(reinterpret_cast<T*>(a.vaccR_out) + (base + w + 1) * vs, sl.VR(), n,
                           nr);
      else
        vec_store<T, NMAX>(
            reinterpret_cast<T*>(a.vaccX) + ((size_t)s * a.npass + a.pass) * vs, sl.VR(), n, nr);
    }
    return;
  } else {
    // ---- last pass: x_1 step (Algorithm 1, the tail steps for the terminal block) ----
    constexpr int LD = Lay<NMAX>::LD;
    T* Ax = sl.A(0);
    T* Cx = sl.Cp(0);
    const double* D0 = a.D + ((size_t)s * N + 0) * nn;
#pragma unroll
    for (int j = 0; j < Share<NMAX>::ELEMS; ++j) {
      const int e = Share<NMAX>::elem(j);
      if (e < NMAX * NMAX) {
        const int r = e / NMAX, c = e % NMAX;
        T v;
        if (r < n && c < n) {
          v = static_cast<T>(r >= c ? D0[r * n + c] : D0[c * n + r]);
          for (int p = 0; p < a.pass; ++p)
            v += reinterpret_cast<const T*>(a.accX)[((size_t)s * a.npass + p) * nn + r * n + c];
          v += sl.AR()[r * LD + c];
        } else {
          v = (r == c) ? T(1) : T(0);
        }
        Ax[r * LD + c] = v;
      }
    }
    slot_load<T, NMAX>(Cx, a.C + (size_t)s * nn, n, false);
    __syncthreads();
    factor_diag<T, NMAX>(Ax, chain_row0 + (unsigned long long)a.permpos[N - 1] * n, n, a.info);
    slot_store_packed<T, NMAX>(Linv + (size_t)(N - 1) * nn, Ax, n);
    // F = C L_X^{-T}
    typename Mfma<T>::acc_t f = mfma_tile_nt<T, NMAX, false>(Cx, Ax);
    __syncthreads();
    mfma_tile_store<T, NMAX, false>(Cx, f, T(1));
    __syncthreads();
    slot_store<T, NMAX>(reinterpret_cast<T*>(a.F) + (size_t)s * nn, Cx, n);
    // U = F F^T in FP64 from the stored F
    double* U = a.U + (size_t)s * nn;
    for (int e = threadIdx.x; e < n * n; e += TileCfg<NMAX>::NT) {
      const int r = e / n, c = e - (e / n) * n;
      double acc = 0.0;
      for (int k = 0; k < n; ++k)
        acc += static_cast<double>(Cx[r * LD + k]) * static_cast<double>(Cx[c * LD + k]);
      U[e] = acc;
    }
    if constexpr (FWD) {
      // Fused forward substitution, X step (the terminal forward step of Algorithm 2):
      // the right-hand side of X is b at stage 0 plus the X updates of every pass (same
      // order as its diagonal block); y_X = L_X^{-1} of it, and w_s = F_s y_X in FP64.
      constexpr int NT = TileCfg<NMAX>::NT;
      constexpr int TPR = NT / NMAX;
      constexpr int CPT = NMAX / TPR;
      const int nr = a.nrhs;
      const int sys_ = s / a.Ssys, sc = s - sys_ * a.Ssys;
      const size_t len = ((size_t)a.Ssys * N + 1) * n;
      const size_t offx = (size_t)sys_ * a.vsys + (size_t)sc * N * n;
      const size_t vs = (size_t)nr * n;
      T* Vx = sl.Y();
      for (int idx = threadIdx.x; idx < nr * NMAX; idx += NT) {
        const int q = idx / NMAX, i = idx % NMAX;
        T v = T(0);
        if (i < n) {
          v = static_cast<T>(a.b[offx + (size_t)q * len + i]);
          for (int p = 0; p < a.pass; ++p)
            v += reinterpret_cast<const T*>(a.vaccX)[((size_t)s * a.npass + p) * vs + q * n + i];
          v += sl.VR()[idx];
        }
        Vx[idx] = v;
      }
      __syncthreads();
      T* yx = reinterpret_cast<T*>(a.y) + ((size_t)s * N + (N - 1)) * vs;
      T* Yx = sl.VR();  // the X updates are folded into Vx; VR now holds y_X
      block_matvec<T, NMAX>(Ax, Vx, nr, [&](int q, int o, T v) {
        Yx[q * NMAX + o] = v;
        if (o < n) yx[q * n + o] = v;
      });
      __syncthreads();
      const int o = threadIdx.x / TPR, p = threadIdx.x % TPR;
      for (int q = 0; q < nr; ++q) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < CPT; ++u)
          acc += static_cast<double>(Cx[o * LD + p * CPT + u]) *
                 static_cast<double>(Yx[q * NMAX + p * CPT + u]);
        acc = lane_group_sum_dpp<TPR>(acc);
        if (p == 0 && o < n) a.w[((size_t)s * nr + q) * n + o] = acc;
      }
    }
  }
}

template <typename T, int NMAX, bool FIRST, bool FINAL, bool FWD, bool FULL>
__global__ void __launch_bounds__(TileCfg<NMAX>::NT,
                                  (pass_min_blocks<T, NMAX, FIRST, FINAL, FULL>()))
    factor_pass_kernel(FactorPassArgs a) {
  factor_pass_body<T, NMAX, FIRST, FINAL, FWD, FULL>(a, blockIdx.x);
}

// LDS entries per block of the level-1 inverse kernels.
template <int NMAX>
constexpr int level1_slot_entries() {
  return NMAX == 32 ? kPacked32 : Lay<NMAX>::SZ;
}

// Level-1 inverses of the first pass.  The odd chain positions (level 1 of Gamma's
// order) take no Schur update from the rest of the chain, so L_jj^{-1} of their
// diagonal blocks depends on D alone (Algorithm 1's diagonal factorizations at the
// lowest level, all independent).  One wave per block (per pair of FP64 32 x 32
// blocks), four waves per workgroup, at full occupancy: the blocks are factored here instead of
// in each window's prologue, where three of a workgroup's four waves would wait on the
// serial factorization.  Block bi of the launch is the (bi % nodd)-th odd position of
// chain bi / nodd; wave wi takes blocks wi * BPW .. wi * BPW + BPW - 1.
template <typename T, int NMAX, bool FULL>
__device__ __attribute__((always_inline)) inline void level1_inverse_body(
    const FactorPassArgs& a_in, unsigned wi, int nodd, unsigned total) {
  FactorPassArgs a = a_in;
  if constexpr (FULL) a.n = NMAX;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // 32 x 32 blocks are held as their packed lower triangles (half the LDS of a padded
  // slot, so that more waves fit on a CU), in FP64 two per wave (the diagonal leaves
  // use 32 lanes, so one wave factors both for the issue slots of one); smaller ones in
  // padded slots; one block per wave but for the FP64 pairs
  constexpr bool PK = NMAX == 32;
  constexpr int BPW = level1_blocks_per_wave(NMAX, sizeof(T) == 8);
  constexpr int E = level1_slot_entries<NMAX>();
  constexpr int LD = Lay<NMAX>::LD;
  typedef typename std::conditional<PK, PackedLower<0>, RowMajor<LD>>::type Ix;
  const unsigned b0 = wi * BPW;
  if (b0 >= total) return;  // the whole wave leaves; no workgroup barrier follows
  T* const slot0 = reinterpret_cast<T*>(smem_raw) + wave_id() * BPW * E;
  const int n = a.n, N = a.N;
  const size_t nn = (size_t)n * n;
  const int lane = threadIdx.x & 63;
  // block h of the wave: chain s[h], odd position j[h]; past the end of the launch the
  // last block again (factored, not reported, not stored)
  int s[BPW], j[BPW];
#pragma unroll
  for (int h = 0; h < BPW; ++h) {
    const unsigned bi = min(b0 + h, total - 1);
    s[h] = (int)(bi / (unsigned)nodd);
    j[h] = 2 * (int)(bi - (unsigned)s[h] * nodd) + 1;
  }
#pragma unroll
  for (int h = 0; h < BPW; ++h) {
    const double* D = a.D + ((size_t)s[h] * N + (N - j[h])) * nn;
    T* slot = slot0 + h * E;
    double dv[NMAX * NMAX / 64];
    if constexpr (FULL && NMAX * NMAX % 128 == 0) {
      // D's lower triangle, two consecutive row entries per 16-byte load; pairs above the
      // diagonal are not fetched (they read as zero) and a pair that starts on it brings
      // one entry above it: the factorization reads only the lower triangle
      const auto rd = block_rsrc(D, (unsigned)(NMAX * NMAX) * 8u);
#pragma unroll
      for (int q = 0; q < NMAX * NMAX / 128; ++q) {
        const int e = 2 * (lane + 64 * q), r = e / NMAX, c = e % NMAX;
        const auto w = __builtin_amdgcn_raw_buffer_load_b128(
            rd, c <= r ? (unsigned)e * 8u : kOutOfRange, 0, 0);
        __builtin_memcpy(&dv[2 * q], &w, 16);
      }
#pragma unroll
      for (int u = 0; u < NMAX * NMAX / 64; ++u) {
        const int e = 2 * (lane + 64 * (u >> 1)) + (u & 1), r = e / NMAX, c = e % NMAX;
        if (!Ix::kLowerOnly || c <= r) slot[Ix::at(r, c)] = static_cast<T>(dv[u]);
      }
    } else {
      // D's lower triangle, identity padded (zeros above the diagonal)
#pragma unroll
      for (int u = 0; u < NMAX * NMAX / 64; ++u) {
        const int e = lane + 64 * u, r = e / NMAX, c = e % NMAX;
        dv[u] = (r < n && c <= r) ? D[r * n + c] : (r == c ? 1.0 : 0.0);
      }
#pragma unroll
      for (int u = 0; u < NMAX * NMAX / 64; ++u) {
        const int e = lane + 64 * u, r = e / NMAX, c = e % NMAX;
        if (!Ix::kLowerOnly || c <= r) slot[Ix::at(r, c)] = static_cast<T>(dv[u]);
      }
    }
  }
  wave_lds_fence();
  int fail;  // pairs: per 32-lane half, that half's block
  if constexpr (PK && BPW == 2)
    fail = wave_potrf_inv_packed_pair<T>(slot0, slot0 + E);
  else if constexpr (PK)
    fail = wave_potrf_inv_packed<T>(slot0);
  else
    fail = wave_potrf_inv<T, NMAX>(slot0);
  {
    const int h = lane >> 5;
    if (h < BPW && (lane & 31) == 0 && b0 + h < total && fail >= 0 && fail < n) {
      const int sh = h ? s[BPW - 1] : s[0], jh = h ? j[BPW - 1] : j[0];
      const int sys = sh / a.Ssys;
      const unsigned long long row0 =
          (unsigned long long)sys * ((unsigned long long)a.Ssys * N + 1) * n +
          (unsigned long long)(sh - sys * a.Ssys) * N * n;
      atomicMin(a.info, row0 + (unsigned long long)a.permpos[jh - 1] * n + fail + 1);
    }
  }
  wave_lds_fence();
  // packed lower triangle (rows of length r + 1 whatever n is, so the n x n block's
  // packing is a prefix of the 32 x 32 one)
  const int np = n * (n + 1) / 2;
#pragma unroll
  for (int h = 0; h < BPW; ++h) {
    if (b0 + h >= total) break;  // wave-uniform
    T* Li = reinterpret_cast<T*>(a.Linv) + ((size_t)s[h] * N + (j[h] - 1)) * nn;
    const T* slot = slot0 + h * E;
#pragma unroll
    for (int p0 = 0; p0 < NMAX * (NMAX + 1) / 2; p0 += 64) {
      const int p = p0 + lane;
      if constexpr (PK) {
        if (p < np) Li[p] = slot[p];
      } else {
        int r = (int)((__fsqrt_rn(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
        r = (r * (r + 1) / 2 > p) ? r - 1 : r;
        r = ((r + 1) * (r + 2) / 2 <= p) ? r + 1 : r;
        if (p < np) Li[p] = slot[r * LD + (p - r * (r + 1) / 2)];
      }
    }
  }
}

template <typename T, int NMAX, bool FULL>
__global__ void __launch_bounds__(256) level1_inverse_kernel(FactorPassArgs a, int nodd,
                                                             unsigned total) {
  level1_inverse_body<T, NMAX, FULL>(a, blockIdx.x * 4u + (unsigned)wave_id(), nodd, total);
}

__global__ void factor_init_kernel(unsigned long long* info) {
  if (threadIdx.x == 0) *info = ~0ull;
}

// part[sys][g][e] = sum of U[s][e] over the scenarios of group g of system sys, in
// scenario order (one workgroup per (system, group), one thread per element).  The
// loads of a group are issued together (clamped to the group's last scenario) and
// added in order afterwards.
__device__ __attribute__((always_inline)) inline void root_reduce_body(
    const double* __restrict__ U, double* part, int S, int nn, int groups, unsigned bx) {
  const int sys = bx / groups;
  const int g = bx - sys * groups;
  const int per = (S + groups - 1) / groups;
  const int s0 = g * per, s1 = min(S, s0 + per);
  const double* Us = U + (size_t)sys * S * nn;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    constexpr int B = 16;
    double acc = 0.0;
    for (int s = s0; s < s1; s += B) {
      double t[B];
#pragma unroll
      for (int u = 0; u < B; ++u) t[u] = Us[(size_t)min(s + u, s1 - 1) * nn + e];
#pragma unroll
      for (int u = 0; u < B; ++u) acc = (s + u < s1) ? acc + t[u] : acc;
    }
    part[((size_t)sys * groups + g) * nn + e] = acc;  // 0 for an empty group
  }
}

__global__ void __launch_bounds__(1024) root_reduce_kernel(const double* __restrict__ U,
                                                           double* part, int S, int nn,
                                                           int groups) {
  root_reduce_body(U, part, S, nn, groups, blockIdx.x);
}

// R~ = R - sum_g part[g] (group order), L_R = chol(R~) in FP64 (Algorithm 1, root
// reduction and root factorization).
// 1024 threads: thread e owns element e of the NMAX x NMAX block (identity padded
// beyond n) and loads all group partials at once.
template <int NMAX>
__device__ __attribute__((always_inline)) inline void root_potrf_body(
    const double* __restrict__ R, const double* __restrict__ part, int groups, int n,
    double* LR, unsigned long long sys_rows, unsigned long long root_row,
    unsigned long long* info, unsigned bx) {
  constexpr int LD = NMAX + 1;
  __shared__ double A[NMAX * LD];
  // one workgroup per system of the batch
  const int sys = bx;
  R += (size_t)sys * n * n;
  part += (size_t)sys * groups * n * n;
  LR += (size_t)sys * n * n;
  const unsigned long long row_base = sys * sys_rows + root_row;
  for (int e = threadIdx.x; e < NMAX * NMAX; e += blockDim.x) {
    const int r = e / NMAX, c = e % NMAX;
    double v = (r == c) ? 1.0 : 0.0;  // identity padding
    if (r < n && c < n) {
      constexpr int B = 32;
      double acc = 0.0;
      for (int g0 = 0; g0 < groups; g0 += B) {
        double t[B];
#pragma unroll
        for (int u = 0; u < B; ++u)
          t[u] = part[(size_t)min(g0 + u, groups - 1) * n * n + r * n + c];
#pragma unroll
        for (int u = 0; u < B; ++u) acc = (g0 + u < groups) ? acc + t[u] : acc;
      }
      const double rv = (r >= c) ? R[r * n + c] : R[c * n + r];
      v = rv - acc;
    }
    A[r * LD + c] = v;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int fail = wave_potrf<double, NMAX>(A);
    if (fail >= 0 && fail < n && threadIdx.x == 0) atomicMin(info, row_base + fail + 1);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NMAX * NMAX; e += blockDim.x) {
    const int r = e / NMAX, c = e % NMAX;
    if (r < n && c < n) LR[r * n + c] = A[r * LD + c];
  }
}

template <int NMAX>
__global__ void __launch_bounds__(1024) root_potrf_kernel(const double* __restrict__ R,
                                                          const double* __restrict__ part,
                                                          int groups, int n, double* LR,
                                                          unsigned long long sys_rows,
                                                          unsigned long long root_row,
                                                          unsigned long long* info) {
  root_potrf_body<NMAX>(R, part, groups, n, LR, sys_rows, root_row, info, blockIdx.x);
}

// ---- one launch over the systems of a ragged batch (see multi.h) ----

template <typename T, int NMAX, bool FIRST, bool FINAL, bool FWD, bool FULL>
__global__ void __launch_bounds__(TileCfg<NMAX>::NT,
                                  (pass_min_blocks<T, NMAX, FIRST, FINAL, FULL>()))
    factor_pass_multi(const MultiItem<FactorPassArgs>* items, int nitems, Reloc r) {
  const MultiItem<FactorPassArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  FactorPassArgs a = it.a;
  a.D = rel(r.D, a.D);
  a.E = rel(r.E, a.E);
  a.C = rel(r.C, a.C);
  a.b = FWD ? rel(r.b, a.b) : nullptr;
  factor_pass_body<T, NMAX, FIRST, FINAL, FWD, FULL>(a, multi_local(it).x);
}

// Ragged batches: item p0 = odd positions per chain, p1 = blocks of the system.
template <typename T, int NMAX, bool FULL>
__global__ void __launch_bounds__(256) level1_inverse_multi(const MultiItem<FactorPassArgs>* items,
                                                            int nitems, Reloc r) {
  const MultiItem<FactorPassArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  FactorPassArgs a = it.a;
  a.D = rel(r.D, a.D);
  level1_inverse_body<T, NMAX, FULL>(a, multi_local(it).x * 4u + (unsigned)wave_id(), it.p0,
                                     (unsigned)it.p1);
}

__global__ void __launch_bounds__(1024) root_reduce_multi(const MultiItem<RootArgs>* items,
                                                          int nitems) {
  const MultiItem<RootArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  root_reduce_body(it.a.U, it.a.part, it.a.S, it.a.n * it.a.n, it.a.groups, multi_local(it).x);
}

template <int NMAX>
__global__ void __launch_bounds__(1024) root_potrf_multi(const MultiItem<RootArgs>* items,
                                                         int nitems, Reloc r) {
  const MultiItem<RootArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  root_potrf_body<NMAX>(rel(r.R, it.a.R), it.a.part, it.a.groups, it.a.n, it.a.LR,
                        it.a.sys_rows, it.a.root_row, it.a.info, multi_local(it).x);
}

__global__ void info_reset_kernel(unsigned long long* info, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    info[i] = ~0ull;
}

template <typename T, int NMAX, bool FIRST, bool FINAL, bool FWD, bool FULL>
void launch_multi_kff(const MultiItem<FactorPassArgs>* items, int nitems, unsigned blocks,
                      size_t lds, const Reloc& r, hipStream_t st) {
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(
        reinterpret_cast<const void*>(&factor_pass_multi<T, NMAX, FIRST, FINAL, FWD, FULL>),
        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL((factor_pass_multi<T, NMAX, FIRST, FINAL, FWD, FULL>), dim3(blocks),
                     dim3(TileCfg<NMAX>::NT), lds, st, items, nitems, r);
}
template <typename T, int NMAX, bool FIRST, bool FINAL, bool FWD>
void launch_multi_kf(const MultiItem<FactorPassArgs>* items, int nitems, unsigned blocks,
                     bool full, size_t lds, const Reloc& r, hipStream_t st) {
  if (full)
    launch_multi_kff<T, NMAX, FIRST, FINAL, FWD, true>(items, nitems, blocks, lds, r, st);
  else
    launch_multi_kff<T, NMAX, FIRST, FINAL, FWD, false>(items, nitems, blocks, lds, r, st);
}

template <typename T, int NMAX>
void launch_multi_pass_t(const MultiItem<FactorPassArgs>* items, int nitems, unsigned blocks,
                         bool first, bool final, bool fwd, bool full, size_t lds,
                         const Reloc& r, hipStream_t st) {
#define BMPC_MULTI_KF(F, L, W)                                                          \
  if (first == F && final == L && fwd == W)                                            \
    return launch_multi_kf<T, NMAX, F, L, W>(items, nitems, blocks, full, lds, r, st);
  BMPC_MULTI_KF(true, true, true)
  BMPC_MULTI_KF(true, true, false)
  BMPC_MULTI_KF(true, false, true)
  BMPC_MULTI_KF(true, false, false)
  BMPC_MULTI_KF(false, true, true)
  BMPC_MULTI_KF(false, true, false)
  BMPC_MULTI_KF(false, false, true)
  BMPC_MULTI_KF(false, false, false)
#undef BMPC_MULTI_KF
}

// Block slots, plus (fused forward substitution) Tw + 5 right-hand-side slots.
template <typename T, int NMAX>
size_t pass_lds_bytes(int Tw, int nrhs_fused) {
  return ((size_t)(2 * Tw + 3) * Lay<NMAX>::SZ + (size_t)(Tw + 5) * nrhs_fused * NMAX) *
         sizeof(T);
}

template <typename T, int NMAX, bool FIRST, bool FINAL, bool FWD, bool FULL>
void launch_pass_kff(const FactorPassArgs& a, hipStream_t st) {
  const size_t lds = pass_lds_bytes<T, NMAX>(a.Tw, FWD ? a.nrhs : 0);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(
        reinterpret_cast<const void*>(&factor_pass_kernel<T, NMAX, FIRST, FINAL, FWD, FULL>),
        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  const unsigned grid = (unsigned)a.S * (unsigned)a.windows;
  hipLaunchKernelGGL((factor_pass_kernel<T, NMAX, FIRST, FINAL, FWD, FULL>), dim3(grid),
                     dim3(TileCfg<NMAX>::NT), lds, st, a);
}
template <typename T, int NMAX, bool FIRST, bool FINAL, bool FWD>
void launch_pass_kf(const FactorPassArgs& a, hipStream_t st) {
  if (a.n == NMAX)
    launch_pass_kff<T, NMAX, FIRST, FINAL, FWD, true>(a, st);
  else
    launch_pass_kff<T, NMAX, FIRST, FINAL, FWD, false>(a, st);
}

// The fused forward substitution is its own kernel symbol, so the plain factorization
// carries none of its registers or code.
template <typename T, int NMAX, bool FIRST, bool FINAL>
void launch_pass_k(const FactorPassArgs& a, hipStream_t st) {
  if (a.b)
    launch_pass_kf<T, NMAX, FIRST, FINAL, true>(a, st);
  else
    launch_pass_kf<T, NMAX, FIRST, FINAL, false>(a, st);
}

template <typename T, int NMAX>
void launch_pass_t(const FactorPassArgs& a, hipStream_t st) {
  const bool first = a.pass == 0;
  if (first && a.is_final)
    launch_pass_k<T, NMAX, true, true>(a, st);
  else if (first)
    launch_pass_k<T, NMAX, true, false>(a, st);
  else if (a.is_final)
    launch_pass_k<T, NMAX, false, true>(a, st);
  else
    launch_pass_k<T, NMAX, false, false>(a, st);
}

}  // namespace

size_t factor_pass_lds_bytes(bool fp64, int nmax, int Tw, int nrhs_fused) {
  if (nmax > 32) return Tw == 1 && nrhs_fused == 0 ? factor64_lds_bytes(fp64) : ~(size_t)0;
  if (fp64) {
    if (nmax <= 8) return pass_lds_bytes<double, 8>(Tw, nrhs_fused);
    if (nmax <= 16) return pass_lds_bytes<double, 16>(Tw, nrhs_fused);
    return pass_lds_bytes<double, 32>(Tw, nrhs_fused);
  }
  if (nmax <= 8) return pass_lds_bytes<float, 8>(Tw, nrhs_fused);
  if (nmax <= 16) return pass_lds_bytes<float, 16>(Tw, nrhs_fused);
  return pass_lds_bytes<float, 32>(Tw, nrhs_fused);
}

template <typename T>
void launch_factor_pass(const FactorPassArgs& a, int nmax, hipStream_t st) {
  if (nmax <= 8)
    launch_pass_t<T, 8>(a, st);
  else if (nmax <= 16)
    launch_pass_t<T, 16>(a, st);
  else if (nmax <= 32)
    launch_pass_t<T, 32>(a, st);
  else
    launch_factor_pass64<T>(a, st);
}
template void launch_factor_pass<double>(const FactorPassArgs&, int, hipStream_t);
template void launch_factor_pass<float>(const FactorPassArgs&, int, hipStream_t);

namespace {
template <typename T, int NMAX>
void launch_l1inv_t(const FactorPassArgs& a, hipStream_t st) {
  const int nodd = (a.m + 1) / 2;
  const unsigned total = (unsigned)a.S * (unsigned)nodd;
  if (total == 0) return;
  constexpr unsigned PER_WG = 4 * level1_blocks_per_wave(NMAX, sizeof(T) == 8);
  const size_t lds = PER_WG * (size_t)level1_slot_entries<NMAX>() * sizeof(T);
  const dim3 grid((total + PER_WG - 1) / PER_WG);
  if (a.n == NMAX)
    hipLaunchKernelGGL((level1_inverse_kernel<T, NMAX, true>), grid, dim3(256), lds, st, a, nodd,
                       total);
  else
    hipLaunchKernelGGL((level1_inverse_kernel<T, NMAX, false>), grid, dim3(256), lds, st, a,
                       nodd, total);
}
template <typename T, int NMAX>
void launch_l1inv_multi_t(const MultiItem<FactorPassArgs>* items, int nitems, unsigned blocks,
                          bool full, const Reloc& r, hipStream_t st) {
  const size_t lds =
      4 * (size_t)level1_blocks_per_wave(NMAX, sizeof(T) == 8) * level1_slot_entries<NMAX>() *
      sizeof(T);
  if (full)
    hipLaunchKernelGGL((level1_inverse_multi<T, NMAX, true>), dim3(blocks), dim3(256), lds, st,
                       items, nitems, r);
  else
    hipLaunchKernelGGL((level1_inverse_multi<T, NMAX, false>), dim3(blocks), dim3(256), lds, st,
                       items, nitems, r);
}
}  // namespace

template <typename T>
void launch_level1_inverse(const FactorPassArgs& a, int nmax, hipStream_t st) {
  if (nmax <= 8)
    launch_l1inv_t<T, 8>(a, st);
  else if (nmax <= 16)
    launch_l1inv_t<T, 16>(a, st);
  else
    launch_l1inv_t<T, 32>(a, st);
}
template void launch_level1_inverse<double>(const FactorPassArgs&, int, hipStream_t);
template void launch_level1_inverse<float>(const FactorPassArgs&, int, hipStream_t);

template <typename T>
void launch_level1_inverse_multi(const MultiItem<FactorPassArgs>* items, int nitems,
                                 unsigned blocks, int nmax, bool full, const Reloc& r,
                                 hipStream_t st) {
  if (nmax <= 8)
    launch_l1inv_multi_t<T, 8>(items, nitems, blocks, full, r, st);
  else if (nmax <= 16)
    launch_l1inv_multi_t<T, 16>(items, nitems, blocks, full, r, st);
  else
    launch_l1inv_multi_t<T, 32>(items, nitems, blocks, full, r, st);
}
template void launch_level1_inverse_multi<double>(const MultiItem<FactorPassArgs>*, int,
                                                  unsigned, int, bool, const Reloc&,
                                                  hipStream_t);
template void launch_level1_inverse_multi<float>(const MultiItem<FactorPassArgs>*, int, unsigned,
                                                 int, bool, const Reloc&, hipStream_t);

template <typename T>
void launch_factor_pass_multi(const MultiItem<FactorPassArgs>* items, int nitems,
                              unsigned blocks, int nmax, bool first, bool final, bool fwd,
                              bool full, size_t lds, const Reloc& r, hipStream_t st) {
  if (nmax <= 8)
    launch_multi_pass_t<T, 8>(items, nitems, blocks, first, final, fwd, full, lds, r, st);
  else if (nmax <= 16)
    launch_multi_pass_t<T, 16>(items, nitems, blocks, first, final, fwd, full, lds, r, st);
  else
    launch_multi_pass_t<T, 32>(items, nitems, blocks, first, final, fwd, full, lds, r, st);
}
template void launch_factor_pass_multi<double>(const MultiItem<FactorPassArgs>*, int, unsigned,
                                               int, bool, bool, bool, bool, size_t,
                                               const Reloc&, hipStream_t);
template void launch_factor_pass_multi<float>(const MultiItem<FactorPassArgs>*, int, unsigned,
                                              int, bool, bool, bool, bool, size_t, const Reloc&,
                                              hipStream_t);

void launch_root_reduce_multi(const MultiItem<RootArgs>* items, int nitems, unsigned blocks,
                              hipStream_t st) {
  hipLaunchKernelGGL(root_reduce_multi, dim3(blocks), dim3(1024), 0, st, items, nitems);
}
void launch_root_potrf_multi(const MultiItem<RootArgs>* items, int nitems, unsigned blocks,
                             int nmax, const Reloc& r, hipStream_t st) {
  if (nmax <= 16)
    hipLaunchKernelGGL(root_potrf_multi<16>, dim3(blocks), dim3(1024), 0, st, items, nitems, r);
  else
    hipLaunchKernelGGL(root_potrf_multi<32>, dim3(blocks), dim3(1024), 0, st, items, nitems, r);
}
void launch_info_reset(unsigned long long* info, int count, hipStream_t st) {
  hipLaunchKernelGGL(info_reset_kernel, dim3((count + 255) / 256), dim3(256), 0, st, info, count);
}

void launch_factor_init(unsigned long long* info, hipStream_t st) {
  hipLaunchKernelGGL(factor_init_kernel, dim3(1), dim3(64), 0, st, info);
}

void launch_root_reduce(const double* U, double* part, int B, int S, int n, int groups,
                        hipStream_t st) {
  hipLaunchKernelGGL(root_reduce_kernel, dim3(B * groups), dim3(1024), 0, st, U, part, S, n * n,
                     groups);
}

void launch_root_potrf(const double* R, const double* part, int B, int groups, int n,
                       double* LR, int64_t sys_rows, int64_t root_row,
                       unsigned long long* info, hipStream_t st) {
  if (n <= 16)
    hipLaunchKernelGGL(root_potrf_kernel<16>, dim3(B), dim3(1024), 0, st, R, part, groups, n,
                       LR, (unsigned long long)sys_rows, (unsigned long long)root_row, info);
  else if (n <= 32)
    hipLaunchKernelGGL(root_potrf_kernel<32>, dim3(B), dim3(1024), 0, st, R, part, groups, n,
                       LR, (unsigned long long)sys_rows, (unsigned long long)root_row, info);
  else
    hipLaunchKernelGGL(root_potrf_kernel<64>, dim3(B), dim3(1024), 0, st, R, part, groups, n,
                       LR, (unsigned long long)sys_rows, (unsigned long long)root_row, info);
}

}  // namespace bmpc
