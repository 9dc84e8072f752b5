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
// F = C L_X^{-T} and the local Schur update U = F F^T (Algorithm 1, lines 4-5).
// FIRST (the pass reading D and E) and FINAL are template flags so that each pass
// kind is its own kernel symbol in profiles.
//
// Elimination of position j with neighbours l (left, optional) and r (right),
// Section IV-B in block form:
//   L_jj = chol(A_j);  G_l = K[l,j] L_jj^{-T};  G_r = K[r,j] L_jj^{-T}
//   A_l -= G_l G_l^T;  A_r -= G_r G_r^T;  K[r,l] = -G_r G_l^T (fill)
#include "bmpc_internal.h"
#include "blockops.h"

namespace bmpc {

namespace {

constexpr int NT = kFactorThreads;

template <typename T, int NMAX>
struct Slots {
  static constexpr int SZ = Lay<NMAX>::SZ;
  T* base;
  int Tw;
  __device__ T* A(int t) const { return base + (2 * t) * SZ; }
  __device__ T* Cp(int t) const { return base + (2 * t + 1) * SZ; }
  __device__ T* AL() const { return base + (2 * Tw) * SZ; }
  __device__ T* CL() const { return base + (2 * Tw + 1) * SZ; }
  __device__ T* AR() const { return base + (2 * Tw + 2) * SZ; }
};

__device__ inline void record_failure(unsigned long long* info, unsigned long long row) {
  atomicMin(info, row);
}

// potrf + inverse of the diagonal block in place, failure recorded with the
// 1-based permuted row index.
template <typename T, int NMAX>
__device__ inline void factor_diag(T* A, int n, unsigned long long perm_row0,
                                   unsigned long long* info) {
  if (threadIdx.x < 64) {
    const int fail = wave_potrf<T, NMAX>(A, n);
    if (fail >= 0 && threadIdx.x == 0) record_failure(info, perm_row0 + fail + 1);
    wave_trtri<T, NMAX>(A, n);
  }
  __syncthreads();
}

template <typename T, int NMAX>
__device__ inline void eliminate(T* Aj, T* Cj, T* Al, T* Cl, T* Ar, int n, T* gLinv,
                                 T* gGl, T* gGr, unsigned long long perm_row0,
                                 unsigned long long* info) {
  factor_diag<T, NMAX>(Aj, n, perm_row0, info);  // Aj := L_jj^{-1}
  // G_r = K[r,j] L^{-T}: Cj holds K[r,j]
  lds_gemm_nt<T, NMAX, NT>(Cj, Cj, false, Aj, T(1), false, n);
  if (Cl) {
    // G_l = K[l,j] L^{-T} = (K[j,l])^T L^{-T}: Cl holds K[j,l]
    lds_gemm_nt<T, NMAX, NT>(Cl, Cl, true, Aj, T(1), false, n);
  }
  lds_store<T, NMAX, NT>(gLinv, Aj, n);
  lds_store<T, NMAX, NT>(gGr, Cj, n);
  if (Cl) lds_store<T, NMAX, NT>(gGl, Cl, n);
  lds_gemm_nt<T, NMAX, NT>(Ar, Cj, false, Cj, T(-1), true, n);     // A_r -= G_r G_r^T
  if (Cl) {
    lds_gemm_nt<T, NMAX, NT>(Al, Cl, false, Cl, T(-1), true, n);   // A_l -= G_l G_l^T
    lds_gemm_nt<T, NMAX, NT>(Cl, Cj, false, Cl, T(-1), false, n);  // K[r,l] = -G_r G_l^T
  }
}

template <typename T, int NMAX, bool FIRST, bool FINAL>
__global__ void __launch_bounds__(NT) factor_pass_kernel(FactorPassArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Slots<T, NMAX> sl{reinterpret_cast<T*>(smem_raw), a.Tw};
  constexpr int SZ = Lay<NMAX>::SZ;
  (void)SZ;
  const int n = a.n, N = a.N;
  const size_t nn = (size_t)n * n;
  const int s = blockIdx.x / a.windows;
  const int w = blockIdx.x - s * a.windows;
  const int lo = w << a.Tw;
  const int hi = min(lo + (1 << a.Tw) - 1, a.mk);
  const bool has_left = lo >= 1;
  const int rb = lo + (1 << a.Tw);
  const bool rb_is_x = rb > a.mk;

  T* Linv = reinterpret_cast<T*>(a.Linv) + (size_t)s * N * nn;
  T* Gl = reinterpret_cast<T*>(a.Gl) + (size_t)s * (N > 1 ? N - 1 : 1) * nn;
  T* Gr = reinterpret_cast<T*>(a.Gr) + (size_t)s * (N > 1 ? N - 1 : 1) * nn;
  const unsigned long long chain_row0 = (unsigned long long)s * N * n;

  // Loads of a node (reduced position q) and of its coupling to its successor.
  auto load_node = [&](T* dst, int q) {
    const int j = q << a.shift;
    lds_load_sym_lower<T, NMAX, NT>(dst, a.D + ((size_t)s * N + (N - j)) * nn, n);
    if (!FIRST) {
      __syncthreads();
      const T* ar = reinterpret_cast<const T*>(a.accR_in) + ((size_t)s * a.stride + q) * nn;
      const T* al = reinterpret_cast<const T*>(a.accL_in) + ((size_t)s * a.stride + q) * nn;
      lds_load<T, NMAX, NT>(dst, ar, n, false, true);
      lds_load<T, NMAX, NT>(dst, al, n, false, true);
    }
  };
  auto load_coupling = [&](T* dst, int q) {
    if (FIRST) {
      // K[pos q+1, pos q] = E[s][N-1-q]^T
      lds_load<T, NMAX, NT>(dst, a.E + ((size_t)s * (N - 1) + (N - 1 - q)) * nn, n, true);
    } else {
      const T* f = reinterpret_cast<const T*>(a.fill_in) + ((size_t)s * a.stride + q) * nn;
      lds_load<T, NMAX, NT>(dst, f, n, false);
    }
  };

  if (has_left) {
    // The left boundary node keeps the updates it received while it was a window
    // boundary in earlier passes; they travel with it in its left accumulator.
    if (!FIRST) {
      const size_t base = (size_t)s * a.stride + lo;
      lds_load<T, NMAX, NT>(sl.AL(), reinterpret_cast<const T*>(a.accR_in) + base * nn, n,
                            false);
      __syncthreads();
      lds_load<T, NMAX, NT>(sl.AL(), reinterpret_cast<const T*>(a.accL_in) + base * nn, n,
                            false, true);
    } else {
      lds_zero<T, NMAX, NT>(sl.AL(), n);
    }
    load_coupling(sl.CL(), lo);
  }
  lds_zero<T, NMAX, NT>(sl.AR(), n);
  __syncthreads();

  unsigned live = 0u;
  // Eliminate the live node of level t whose right neighbour's A slot is Ar.
  auto elim_level = [&](int t, int pos_q, T* Ar) {
    const unsigned above = live & ~((2u << t) - 1u);
    T* Al = nullptr;
    T* Cl = nullptr;
    if (above) {
      const int u = __builtin_ctz(above);
      Al = sl.A(u);
      Cl = sl.Cp(u);
    } else if (has_left) {
      Al = sl.AL();
      Cl = sl.CL();
    }
    const int j = pos_q << a.shift;  // original chain position
    const unsigned long long prow = chain_row0 + (unsigned long long)a.permpos[j - 1] * n;
    eliminate<T, NMAX>(sl.A(t), sl.Cp(t), Al, Cl, Ar, n, Linv + (size_t)(j - 1) * nn,
                       Gl + (size_t)(j - 1) * nn, Gr + (size_t)(j - 1) * nn, prow, a.info);
    live &= ~(1u << t);
  };

  for (int q = lo + 1; q <= hi; ++q) {
    const int v = __builtin_ctz((unsigned)q);
    load_node(sl.A(v), q);
    load_coupling(sl.Cp(v), q);
    __syncthreads();
    for (int t = 0; t < v; ++t) {
      if (live & (1u << t)) elim_level(t, q - (1 << t), sl.A(v));
    }
    live |= (1u << v);
  }
  // Right boundary read: eliminate every remaining live level, lowest first.
  while (live) {
    const int t = __builtin_ctz(live);
    // position of the live node of level t: rb - 2^t for a node boundary; for X the
    // live nodes are the ones whose level-neighbour lies beyond the chain end.
    const int pos = rb_is_x ? ((hi >> t) << t) : rb - (1 << t);
    elim_level(t, pos, sl.AR());
  }

  if (!FINAL) {
    const size_t base = (size_t)s * a.stride;
    if (has_left) {
      lds_store<T, NMAX, NT>(reinterpret_cast<T*>(a.accL_out) + (base + w) * nn, sl.AL(), n);
      lds_store<T, NMAX, NT>(reinterpret_cast<T*>(a.fill_out) + (base + w) * nn, sl.CL(), n);
    }
    if (!rb_is_x) {
      lds_store<T, NMAX, NT>(reinterpret_cast<T*>(a.accR_out) + (base + w + 1) * nn, sl.AR(), n);
    } else {
      lds_store<T, NMAX, NT>(reinterpret_cast<T*>(a.accX) + ((size_t)s * a.npass + a.pass) * nn,
                             sl.AR(), n);
    }
    return;
  }

  // ---- last pass: x_1 step (Algorithm 1, lines 3-5 for the terminal block) ----
  T* Ax = sl.A(0);
  T* Cx = sl.Cp(0);
  lds_load_sym_lower<T, NMAX, NT>(Ax, a.D + ((size_t)s * N + 0) * nn, n);
  __syncthreads();
  for (int p = 0; p < a.pass; ++p)
    lds_load<T, NMAX, NT>(Ax, reinterpret_cast<const T*>(a.accX) + ((size_t)s * a.npass + p) * nn,
                          n, false, true);
  __syncthreads();
  {
    constexpr int LD = Lay<NMAX>::LD;
    for (int e = threadIdx.x; e < n * n; e += NT) {
      const int r = e / n, c = e - (e / n) * n;
      Ax[r * LD + c] += sl.AR()[r * LD + c];
    }
  }
  __syncthreads();
  factor_diag<T, NMAX>(Ax, n, chain_row0 + (unsigned long long)a.permpos[N - 1] * n, a.info);
  lds_store<T, NMAX, NT>(Linv + (size_t)(N - 1) * nn, Ax, n);
  // F = C L_X^{-T}
  lds_load<T, NMAX, NT>(Cx, a.C + (size_t)s * nn, n, false);
  __syncthreads();
  lds_gemm_nt<T, NMAX, NT>(Cx, Cx, false, Ax, T(1), false, n);
  lds_store<T, NMAX, NT>(reinterpret_cast<T*>(a.F) + (size_t)s * nn, Cx, n);
  // U = F F^T in FP64 from the stored F
  {
    constexpr int LD = Lay<NMAX>::LD;
    double* U = a.U + (size_t)s * nn;
    for (int e = threadIdx.x; e < n * n; e += NT) {
      const int r = e / n, c = e - (e / n) * n;
      double acc = 0.0;
      for (int k = 0; k < n; ++k)
        acc += static_cast<double>(Cx[r * LD + k]) * static_cast<double>(Cx[c * LD + k]);
      U[e] = acc;
    }
  }
}

__global__ void factor_init_kernel(unsigned long long* info) {
  if (threadIdx.x == 0) *info = ~0ull;
}

// part[g][e] = sum of U[s][e] over the scenarios of group g, in scenario order.
__global__ void __launch_bounds__(256) root_reduce_kernel(const double* __restrict__ U,
                                                          double* part, int S, int nn,
                                                          int groups) {
  const int g = blockIdx.x;
  const int per = (S + groups - 1) / groups;
  const int s0 = g * per, s1 = min(S, s0 + per);
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    double acc = 0.0;
    for (int s = s0; s < s1; ++s) acc += U[(size_t)s * nn + e];
    part[(size_t)g * nn + e] = acc;
  }
}

// R~ = R - sum_g part[g] (group order), L_R = chol(R~) in FP64 (Algorithm 1, 7-8).
__global__ void __launch_bounds__(256) root_potrf_kernel(const double* __restrict__ R,
                                                         const double* __restrict__ part,
                                                         int groups, int n, double* LR,
                                                         unsigned long long row_base,
                                                         unsigned long long* info) {
  __shared__ double A[32 * 33];
  constexpr int LD = 33;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e - (e / n) * n;
    const double rv = (r >= c) ? R[r * n + c] : R[c * n + r];
    double acc = 0.0;
    for (int g = 0; g < groups; ++g) acc += part[(size_t)g * n * n + e];
    A[r * LD + c] = rv - acc;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int fail = wave_potrf<double, 32>(A, n);
    if (fail >= 0 && threadIdx.x == 0) atomicMin(info, row_base + fail + 1);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e - (e / n) * n;
    LR[e] = A[r * LD + c];
  }
}

template <typename T, int NMAX>
size_t pass_lds_bytes(int Tw) {
  return (size_t)(2 * Tw + 3) * Lay<NMAX>::SZ * sizeof(T);
}

template <typename T, int NMAX, bool FIRST, bool FINAL>
void launch_pass_k(const FactorPassArgs& a, hipStream_t st) {
  const size_t lds = pass_lds_bytes<T, NMAX>(a.Tw);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(
        reinterpret_cast<const void*>(&factor_pass_kernel<T, NMAX, FIRST, FINAL>),
        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  const unsigned grid = (unsigned)a.S * (unsigned)a.windows;
  hipLaunchKernelGGL((factor_pass_kernel<T, NMAX, FIRST, FINAL>), dim3(grid), dim3(NT), lds,
                     st, a);
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

size_t factor_pass_lds_bytes(bool fp64, int nmax, int Tw) {
  if (fp64) {
    if (nmax <= 8) return pass_lds_bytes<double, 8>(Tw);
    if (nmax <= 16) return pass_lds_bytes<double, 16>(Tw);
    return pass_lds_bytes<double, 32>(Tw);
  }
  if (nmax <= 8) return pass_lds_bytes<float, 8>(Tw);
  if (nmax <= 16) return pass_lds_bytes<float, 16>(Tw);
  return pass_lds_bytes<float, 32>(Tw);
}

template <typename T>
void launch_factor_pass(const FactorPassArgs& a, int nmax, hipStream_t st) {
  if (nmax <= 8)
    launch_pass_t<T, 8>(a, st);
  else if (nmax <= 16)
    launch_pass_t<T, 16>(a, st);
  else
    launch_pass_t<T, 32>(a, st);
}
template void launch_factor_pass<double>(const FactorPassArgs&, int, hipStream_t);
template void launch_factor_pass<float>(const FactorPassArgs&, int, hipStream_t);

void launch_factor_init(unsigned long long* info, hipStream_t st) {
  hipLaunchKernelGGL(factor_init_kernel, dim3(1), dim3(64), 0, st, info);
}

void launch_root_reduce(const double* U, double* part, int S, int n, int groups,
                        hipStream_t st) {
  hipLaunchKernelGGL(root_reduce_kernel, dim3(groups), dim3(256), 0, st, U, part, S, n * n,
                     groups);
}

void launch_root_potrf(const double* R, const double* part, int groups, int n, double* LR,
                       int64_t row_base, unsigned long long* info, hipStream_t st) {
  hipLaunchKernelGGL(root_potrf_kernel, dim3(1), dim3(256), 0, st, R, part, groups, n, LR,
                     (unsigned long long)row_base, info);
}

}  // namespace bmpc
