// Two-level triangular solves (Algorithm 2) for gfx950.
//
// Forward substitution L dy = Pi r, one launch per Gamma level: a position j of
// level l pulls the contributions of the positions that precede it in the factor's
// row j -- the left neighbours j-2^t and right neighbours j+2^t of levels t+1 < l --
// so every factor block is read exactly once per sweep and no two work items write
// the same vector (no atomics, fixed summation order).  Then X (x_1), whose row holds
// the G_r blocks of the last position of every level with an odd chain length, and
// the FP64 root step (Algorithm 2, root step).  Backward substitution walks the
// levels in reverse; position j reads the already known x of its two neighbours.
// The permutation Pi_i (Algorithm 2, gather and scatter) is applied as an index map:
// chain position j reads and writes stage N-j of the natural-order vectors.
//
// Factor blocks are held in registers (RegBlock).  In the level kernels every block
// a position needs is loaded at once, spread over up to four waves; the x_1 kernels
// pipeline their pulls two deep through a double-buffered LDS vector array.
#include <algorithm>

#include "bmpc_internal.h"
#include "blockops.h"
#include "multi.h"
#include "regblock.h"
#include "solve_common.h"

namespace bmpc {

namespace {

constexpr int NT = kSolveThreads;

// Gathered right-hand side of a position: dst[q][i] = b[off + q*len + i] / rnorm, zero
// padded to NMAX (seg0 = norm index of q = 0).
template <typename T, int NMAX>
__device__ inline void gather_rhs(const SolveArgs& a, T (*dst)[NMAX], size_t off, int seg0) {
  const size_t len = vec_len(a);
  for (int idx = threadIdx.x; idx < a.nrhs * NMAX; idx += NT) {
    const int q = idx / NMAX, i = idx % NMAX;
    T v = T(0);
    if (i < a.n) {
      double bv = a.b[(size_t)q * len + off + i];
      if (a.rnorm) {
        const double rn = a.rnorm[seg0 + q];
        bv = rn > 0.0 ? bv / rn : 0.0;
      }
      v = static_cast<T>(bv);
    }
    dst[q][i] = v;
  }
}

// Per-lane staging of one neighbour vector (nrhs x n values, zero padded).
template <typename T, int NMAX>
struct VecStage {
  static constexpr int PER = (kMaxRhs * NMAX + NT - 1) / NT;
  T v[PER];
  __device__ void load(const T* __restrict__ src, int n, int nrhs) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = threadIdx.x + k * NT;
      const int q = idx / NMAX, i = idx % NMAX;
      v[k] = (q < nrhs && i < n) ? src[q * n + i] : T(0);
    }
  }
  __device__ void store(T (*dst)[NMAX], int nrhs) const {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = threadIdx.x + k * NT;
      const int q = idx / NMAX;
      if (q < nrhs) dst[q][idx % NMAX] = v[k];
    }
  }
};

// Accumulate sum_p op(M_p) v_p over a list of pulls with a two-deep pipeline.
// pull(p, &blk, &vec) returns false when pull p does not exist.
template <typename T, int NMAX, bool TRANS, typename PullFn>
__device__ inline void pull_products(int npull, PullFn pull, int n, int nrhs,
                                     T (*vbuf)[kMaxRhs][NMAX], T* part) {
  typedef RegBlock<T, NMAX> RB;
  const T* blk = nullptr;
  const T* vec = nullptr;
  int p = 0;
  while (p < npull && !pull(p, blk, vec)) ++p;
  if (p >= npull) return;
  RB cur;
  cur.template load<TRANS>(blk, n);
  {
    VecStage<T, NMAX> vs;
    vs.load(vec, n, nrhs);
    vs.store(vbuf[0], nrhs);
  }
  __syncthreads();
  int buf = 0;
  while (p < npull) {
    int pn = p + 1;
    const T* nblk = nullptr;
    const T* nvec = nullptr;
    while (pn < npull && !pull(pn, nblk, nvec)) ++pn;
    RB nxt;
    VecStage<T, NMAX> vs;
    if (pn < npull) {
      nxt.template load<TRANS>(nblk, n);
      vs.load(nvec, n, nrhs);
    }
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q)
      if (q < nrhs) part[q] += cur.dot(vbuf[buf][q]);
    if (pn < npull) vs.store(vbuf[buf ^ 1], nrhs);
    __syncthreads();
    cur = nxt;
    buf ^= 1;
    p = pn;
  }
}

// dst[q][o] -= (reduced partial sums); lanes of one output index share a sum.
template <typename T, int NMAX>
__device__ inline void subtract_reduced(T (*dst)[NMAX], const T* part, int nrhs) {
  typedef RegBlock<T, NMAX> RB;
#pragma unroll
  for (int q = 0; q < kMaxRhs; ++q) {
    if (q < nrhs) {
      const T s = lane_group_sum<RB::LPR>(part[q]);
      if (RB::base() == 0) dst[q][RB::out_index()] -= s;
    }
  }
}

template <typename T, int NMAX>
struct SolveSmem {
  T vbuf[2][kMaxRhs][NMAX];
  T rhs[kMaxRhs][NMAX];
};

// Level kernels of both sweeps.  A position applies its own L_jj^{-1} after
// subtracting the products of the factor blocks it pulls, each with the vector of a
// neighbour.  Forward (position j of level l): pull 2t is the G_r of the left
// neighbour j-2^t, pull 2t+1 the G_l of the right neighbour j+2^t (t < l-1).
// Backward: pull 0 is G_l(j)^T with x of the left neighbour, pull 1 is G_r(j)^T with
// x of the right neighbour (or of X).  Each wave takes kPullsPerWave consecutive pulls
// and issues all of their loads at once (wave 0 also loads L_jj^{-1}); the workgroup
// has up to kLevelMaxWaves waves and further pulls go round in turns.  Partial sums
// are combined in wave order.
constexpr int kPullsPerWave = 2;
constexpr int kLevelMaxWaves = 4;

// Dynamic LDS of a level workgroup with W waves and nrhs right-hand sides:
// vbuf[W][kPullsPerWave][nrhs][NMAX], partial[W][nrhs][NMAX], rhs[nrhs][NMAX].
template <typename T, int NMAX>
inline size_t level_smem_bytes(int waves, int nrhs) {
  return (size_t)(waves * kPullsPerWave + waves + 1) * nrhs * NMAX * sizeof(T);
}

// One neighbour vector (nrhs x n, zero padded) staged by the lanes of one wave.
template <typename T, int NMAX>
struct WaveVec {
  static constexpr int PER = (kMaxRhs * NMAX + 63) / 64;
  T v[PER];
  __device__ void load(const T* __restrict__ src, int n, int nrhs) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = lane + k * 64;
      const int q = idx / NMAX, i = idx % NMAX;
      v[k] = (q < nrhs && i < n) ? src[q * n + i] : T(0);
    }
  }
  // n == NMAX: the nrhs x n values are contiguous; a buffer resource over them reads
  // the padding past nrhs as zero, and rounds past it are skipped wave-uniformly.
  __device__ void load_full(const T* __restrict__ src, int nrhs) {
    const int lane = threadIdx.x & 63;
    const auto rs = block_rsrc(src, (unsigned)(nrhs * NMAX) * sizeof(T));
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (k * 64 < nrhs * NMAX) {
        const unsigned off = (unsigned)(lane + k * 64) * sizeof(T);
        if constexpr (sizeof(T) == 8)
          v[k] = buf_load_f64(rs, off);
        else
          v[k] = buf_load_f32(rs, off);
      }
    }
  }
  __device__ void store_full(T (*dst)[NMAX], int nrhs) const {
    const int lane = threadIdx.x & 63;
    T* d = &dst[0][0];
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (k * 64 < nrhs * NMAX && lane + k * 64 < nrhs * NMAX) d[lane + k * 64] = v[k];
  }
  __device__ void store(T (*dst)[NMAX], int nrhs) const {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = lane + k * 64;
      const int q = idx / NMAX;
      if (q < nrhs) dst[q][idx % NMAX] = v[k];
    }
  }
};

// Right-hand side of a position, held in registers by wave 0 until the pull loads are
// in flight: the gathered b scaled by 1/rnorm (forward) or the position's y (backward).
template <typename T, int NMAX, bool FWD>
struct RhsRegs {
  static constexpr int PER = (kMaxRhs * NMAX + 63) / 64;
  typedef typename std::conditional<FWD, double, T>::type RT;
  RT v[PER];
  double rn[FWD ? PER : 1];
  // Lanes past the data read a clamped in-range element; store() drops them, so no
  // loaded value is used before the factor loads are issued.
  __device__ void load(const SolveArgs& a, size_t off, int seg0, const T* yj) {
    const int lane = threadIdx.x & 63;
    const size_t len = vec_len(a);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (k * 64 >= a.nrhs * NMAX) continue;  // wave-uniform
      const int idx = lane + k * 64;
      const int q = min(idx / NMAX, a.nrhs - 1), ii = min(idx % NMAX, a.n - 1);
      if constexpr (FWD) {
        v[k] = a.b[(size_t)q * len + off + ii];
        if (a.rnorm) rn[k] = a.rnorm[seg0 + q];
      } else {
        v[k] = yj[q * a.n + ii];
      }
    }
  }
  __device__ void store(const SolveArgs& a, T (*dst)[NMAX]) const {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (k * 64 >= a.nrhs * NMAX) continue;  // wave-uniform
      const int idx = lane + k * 64;
      const int q = idx / NMAX, ii = idx % NMAX;
      if (q < a.nrhs) {
        T t = T(0);
        if (ii < a.n) {
          if constexpr (FWD) {
            const double r = a.rnorm ? rn[k] : 1.0;
            t = static_cast<T>(r > 0.0 ? v[k] / r : 0.0);
          } else {
            t = v[k];
          }
        }
        dst[q][ii] = t;
      }
    }
  }
};

// Right-hand sides whose refinement update (x += rnorm * d) has x and rnorm fetched
// together with the factor blocks; further ones are read when they are written.
constexpr int kUpdatePrefetch = 2;

template <typename T, int NMAX, bool FWD, bool FULL>
__device__ __attribute__((always_inline)) inline void solve_level_body(const SolveArgs& a,
                                                                       int level, int count,
                                                                       unsigned bx) {
  if (a.done && *a.done) return;
  typedef RegBlock<T, NMAX> RB;
  constexpr int P = kPullsPerWave;
  const int n = a.n, N = a.N, nrhs = a.nrhs, m = a.m;
  const size_t nn = (size_t)n * n;
  const int W = blockDim.x >> 6, wv = threadIdx.x >> 6;
  extern __shared__ __align__(16) unsigned char level_smem[];
  typedef T Vec[NMAX];
  Vec* vbuf = reinterpret_cast<Vec*>(level_smem);          // [(w * P + u) * nrhs + q]
  Vec* partial = vbuf + (size_t)W * P * nrhs;              // [w * nrhs + q]
  Vec* rhs = partial + (size_t)W * nrhs;                   // [q]
  const int s = bx / count;
  const int i = bx - s * count;
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
  const size_t len = vec_len(a);
  const int o = RB::out_index();
  const bool writer = RB::base() == 0 && o < n;

  auto pull = [&](int p, const T*& blk, const T*& vec) -> bool {
    if constexpr (FWD) {
      const int t = p >> 1;
      const int c = (p & 1) ? j + (1 << t) : j - (1 << t);
      if (c > m) return false;
      blk = ((p & 1) ? Gl : Gr) + (size_t)(c - 1) * nn;
      vec = y + (size_t)(c - 1) * nrhs * n;
    } else {
      if (p == 0) {
        if (j - half < 1) return false;
        blk = Gl + (size_t)(j - 1) * nn;
        vec = y + (size_t)(j - half - 1) * nrhs * n;
      } else {
        const int ir = j + half <= m ? j + half - 1 : N - 1;
        blk = Gr + (size_t)(j - 1) * nn;
        vec = y + (size_t)ir * nrhs * n;
      }
    }
    return true;
  };

  // Every global load of the first round goes out before the first wait: wave 0 takes
  // L_jj^{-1}, the right-hand side and (backward refinement update) x and rnorm; each
  // wave its pulls.
  RB lin;
  RhsRegs<T, NMAX, FWD> rr;
  double xold[kUpdatePrefetch] = {}, rnq[kUpdatePrefetch] = {};
  if (wv == 0) {
    if constexpr (FULL)
      lin.template load_packed_raw<!FWD>(Linv + (size_t)(j - 1) * nn);
    else
      lin.template load_packed<!FWD>(Linv + (size_t)(j - 1) * nn, n);
    rr.load(a, off, seg0, yj);
    if constexpr (!FWD) {
      if (a.accumulate) {  // wave-uniform; the writer lanes use the values
        const int oc = min(o, n - 1);
#pragma unroll
        for (int q = 0; q < kUpdatePrefetch; ++q) {
          if (q < nrhs) {
            xold[q] = a.x[(size_t)q * len + off + oc];
            rnq[q] = a.rnorm[seg0 + q];
          }
        }
      }
    }
  }
  // One round: this wave's pulls base + wv*P + u.  The first round is peeled so that
  // wave 0 stores the right-hand side right after that round's loads are issued.
  auto round = [&](int base, bool first) {
    RB blk[P];
    WaveVec<T, NMAX> vs[P];
    bool has[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int p = base + wv * P + u;
      const T* bp = nullptr;
      const T* vp = nullptr;
      has[u] = p < npull && pull(p, bp, vp);
      if (has[u]) {
        blk[u].template load_fixed<!FWD, FULL>(bp, n);
        if constexpr (FULL)
          vs[u].load_full(vp, nrhs);
        else
          vs[u].load(vp, n, nrhs);
      }
    }
    if (first && wv == 0) rr.store(a, rhs);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      if (has[u]) {
        if constexpr (FULL)
          vs[u].store_full(vbuf + (size_t)(wv * P + u) * nrhs, nrhs);
        else
          vs[u].store(vbuf + (size_t)(wv * P + u) * nrhs, nrhs);
      }
    }
    wave_lds_fence();
    // this wave's partial sums, accumulated over the rounds in its LDS row
#pragma unroll 1
    for (int q = 0; q < nrhs; ++q) {
      T acc = T(0);
#pragma unroll
      for (int u = 0; u < P; ++u)
        if (has[u]) acc += blk[u].dot(vbuf[(size_t)(wv * P + u) * nrhs + q]);
      acc = lane_group_sum<RB::LPR>(acc);
      if (RB::base() == 0) {
        T* dst = &partial[wv * nrhs + q][o];
        *dst = first ? acc : *dst + acc;
      }
    }
    wave_lds_fence();
  };
  round(0, true);
  for (int base = W * P; base < npull; base += W * P) round(base, false);
  __syncthreads();
  if (wv != 0) return;
  if constexpr (FULL) lin.template mask_packed<!FWD>();
  for (int idx = threadIdx.x; idx < nrhs * NMAX; idx += 64) {
    const int q = idx / NMAX, ii = idx % NMAX;
    T acc = partial[q][ii];
    for (int w = 1; w < W; ++w) acc += partial[w * nrhs + q][ii];
    rhs[q][ii] -= acc;
  }
  wave_lds_fence();
  // x[off + q*len] = d, or x += rnorm * d with rnorm * d kept in dstore
  auto finish = [&](int q, double xo, double rn) {
    const T v = lane_group_sum<RB::LPR>(lin.dot(rhs[q]));
    if (writer) {
      yj[q * n + o] = v;
      if constexpr (!FWD) {
        const size_t idx = (size_t)q * len + off + o;
        const double d = static_cast<double>(v);
        if (a.accumulate) {
          const double dd = rn * d;
          a.x[idx] = xo + dd;
          a.dstore[idx] = dd;
        } else {
          a.x[idx] = d;
        }
      }
    }
  };
  if constexpr (FWD) {
#pragma unroll 1
    for (int q = 0; q < nrhs; ++q) finish(q, 0.0, 0.0);
  } else {
#pragma unroll
    for (int q = 0; q < kUpdatePrefetch; ++q)
      if (q < nrhs) finish(q, xold[q], rnq[q]);
#pragma unroll 1
    for (int q = kUpdatePrefetch; q < nrhs; ++q) {
      const size_t idx = (size_t)q * len + off + o;
      const bool ok = a.accumulate && writer;
      finish(q, ok ? a.x[idx] : 0.0, ok ? a.rnorm[seg0 + q] : 0.0);
    }
  }
}

template <typename T, int NMAX, bool FWD, bool FULL>
__global__ void __launch_bounds__(64 * kLevelMaxWaves) solve_level_kernel(SolveArgs a, int level,
                                                                         int count) {
  solve_level_body<T, NMAX, FWD, FULL>(a, level, count, blockIdx.x);
}

// Level kernel for one right-hand side and n == NMAX (the common case): the same
// products and summation order as solve_level_kernel with the per-element staging of
// several right-hand sides taken out.  Lane l holds element l % NMAX of each vector it
// stages; the chain comes from the grid (position index, scenario, system), and each
// wave keeps its partial sums in a register across rounds.
// One position (index i of the level, scenario sl, system sys) served by W waves, this
// thread's wave being wv; smem holds (W * kPullsPerWave + W + 1) * NMAX elements.
template <typename T, int NMAX, bool FWD>
__device__ __attribute__((always_inline)) inline void level_one_position(
    const SolveArgs& a, int level, int i, int sl, int sys, int W, int wv,
    unsigned char* smem) {
  typedef RegBlock<T, NMAX> RB;
  constexpr int P = kPullsPerWave;
  constexpr int n = NMAX;
  constexpr size_t nn = (size_t)NMAX * NMAX;
  const int N = a.N, m = a.m;
  const int lane = threadIdx.x & 63;
  typedef T Vec[NMAX];
  Vec* vbuf = reinterpret_cast<Vec*>(smem);  // [w * P + u]
  Vec* partial = vbuf + W * P;               // [w]
  T* t = partial[W];                         // right-hand side, then residual
  const size_t s = (size_t)sys * a.S + sl;
  const int j = (2 * i + 1) << (level - 1);
  const size_t gstride = g_chain_blocks(N);
  const T* Gl = reinterpret_cast<const T*>(a.Gl) + s * gstride * nn;
  const T* Gr = reinterpret_cast<const T*>(a.Gr) + s * gstride * nn;
  const T* Linv = reinterpret_cast<const T*>(a.Linv) + s * N * nn;
  T* y = reinterpret_cast<T*>(a.y) + s * N * n;
  T* yj = y + (size_t)(j - 1) * n;
  const int half = 1 << (level - 1);
  const int npull = FWD ? 2 * (level - 1) : 2;
  const size_t off = (size_t)sys * a.vsys + ((size_t)sl * N + (N - j)) * n;
  const int seg = sys * a.seg_sys;
  const int o = RB::out_index();
  const bool writer = RB::base() == 0;
  const int vl = lane & (NMAX - 1);

  auto pull = [&](int p, const T*& blk, const T*& vec) -> bool {
    if constexpr (FWD) {
      const int tt = p >> 1;
      const int c = (p & 1) ? j + (1 << tt) : j - (1 << tt);
      if (c > m) return false;
      blk = ((p & 1) ? Gl : Gr) + (size_t)(c - 1) * nn;
      vec = y + (size_t)(c - 1) * n;
    } else {
      if (p == 0) {
        if (j - half < 1) return false;
        blk = Gl + (size_t)(j - 1) * nn;
        vec = y + (size_t)(j - half - 1) * n;
      } else {
        const int ir = j + half <= m ? j + half - 1 : N - 1;
        blk = Gr + (size_t)(j - 1) * nn;
        vec = y + (size_t)ir * n;
      }
    }
    return true;
  };

  // All loads of the first round are issued before the first wait.
  RB lin;
  T rv = T(0);
  double rb = 0.0, xo = 0.0;
  if (wv == 0) {
    lin.template load_packed_raw<!FWD>(Linv + (size_t)(j - 1) * nn);
    if constexpr (FWD)
      rb = a.b[off + vl];
    else
      rv = yj[vl];
    if (!FWD && a.accumulate) xo = a.x[off + o];
  }
  T tot = T(0);
  auto round = [&](int base, bool first) {
    RB blk[P];
    T vv[P];
    bool has[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int p = base + wv * P + u;
      const T* bp = nullptr;
      const T* vp = nullptr;
      has[u] = p < npull && pull(p, bp, vp);
      if (has[u]) {
        blk[u].template load_fixed<!FWD, true>(bp, n);
        vv[u] = vp[vl];
      }
    }
    if (first && wv == 0 && lane < NMAX) {
      if constexpr (FWD) {
        const double rn = a.rnorm ? a.rnorm[seg] : 1.0;
        t[lane] = static_cast<T>(rn > 0.0 ? rb / rn : 0.0);
      } else {
        t[lane] = rv;
      }
    }
#pragma unroll
    for (int u = 0; u < P; ++u)
      if (has[u] && lane < NMAX) vbuf[wv * P + u][lane] = vv[u];
    wave_lds_fence();
    T acc = T(0);
#pragma unroll
    for (int u = 0; u < P; ++u)
      if (has[u]) acc += blk[u].dot(vbuf[wv * P + u]);
    acc = lane_group_sum_dpp<RB::LPR>(acc);
    tot = first ? acc : tot + acc;
    wave_lds_fence();
  };
  round(0, true);
  for (int base = W * P; base < npull; base += W * P) round(base, false);
  if (W > 1) {
    if (writer) partial[wv][o] = tot;
    __syncthreads();
    if (wv != 0) return;
    T sum = partial[0][o];
    for (int w = 1; w < W; ++w) sum += partial[w][o];
    tot = sum;
  }
  // residual of the position, then L_jj^{-1} (forward) or L_jj^{-T} (backward) on it
  const T r = t[o] - tot;
  wave_lds_fence();
  if (writer) t[o] = r;
  wave_lds_fence();
  lin.template mask_packed<!FWD>();
  const T v = lane_group_sum_dpp<RB::LPR>(lin.dot(t));
  if (writer) {
    yj[o] = v;
    if constexpr (!FWD) {
      const size_t idx = off + o;
      const double d = static_cast<double>(v);
      if (a.accumulate) {
        const double dd = a.rnorm[seg] * d;
        a.x[idx] = xo + dd;
        a.dstore[idx] = dd;
      } else {
        a.x[idx] = d;
      }
    }
  }
}

template <typename T, int NMAX, bool FWD>
__global__ void __launch_bounds__(64 * kLevelMaxWaves) solve_level_one_kernel(SolveArgs a,
                                                                             int level) {
  if (a.done && *a.done) return;
  extern __shared__ __align__(16) unsigned char level_smem[];
  level_one_position<T, NMAX, FWD>(a, level, blockIdx.x, blockIdx.y, blockIdx.z,
                                   (int)(blockDim.x >> 6), (int)(threadIdx.x >> 6), level_smem);
}

// Backward level kernel for one right-hand side and n = 32 that reads every block by
// rows: lane l holds the 16-byte piece (VEC elements) at columns VEC*q of rows
// mrow + RPI*k (q = l % QPR, mrow = l / QPR, k < K), so one load instruction covers RPI
// whole rows of a block, as in the forward sweep, instead of reading columns with
// dword loads.  The transposed products G^T x and L_jj^{-T} r sum over rows, i.e. over
// the lanes that share q (column_group_sum); the residual r, produced by columns, is
// re-indexed by rows through LDS.  Position j's own G_l slot is read even without a
// left neighbour (it is then never written and not used), so that no load waits on a
// branch.  Same result as solve_level_one_kernel<T, 32, false> up to summation order.
template <typename T>
__device__ __attribute__((always_inline)) inline void bwd_rows_position(
    const SolveArgs& a, int level, int i, int sl, int sys, T (*xs)[32]) {
  constexpr int NMAX = 32;
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int QPR = NMAX / VEC;
  constexpr int RPI = 64 / QPR;
  constexpr int K = NMAX / RPI;
  constexpr int n = NMAX;
  constexpr size_t nn = (size_t)NMAX * NMAX;
  typedef T vt __attribute__((ext_vector_type(VEC)));
  // xs[3][NMAX] (this wave's LDS): x of the left and right neighbours, y_j; then r by rows
  const int lane = threadIdx.x & 63, q = lane % QPR, mrow = lane / QPR;
  const int N = a.N, m = a.m;
  const size_t s = (size_t)sys * a.S + sl;
  const int j = (2 * i + 1) << (level - 1);
  const int half = 1 << (level - 1);
  const size_t gstride = g_chain_blocks(N);
  const T* Glb = reinterpret_cast<const T*>(a.Gl) + (s * gstride + (j - 1)) * nn;
  const T* Grb = reinterpret_cast<const T*>(a.Gr) + (s * gstride + (j - 1)) * nn;
  const T* Lb = reinterpret_cast<const T*>(a.Linv) + (s * N + (j - 1)) * nn;
  T* y = reinterpret_cast<T*>(a.y) + s * N * n;
  T* yj = y + (size_t)(j - 1) * n;
  const bool has_left = j - half >= 1;
  const int ir = j + half <= m ? j + half - 1 : N - 1;
  const size_t off = (size_t)sys * a.vsys + ((size_t)sl * N + (N - j)) * n;
  vt gl[K], gr[K];
  T li[K][VEC];
  const auto rsL = block_rsrc(Lb, (unsigned)(NMAX * (NMAX + 1) / 2) * sizeof(T));
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int R = mrow + RPI * k;
    gr[k] = *reinterpret_cast<const vt*>(Grb + R * NMAX + VEC * q);
    gl[k] = *reinterpret_cast<const vt*>(Glb + R * NMAX + VEC * q);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const unsigned o = (unsigned)(R * (R + 1) / 2 + VEC * q + e) * sizeof(T);
      if constexpr (sizeof(T) == 8)
        li[k][e] = buf_load_f64(rsL, o);
      else
        li[k][e] = buf_load_f32(rsL, o);
    }
  }
  const int vl = lane & (NMAX - 1);
  const T v0 = y[(size_t)(has_left ? j - half - 1 : j - 1) * n + vl];
  const T v1 = y[(size_t)ir * n + vl];
  const T v2 = yj[vl];
  double xo[VEC];
  if (a.accumulate) {  // wave-uniform; the x being updated, at the output lanes' columns
#pragma unroll
    for (int e = 0; e < VEC; ++e) xo[e] = a.x[off + VEC * q + e];
  }
  if (lane < NMAX) {
    xs[0][lane] = has_left ? v0 : T(0);
    xs[1][lane] = v1;
    xs[2][lane] = v2;
  }
  wave_lds_fence();
  // r = y_j - G_l^T x_l - G_r^T x_r, by columns c = VEC*q + e
  T p[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) p[e] = T(0);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int R = mrow + RPI * k;
    const T al = xs[0][R], ar = xs[1][R];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      if (has_left) p[e] += gl[k][e] * al;
      p[e] += gr[k][e] * ar;
    }
  }
  T r[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) r[e] = xs[2][VEC * q + e] - column_group_sum<QPR>(p[e]);
  wave_lds_fence();
  if (mrow == 0) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) xs[0][VEC * q + e] = r[e];
  }
  wave_lds_fence();
  // x_j = L_jj^{-T} r: sum over rows R >= c of L^{-1}[R][c] r[R]
  T x[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) x[e] = T(0);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int R = mrow + RPI * k;
    const T rr = xs[0][R];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      if (VEC * q + e <= R) x[e] += li[k][e] * rr;
  }
#pragma unroll
  for (int e = 0; e < VEC; ++e) x[e] = column_group_sum<QPR>(x[e]);
  if (mrow == 0) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int c = VEC * q + e;
      yj[c] = x[e];
      const size_t idx = off + c;
      const double d = static_cast<double>(x[e]);
      if (a.accumulate) {
        const double dd = a.rnorm[sys * a.seg_sys] * d;
        a.x[idx] = xo[e] + dd;
        a.dstore[idx] = dd;
      } else {
        a.x[idx] = d;
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(64) solve_bwd_rows_kernel(SolveArgs a, int level) {
  if (a.done && *a.done) return;
  __shared__ T xs[3][32];
  bwd_rows_position<T>(a, level, blockIdx.x, blockIdx.y, blockIdx.z, xs);
}

// The top backward levels of every chain in one launch: one workgroup per chain (grid
// y: system), wave w solves position w of each level from the top level down to
// level_lo (at most kBwdTopWaves positions per level), with a barrier between levels.
// A position reads the x of its neighbours from y, written by other waves of the
// workgroup at higher levels; the barrier orders those stores before the reads (the
// waves of a workgroup share one CU and its vector cache).  Each position runs the code
// of the single-level kernel (row reads at n = 32, one wave of the general one-vector
// kernel otherwise), so the results are bitwise those of the launches level by level.
template <typename T, int NMAX>
__device__ __attribute__((always_inline)) inline void solve_bwd_top_body(const SolveArgs& a,
                                                                         int level_lo,
                                                                         unsigned bx,
                                                                         unsigned by) {
  if (a.done && *a.done) return;
  constexpr int PER = NMAX == 32 ? 3 * NMAX : (kPullsPerWave + 2) * NMAX;  // per wave
  __shared__ __align__(16) T sm[kBwdTopWaves * PER];
  const int w = threadIdx.x >> 6;
  for (int level = chain_levels(a.m); level >= level_lo; --level) {
    if (w < level_count(a.m, level)) {
      if constexpr (NMAX == 32)
        bwd_rows_position<T>(a, level, w, bx, by,
                             reinterpret_cast<T(*)[NMAX]>(sm + w * PER));
      else
        level_one_position<T, NMAX, false>(a, level, w, bx, by, 1, 0,
                                           reinterpret_cast<unsigned char*>(sm + w * PER));
    }
    __syncthreads();
  }
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(64 * kBwdTopWaves) solve_bwd_top_kernel(SolveArgs a,
                                                                          int level_lo) {
  solve_bwd_top_body<T, NMAX>(a, level_lo, blockIdx.x, blockIdx.y);
}

template <typename T, int NMAX>
__device__ __attribute__((always_inline)) inline void solve_x_fwd_body(const SolveArgs& a,
                                                                  unsigned bx) {
  if (a.done && *a.done) return;
  typedef RegBlock<T, NMAX> RB;
  __shared__ SolveSmem<T, NMAX> sm;
  const int n = a.n, N = a.N, nrhs = a.nrhs, m = a.m;
  const size_t nn = (size_t)n * n;
  const int s = bx;
  const size_t gstride = g_chain_blocks(N);
  const T* Gr = reinterpret_cast<const T*>(a.Gr) + (size_t)s * gstride * nn;
  const T* Linv = reinterpret_cast<const T*>(a.Linv) + (size_t)s * N * nn;
  T* y = reinterpret_cast<T*>(a.y) + (size_t)s * N * nrhs * n;

  RB lin, fb;
  lin.template load_packed<false>(Linv + (size_t)(N - 1) * nn, n);
  fb.template load<false>(reinterpret_cast<const T*>(a.F) + (size_t)s * nn, n);
  gather_rhs<T, NMAX>(a, sm.rhs, vec_off(a, s, 0), seg_of(a, s));
  T part[kMaxRhs];
#pragma unroll
  for (int q = 0; q < kMaxRhs; ++q) part[q] = T(0);
  // The last position of level t+1 has X as its right neighbour iff floor(m/2^t) is odd.
  auto pull = [&](int t, const T*& blk, const T*& vec) -> bool {
    if (((m >> t) & 1) == 0) return false;
    const int c = (m >> t) << t;
    blk = Gr + (size_t)(c - 1) * nn;
    vec = y + (size_t)(c - 1) * nrhs * n;
    return true;
  };
  pull_products<T, NMAX, false>(chain_levels(m), pull, n, nrhs, sm.vbuf, part);
  __syncthreads();
  subtract_reduced<T, NMAX>(sm.rhs, part, nrhs);
  __syncthreads();
  T* yx = y + (size_t)(N - 1) * nrhs * n;
#pragma unroll
  for (int q = 0; q < kMaxRhs; ++q) {
    if (q < nrhs) {
      const T v = lane_group_sum<RB::LPR>(lin.dot(sm.rhs[q]));
      if (RB::base() == 0 && RB::out_index() < n) {
        yx[q * n + RB::out_index()] = v;
        sm.vbuf[0][q][RB::out_index()] = v;
      }
    }
  }
  __syncthreads();
  // w_s = F_s y_X in FP64 (the root reduction input of Algorithm 2)
  const int b = RB::base(), o = RB::out_index();
#pragma unroll
  for (int q = 0; q < kMaxRhs; ++q) {
    if (q < nrhs) {
      double p = 0.0;
#pragma unroll
      for (int e = 0; e < RB::EPL; ++e)
        p += static_cast<double>(fb.v[e]) * static_cast<double>(sm.vbuf[0][q][b + e]);
      p = lane_group_sum<RB::LPR>(p);
      if (b == 0 && o < n) a.w[((size_t)s * nrhs + q) * n + o] = p;
    }
  }
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(NT) solve_x_fwd_kernel(SolveArgs a) {
  solve_x_fwd_body<T, NMAX>(a, blockIdx.x);
}

// Root step in FP64 (Algorithm 2, root step).  One workgroup of 1024 threads per
// system of the batch:
// r~_0 = r_0 - sum_s w_s with thread (g, i) summing the scenarios s = g mod G of
// element i (G = 1024 / NMAX groups) and the G group partials combined in order; then
// the two triangular solves with L_R in LDS, one wave per right-hand side, lane i
// owning row i.
template <int NMAX>
__device__ __attribute__((always_inline)) inline void solve_root_body(const SolveArgs& a,
                                                                      unsigned bx) {
  if (a.done && *a.done) return;
  constexpr int G = 1024 / NMAX, LD = NMAX + 1;
  __shared__ double part[G][LD];
  __shared__ double L[NMAX * LD];
  __shared__ double r0[kMaxRhs][NMAX];
  const int n = a.n, S = a.S, nrhs = a.nrhs;
  const int sys = bx;
  const size_t len = vec_len(a);
  const size_t root_off = (size_t)sys * a.vsys + (size_t)S * a.N * n;
  const int seg0 = sys * a.seg_sys;
  const double* w = a.w + (size_t)sys * S * nrhs * n;  // this system's chains
  const int t = threadIdx.x, i = t % NMAX, g = t / NMAX;
  for (int e = t; e < NMAX * NMAX; e += 1024) {
    const int r = e / NMAX, c = e % NMAX;
    L[r * LD + c] = (r < n && c < n) ? a.LR[(size_t)sys * n * n + r * n + c]
                                     : (r == c ? 1.0 : 0.0);  // identity padding
  }
  for (int q = 0; q < nrhs; ++q) {
    double acc = 0.0;
    if (i < n) {
      constexpr int B = 8;
      for (int s0 = g; s0 < S; s0 += G * B) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const int sc = s0 + G * u;
          v[u] = sc < S ? w[((size_t)sc * nrhs + q) * n + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) acc += v[u];
      }
    }
    part[g][i] = acc;
    __syncthreads();
    if (t < n) {
      double sum = 0.0;
      for (int gg = 0; gg < G; ++gg) sum += part[gg][t];
      double bv = a.b[(size_t)q * len + root_off + t];
      if (a.rnorm) {
        const double rn = a.rnorm[seg0 + q];
        bv = rn > 0.0 ? bv / rn : 0.0;
      }
      r0[q][t] = bv - sum;
    }
    __syncthreads();
  }
  // L_R y = r, then L_R^T x = y: wave q handles right-hand side q, lane k row k.  L is
  // identity padded to NMAX x NMAX, so both sweeps run NMAX unrolled steps (the padded
  // unknowns stay 0); each lane holds the row (forward) or column (backward) of L it
  // updates with, and 1 / L[k][k] is formed once per lane and broadcast with x_k.
  const int wv = t >> 6, lane = t & 63;
  if (wv < nrhs) {
    const int row = lane < NMAX ? lane : NMAX - 1;
    double v = (lane < n) ? r0[wv][lane] : 0.0;
    const double rd = 1.0 / L[row * LD + row];
    double lk[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) lk[k] = L[row * LD + k];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
      const double xk = wave_bcast(v, k) * wave_bcast(rd, k);
      v = (lane == k) ? xk : (lane > k ? v - lk[k] * xk : v);
    }
#pragma unroll
    for (int k = 0; k < NMAX; ++k) lk[k] = L[k * LD + row];
#pragma unroll
    for (int k = NMAX - 1; k >= 0; --k) {
      const double xk = wave_bcast(v, k) * wave_bcast(rd, k);
      v = (lane == k) ? xk : (lane < k ? v - lk[k] * xk : v);
    }
    if (lane < n) r0[wv][lane] = v;
  }
  __syncthreads();
  for (int idx = t; idx < n * nrhs; idx += 1024) {
    const int q = idx / n, ii = idx - (idx / n) * n;
    a.x0[(size_t)sys * nrhs * n + idx] = r0[q][ii];
    scatter_value(a, q, root_off + ii, seg0, r0[q][ii]);
  }
}

template <int NMAX>
__global__ void __launch_bounds__(1024) solve_root_kernel(SolveArgs a) {
  solve_root_body<NMAX>(a, blockIdx.x);
}

template <typename T, int NMAX>
__device__ __attribute__((always_inline)) inline void solve_x_bwd_body(const SolveArgs& a,
                                                                  unsigned bx) {
  if (a.done && *a.done) return;
  typedef RegBlock<T, NMAX> RB;
  __shared__ SolveSmem<T, NMAX> sm;
  __shared__ double x0s[kMaxRhs][NMAX];
  const int n = a.n, N = a.N, nrhs = a.nrhs;
  const size_t nn = (size_t)n * n;
  const int s = bx;
  const T* Linv = reinterpret_cast<const T*>(a.Linv) + (size_t)s * N * nn;
  T* yx = reinterpret_cast<T*>(a.y) + ((size_t)s * N + (N - 1)) * nrhs * n;
  RB lin, fb;
  lin.template load_packed<true>(Linv + (size_t)(N - 1) * nn, n);
  fb.template load<true>(reinterpret_cast<const T*>(a.F) + (size_t)s * nn, n);
  for (int idx = threadIdx.x; idx < nrhs * NMAX; idx += NT) {
    const int q = idx / NMAX, i = idx % NMAX;
    x0s[q][i] = i < n ? a.x0[((size_t)(s / a.S) * nrhs + q) * n + i] : 0.0;
    sm.rhs[q][i] = i < n ? yx[q * n + i] : T(0);
  }
  __syncthreads();
  // dy_X -= F^T x_0 (root propagation of Algorithm 2), product in FP64
  const int b = RB::base(), o = RB::out_index();
#pragma unroll
  for (int q = 0; q < kMaxRhs; ++q) {
    if (q < nrhs) {
      double p = 0.0;
#pragma unroll
      for (int e = 0; e < RB::EPL; ++e) p += static_cast<double>(fb.v[e]) * x0s[q][b + e];
      p = lane_group_sum<RB::LPR>(p);
      if (b == 0) sm.rhs[q][o] = static_cast<T>(static_cast<double>(sm.rhs[q][o]) - p);
    }
  }
  __syncthreads();
  const size_t off = vec_off(a, s, 0);
  const int seg0 = seg_of(a, s);
#pragma unroll
  for (int q = 0; q < kMaxRhs; ++q) {
    if (q < nrhs) {
      const T v = lane_group_sum<RB::LPR>(lin.dot(sm.rhs[q]));
      if (b == 0 && o < n) {
        yx[q * n + o] = v;
        scatter_value(a, q, off + o, seg0, static_cast<double>(v));
      }
    }
  }
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(NT) solve_x_bwd_kernel(SolveArgs a) {
  solve_x_bwd_body<T, NMAX>(a, blockIdx.x);
}

// ---- one launch over the systems of a ragged batch (see multi.h) ----
// Items of the level kinds carry (level, count) in p0, p1; the merged backward top
// levels carry level_lo in p0.

__device__ inline SolveArgs relocate_solve(const SolveArgs& t, const Reloc& r) {
  SolveArgs a = t;
  a.b = rel(r.b, t.b);
  a.x = rel(r.x, t.x);
  a.dstore = rel(r.r, t.dstore);
  return a;
}

template <typename T, int NMAX, bool FWD, bool FULL>
__global__ void __launch_bounds__(64 * kLevelMaxWaves) solve_level_multi(
    const MultiItem<SolveArgs>* items, int nitems, Reloc r) {
  const MultiItem<SolveArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  const SolveArgs a = relocate_solve(it.a, r);
  solve_level_body<T, NMAX, FWD, FULL>(a, it.p0, it.p1, multi_local(it).x);
}

template <typename T, int NMAX, bool FWD>
__global__ void __launch_bounds__(64 * kLevelMaxWaves) solve_level_one_multi(
    const MultiItem<SolveArgs>* items, int nitems, Reloc r) {
  const MultiItem<SolveArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  const SolveArgs a = relocate_solve(it.a, r);
  if (a.done && *a.done) return;
  extern __shared__ __align__(16) unsigned char level_smem[];
  const LocalBlock lb = multi_local(it);
  level_one_position<T, NMAX, FWD>(a, it.p0, lb.x, lb.y, lb.z, (int)(blockDim.x >> 6),
                                   (int)(threadIdx.x >> 6), level_smem);
}

template <typename T>
__global__ void __launch_bounds__(64) solve_bwd_rows_multi(const MultiItem<SolveArgs>* items,
                                                           int nitems, Reloc r) {
  const MultiItem<SolveArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  const SolveArgs a = relocate_solve(it.a, r);
  if (a.done && *a.done) return;
  __shared__ T xs[3][32];
  const LocalBlock lb = multi_local(it);
  bwd_rows_position<T>(a, it.p0, lb.x, lb.y, lb.z, xs);
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(64 * kBwdTopWaves) solve_bwd_top_multi(
    const MultiItem<SolveArgs>* items, int nitems, Reloc r) {
  const MultiItem<SolveArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  const SolveArgs a = relocate_solve(it.a, r);
  const LocalBlock lb = multi_local(it);
  solve_bwd_top_body<T, NMAX>(a, it.p0, lb.x, lb.y);
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(NT) solve_x_fwd_multi(const MultiItem<SolveArgs>* items,
                                                        int nitems, Reloc r) {
  const MultiItem<SolveArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  solve_x_fwd_body<T, NMAX>(relocate_solve(it.a, r), multi_local(it).x);
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(NT) solve_x_bwd_multi(const MultiItem<SolveArgs>* items,
                                                        int nitems, Reloc r) {
  const MultiItem<SolveArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  solve_x_bwd_body<T, NMAX>(relocate_solve(it.a, r), multi_local(it).x);
}

template <int NMAX>
__global__ void __launch_bounds__(1024) solve_root_multi(const MultiItem<SolveArgs>* items,
                                                         int nitems, Reloc r) {
  const MultiItem<SolveArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  solve_root_body<NMAX>(relocate_solve(it.a, r), multi_local(it).x);
}

template <typename T, int NMAX>
void solve_multi_t(int kind, bool fwd, bool full, const MultiItem<SolveArgs>* items, int nitems,
                   unsigned blocks, unsigned threads, size_t lds, const Reloc& r, hipStream_t st) {
  const dim3 g(blocks), b(threads);
  switch (kind) {
    case SK_LEVEL:
      if (fwd && full)
        hipLaunchKernelGGL((solve_level_multi<T, NMAX, true, true>), g, b, lds, st, items, nitems, r);
      else if (fwd)
        hipLaunchKernelGGL((solve_level_multi<T, NMAX, true, false>), g, b, lds, st, items, nitems, r);
      else if (full)
        hipLaunchKernelGGL((solve_level_multi<T, NMAX, false, true>), g, b, lds, st, items, nitems, r);
      else
        hipLaunchKernelGGL((solve_level_multi<T, NMAX, false, false>), g, b, lds, st, items, nitems, r);
      break;
    case SK_LEVEL_ONE:
      if (fwd)
        hipLaunchKernelGGL((solve_level_one_multi<T, NMAX, true>), g, b, lds, st, items, nitems, r);
      else
        hipLaunchKernelGGL((solve_level_one_multi<T, NMAX, false>), g, b, lds, st, items, nitems, r);
      break;
    case SK_BWD_ROWS:
      if constexpr (NMAX == 32)
        hipLaunchKernelGGL((solve_bwd_rows_multi<T>), g, b, 0, st, items, nitems, r);
      break;
    case SK_BWD_TOP:
      hipLaunchKernelGGL((solve_bwd_top_multi<T, NMAX>), g, b, 0, st, items, nitems, r);
      break;
    case SK_X_FWD:
      hipLaunchKernelGGL((solve_x_fwd_multi<T, NMAX>), g, b, 0, st, items, nitems, r);
      break;
    case SK_X_BWD:
      hipLaunchKernelGGL((solve_x_bwd_multi<T, NMAX>), g, b, 0, st, items, nitems, r);
      break;
    case SK_ROOT:
      hipLaunchKernelGGL((solve_root_multi<32>), g, b, 0, st, items, nitems, r);
      break;
  }
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
void level_t(const SolveArgs& a, int level, bool fwd, hipStream_t st) {
  const LevelCfg c = solve_level_config(a, level, fwd, NMAX, sizeof(T) == 8);
  if (c.count <= 0) return;
  const dim3 g(c.gx, c.gy, c.gz), b(c.threads);
  switch (c.kind) {
    case SK_BWD_ROWS:
      if constexpr (NMAX == 32) hipLaunchKernelGGL((solve_bwd_rows_kernel<T>), g, b, 0, st, a, level);
      break;
    case SK_LEVEL_ONE:
      if (fwd)
        hipLaunchKernelGGL((solve_level_one_kernel<T, NMAX, true>), g, b, c.lds, st, a, level);
      else
        hipLaunchKernelGGL((solve_level_one_kernel<T, NMAX, false>), g, b, c.lds, st, a, level);
      break;
    default:
      if (fwd && c.full)
        hipLaunchKernelGGL((solve_level_kernel<T, NMAX, true, true>), g, b, c.lds, st, a, level, c.count);
      else if (fwd)
        hipLaunchKernelGGL((solve_level_kernel<T, NMAX, true, false>), g, b, c.lds, st, a, level, c.count);
      else if (c.full)
        hipLaunchKernelGGL((solve_level_kernel<T, NMAX, false, true>), g, b, c.lds, st, a, level, c.count);
      else
        hipLaunchKernelGGL((solve_level_kernel<T, NMAX, false, false>), g, b, c.lds, st, a, level, c.count);
  }
}
template <typename T, int NMAX>
void fwd_level_t(const SolveArgs& a, int level, hipStream_t st) {
  level_t<T, NMAX>(a, level, true, st);
}
template <typename T, int NMAX>
void bwd_level_t(const SolveArgs& a, int level, hipStream_t st) {
  level_t<T, NMAX>(a, level, false, st);
}
template <typename T, int NMAX>
void x_fwd_t(const SolveArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((solve_x_fwd_kernel<T, NMAX>), dim3(a.B * a.S), dim3(NT), 0, st, a);
}
template <typename T, int NMAX>
void x_bwd_t(const SolveArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((solve_x_bwd_kernel<T, NMAX>), dim3(a.B * a.S), dim3(NT), 0, st, a);
}

}  // namespace

// Kernel, grid and LDS of one level of a sweep (n <= 32).  One right-hand side with
// full blocks and a grid of (positions, scenarios, systems) within the y and z launch
// limits takes the one-vector kernels (row reads for the backward sweep at n = 32),
// everything else the general level kernel on a flat grid.  Forward positions of level
// l pull 2 (l - 1) blocks, kPullsPerWave per wave, on up to kLevelMaxWaves waves (or
// a.fwd_waves: one wave per position when the plan asks for it).
LevelCfg solve_level_config(const SolveArgs& a, int level, bool fwd, int nmax, bool fp64) {
  LevelCfg c{};
  c.count = level_count(a.m, level);
  const bool one = a.nrhs == 1 && a.n == nmax && a.S <= 65535 && a.B <= 65535;
  int waves = 1;
  if (fwd) {
    const int pulls = 2 * (level - 1);
    const int cap = a.fwd_waves > 0 ? std::min(a.fwd_waves, kLevelMaxWaves) : kLevelMaxWaves;
    waves = std::max(1, std::min(cap, (pulls + kPullsPerWave - 1) / kPullsPerWave));
  }
  c.threads = 64 * waves;
  c.lds = solve_level_lds(fp64, nmax, waves, a.nrhs);
  c.full = a.n == nmax;
  if (one) {
    c.kind = (!fwd && nmax == 32) ? SK_BWD_ROWS : SK_LEVEL_ONE;
    if (c.kind == SK_BWD_ROWS) c.lds = 0;
    c.gx = (unsigned)c.count;
    c.gy = (unsigned)a.S;
    c.gz = (unsigned)a.B;
  } else {
    c.kind = SK_LEVEL;
    c.gx = (unsigned)(a.B * a.S) * (unsigned)std::max(c.count, 0);
    c.gy = c.gz = 1;
  }
  return c;
}

template <typename T>
void launch_solve_fwd_level(const SolveArgs& a, int level, int nmax, hipStream_t st) {
  if (nmax > 32) return launch_solve64_level<T>(a, level, true, st);
  BMPC_DISPATCH_NMAX(nmax, fwd_level_t, a, level, st);
}
template <typename T>
void launch_solve_bwd_level(const SolveArgs& a, int level, int nmax, hipStream_t st) {
  if (nmax > 32) return launch_solve64_level<T>(a, level, false, st);
  BMPC_DISPATCH_NMAX(nmax, bwd_level_t, a, level, st);
}
template <typename T>
void launch_solve_bwd_top(const SolveArgs& a, int level_lo, hipStream_t st) {
  const int waves = level_count(a.m, level_lo);
  if (waves < 1 || waves > kBwdTopWaves) return;
  const dim3 grid(a.S, a.B), block(64 * waves);
  if (a.n == 32)
    hipLaunchKernelGGL((solve_bwd_top_kernel<T, 32>), grid, block, 0, st, a, level_lo);
  else if (a.n == 16)
    hipLaunchKernelGGL((solve_bwd_top_kernel<T, 16>), grid, block, 0, st, a, level_lo);
  else if (a.n == 8)
    hipLaunchKernelGGL((solve_bwd_top_kernel<T, 8>), grid, block, 0, st, a, level_lo);
}
template <typename T>
void launch_solve_x_fwd(const SolveArgs& a, int nmax, hipStream_t st) {
  if (nmax > 32) return launch_solve64_x<T>(a, true, st);
  BMPC_DISPATCH_NMAX(nmax, x_fwd_t, a, st);
}
template <typename T>
void launch_solve_x_bwd(const SolveArgs& a, int nmax, hipStream_t st) {
  if (nmax > 32) return launch_solve64_x<T>(a, false, st);
  BMPC_DISPATCH_NMAX(nmax, x_bwd_t, a, st);
}
void launch_solve_root(const SolveArgs& a, hipStream_t st) {
  if (a.n > 32)
    hipLaunchKernelGGL(solve_root_kernel<64>, dim3(a.B), dim3(1024), 0, st, a);
  else
    hipLaunchKernelGGL(solve_root_kernel<32>, dim3(a.B), dim3(1024), 0, st, a);
}

size_t solve_level_lds(bool fp64, int nmax, int waves, int nrhs) {
  return fp64 ? (nmax <= 8 ? level_smem_bytes<double, 8>(waves, nrhs)
                          : nmax <= 16 ? level_smem_bytes<double, 16>(waves, nrhs)
                                       : level_smem_bytes<double, 32>(waves, nrhs))
              : (nmax <= 8 ? level_smem_bytes<float, 8>(waves, nrhs)
                           : nmax <= 16 ? level_smem_bytes<float, 16>(waves, nrhs)
                                        : level_smem_bytes<float, 32>(waves, nrhs));
}

template <typename T>
void launch_solve_multi(int kind, bool fwd, bool full, int nmax,
                        const MultiItem<SolveArgs>* items, int nitems, unsigned blocks,
                        unsigned threads, size_t lds, const Reloc& r, hipStream_t st) {
  if (nmax <= 8)
    solve_multi_t<T, 8>(kind, fwd, full, items, nitems, blocks, threads, lds, r, st);
  else if (nmax <= 16)
    solve_multi_t<T, 16>(kind, fwd, full, items, nitems, blocks, threads, lds, r, st);
  else
    solve_multi_t<T, 32>(kind, fwd, full, items, nitems, blocks, threads, lds, r, st);
}
template void launch_solve_multi<double>(int, bool, bool, int, const MultiItem<SolveArgs>*, int,
                                         unsigned, unsigned, size_t, const Reloc&, hipStream_t);
template void launch_solve_multi<float>(int, bool, bool, int, const MultiItem<SolveArgs>*, int,
                                        unsigned, unsigned, size_t, const Reloc&, hipStream_t);

template void launch_solve_fwd_level<double>(const SolveArgs&, int, int, hipStream_t);
template void launch_solve_fwd_level<float>(const SolveArgs&, int, int, hipStream_t);
template void launch_solve_bwd_level<double>(const SolveArgs&, int, int, hipStream_t);
template void launch_solve_bwd_level<float>(const SolveArgs&, int, int, hipStream_t);
template void launch_solve_bwd_top<double>(const SolveArgs&, int, hipStream_t);
template void launch_solve_bwd_top<float>(const SolveArgs&, int, hipStream_t);
template void launch_solve_x_fwd<double>(const SolveArgs&, int, hipStream_t);
template void launch_solve_x_fwd<float>(const SolveArgs&, int, hipStream_t);
template void launch_solve_x_bwd<double>(const SolveArgs&, int, hipStream_t);
template void launch_solve_x_bwd<float>(const SolveArgs&, int, hipStream_t);

}  // namespace bmpc
