// Mixed-precision iterative refinement support (FP64 residual r = b - K x).
//
// The residual is formed from the caller's FP64 blocks exactly as K is defined in
// eq. (root_coupled_matrix) / eq. (tail_block_tridiagonal): row block (s,k) of a
// tail is D_{s,k} x_{s,k} + E_{s,k-1} x_{s,k-1} + E_{s,k}^T x_{s,k+1} (+ C_s^T x_0
// for k = 0); the root row block is R x_0 + sum_s C_s x_{s,0}, with the sum over s
// taken in scenario order.  One wave walks a chunk of consecutive stages of one tail,
// so each E block is fetched from HBM once and used for both rows it touches; the
// blocks of the next stage are loaded while the current one is applied.  Infinity
// norms are maxima taken by a two-stage reduction (per-block partial maxima, then
// one block), so they are deterministic and need no atomics.
#include "bmpc_internal.h"
#include "multi.h"
#include "regblock.h"

namespace bmpc {

namespace {

// One 256-thread workgroup walks a chunk of consecutive stages of one tail.  The
// blocks of a stage (the lower triangle of D, all of E) are read with coalesced 8-byte
// loads into registers two stages ahead, together with the x of the next stage and the
// b of the stage, then staged in double-buffered LDS, where the symmetric product with
// D and the product with E^T read them transposed; so each E block leaves HBM once and
// serves both rows it touches.  Nothing fetched ahead is used before the step that
// needs it, so the loads of two stages stay in flight while a stage is applied.  Row o
// of the stage's result is summed by RT = min(256 / NMAX, NMAX) threads, each over
// NMAX / RT columns (at NMAX = 8 only the first 64 threads have a row).
constexpr int RES_T = 256;

// LDS of a residual workgroup: Ds[2][NMAX][NMAX+1] (D of stage k in Ds[k & 1]),
// Es[2][NMAX][NMAX+1] (E of stage k in Es[k & 1]; C in Es[1] at stage 0), then
// xs[3][nrhs][NMAX], x0s[nrhs][NMAX], bs[2][nrhs][NMAX], rs[nrhs][NMAX] and
// ws[nrhs][NMAX] (dynamic, sized by nrhs).
template <int NMAX>
inline size_t residual_lds_bytes(int nrhs) {
  return (size_t)(4 * NMAX * (NMAX + 1) + 8 * nrhs * NMAX) * sizeof(double);
}

// The blocks and vectors of one stage k, in registers: D_k (lower triangle), E_k (if
// k + 1 < N), x_{k+1} and b_k.  With FULL (n == NMAX) the blocks are read through a
// buffer resource (entries above the diagonal of D at an out-of-range offset, so they
// read as zero and are not fetched); vector lanes past the data read a clamped
// in-range element.  commit() writes the stage into LDS, zero padded, so the LDS copy
// never holds stale values.
template <int NMAX, bool FULL>
struct StageFetch {
  static constexpr int PER = (NMAX * NMAX + RES_T - 1) / RES_T;
  static constexpr int VPER = (rhs_chunk(NMAX) * NMAX + RES_T - 1) / RES_T;
  double d[PER], e[PER], xv[VPER], bv[VPER];

  // Element of the block held in v[u]: with PAIRS, v[2h] and v[2h+1] are two
  // consecutive elements of a row, read by one 16-byte load.
  static constexpr bool PAIRS = FULL && NMAX * NMAX % (2 * RES_T) == 0;
  __device__ static int elem(int u) {
    if constexpr (PAIRS)
      return 2 * ((int)threadIdx.x + (u >> 1) * RES_T) + (u & 1);
    else
      return (int)threadIdx.x + u * RES_T;
  }

  // A block that does not exist (exists = false) is read as zero without a memory
  // access, so every fetch issues the same loads.
  template <bool LOWER>
  __device__ static void block(double (&v)[PER], const double* __restrict__ g, int n,
                               bool exists) {
    if constexpr (PAIRS) {
      // pairs past the diagonal of a lower triangle are not fetched; a pair that starts
      // on the diagonal brings one entry above it, which is never read
      const auto rs = block_rsrc(g, exists ? (unsigned)(NMAX * NMAX) * 8u : 0u);
#pragma unroll
      for (int h = 0; h < PER / 2; ++h) {
        const int el = elem(2 * h);
        const int r = el / NMAX, c = el % NMAX;
        const bool ok = !LOWER || c <= r;
        const auto w = __builtin_amdgcn_raw_buffer_load_b128(rs, ok ? (unsigned)el * 8u
                                                                    : kOutOfRange, 0, 0);
        __builtin_memcpy(&v[2 * h], &w, 16);
      }
    } else if constexpr (FULL) {
      const auto rs = block_rsrc(g, exists ? (unsigned)(NMAX * NMAX) * 8u : 0u);
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int el = threadIdx.x + u * RES_T;
        const int r = el / NMAX, c = el % NMAX;
        const bool ok = el < NMAX * NMAX && (!LOWER || c <= r);
        v[u] = buf_load_f64(rs, ok ? (unsigned)el * 8u : kOutOfRange);
      }
    } else {
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int el = threadIdx.x + u * RES_T;
        const int r = el / NMAX, c = el % NMAX;
        const bool ok = exists && el < NMAX * NMAX && r < n && c < n && (!LOWER || c <= r);
        v[u] = ok ? g[r * n + c] : 0.0;
      }
    }
  }
  __device__ static void put(double* dst, const double (&v)[PER]) {
    constexpr int LD = NMAX + 1;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int el = elem(u);
      if (el < NMAX * NMAX) dst[(el / NMAX) * LD + el % NMAX] = v[u];
    }
  }
  // xk = offset of stage 0 of the chain's vectors (right-hand side 0).  Stages at or
  // past k1 (the end of the chunk) fetch nothing from the blocks and clamped vectors.
  __device__ void issue(const ResidualArgs& a, const double* Dc, const double* Ec, size_t xk,
                        size_t len, int k, int k1) {
    static_assert(VPER == 1, "one vector element per thread");
    const int n = a.n, N = a.N, nrhs = a.nrhs;
    const size_t nn = (size_t)n * n;
    const int kc = min(k, N - 1);
    block<true>(d, Dc + (size_t)kc * nn, n, k < k1);
    block<false>(e, Ec + (size_t)min(kc, N - 2 < 0 ? 0 : N - 2) * nn, n, k < k1 && k + 1 < N);
    const int idx = threadIdx.x;
    const int q = min(idx / NMAX, nrhs - 1), i = min(idx % NMAX, n - 1);
    const size_t base = xk + (size_t)q * len + i;
    xv[0] = a.x[base + (size_t)min(k + 1, N - 1) * n];
    bv[0] = a.b[base + (size_t)kc * n];
  }
  // stage k into D/E slots, x_{k+1} into xslot, b_k into bslot
  __device__ void commit(const ResidualArgs& a, int k, double* Dsl, double* Esl, double* xslot,
                         double* bslot) const {
    const int n = a.n, N = a.N, nrhs = a.nrhs;
    put(Dsl, d);
    if (k + 1 < N) put(Esl, e);
    const int idx = threadIdx.x;
    if (idx < nrhs * NMAX) {
      const bool ok = idx % NMAX < n;
      xslot[idx] = ok && k + 1 < N ? xv[0] : 0.0;
      bslot[idx] = ok ? bv[0] : 0.0;
    }
  }
};

template <int NMAX, bool FULL>
__device__ __attribute__((always_inline)) inline void residual_body(const ResidualArgs& a,
                                                                    int chunks, unsigned bx) {
  if (a.done && *a.done) return;
  constexpr int LD = NMAX + 1;
  constexpr int BS = NMAX * LD;
  constexpr int RT = RES_T / NMAX < NMAX ? RES_T / NMAX : NMAX;  // threads per row
  constexpr int CPT = NMAX / RT;                                 // columns per thread
  static_assert(CPT >= 1 && RT * CPT == NMAX, "row split");
  typedef StageFetch<NMAX, FULL> SF;
  extern __shared__ __align__(16) double res_lds[];
  const int n = a.n, N = a.N, S = a.S, nrhs = a.nrhs;
  const int VS = nrhs * NMAX;          // one vector slot
  double* Ds = res_lds;                // [2][BS]
  double* Es = res_lds + 2 * BS;       // [2][BS]
  double* xs = res_lds + 4 * BS;       // [3][nrhs][NMAX]
  double* x0s = xs + 3 * VS;           // [nrhs][NMAX]
  double* bs = x0s + VS;               // [2][nrhs][NMAX]
  double* rs = bs + 2 * VS;            // [nrhs][NMAX] residual of the current stage
  double* ws = rs + VS;                // [nrhs][NMAX] C_s x_{s,0} (stage 0)
  const size_t nn = (size_t)n * n;
  const size_t len = ((size_t)S * N + 1) * n;
  const int s = bx / chunks;  // chain of the batch
  const int ch = bx - s * chunks;
  const int sys = s / S, sl = s - sys * S;
  const size_t vbase = (size_t)sys * a.vsys;
  const size_t xk = vbase + (size_t)sl * N * n;  // stage 0 of this chain, q = 0
  const int k0 = ch * a.chunk, k1 = min(N, k0 + a.chunk);
  const double* Dc = a.D + (size_t)s * N * nn;
  const double* Ec = a.E + (size_t)s * (N > 1 ? N - 1 : 0) * nn;
  const int t = threadIdx.x, orow = t / RT, p = t - orow * RT;
  const int o = orow < NMAX ? orow : 0;  // rows past NMAX (NMAX = 8) compute row 0, unused
  double kmax = 0.0;  // largest row sum of |K| over this workgroup's rows (knorm_part)

  // Prologue: stage k0 with x_{k0+1} and b_{k0}, E_{k0-1} (or C_s at k0 = 0), x_{k0-1},
  // x_{k0} and (k0 = 0) the root x, all straight into LDS.
  {
    SF f0;
    double pv[SF::PER];
    f0.issue(a, Dc, Ec, xk, len, k0, k1);
    if (k0 > 0)
      SF::template block<false>(pv, Ec + (size_t)(k0 - 1) * nn, n, true);
    else
      SF::template block<false>(pv, a.C + (size_t)s * nn, n, true);
    for (int idx = t; idx < VS; idx += RES_T) {
      const int q = idx / NMAX, i = idx % NMAX;
      const size_t b0 = xk + (size_t)q * len + i;
      xs[((k0 + 2) % 3) * VS + idx] = (k0 > 0 && i < n) ? a.x[b0 + (size_t)(k0 - 1) * n] : 0.0;
      xs[(k0 % 3) * VS + idx] = i < n ? a.x[b0 + (size_t)k0 * n] : 0.0;
      if (k0 == 0)
        x0s[idx] = i < n ? a.x[vbase + (size_t)q * len + (size_t)S * N * n + i] : 0.0;
    }
    f0.commit(a, k0, Ds + (k0 & 1) * BS, Es + (k0 & 1) * BS, xs + ((k0 + 1) % 3) * VS,
              bs + (k0 & 1) * VS);
    SF::put(Es + ((k0 + 1) & 1) * BS, pv);
  }
  // Two stages in flight: fa holds stage k+1 and fb stage k+2 when step k starts.  Every
  // step issues the same loads (past the chunk they fetch nothing) and stores its
  // residual after the next fetch is issued, so the wait for a stage covers only the
  // loads issued before it.
  SF fa, fb;
  fa.issue(a, Dc, Ec, xk, len, k0 + 1, k1);
  __builtin_amdgcn_sched_barrier(0);  // keep stage k0+1 ahead of k0+2 in the load queue
  fb.issue(a, Dc, Ec, xk, len, k0 + 2, k1);
  auto step = [&](int k, SF& f) {
    __syncthreads();
    if (k < k1) {
      const double* D = Ds + (k & 1) * BS;
      const double* Ek = Es + (k & 1) * BS;
      const double* Ep = Es + ((k + 1) & 1) * BS;  // E of stage k-1 (or C at k = 0)
      const double* xm = xs + ((k + 2) % 3) * VS;
      const double* xkk = xs + (k % 3) * VS;
      const double* xp = xs + ((k + 1) % 3) * VS;
      const double* bk = bs + (k & 1) * VS;
      const bool has_prev = k > 0, has_next = k + 1 < N;
#pragma unroll 1
      for (int q = 0; q < nrhs; ++q) {
        double acc = 0.0, accw = 0.0;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
          const int c = p * CPT + u;
          const double dv = c <= o ? D[o * LD + c] : D[c * LD + o];
          acc += dv * xkk[q * NMAX + c];
          if (has_prev) acc += Ep[o * LD + c] * xm[q * NMAX + c];  // E_{k-1} x_{k-1}
          if (has_next) acc += Ek[c * LD + o] * xp[q * NMAX + c];  // E_k^T x_{k+1}
          if (!has_prev) {                                        // k = 0: C^T x_0, C x_{s,0}
            acc += Ep[c * LD + o] * x0s[q * NMAX + c];
            accw += Ep[o * LD + c] * xkk[q * NMAX + c];
          }
        }
        acc = lane_group_sum_dpp<RT>(acc);
        if (p == 0 && orow < NMAX) rs[q * NMAX + o] = bk[q * NMAX + o] - acc;
        if (!has_prev) {
          accw = lane_group_sum_dpp<RT>(accw);
          if (p == 0 && orow < NMAX) ws[q * NMAX + o] = accw;
        }
      }
      if (a.knorm_part) {
        // row sums of |K| over the same entries (independent of the right-hand side):
        // the largest one goes into the norm; at stage 0 the rows of |C_s| are kept for
        // the root rows (zero padding adds nothing)
        double ab = 0.0, abc = 0.0;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
          const int c = p * CPT + u;
          ab += fabs(c <= o ? D[o * LD + c] : D[c * LD + o]);
          if (has_prev) ab += fabs(Ep[o * LD + c]);
          if (has_next) ab += fabs(Ek[c * LD + o]);
          if (!has_prev) {
            ab += fabs(Ep[c * LD + o]);
            abc += fabs(Ep[o * LD + c]);
          }
        }
        ab = lane_group_sum_dpp<RT>(ab);
        kmax = fmax(kmax, ab);
        if (!has_prev) {
          abc = lane_group_sum_dpp<RT>(abc);
          if (p == 0 && orow < n) a.crow[(size_t)s * n + o] = abc;
        }
      }
    }
    __syncthreads();
    f.commit(a, k + 1, Ds + ((k + 1) & 1) * BS, Es + ((k + 1) & 1) * BS,
             xs + ((k + 2) % 3) * VS, bs + ((k + 1) & 1) * VS);
    f.issue(a, Dc, Ec, xk, len, k + 3, k1);
    if (k < k1 && t < VS && t % NMAX < n) {
      const int q = t / NMAX, i = t % NMAX;
      a.r[xk + (size_t)q * len + (size_t)k * n + i] = rs[t];
      if (k == 0) a.w[((size_t)s * nrhs + q) * n + i] = ws[t];
    }
  };
  for (int k = k0; k < k1; k += 2) {
    step(k, fa);
    step(k + 1, fb);
  }
  if (a.knorm_part) {
    __shared__ double wmax[RES_T / 64];
    for (int off = 32; off > 0; off >>= 1) kmax = fmax(kmax, __shfl_xor(kmax, off));
    if ((t & 63) == 0) wmax[t >> 6] = kmax;
    __syncthreads();
    if (t == 0) {
      double m = 0.0;
      for (int i = 0; i < RES_T / 64; ++i) m = fmax(m, wmax[i]);
      a.knorm_part[bx] = m;
    }
  }
}

template <int NMAX, bool FULL>
__global__ void __launch_bounds__(RES_T) residual_kernel(ResidualArgs a, int chunks) {
  residual_body<NMAX, FULL>(a, chunks, blockIdx.x);
}

// One workgroup per system; thread (g, i) sums element i of the products C_s x_{s,0}
// over the scenarios s = g mod G (G = 1024 / NMAX groups), the groups in order.
template <int NMAX>
__device__ __attribute__((always_inline)) inline void residual_root_body(const ResidualArgs& a,
                                                                         unsigned bx) {
  if (a.done && *a.done) return;
  constexpr int G = 1024 / NMAX;
  __shared__ double part[G][NMAX + 1];
  const int n = a.n, N = a.N, S = a.S, nrhs = a.nrhs;
  const int sys = bx;  // one workgroup per system
  const size_t len = ((size_t)S * N + 1) * n;
  const size_t root = (size_t)sys * a.vsys + (size_t)S * N * n;
  const double* w = a.w + (size_t)sys * S * nrhs * n;
  const double* R = a.R + (size_t)sys * n * n;
  const int t = threadIdx.x, i = t % NMAX, g = t / NMAX;
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
      const int row = t;
      double sum = 0.0;
      for (int gg = 0; gg < G; ++gg) sum += part[gg][row];
      double rx = 0.0;
      for (int c = 0; c < n; ++c) {
        const double rv = (row >= c) ? R[row * n + c] : R[c * n + row];
        rx += rv * a.x[(size_t)q * len + root + c];
      }
      a.r[(size_t)q * len + root + row] = a.b[(size_t)q * len + root + row] - rx - sum;
    }
    __syncthreads();
  }
  if (a.knorm_root) {
    // root rows of |K|: the |C_s| row sums of the scenarios (G interleaved groups, each
    // in scenario order, then the groups in order, as the sum of w above), plus |R|
    const double* cr = a.crow + (size_t)sys * S * n;
    double acc = 0.0;
    if (i < n) {
      constexpr int B = 8;
      for (int s0 = g; s0 < S; s0 += G * B) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const int sc = s0 + G * u;
          v[u] = sc < S ? cr[(size_t)sc * n + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) acc += v[u];
      }
    }
    part[g][i] = acc;
    __syncthreads();
    double m = 0.0;
    if (t < n) {
      double sum = 0.0;
      for (int gg = 0; gg < G; ++gg) sum += part[gg][t];
      for (int c = 0; c < n; ++c) sum += fabs(t >= c ? R[t * n + c] : R[c * n + t]);
      m = sum;
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (t == 0) a.knorm_root[sys] = m;  // n <= 64: the rows sit in wave 0
  }
}

template <int NMAX>
__global__ void __launch_bounds__(1024) residual_root_kernel(ResidualArgs a) {
  residual_root_body<NMAX>(a, blockIdx.x);
}

// Maximum that propagates NaN (so a NaN residual or correction fails the stop test).
__device__ inline double nan_max(double a, double b) { return (a != a || a > b) ? a : b; }

__device__ inline double block_max(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_xor(v, off));
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wv] = v;
  __syncthreads();
  double m = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = nan_max(m, sh[i]);
  __syncthreads();
  return m;
}

// partial[t][q][blk] = max over this block's slice of |v_t[q][.]| (t = 0: v, 1: v2).
// Each thread keeps four independent loads in flight per iteration.
__global__ void __launch_bounds__(256) maxabs_partial_kernel(const double* v, const double* v2,
                                                             int nrhs, size_t len,
                                                             double* partial, const int* done) {
  if (done && *done) return;
  __shared__ double sh[4];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int t = 0; t < (v2 ? 2 : 1); ++t) {
    const double* src = t == 0 ? v : v2;
    for (int q = 0; q < nrhs; ++q) {
      const double* p = src + (size_t)q * len;
      double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
      size_t i = t0;
      for (; i + 3 * stride < len; i += 4 * stride) {
        const double a0 = p[i], a1 = p[i + stride], a2 = p[i + 2 * stride], a3 = p[i + 3 * stride];
        m0 = nan_max(fabs(a0), m0);
        m1 = nan_max(fabs(a1), m1);
        m2 = nan_max(fabs(a2), m2);
        m3 = nan_max(fabs(a3), m3);
      }
      for (; i < len; i += stride) m0 = nan_max(fabs(p[i]), m0);
      double mx = block_max(nan_max(nan_max(m0, m1), nan_max(m2, m3)), sh);
      if (threadIdx.x == 0) partial[((size_t)t * nrhs + q) * gridDim.x + blockIdx.x] = mx;
    }
  }
}

// max of the non-negative (or NaN) p[i] over i = t0, t0 + step, .. < cnt, 0 if none.
// U loads are issued together per round (indices clamped into range, the extra ones
// not counted), so that a thread waits once per round rather than once per load.
template <int U>
__device__ inline double strided_max(const double* p, int cnt, int t0, int step) {
  double m = 0.0;
  for (int i0 = t0; i0 < cnt; i0 += U * step) {
    double t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = p[min(i0 + u * step, cnt - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) m = i0 + u * step < cnt ? nan_max(t[u], m) : m;
  }
  return m;
}

// max over the block partials of one vector and right-hand side, on one wave
__device__ inline double wave_reduce_partials(const double* part, int blocks) {
  double mx = strided_max<16>(part, blocks, (int)threadIdx.x, 64);
  for (int off = 32; off > 0; off >>= 1) mx = nan_max(mx, __shfl_xor(mx, off));
  return mx;
}

__global__ void __launch_bounds__(64) maxabs_final_kernel(const double* partial, int blocks,
                                                          int nrhs, double* out,
                                                          const int* done) {
  if (done && *done) return;
  for (int q = 0; q < nrhs; ++q) {
    const double mx = wave_reduce_partials(partial + (size_t)q * blocks, blocks);
    if (threadIdx.x == 0) out[q] = mx;
  }
}

// flags[0] = done, flags[1] = corrections applied
__global__ void refine_reset_kernel(int* flags) {
  if (threadIdx.x == 0) {
    flags[0] = 0;
    flags[1] = 0;
  }
}

// |d|_inf and |x|_inf from the block partials, then the stop test
// |d_q|_inf <= tol |x_q|_inf for every right-hand side.
__global__ void __launch_bounds__(64) refine_check_kernel(const double* partial, int blocks,
                                                          int nrhs, double tol, int* flags,
                                                          double* relcorr, double* dnorm,
                                                          double* xnorm) {
  if (flags[0]) return;
  bool ok = true;
  double worst = 0.0;
  for (int q = 0; q < nrhs; ++q) {
    const double d = wave_reduce_partials(partial + (size_t)q * blocks, blocks);
    const double xv = wave_reduce_partials(partial + ((size_t)nrhs + q) * blocks, blocks);
    const double rel = xv > 0.0 ? d / xv : d;
    worst = nan_max(worst, rel);
    if (!(d <= tol * xv)) ok = false;
    if (threadIdx.x == 0) {
      dnorm[q] = d;
      xnorm[q] = xv;
    }
  }
  if (threadIdx.x == 0) {
    flags[1] += 1;
    *relcorr = worst;
    if (ok) flags[0] = 1;
  }
}

// Backward-error stop test (one workgroup).  For every system sys and right-hand side q
// (segment sys * nrhs + q): |r|_inf and |x|_inf from the block partials of
// maxabs_partial_kernel (partial[0] over r, partial[1] over x), |b|_inf from bnorm and
// |K|_inf of the system (reduced here from the residual's per-workgroup row-sum maxima
// and its root rows when kpart is not null, kept in knorm); then
// eta = |r| / (|K| |x| + |b|), the normwise backward error of x.  The loop is done
// (flags[0] = 1) when eta <= tol for every segment; otherwise flags[1] counts one more
// correction if count is set.  rnorm receives |r| for the correction solve, relcorr the
// largest eta.
__global__ void __launch_bounds__(256) refine_be_check_kernel(
    const double* partial, int blocks, int B, int nrhs, const double* kpart, int kper,
    const double* kroot, double* knorm, const double* bnorm, double tol, int count, int* flags,
    double* relcorr, double* rnorm) {
  if (flags[0]) return;
  __shared__ double sh[4];
  const int segs = B * nrhs;
  bool ok = true;
  double worst = 0.0;
  for (int sys = 0; sys < B; ++sys) {
    if (kpart) {
      double m = strided_max<8>(kpart + (size_t)sys * kper, kper, (int)threadIdx.x, (int)blockDim.x);
      m = block_max(m, sh);
      if (threadIdx.x == 0) knorm[sys] = nan_max(m, kroot[sys]);
      __syncthreads();
    }
    const double kn = knorm[sys];
    for (int q = 0; q < nrhs; ++q) {
      const int seg = sys * nrhs + q;
      double mr = strided_max<4>(partial + (size_t)seg * blocks, blocks, (int)threadIdx.x,
                                 (int)blockDim.x);
      double mx = strided_max<4>(partial + ((size_t)segs + seg) * blocks, blocks,
                                 (int)threadIdx.x, (int)blockDim.x);
      mr = block_max(mr, sh);
      mx = block_max(mx, sh);
      if (threadIdx.x == 0) {
        const double den = kn * mx + bnorm[seg];
        const double eta = den > 0.0 ? mr / den : (mr > 0.0 ? HUGE_VAL : 0.0);
        worst = nan_max(worst, eta);
        if (!(eta <= tol)) ok = false;
        rnorm[seg] = mr;
      }
    }
  }
  if (threadIdx.x == 0) {
    *relcorr = worst;
    if (ok)
      flags[0] = 1;
    else if (count)
      flags[1] += 1;
  }
}

// ---- ragged batches (see multi.h) ----

__device__ inline ResidualArgs relocate_residual(const ResidualArgs& t, const Reloc& r) {
  ResidualArgs a = t;
  a.D = rel(r.D, t.D);
  a.E = rel(r.E, t.E);
  a.C = rel(r.C, t.C);
  a.R = rel(r.R, t.R);
  a.b = rel(r.b, t.b);
  a.x = rel(r.x, t.x);
  a.r = rel(r.r, t.r);
  return a;
}

template <int NMAX, bool FULL>
__global__ void __launch_bounds__(RES_T) residual_multi(const MultiItem<ResidualArgs>* items,
                                                        int nitems, Reloc r) {
  const MultiItem<ResidualArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  residual_body<NMAX, FULL>(relocate_residual(it.a, r), it.p0, multi_local(it).x);
}

template <int NMAX>
__global__ void __launch_bounds__(1024) residual_root_multi(const MultiItem<ResidualArgs>* items,
                                                            int nitems, Reloc r) {
  const MultiItem<ResidualArgs>& it = items[multi_find(items, nitems, blockIdx.x)];
  residual_root_body<NMAX>(relocate_residual(it.a, r), multi_local(it).x);
}

__global__ void __launch_bounds__(256) seg_maxabs_kernel(const double* v, const double* v2,
                                                         const SegRec* segs, double* out,
                                                         double* out2, const int* done) {
  if (done && *done) return;
  __shared__ double sh[4];
  const SegRec sg = segs[blockIdx.x];
  for (int t = 0; t < (v2 ? 2 : 1); ++t) {
    const double* p = (t == 0 ? v : v2) + sg.off;
    double m0 = 0.0, m1 = 0.0;
    size_t i = threadIdx.x;
    for (; i + 256 < sg.len; i += 512) {
      m0 = nan_max(fabs(p[i]), m0);
      m1 = nan_max(fabs(p[i + 256]), m1);
    }
    for (; i < sg.len; i += 256) m0 = nan_max(fabs(p[i]), m0);
    const double mx = block_max(nan_max(m0, m1), sh);
    if (threadIdx.x == 0) (t == 0 ? out : out2)[blockIdx.x] = mx;
  }
}

// Per system (one workgroup each): its |K| (backward-error mode, when kpart is set) and
// whether all its segments pass; sys_worst = the largest test quantity.
__global__ void __launch_bounds__(256) ragged_sys_check_kernel(
    int mode, const double* dr, const double* xn, const double* bn, const int* seg_sys,
    int nseg, const double* kpart, const int* kp_off, const double* kroot, double* knorm,
    double tol, const int* flags, int* sys_ok, double* sys_worst) {
  if (flags[0]) return;
  __shared__ double sh[4];
  const int sys = blockIdx.x;
  if (mode == 1 && kpart) {
    double m = strided_max<8>(kpart + kp_off[sys], kp_off[sys + 1] - kp_off[sys],
                              (int)threadIdx.x, (int)blockDim.x);
    m = block_max(m, sh);
    if (threadIdx.x == 0) knorm[sys] = nan_max(m, kroot[sys]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  bool ok = true;
  double worst = 0.0;
  // the segments of a system are consecutive; find them by a scan of seg_sys
  int lo = 0, hi = nseg;
  while (lo < hi) {  // first segment of sys
    const int mid = (lo + hi) >> 1;
    if (seg_sys[mid] < sys) lo = mid + 1; else hi = mid;
  }
  for (int k = lo; k < nseg && seg_sys[k] == sys; ++k) {
    double q;
    if (mode == 1) {
      const double den = knorm[sys] * xn[k] + bn[k];
      q = den > 0.0 ? dr[k] / den : (dr[k] > 0.0 ? HUGE_VAL : 0.0);
    } else {
      q = xn[k] > 0.0 ? dr[k] / xn[k] : dr[k];
    }
    worst = nan_max(worst, q);
    if (!(q <= tol)) ok = false;
  }
  sys_ok[sys] = ok ? 1 : 0;
  sys_worst[sys] = worst;
}

__global__ void __launch_bounds__(256) ragged_final_check_kernel(int B, int count, int* flags,
                                                                 double* relcorr,
                                                                 const int* sys_ok,
                                                                 const double* sys_worst) {
  if (flags[0]) return;
  __shared__ double sh[4];
  double w = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < B; i += blockDim.x) {
    w = nan_max(sys_worst[i], w);
    if (!sys_ok[i]) bad = 1.0;
  }
  w = block_max(w, sh);
  bad = block_max(bad, sh);
  if (threadIdx.x == 0) {
    *relcorr = w;
    // count: 2 = a correction was applied before this test (correction-size test),
    // 1 = one is applied after it unless the test holds (backward error), 0 = none
    if (count == 2 || (count == 1 && bad != 0.0)) flags[1] += 1;
    if (bad == 0.0) flags[0] = 1;
  }
}

}  // namespace

size_t residual_lds(int nmax, int nrhs) {
  return nmax <= 8 ? residual_lds_bytes<8>(nrhs)
                   : nmax <= 16 ? residual_lds_bytes<16>(nrhs) : residual_lds_bytes<32>(nrhs);
}

void launch_residual_multi(int nmax, bool full, const MultiItem<ResidualArgs>* items, int nitems,
                           unsigned blocks, size_t lds, const Reloc& r, hipStream_t st) {
  const dim3 g(blocks), b(RES_T);
#define BMPC_RES_MULTI(NM)                                                             \
  if (full)                                                                            \
    hipLaunchKernelGGL((residual_multi<NM, true>), g, b, lds, st, items, nitems, r);     \
  else                                                                                 \
    hipLaunchKernelGGL((residual_multi<NM, false>), g, b, lds, st, items, nitems, r);
  if (nmax <= 8) {
    BMPC_RES_MULTI(8)
  } else if (nmax <= 16) {
    BMPC_RES_MULTI(16)
  } else {
    BMPC_RES_MULTI(32)
  }
#undef BMPC_RES_MULTI
}

void launch_residual_root_multi(const MultiItem<ResidualArgs>* items, int nitems, unsigned blocks,
                                const Reloc& r, hipStream_t st) {
  hipLaunchKernelGGL(residual_root_multi<32>, dim3(blocks), dim3(1024), 0, st, items, nitems, r);
}

void launch_seg_maxabs(const double* v, const double* v2, const SegRec* segs, int nseg,
                       double* out, double* out2, const int* done, hipStream_t st) {
  hipLaunchKernelGGL(seg_maxabs_kernel, dim3(nseg), dim3(256), 0, st, v, v2, segs, out, out2,
                     done);
}

void launch_ragged_check(int mode, const double* dn_or_rn, const double* xn, const double* bn,
                         const int* seg_sys, int nseg, int B, const double* kpart,
                         const int* kp_off, const double* kroot, double* knorm, double tol,
                         int count, int* flags, double* relcorr, int* sys_ok,
                         double* sys_worst, hipStream_t st) {
  hipLaunchKernelGGL(ragged_sys_check_kernel, dim3(B), dim3(256), 0, st, mode, dn_or_rn, xn, bn,
                     seg_sys, nseg, kpart, kp_off, kroot, knorm, tol, (const int*)flags, sys_ok,
                     sys_worst);
  hipLaunchKernelGGL(ragged_final_check_kernel, dim3(1), dim3(256), 0, st, B, count, flags,
                     relcorr, (const int*)sys_ok, (const double*)sys_worst);
}

void launch_refine_be_check(const double* r, const double* x, int B, int nrhs, size_t len,
                            double* partial, const double* kpart, int kper,
                            const double* kroot, double* knorm, const double* bnorm,
                            double tol, int count, int* flags, double* relcorr, double* rnorm,
                            hipStream_t st) {
  hipLaunchKernelGGL(maxabs_partial_kernel, dim3(kNormBlocks), dim3(256), 0, st, r, x, B * nrhs,
                     len, partial, (const int*)flags);
  hipLaunchKernelGGL(refine_be_check_kernel, dim3(1), dim3(256), 0, st, (const double*)partial,
                     kNormBlocks, B, nrhs, kpart, kper, kroot, knorm, bnorm, tol, count, flags,
                     relcorr, rnorm);
}

template <int NMAX>
static void launch_residual_t(const ResidualArgs& a, dim3 grid, int chunks, hipStream_t st) {
  const size_t lds = residual_lds_bytes<NMAX>(a.nrhs);
  if (NMAX > 32) {  // beyond the default 64 KB of dynamic LDS
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&residual_kernel<NMAX, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)residual_lds_bytes<NMAX>(rhs_chunk(NMAX)));
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&residual_kernel<NMAX, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)residual_lds_bytes<NMAX>(rhs_chunk(NMAX)));
      attr_set = true;
    }
  }
  if (a.n == NMAX)
    hipLaunchKernelGGL((residual_kernel<NMAX, true>), grid, dim3(RES_T), lds, st, a, chunks);
  else
    hipLaunchKernelGGL((residual_kernel<NMAX, false>), grid, dim3(RES_T), lds, st, a, chunks);
}

void launch_residual(const ResidualArgs& a, int nmax, hipStream_t st) {
  const int chunks = (a.N + a.chunk - 1) / a.chunk;
  const dim3 grid((unsigned)(a.B * a.S) * (unsigned)chunks);
  if (nmax <= 8)
    launch_residual_t<8>(a, grid, chunks, st);
  else if (nmax <= 16)
    launch_residual_t<16>(a, grid, chunks, st);
  else if (nmax <= 32)
    launch_residual_t<32>(a, grid, chunks, st);
  else
    launch_residual_t<64>(a, grid, chunks, st);
}

void launch_residual_root(const ResidualArgs& a, hipStream_t st) {
  if (a.n > 32)
    hipLaunchKernelGGL(residual_root_kernel<64>, dim3(a.B), dim3(1024), 0, st, a);
  else
    hipLaunchKernelGGL(residual_root_kernel<32>, dim3(a.B), dim3(1024), 0, st, a);
}

void launch_maxabs(const double* v, int nrhs, size_t len, double* partial, double* out,
                   const int* done, hipStream_t st) {
  hipLaunchKernelGGL(maxabs_partial_kernel, dim3(kNormBlocks), dim3(256), 0, st, v,
                     (const double*)nullptr, nrhs, len, partial, done);
  hipLaunchKernelGGL(maxabs_final_kernel, dim3(1), dim3(64), 0, st, partial, kNormBlocks, nrhs,
                     out, done);
}

void launch_refine_reset(int* flags, hipStream_t st) {
  hipLaunchKernelGGL(refine_reset_kernel, dim3(1), dim3(64), 0, st, flags);
}

void launch_refine_check(const double* d, const double* x, int nrhs, size_t len,
                         double* partial, double tol, int* flags, double* relcorr,
                         double* dnorm, double* xnorm, hipStream_t st) {
  hipLaunchKernelGGL(maxabs_partial_kernel, dim3(kNormBlocks), dim3(256), 0, st, d, x, nrhs, len,
                     partial, (const int*)flags);
  hipLaunchKernelGGL(refine_check_kernel, dim3(1), dim3(64), 0, st, (const double*)partial,
                     kNormBlocks, nrhs, tol, flags, relcorr, dnorm, xnorm);
}

}  // namespace bmpc
