// Assembly of the reduced IPM system of a branch-MPC QP (gfx950).
//
// The regularized primal-dual IPM KKT matrix [[P + tau I, A^T, G^T], [A, -delta I, 0],
// [G, 0, -(W + delta I)]] reduces, by eliminating its second and third block rows, to
// the SPD matrix K = P + tau I + delta^{-1} A^T A + G^T (W + delta I)^{-1} G (appendix
// on the linear systems of IPM and ADMM).  In branch MPC every cost and constraint
// term touches two neighbouring blocks, stored per link j of scenario s: link 0 couples
// (u, v) = (x_0, x_{s,0}), link k couples (x_{s,k-1}, x_{s,k}), link N is the terminal
// term on u = x_{s,N-1}.  With X_j = [A_j / sqrt(delta); diag(w_j + delta)^{-1/2} G_j]
// the link's share of K is M_j = Q_j + X_j^T X_j (2n x 2n, quadrants uu, uv, vu, vv):
//   D_{s,k} = tau I + M_{s,k}[vv] + M_{s,k+1}[uu]      E_{s,k} = M_{s,k+1}[vu]
//   C_s     = M_{s,0}[uv]                             R = tau I + sum_s M_{s,0}[uu]
// so K has exactly the root-coupled block structure the solver takes.  One workgroup
// per tail stage stages the scaled rows of its two links in LDS, one link at a time;
// the root block is a fixed-order sum over the scenarios.
#include <mutex>

#include "bmpc.h"
#include "bmpc_internal.h"

namespace bmpc {

namespace {

constexpr int QT = 256;

struct QpArgs {
  int S, N, n, me, mi;
  const double* Q;
  const double* A;
  const double* G;
  const double* w;
  double tau, delta;
  double* D;
  double* E;
  double* C;
  double* Rpart;  // [S][n][n] link-0 uu parts
};

// X (rows x 2n, row-major in LDS) of link j of scenario s: A / sqrt(delta), then the
// G rows divided by sqrt(w + delta).
__device__ void stage_link(const QpArgs& a, int s, int j, double* X) {
  const int n2 = 2 * a.n, rows = a.me + a.mi;
  const size_t link = (size_t)s * (a.N + 1) + j;
  const double sa = 1.0 / sqrt(a.delta);
  for (int e = threadIdx.x; e < rows * n2; e += QT) {
    const int r = e / n2, c = e - r * n2;
    double v;
    if (r < a.me) {
      v = a.A[(link * a.me + r) * n2 + c] * sa;
    } else {
      const int i = r - a.me;
      v = a.G[(link * a.mi + i) * n2 + c] / sqrt(a.w[link * a.mi + i] + a.delta);
    }
    X[e] = v;
  }
}

// M_j[p][q] for rows p, q of the 2n-sized link variable (X staged in LDS)
__device__ inline double link_entry(const QpArgs& a, int s, int j, const double* X, int p,
                                   int q) {
  const int n2 = 2 * a.n, rows = a.me + a.mi;
  double acc = a.Q[(((size_t)s * (a.N + 1) + j) * n2 + p) * n2 + q];
  for (int r = 0; r < rows; ++r) acc += X[r * n2 + p] * X[r * n2 + q];
  return acc;
}

__global__ void __launch_bounds__(QT) qp_stage_kernel(QpArgs a) {
  extern __shared__ double X[];  // (me + mi) x 2n
  const int s = blockIdx.x / a.N;
  const int k = blockIdx.x - s * a.N;
  const int n = a.n, N = a.N;
  const size_t nn = (size_t)n * n;
  const size_t blk = (size_t)s * N + k;
  // link k: its v part is stage k (D's vv share); for k = 0 also C and the root share
  stage_link(a, s, k, X);
  __syncthreads();
  double dacc[(32 * 32 + QT - 1) / QT];
  int t = 0;
  for (int e = threadIdx.x; e < n * n; e += QT, ++t) {
    const int r = e / n, c = e - r * n;
    dacc[t] = (r == c ? a.tau : 0.0) + link_entry(a, s, k, X, n + r, n + c);
    if (k == 0) {
      a.C[(size_t)s * nn + e] = link_entry(a, s, 0, X, r, n + c);
      a.Rpart[(size_t)s * nn + e] = link_entry(a, s, 0, X, r, c);
    }
  }
  __syncthreads();
  // link k+1: its u part is stage k (D's uu share) and, below the last stage, its
  // vu quadrant is E_{s,k}
  stage_link(a, s, k + 1, X);
  __syncthreads();
  t = 0;
  for (int e = threadIdx.x; e < n * n; e += QT, ++t) {
    const int r = e / n, c = e - r * n;
    a.D[blk * nn + e] = dacc[t] + link_entry(a, s, k + 1, X, r, c);
    if (k + 1 < N) a.E[((size_t)s * (N - 1) + k) * nn + e] = link_entry(a, s, k + 1, X, n + r, c);
  }
}

// R = tau I + sum_s Rpart[s], in scenario order (thread per element)
__global__ void __launch_bounds__(1024) qp_root_kernel(const double* Rpart, int S, int n,
                                                       double tau, double* R) {
  const int e = threadIdx.x;
  if (e >= n * n) return;
  const size_t nn = (size_t)n * n;
  double acc = 0.0;
  constexpr int U = 8;
  for (int s0 = 0; s0 < S; s0 += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = s0 + u < S ? Rpart[(size_t)(s0 + u) * nn + e] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  R[e] = acc + ((e / n) == (e % n) ? tau : 0.0);
}

}  // namespace

}  // namespace bmpc

namespace {

// Scratch of bmpc_assemble_qp_noalloc: the per-scenario root shares (S * n * n doubles)
// in a file-scope device array, one copy per GPU, so that the entry point allocates
// nothing.  Host code never uses the array's name as an address: the device address of
// each GPU's copy is looked up once per device (hipGetSymbolAddress with that device
// current) and kept here.
constexpr size_t kQpScratchDoubles = (size_t)512 * 32 * 32;  // 4 MiB
static __device__ __align__(256) double scratch[kQpScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch (null on failure).
double* device_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" bmpc_status bmpc_assemble_qp(const bmpc_qp_dims* d, const double* Q, const double* A,
                                        const double* G, const double* w, double tau,
                                        double delta, double* D, double* E, double* C,
                                        double* R, double* work, void* stream) {
  using namespace bmpc;
  if (!d || d->S < 1 || d->N < 1 || d->n < 1 || d->n > 32 || d->me < 0 || d->me > 64 ||
      d->mi < 0 || d->mi > 128 || !(tau >= 0.0) || !(delta > 0.0) || !Q || !D || !C || !R ||
      !work || (d->N > 1 && !E) || (d->me > 0 && !A) || (d->mi > 0 && (!G || !w)))
    return BMPC_ERR_INVALID;
  QpArgs a{};
  a.S = d->S;
  a.N = d->N;
  a.n = d->n;
  a.me = d->me;
  a.mi = d->mi;
  a.Q = Q;
  a.A = A;
  a.G = G;
  a.w = w;
  a.tau = tau;
  a.delta = delta;
  a.D = D;
  a.E = E;
  a.C = C;
  a.Rpart = work;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t lds = (size_t)(d->me + d->mi) * 2 * d->n * sizeof(double);
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(qp_stage_kernel),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return BMPC_ERR_DEVICE;
  hipLaunchKernelGGL(qp_stage_kernel, dim3((unsigned)(d->S * d->N)), dim3(QT), lds, st, a);
  hipLaunchKernelGGL(qp_root_kernel, dim3(1), dim3(1024), 0, st, (const double*)work, d->S,
                     d->n, tau, R);
  return hipGetLastError() == hipSuccess ? BMPC_OK : BMPC_ERR_DEVICE;
}

extern "C" bmpc_status bmpc_assemble_qp_noalloc(const bmpc_qp_dims* d, const double* Q,
                                                const double* A, const double* G, const double* w,
                                                double tau, double delta, double* D, double* E,
                                                double* C, double* R, void* stream) {
  if (!d || d->S < 1 || d->n < 1 || d->n > 32 ||
      (size_t)d->S * d->n * d->n > kQpScratchDoubles)
    return BMPC_ERR_INVALID;
  double* work = device_scratch();
  if (!work) return BMPC_ERR_DEVICE;
  return bmpc_assemble_qp(d, Q, A, G, w, tau, delta, D, E, C, R, work, stream);
}
