// Autotuner of a plan's launch configuration (gfx950).
//
// For one shape (S, N, n, nrhs), a batch count and a precision it builds a plan for every candidate
// configuration -- levels per factor pass (window depth), the backward sweep's top
// levels in one launch with one workgroup per chain or one launch per level with one
// wave per position, the forward sweep's positions on up to four waves or on one --
// and times the plan's own step (FP64: factor + solve; FP32: factor + one refinement
// correction) on synthetic data in HBM with HIP events, the median of a few runs.  One
// system of a small shape leaves most of the GPU idle and is timed for its latency; a
// batch of systems (num_systems > 1, the arrays stacked as in a batch plan) is timed for
// its throughput, which is what a system sharing the GPU with many others sees.  The
// data is a block-diagonally dominant SPD system; the kernels' timing does not depend
// on the values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "plan.h"

namespace bmpc {

namespace {

// D = 2 I, E and C entries 1 / (4 n) (spectral norms <= 1/4), R = (S / 4 + 1) I, b = 1:
// every row block's diagonal exceeds its off-diagonal norms, so K is SPD.
__global__ void tune_fill_kernel(double* D, double* E, double* C, double* R, double* b,
                                 size_t nD, size_t nE, size_t nC, size_t nR, size_t nb, int n,
                                 int S) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nn = (size_t)n * n;
  const double off = 0.25 / n;
  for (size_t i = t0; i < nD; i += stride) {
    const size_t e = i % nn;
    D[i] = (e / n == e % n) ? 2.0 : 0.0;
  }
  for (size_t i = t0; i < nE; i += stride) E[i] = off;
  for (size_t i = t0; i < nC; i += stride) C[i] = off;
  for (size_t i = t0; i < nR; i += stride) {
    const size_t e = i % nn;
    R[i] = (e / n == e % n) ? 0.25 * S + 1.0 : 0.0;
  }
  for (size_t i = t0; i < nb; i += stride) b[i] = 1.0;
}

}  // namespace

}  // namespace bmpc

using namespace bmpc;

extern "C" bmpc_status bmpc_autotune(const bmpc_dims* dims, int32_t num_systems,
                                     bmpc_precision prec, void* stream, int32_t reps,
                                     bmpc_options* best, double* best_ms, double* times,
                                     int32_t cap, int32_t* count) {
  const int B = num_systems > 0 ? num_systems : 1;
  if (!dims_ok(dims, B) || !best || reps < 1 || reps > 100 || cap < 0 || (cap > 0 && !times) ||
      (prec != BMPC_FP64 && prec != BMPC_FP32_REFINE))
    return BMPC_ERR_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bmpc_dims& d = *dims;
  const size_t nn = (size_t)d.n * d.n;
  const size_t nD = (size_t)B * d.S * d.N * nn, nE = (size_t)B * d.S * (d.N - 1) * nn;
  const size_t nC = (size_t)B * d.S * nn, nR = (size_t)B * nn;
  const size_t nb = (size_t)B * d.nrhs * ((size_t)d.S * d.N + 1) * d.n;
  double *D = nullptr, *E = nullptr, *C = nullptr, *R = nullptr, *b = nullptr, *x = nullptr;
  auto release = [&] {
    for (double* p : {D, E, C, R, b, x})
      if (p) (void)hipFree(p);
  };
  if (hipMalloc((void**)&D, nD * 8) != hipSuccess ||
      hipMalloc((void**)&E, std::max<size_t>(nE, 1) * 8) != hipSuccess ||
      hipMalloc((void**)&C, nC * 8) != hipSuccess || hipMalloc((void**)&R, nR * 8) != hipSuccess ||
      hipMalloc((void**)&b, nb * 8) != hipSuccess || hipMalloc((void**)&x, nb * 8) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return BMPC_ERR_ALLOC;
  }
  hipLaunchKernelGGL(tune_fill_kernel, dim3(1024), dim3(256), 0, st, D, E, C, R, b, nD, nE, nC,
                     nR, nb, d.n, d.S);
  // candidates: every window depth the shared memory allows, crossed with the two sweep
  // mappings
  const bool fp64 = prec == BMPC_FP64;
  bmpc_options probe{};
  probe.window_depth = kMaxWindowDepth;
  const int maxTw = pick_window_depth(fp64, nmax_for(d.n), d.nrhs, &probe);
  std::vector<bmpc_options> cands;
  for (int tw = 1; tw <= maxTw; ++tw)
    for (int f : {0, BMPC_FLAG_NO_BWD_TOP_MERGE, BMPC_FLAG_FWD_ONE_WAVE,
                  BMPC_FLAG_NO_BWD_TOP_MERGE | BMPC_FLAG_FWD_ONE_WAVE}) {
      bmpc_options o{};
      o.window_depth = tw;
      o.flags = f;
      o.num_systems = B;
      cands.push_back(o);
    }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double best_t = -1.0;
  int tried = 0;
  bmpc_status status = BMPC_OK;
  for (const bmpc_options& o : cands) {
    bmpc_plan p = nullptr;
    const bmpc_status a = bmpc_analyze_ex(dims, prec, stream, &o, &p);
    if (a == BMPC_ERR_ALLOC) continue;  // too large with this configuration
    if (a != BMPC_OK) {
      status = a;
      break;
    }
    auto step = [&] {
      if (fp64)
        (void)bmpc_factor_solve(p, D, E, C, R, b, x);
      else
        (void)bmpc_factor_refine(p, D, E, C, R, b, x, 0.0, 1);
    };
    step();  // warm-up
    std::vector<double> ms;
    for (int r = 0; r < reps; ++r) {
      (void)hipEventRecord(e0, st);
      step();
      (void)hipEventRecord(e1, st);
      float t = 0.f;
      (void)hipEventSynchronize(e1);
      (void)hipEventElapsedTime(&t, e0, e1);
      ms.push_back(t);
    }
    std::sort(ms.begin(), ms.end());
    const double med = ms[ms.size() / 2];
    int64_t info = 0;
    const bool ok = bmpc_get_info(p, &info) == BMPC_OK && last_error_status() == BMPC_OK;
    (void)bmpc_destroy(p);
    if (!ok) {
      status = BMPC_ERR_DEVICE;
      break;
    }
    if (tried < cap) times[tried] = med;
    ++tried;
    if (best_t < 0.0 || med < best_t) {
      best_t = med;
      *best = o;
      best->num_systems = 0;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  release();
  if (count) *count = tried;
  if (best_ms) *best_ms = best_t;
  if (status == BMPC_OK && tried == 0) status = BMPC_ERR_ALLOC;
  return status;
}
