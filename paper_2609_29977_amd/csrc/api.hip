// C ABI of the bmpc library: analysis, plan-owned workspaces and the launch
// sequences of Algorithm 1 (factor), Algorithm 2 (solve) and mixed-precision
// iterative refinement.  Host code; kernels live in factor.hip, solve.hip and
// refine.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "bmpc.h"
#include "bmpc_internal.h"
#include "plan.h"

using namespace bmpc;

namespace bmpc {

int nmax_for(int n) { return n <= 8 ? 8 : (n <= 16 ? 16 : (n <= 32 ? 32 : 64)); }

double potrf_flops(double n) { return n * n * n / 3.0 + n * n / 2.0 + n / 6.0; }
double trsm_flops(double n) { return n * n * n; }
double syrk_flops(double n) { return n * n * n + n * n; }
double gemm_flops(double n) { return 2.0 * n * n * n; }

// Levels per factor pass.  Measured on n = 16 and n = 32 workloads (S up to 512, N up
// to 256): deeper windows save pass launches and boundary traffic but lengthen the
// serial walk of each window, which sets the pass time once the chains are short or
// few; 3 (FP64) and 4 (FP32) were fastest or within a few percent of it throughout.
// Levels per pass, measured on the paper-grid and c2/c3 shapes: four for FP32 blocks
// up to 16, three otherwise (FP64, whose slots are twice as large; FP32 32 x 32 blocks,
// where three levels let four workgroups share a CU).
int default_window_depth(bool fp64, int nmax) {
  if (nmax > 32) return 1;  // blocks of 33..64: one level per pass (factor64.hip)
  return (fp64 || nmax == 32) ? 3 : 4;
}

int ctz_host(unsigned v) { return __builtin_ctz(v); }


// Permuted position of every chain position (Gamma_{N-1} on the reversed tail,
// Section IV-A): level-major, positions in increasing order inside a level; X last.
std::vector<int> make_permpos(int N) {
  const int m = N - 1;
  std::vector<int> pp(N, 0);
  int pos = 0;
  for (int l = 1; l <= chain_levels(m); ++l)
    for (int j = 1 << (l - 1); j <= m; j += 1 << l) pp[j - 1] = pos++;
  pp[N - 1] = pos;  // X = stage 0, last
  return pp;
}

std::vector<int> make_perm(int N) {
  std::vector<int> pp = make_permpos(N), perm(N);
  for (int j = 1; j <= N; ++j) perm[pp[j - 1]] = N - j;  // position j holds stage N-j
  return perm;
}

Costs make_costs(const bmpc_dims& d, bool fp64, int Tw1, int Tw2, int B, bool no_top_merge) {
  Costs c;
  c.Tw = Tw1;
  c.Tw2 = Tw2;
  const int S = d.S, N = d.N, n = d.n, m = N - 1;
  const double tb = fp64 ? 8.0 : 4.0;
  const double nn = (double)n * n, tri = (double)n * (n + 1) / 2.0;
  const double len = ((double)S * N + 1) * n;
  int mk = m, shift = 0;
  double nG = 0;  // off-diagonal factor blocks per tail
  // the odd positions' inverses of the first pass come from their own kernel (n <= 32)
  const bool level1 = n <= 32 && m >= 1;
  double l1_fl = 0, l1_by = 0;
  for (;;) {
    PassPlan p{};
    const int Tw = shift == 0 ? Tw1 : Tw2;
    p.tw = Tw;
    p.is_final = mk < (1 << Tw);
    p.windows = p.is_final ? 1 : (mk >> Tw) + 1;
    p.mk = mk;
    p.shift = shift;
    double fl = 0, by = 0;
    for (int q = 1; q <= mk; ++q) {
      const int v = ctz_host((unsigned)q);
      if (!p.is_final && v >= Tw) continue;  // a window boundary, eliminated later
      const int hl = (q != (1 << v)) ? 1 : 0;
      nG += 1 + hl;
      if (shift == 0 && level1 && v == 0) {
        // inverted beforehand (level1_inverse_kernel: read D, write L_jj^{-1}); the pass
        // reads the inverse back and writes the G's
        l1_fl += potrf_flops(n);
        l1_by += 8.0 * tri + tb * tri;
        fl += (1 + hl) * (trsm_flops(n) + syrk_flops(n)) + hl * gemm_flops(n);
        by += tb * (tri + (1 + hl) * nn);
        continue;
      }
      fl += potrf_flops(n) + (1 + hl) * (trsm_flops(n) + syrk_flops(n)) + hl * gemm_flops(n);
      by += 8.0 * tri + tb * (tri + (1 + hl) * nn);  // read D, write L_jj^{-1}, G's
    }
    if (shift == 0) by += 8.0 * nn * m;  // every E block is read by the first pass
    if (p.is_final) {
      // x_1 step: read D_0 and C, write L_X^{-1} and F; U = F F^T
      fl += potrf_flops(n) + trsm_flops(n) + syrk_flops(n);
      by += 8.0 * tri + 8.0 * nn + tb * (tri + nn);
    }
    p.flops = fl * S;
    p.bytes = by * S;
    c.passes.push_back(p);
    if (p.is_final) break;
    mk >>= Tw;
    shift += Tw;
  }
  for (size_t i = 0; i < c.passes.size(); ++i) {
    const PassPlan& p = c.passes[i];
    const int cls = p.is_final ? KC_FACTOR_FINAL : (i == 0 ? KC_FACTOR_FIRST : KC_FACTOR_MID);
    c.pass_flops[cls] += p.flops;
    c.pass_bytes[cls] += p.bytes;
    c.factor_flops += p.flops;
  }
  c.pass_flops[KC_FACTOR_L1INV] = l1_fl * S;
  c.pass_bytes[KC_FACTOR_L1INV] = l1_by * S;
  c.factor_flops += l1_fl * S;
  c.factor_flops += (double)S * nn + potrf_flops(n);  // root reduction + root Cholesky
  c.pass_flops[KC_ROOT_POTRF] = potrf_flops(n) + (double)S * nn;
  const double K_bytes = 8.0 * ((double)S * N * tri + (double)S * m * nn + (double)S * nn + tri);
  c.L_bytes = tb * ((double)S * N * tri + (double)S * nG * nn + (double)S * nn) + 8.0 * tri;
  c.factor_bytes = K_bytes + c.L_bytes;
  c.pass_bytes[KC_ROOT_REDUCE] = 8.0 * S * nn;
  c.pass_bytes[KC_ROOT_POTRF] = 8.0 * (tri + tri);
  const double rhs_bytes = 8.0 * len * d.nrhs;
  c.solve_bytes = 2.0 * c.L_bytes + 2.0 * rhs_bytes;
  c.residual_bytes = K_bytes + 3.0 * rhs_bytes;
  c.solve_flops = d.nrhs * ((double)S * (2.0 * N * nn + 4.0 * nG * nn + 4.0 * nn) +
                            (double)S * n + 2.0 * nn);
  c.levels = chain_levels(m) + 1;
  // Per-call solve / residual classes: factor blocks read once per sweep, the
  // right-hand side gathered once, x scattered once, the y scratch written and read.
  const double q = d.nrhs, vec_t = tb * n * q;
  const double chain_blocks = (double)S * (m * tri + nG * nn) * tb;
  c.pass_bytes[KC_SOLVE_FWD] = chain_blocks + (double)S * m * (8.0 * n * q + vec_t) +
                               (double)S * nG * vec_t;
  c.pass_flops[KC_SOLVE_FWD] = q * (double)S * (2.0 * m * nn + 2.0 * nG * nn);
  c.pass_bytes[KC_SOLVE_BWD] = chain_blocks + (double)S * m * (8.0 * n * q + 2.0 * vec_t) +
                               (double)S * nG * vec_t;
  c.pass_flops[KC_SOLVE_BWD] = c.pass_flops[KC_SOLVE_FWD];
  c.pass_bytes[KC_SOLVE_X_FWD] = (double)S * (2.0 * tb * nn + 8.0 * n * q + 8.0 * n * q);
  c.pass_bytes[KC_SOLVE_X_BWD] = (double)S * (2.0 * tb * nn + 8.0 * n * q + vec_t);
  c.pass_bytes[KC_SOLVE_ROOT] = 8.0 * ((double)S * n * q + 2.0 * n * q + tri);
  c.pass_bytes[KC_RESIDUAL] = K_bytes - 8.0 * tri + 3.0 * 8.0 * (double)S * N * n * q;
  c.pass_bytes[KC_RESIDUAL_ROOT] = 8.0 * (tri + (double)S * n * q + 3.0 * n * q);
  // r = b - K x: one multiply-add per stored block entry and side it acts on (D
  // symmetric, E and C each acting as themselves and transposed)
  c.pass_flops[KC_RESIDUAL] = q * 2.0 * (double)S * (N * nn + 2.0 * m * nn + nn);
  c.pass_flops[KC_RESIDUAL_ROOT] = q * 2.0 * ((double)S * nn + nn);
  const int L = chain_levels(m);
  for (int k = 0; k < KC_COUNT; ++k) c.launches[k] = 1;
  if (!level1) c.launches[KC_FACTOR_L1INV] = 0;
  // the solve and residual classes run once per chunk of right-hand sides
  const int ck = rhs_chunk(nmax_for(n));
  const int chunks = (d.nrhs + ck - 1) / ck, last = d.nrhs - (chunks - 1) * ck;
  for (int k : {KC_SOLVE_X_FWD, KC_SOLVE_ROOT, KC_SOLVE_X_BWD, KC_RESIDUAL, KC_RESIDUAL_ROOT})
    c.launches[k] = chunks;
  c.launches[KC_SOLVE_FWD] = L * chunks;
  auto bwd_launches = [&](int q) {
    const int top = no_top_merge ? L + 1 : bwd_top_level(m, n, q, S, B);
    return top <= L ? top : L;  // levels below top, plus one for the rest
  };
  c.launches[KC_SOLVE_BWD] = (chunks - 1) * bwd_launches(ck) + bwd_launches(last);
  // a batch of B systems does B times the work in the same launches
  for (PassPlan& pp : c.passes) {
    pp.flops *= B;
    pp.bytes *= B;
  }
  for (int k = 0; k < KC_COUNT; ++k) {
    c.pass_flops[k] *= B;
    c.pass_bytes[k] *= B;
  }
  c.factor_flops *= B;
  c.solve_flops *= B;
  c.factor_bytes *= B;
  c.solve_bytes *= B;
  c.residual_bytes *= B;
  c.L_bytes *= B;
  return c;
}

}  // namespace bmpc


namespace bmpc {

bool dims_ok(const bmpc_dims* d, int B) {
  return d && d->S >= 1 && d->N >= 1 && d->n >= 1 && d->n <= 64 && d->nrhs >= 1 &&
         d->nrhs <= kMaxPlanRhs && B >= 1 && (double)B * d->S * d->N * d->n < 2.0e9 &&
         (double)B * d->S * d->N < 2.0e9 / 64 &&
         (double)B * d->nrhs * ((double)d->S * d->N + 1) * d->n < 4.0e9;
}

int flags_of(const bmpc_options* o) { return o ? o->flags : 0; }
bool no_top_merge_of(const bmpc_options* o) { return (flags_of(o) & BMPC_FLAG_NO_BWD_TOP_MERGE) != 0; }

int systems_of(const bmpc_options* o) { return (o && o->num_systems > 0) ? o->num_systems : 1; }

void free_plan_memory(bmpc_plan p) {
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
  if (p->hflag) (void)hipHostFree(p->hflag);
  p->hflag = nullptr;
  for (const Timing& t : p->timings) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  p->timings.clear();
  for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
  p->event_pool.clear();
}

bool dalloc(bmpc_plan p, void** ptr, size_t bytes) {
  bytes = (std::max<size_t>(bytes, 256) + 255) & ~(size_t)255;
  if (p->measure || p->arena) {
    *ptr = p->measure ? reinterpret_cast<void*>(256) : p->arena + p->arena_used;
    p->arena_used += bytes;
    p->workspace_bytes += (double)bytes;
    return true;
  }
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    *ptr = nullptr;
    // the runtime keeps the failure as its last error; cleared here, since it is reported
    // as BMPC_ERR_ALLOC and would otherwise surface in the next call that checks it
    (void)hipGetLastError();
    return false;
  }
  p->allocs.push_back(*ptr);
  p->workspace_bytes += (double)bytes;
  return true;
}

// The LDS of a pass includes the right-hand-side slots of the fused forward
// substitution for one chunk of the plan's right-hand sides, so that path always fits.
int pick_window_depth(bool fp64, int nmax, int nrhs, const bmpc_options* o) {
  if (nmax > 32) return 1;
  int Tw = (o && o->window_depth > 0) ? o->window_depth : default_window_depth(fp64, nmax);
  Tw = std::min(Tw, kMaxWindowDepth);
  const int q = std::min(nrhs, rhs_chunk(nmax));
  while (Tw > 1 && factor_pass_lds_bytes(fp64, nmax, Tw, q) > (size_t)kLdsBudget) --Tw;
  return Tw;
}

// Levels of the passes after the first: the option, else the first pass's depth.  A
// smaller depth gives the later passes more workgroups per chain and the final pass a
// shorter walk, but adds passes; on the c2 and c3 shapes the extra passes cost more
// than the shorter walks save.
int pick_later_depth(bool fp64, int nmax, int nrhs, int Tw, const bmpc_options* o) {
  if (nmax > 32) return 1;
  bmpc_options lo{};
  if (o) lo = *o;
  lo.window_depth = std::min((o && o->later_depth > 0) ? o->later_depth : Tw, kMaxWindowDepth);
  return pick_window_depth(fp64, nmax, nrhs, &lo);
}

// Factor passes and root factor; a non-null b also runs the tail forward substitution
// of that right-hand side inside the passes (y and w as the forward sweep and the X
// step of the solve leave them).
// Arguments of factor pass k; a non-null b adds the forward substitution of nq
// right-hand sides starting at b (the first chunk).
FactorPassArgs factor_pass_args(bmpc_plan p, int k, const double* D, const double* E,
                                const double* C, const double* b, int nq) {
  const bmpc_dims& d = p->d;
  const int npass = (int)p->costs.passes.size();
  const PassPlan& pp = p->costs.passes[k];
  FactorPassArgs a{};
  a.S = p->B * d.S;
  a.Ssys = d.S;
  a.N = d.N;
  a.n = d.n;
  a.m = p->m;
  a.Tw = pp.tw;
  a.pass = k;
  a.npass = npass;
  a.mk = pp.mk;
  a.shift = pp.shift;
  a.windows = pp.windows;
  a.is_final = pp.is_final;
  a.D = D;
  a.E = E;
  a.C = C;
  const int in = (k + 1) & 1, out = k & 1;
  a.accR_in = k > 0 ? p->acc[in][0] : nullptr;
  a.accL_in = k > 0 ? p->acc[in][1] : nullptr;
  a.fill_in = k > 0 ? p->acc[in][2] : nullptr;
  a.accR_out = p->acc[out][0];
  a.accL_out = p->acc[out][1];
  a.fill_out = p->acc[out][2];
  a.stride = p->stride;
  a.accX = p->accX;
  a.Linv = p->Linv;
  a.Gl = p->Gl;
  a.Gr = p->Gr;
  a.F = p->F;
  a.U = p->U;
  a.permpos = p->d_permpos;
  a.info = p->d_info;
  if (b) {
    a.b = b;
    a.nrhs = nq;
    a.vsys = (size_t)d.nrhs * (((size_t)d.S * d.N + 1) * d.n);
    a.y = p->y;
    a.w = p->w;
    a.vaccR_in = k > 0 ? p->vacc[in][0] : nullptr;
    a.vaccL_in = k > 0 ? p->vacc[in][1] : nullptr;
    a.vaccR_out = p->vacc[out][0];
    a.vaccL_out = p->vacc[out][1];
    a.vaccX = p->vaccX;
  }
  return a;
}

// Arguments of the residual of chunk c of the right-hand sides (b, x, r at their
// bases; knorm adds the row sums of |K|).
ResidualArgs residual_args(bmpc_plan p, int c, const double* D, const double* E,
                           const double* C, const double* R, const double* b, const double* x,
                           double* r, bool knorm) {
  const size_t off = (size_t)c * p->chunk * vec_len(p);
  ResidualArgs ra{};
  ra.S = p->d.S;
  ra.B = p->B;
  ra.N = p->d.N;
  ra.n = p->d.n;
  ra.nrhs = chunk_rhs(p, c);
  ra.vsys = (size_t)p->d.nrhs * vec_len(p);
  ra.chunk = 16;
  ra.D = D;
  ra.E = E;
  ra.C = C;
  ra.R = R;
  ra.b = b + off;
  ra.x = x + off;
  ra.r = r + off;
  ra.w = p->w;
  ra.done = p->flags;
  if (knorm) {
    ra.knorm_part = p->kpart;
    ra.knorm_root = p->kroot;
    ra.crow = p->crow;
  }
  return ra;
}

template <typename T>
void enqueue_factor(bmpc_plan p, const double* D, const double* E, const double* C,
                    const double* R, const double* b = nullptr, int nq = 0) {
  const bmpc_dims& d = p->d;
  hipStream_t st = p->stream;
  timed(p, KC_FACTOR_INIT, [&] { launch_factor_init(p->d_info, st); });
  const int npass = (int)p->costs.passes.size();
  if (p->nmax <= 32 && d.N > 1) {
    const FactorPassArgs a0 = factor_pass_args(p, 0, D, E, C, nullptr, 0);
    timed(p, KC_FACTOR_L1INV, [&] { launch_level1_inverse<T>(a0, p->nmax, st); });
  }
  for (int k = 0; k < npass; ++k) {
    const PassPlan& pp = p->costs.passes[k];
    const FactorPassArgs a = factor_pass_args(p, k, D, E, C, b, nq);
    const int cls = pp.is_final ? KC_FACTOR_FINAL : (k == 0 ? KC_FACTOR_FIRST : KC_FACTOR_MID);
    timed(p, cls, [&] { launch_factor_pass<T>(a, p->nmax, st); });
  }
  timed(p, KC_ROOT_REDUCE,
        [&] { launch_root_reduce(p->U, p->Upart, p->B, d.S, d.n, p->groups, st); });
  const int64_t root_row = (int64_t)d.S * d.N * d.n;
  const int64_t sys_rows = root_row + d.n;
  timed(p, KC_ROOT_POTRF, [&] {
    launch_root_potrf(R, p->Upart, p->B, p->groups, d.n, p->LR, sys_rows, root_row, p->d_info,
                      st);
  });
}

size_t vec_len(bmpc_plan p) { return ((size_t)p->d.S * p->d.N + 1) * p->d.n; }
int chunks_of(bmpc_plan p) { return (p->d.nrhs + p->chunk - 1) / p->chunk; }
int chunk_rhs(bmpc_plan p, int c) { return std::min(p->chunk, p->d.nrhs - c * p->chunk); }

// Arguments of a solve of the chunk of right-hand sides starting at q0 (nq of them).
SolveArgs solve_args(bmpc_plan p, const double* b, double* x, int q0, int nq) {
  SolveArgs a{};
  const size_t off = (size_t)q0 * vec_len(p);
  a.S = p->d.S;
  a.B = p->B;
  a.N = p->d.N;
  a.n = p->d.n;
  a.m = p->m;
  a.nrhs = nq;
  a.vsys = (size_t)p->d.nrhs * vec_len(p);
  a.seg_sys = p->d.nrhs;
  a.fwd_waves = (p->opt_flags & BMPC_FLAG_FWD_ONE_WAVE) ? 1 : 0;
  a.Linv = p->Linv;
  a.Gl = p->Gl;
  a.Gr = p->Gr;
  a.F = p->F;
  a.LR = p->LR;
  a.b = b + off;
  a.x = x + off;
  a.y = p->y;
  a.w = p->w;
  a.x0 = p->x0;
  return a;
}

// Root step, root propagation and tail backward substitution (Algorithm 2 from its root
// step on), given the y and w of the forward part.
template <typename T>
void enqueue_solve_back(bmpc_plan p, const SolveArgs& a) {
  hipStream_t st = p->stream;
  const int L = chain_levels(p->m);
  timed(p, KC_SOLVE_ROOT, [&] { launch_solve_root(a, st); });
  timed(p, KC_SOLVE_X_BWD, [&] { launch_solve_x_bwd<T>(a, p->nmax, st); });
  // the top levels (few positions per chain) in one launch, the others one by one
  const int top = (p->opt_flags & BMPC_FLAG_NO_BWD_TOP_MERGE)
                      ? L + 1
                      : bwd_top_level(p->m, p->d.n, a.nrhs, p->d.S, p->B);
  if (top <= L) timed(p, KC_SOLVE_BWD, [&] { launch_solve_bwd_top<T>(a, top, st); });
  for (int l = std::min(L, top - 1); l >= 1; --l)
    timed(p, KC_SOLVE_BWD, [&] { launch_solve_bwd_level<T>(a, l, p->nmax, st); });
}

template <typename T>
void enqueue_solve_chunk(bmpc_plan p, const SolveArgs& a) {
  hipStream_t st = p->stream;
  const int L = chain_levels(p->m);
  for (int l = 1; l <= L; ++l)
    timed(p, KC_SOLVE_FWD, [&] { launch_solve_fwd_level<T>(a, l, p->nmax, st); });
  timed(p, KC_SOLVE_X_FWD, [&] { launch_solve_x_fwd<T>(a, p->nmax, st); });
  enqueue_solve_back<T>(p, a);
}

// Algorithm 2 for every chunk of right-hand sides in turn (the scratch y, w, x0 is
// sized for one chunk); mod adjusts each chunk's arguments (refinement scaling).
template <typename T, typename Mod>
void enqueue_solve(bmpc_plan p, const double* b, double* x, int first_chunk, Mod mod) {
  for (int c = first_chunk; c < chunks_of(p); ++c) {
    SolveArgs a = solve_args(p, b, x, c * p->chunk, chunk_rhs(p, c));
    mod(a, c * p->chunk);
    enqueue_solve_chunk<T>(p, a);
  }
}
template <typename T>
void enqueue_solve(bmpc_plan p, const double* b, double* x, int first_chunk = 0) {
  enqueue_solve<T>(p, b, x, first_chunk, [](SolveArgs&, int) {});
}

// Factor, then the whole solve of b into x with the first chunk's forward substitution
// inside the factorization.
template <typename T>
void enqueue_factor_solve(bmpc_plan p, const double* D, const double* E, const double* C,
                          const double* R, const double* b, double* x) {
  if (p->nmax > 32) {  // no forward substitution inside the n > 32 factor passes
    enqueue_factor<T>(p, D, E, C, R);
    enqueue_solve<T>(p, b, x);
    return;
  }
  enqueue_factor<T>(p, D, E, C, R, b, chunk_rhs(p, 0));
  enqueue_solve_back<T>(p, solve_args(p, b, x, 0, chunk_rhs(p, 0)));
  enqueue_solve<T>(p, b, x, 1);
}

bmpc_status last_error_status() {
  return hipGetLastError() == hipSuccess ? BMPC_OK : BMPC_ERR_DEVICE;
}

// Whether the refinement's stop test already holds, read on the host.  Outside stream
// capture the loop stops issuing launches once it holds (the device-side flag would
// make them return at once, but each still costs a launch); under capture the launch
// sequence stays fixed and the flag alone decides.
bool stop_reached(bmpc_plan p) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(p->stream, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (cs != hipStreamCaptureStatusNone) return false;
  if (hipMemcpyAsync(p->hflag, p->flags, sizeof(int), hipMemcpyDeviceToHost, p->stream) !=
          hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return p->hflag[0] != 0;
}

// Analysis and workspaces of a plan (bmpc_analyze_ex after its argument checks).  A
// plan with a ragged parent shares the parent's residual vector and stop flags, which
// the parent sets.
bmpc_status init_plan(bmpc_plan p, const bmpc_dims* dims, bmpc_precision prec, void* stream,
                      const bmpc_options* opts) {
  p->d = *dims;
  p->prec = prec;
  p->fp64 = prec == BMPC_FP64;
  p->m = dims->N - 1;
  p->nmax = nmax_for(dims->n);
  p->Tw = pick_window_depth(p->fp64, p->nmax, dims->nrhs, opts);
  p->Tw2 = pick_later_depth(p->fp64, p->nmax, dims->nrhs, p->Tw, opts);
  p->B = systems_of(opts);
  p->opt_flags = flags_of(opts);
  p->chunk = rhs_chunk(p->nmax);
  p->stream = reinterpret_cast<hipStream_t>(stream);
  p->costs = make_costs(*dims, p->fp64, p->Tw, p->Tw2, p->B, no_top_merge_of(opts));
  p->perm = make_perm(dims->N);
  p->permpos = make_permpos(dims->N);
  p->groups = std::min(dims->S, 32);
  const int B = p->B, N = dims->N, n = dims->n, nrhs = dims->nrhs;
  const int cq = std::min(nrhs, p->chunk);  // right-hand sides of one chunk
  const size_t S = (size_t)B * dims->S;  // chains of the batch
  const size_t nn = (size_t)n * n, tb = p->fp64 ? 8 : 4;
  const size_t len = ((size_t)dims->S * N + 1) * n;
  const size_t segs = (size_t)B * nrhs;  // (system, right-hand side) vectors
  const int res_chunks = (N + 15) / 16;   // tail residual workgroups per chain
  p->kper = dims->S * res_chunks;
  const int npass = (int)p->costs.passes.size();
  p->stride = (npass > 1 ? p->costs.passes[0].windows : 1) + 1;
  const size_t gblocks = g_chain_blocks(N);
  bool ok = dalloc(p, &p->Linv, S * N * nn * tb) &&
            dalloc(p, &p->Gl, S * gblocks * nn * tb) &&
            dalloc(p, &p->Gr, S * gblocks * nn * tb) &&
            dalloc(p, &p->F, S * nn * tb) &&
            dalloc(p, (void**)&p->U, S * nn * 8) &&
            dalloc(p, (void**)&p->Upart, (size_t)B * p->groups * nn * 8) &&
            dalloc(p, (void**)&p->LR, (size_t)B * nn * 8) &&
            dalloc(p, &p->accX, S * npass * nn * tb) &&
            dalloc(p, &p->vaccX, S * npass * cq * n * tb) &&
            dalloc(p, (void**)&p->d_permpos, (size_t)N * sizeof(int)) &&
            dalloc(p, (void**)&p->d_info, sizeof(unsigned long long)) &&
            dalloc(p, &p->y, S * N * cq * n * tb) &&
            dalloc(p, (void**)&p->w, S * cq * n * 8) &&
            dalloc(p, (void**)&p->x0, (size_t)B * cq * n * 8) &&
            (p->parent || dalloc(p, (void**)&p->rbuf, segs * len * 8)) &&
            dalloc(p, (void**)&p->norms, 3 * segs * 8) &&
            dalloc(p, (void**)&p->npart, 2 * segs * kNormBlocks * 8) &&
            (p->parent || dalloc(p, (void**)&p->flags, 2 * sizeof(int))) &&
            dalloc(p, (void**)&p->relcorr, sizeof(double)) &&
            dalloc(p, (void**)&p->bnorm, segs * 8) &&
            dalloc(p, (void**)&p->knorm, (size_t)B * 8) &&
            dalloc(p, (void**)&p->kpart, S * res_chunks * 8) &&
            dalloc(p, (void**)&p->kroot, (size_t)B * 8) &&
            dalloc(p, (void**)&p->crow, S * n * 8);
  if (ok && !p->parent && !p->measure &&
      hipHostMalloc((void**)&p->hflag, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    p->hflag = nullptr;
    (void)hipGetLastError();
    ok = false;
  }
  if (ok && npass > 1) {
    for (int set = 0; set < 2 && ok; ++set) {
      for (int b = 0; b < 3 && ok; ++b)
        ok = dalloc(p, &p->acc[set][b], S * p->stride * nn * tb);
      for (int b = 0; b < 2 && ok; ++b)
        ok = dalloc(p, &p->vacc[set][b], S * p->stride * cq * n * tb);
    }
  }
  if (!ok) return BMPC_ERR_ALLOC;
  if (p->measure) return BMPC_OK;
  if (hipMemcpy(p->d_permpos, p->permpos.data(), (size_t)N * sizeof(int),
                hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();  // reported here, not by a later call
    return BMPC_ERR_DEVICE;
  }
  return BMPC_OK;
}


}  // namespace bmpc

extern "C" {

const char* bmpc_status_string(bmpc_status st) {
  switch (st) {
    case BMPC_OK: return "ok";
    case BMPC_ERR_INVALID: return "invalid argument";
    case BMPC_ERR_NOT_SPD: return "matrix not positive definite";
    case BMPC_ERR_ALLOC: return "device allocation failed";
    case BMPC_ERR_DEVICE: return "HIP runtime error";
    case BMPC_ERR_STATE: return "solve before factor";
    case BMPC_ERR_NOT_CONVERGED: return "refinement did not converge";
  }
  return "unknown status";
}

bmpc_status bmpc_ordering(int32_t N, int32_t* perm) {
  if (N < 1 || !perm) return BMPC_ERR_INVALID;
  std::vector<int> pr = make_perm(N);
  for (int i = 0; i < N; ++i) perm[i] = pr[i];
  return BMPC_OK;
}

bmpc_status bmpc_structure(int32_t N, int32_t* rows, int32_t* cols, int64_t cap,
                           int64_t* count) {
  if (N < 1 || !count || cap < 0 || (cap > 0 && (!rows || !cols))) return BMPC_ERR_INVALID;
  const int m = N - 1;
  std::vector<int> pp = make_permpos(N);
  std::vector<std::pair<int, int>> b;
  for (int j = 1; j <= N; ++j) b.push_back({pp[j - 1], pp[j - 1]});
  for (int j = 1; j <= m; ++j) {
    const int v = ctz_host((unsigned)j);
    const int jl = j - (1 << v), jr = j + (1 << v);
    if (jl >= 1) b.push_back({pp[jl - 1], pp[j - 1]});
    b.push_back({jr <= m ? pp[jr - 1] : pp[N - 1], pp[j - 1]});
  }
  b.push_back({N, pp[N - 1]});  // F: the root row holds the terminal block only
  b.push_back({N, N});          // L_R
  std::sort(b.begin(), b.end());
  *count = (int64_t)b.size();
  for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)b.size()); ++i) {
    rows[i] = b[i].first;
    cols[i] = b[i].second;
  }
  return BMPC_OK;
}

bmpc_status bmpc_cost_model(const bmpc_dims* dims, bmpc_precision prec,
                            const bmpc_options* opts, bmpc_cost* cost) {
  if (!dims_ok(dims, systems_of(opts)) || !cost ||
      (prec != BMPC_FP64 && prec != BMPC_FP32_REFINE))
    return BMPC_ERR_INVALID;
  const bool fp64 = prec == BMPC_FP64;
  const int Tw = pick_window_depth(fp64, nmax_for(dims->n), dims->nrhs, opts);
  const int Tw2 = pick_later_depth(fp64, nmax_for(dims->n), dims->nrhs, Tw, opts);
  Costs c = make_costs(*dims, fp64, Tw, Tw2, systems_of(opts), no_top_merge_of(opts));
  std::memset(cost, 0, sizeof(*cost));
  cost->factor_flops = c.factor_flops;
  cost->solve_flops = c.solve_flops;
  cost->factor_bytes = c.factor_bytes;
  cost->solve_bytes = c.solve_bytes;
  cost->residual_bytes = c.residual_bytes;
  cost->levels = c.levels;
  cost->passes = (int32_t)c.passes.size();
  cost->window_depth = Tw;
  cost->later_depth = Tw2;
  return BMPC_OK;
}

bmpc_status bmpc_analyze_ex(const bmpc_dims* dims, bmpc_precision prec, void* stream,
                            const bmpc_options* opts, bmpc_plan* out) {
  if (!out) return BMPC_ERR_INVALID;
  *out = nullptr;
  if (!dims_ok(dims, systems_of(opts)) || (prec != BMPC_FP64 && prec != BMPC_FP32_REFINE))
    return BMPC_ERR_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return BMPC_ERR_DEVICE;
  bmpc_plan p = new (std::nothrow) bmpc_plan_s();
  if (!p) return BMPC_ERR_ALLOC;
  const bmpc_status st = init_plan(p, dims, prec, stream, opts);
  if (st != BMPC_OK) {
    free_plan_memory(p);
    delete p;
    return st;
  }
  *out = p;
  return BMPC_OK;
}

bmpc_status bmpc_analyze(const bmpc_dims* dims, bmpc_precision prec, void* stream,
                         bmpc_plan* out) {
  return bmpc_analyze_ex(dims, prec, stream, nullptr, out);
}

bmpc_status bmpc_set_stream(bmpc_plan plan, void* stream) {
  if (!plan) return BMPC_ERR_INVALID;
  plan->stream = reinterpret_cast<hipStream_t>(stream);
  if (plan->ragged)
    for (bmpc_plan s : ragged_subs(plan)) s->stream = plan->stream;
  return BMPC_OK;
}

bmpc_status bmpc_factor(bmpc_plan p, const double* D, const double* E, const double* C,
                        const double* R) {
  if (p && p->ragged) return (D && E && C && R) ? ragged_factor(p, D, E, C, R, nullptr, nullptr)
                                                : BMPC_ERR_INVALID;
  if (!p || !D || !C || !R || (p->d.N > 1 && !E)) return BMPC_ERR_INVALID;
  if (p->fp64)
    enqueue_factor<double>(p, D, E, C, R);
  else
    enqueue_factor<float>(p, D, E, C, R);
  const bmpc_status st = last_error_status();
  if (st == BMPC_OK) p->factored = true;
  return st;
}

bmpc_status bmpc_solve(bmpc_plan p, const double* b, double* x) {
  if (!p || !b || !x) return BMPC_ERR_INVALID;
  if (!p->factored) return BMPC_ERR_STATE;
  if (p->ragged) return ragged_solve(p, b, x);
  if (p->fp64)
    enqueue_solve<double>(p, b, x);
  else
    enqueue_solve<float>(p, b, x);
  return last_error_status();
}

// x = K^{-1} b by refinement (see bmpc_refine); with fused, the factor is issued here
// and the first solve's forward part (first chunk of right-hand sides) runs inside it.
static bmpc_status refine_impl(bmpc_plan p, const double* D, const double* E, const double* C,
                               const double* R, const double* b, double* x, double tol,
                               int32_t max_iters, bool fused) {
  if (!p || !D || !C || !R || !b || !x || (p->d.N > 1 && !E)) return BMPC_ERR_INVALID;
  if (max_iters < 0 || max_iters > 100 || !(tol >= 0.0) || x == b) return BMPC_ERR_INVALID;
  if (!fused && !p->factored) return BMPC_ERR_STATE;
  if (p->ragged) {
    if (!E) return BMPC_ERR_INVALID;
    return ragged_refine(p, D, E, C, R, b, x, tol, max_iters, fused);
  }
  hipStream_t st = p->stream;
  const int nrhs = p->d.nrhs;
  const int segs = p->B * nrhs;  // norms per (system, right-hand side)
  const size_t len = vec_len(p);
  const bool be = p->refine_stop == BMPC_STOP_BACKWARD_ERROR;
  double* rnorm = p->norms;
  double* dnorm = p->norms + segs;
  double* xnorm = p->norms + 2 * segs;
  timed(p, KC_REFINE_MISC, [&] { launch_refine_reset(p->flags, st); });
  if (fused) {
    if (p->fp64)
      enqueue_factor_solve<double>(p, D, E, C, R, b, x);
    else
      enqueue_factor_solve<float>(p, D, E, C, R, b, x);
    if (last_error_status() != BMPC_OK) return BMPC_ERR_DEVICE;
    p->factored = true;
  } else {
    if (p->fp64)
      enqueue_solve<double>(p, b, x);
    else
      enqueue_solve<float>(p, b, x);
  }
  if (be && max_iters >= 0)
    timed(p, KC_REFINE_MISC, [&] { launch_maxabs(b, segs, len, p->npart, p->bnorm, nullptr, st); });
  // r = b - K x for every chunk; the first residual of a backward-error loop also takes
  // the row sums of |K|
  auto residual = [&](bool knorm) {
    for (int c = 0; c < chunks_of(p); ++c) {
      const ResidualArgs ra = residual_args(p, c, D, E, C, R, b, x, p->rbuf, knorm && c == 0);
      timed(p, KC_RESIDUAL, [&] { launch_residual(ra, p->nmax, st); });
      timed(p, KC_RESIDUAL_ROOT, [&] { launch_residual_root(ra, st); });
    }
  };
  // correction solve: reads r / |r|, adds |r| d to x and keeps |r| d in place of r
  auto correction = [&] {
    auto mod = [&](SolveArgs& c, int q0) {
      c.rnorm = rnorm + q0;
      c.dstore = p->rbuf + (size_t)q0 * len;
      c.done = p->flags;
      c.accumulate = 1;
    };
    if (p->fp64)
      enqueue_solve<double>(p, p->rbuf, x, 0, mod);
    else
      enqueue_solve<float>(p, p->rbuf, x, 0, mod);
  };
  bool stopped = false;  // the host saw the stop test hold
  for (int it = 0; it < max_iters; ++it) {
    residual(be && it == 0);
    if (be) {
      // stop before the correction when x is already backward stable
      timed(p, KC_REFINE_MISC, [&] {
        launch_refine_be_check(p->rbuf, x, p->B, nrhs, len, p->npart, it == 0 ? p->kpart : nullptr,
                               p->kper, p->kroot, p->knorm, p->bnorm, tol, 1, p->flags,
                               p->relcorr, rnorm, st);
      });
      // The first solve of an FP32 plan cannot meet a tolerance far below FP32's
      // rounding, so the host does not wait for that check (the device still applies it:
      // the later launches of a converged loop return at once).
      const bool hopeless = it == 0 && !p->fp64 && tol < 0x1p-30;
      if (!hopeless && (stopped = stop_reached(p))) break;
    } else {
      timed(p, KC_REFINE_MISC, [&] {
        launch_maxabs(p->rbuf, segs, len, p->npart, rnorm, p->flags, st);
      });
    }
    correction();
    if (!be) {
      timed(p, KC_REFINE_MISC, [&] {
        launch_refine_check(p->rbuf, x, segs, len, p->npart, tol, p->flags, p->relcorr, dnorm,
                            xnorm, st);
      });
      if (it + 1 < max_iters && (stopped = stop_reached(p))) break;
    }
  }
  if (be && !stopped) {
    // the returned x is certified by its own residual
    residual(max_iters == 0);
    timed(p, KC_REFINE_MISC, [&] {
      launch_refine_be_check(p->rbuf, x, p->B, nrhs, len, p->npart,
                             max_iters == 0 ? p->kpart : nullptr, p->kper, p->kroot, p->knorm,
                             p->bnorm, tol, 0, p->flags, p->relcorr, rnorm, st);
    });
  }
  p->last_max_iters = be ? std::max(max_iters, 1) : max_iters;
  return last_error_status();
}

bmpc_status bmpc_refine(bmpc_plan p, const double* D, const double* E, const double* C,
                        const double* R, const double* b, double* x, double tol,
                        int32_t max_iters) {
  return refine_impl(p, D, E, C, R, b, x, tol, max_iters, false);
}

bmpc_status bmpc_factor_refine(bmpc_plan p, const double* D, const double* E, const double* C,
                               const double* R, const double* b, double* x, double tol,
                               int32_t max_iters) {
  return refine_impl(p, D, E, C, R, b, x, tol, max_iters, true);
}

bmpc_status bmpc_factor_solve(bmpc_plan p, const double* D, const double* E, const double* C,
                              const double* R, const double* b, double* x) {
  if (!p || !D || !C || !R || !b || !x || (p->d.N > 1 && !E)) return BMPC_ERR_INVALID;
  if (p->ragged) return E ? ragged_factor(p, D, E, C, R, b, x) : BMPC_ERR_INVALID;
  if (p->fp64)
    enqueue_factor_solve<double>(p, D, E, C, R, b, x);
  else
    enqueue_factor_solve<float>(p, D, E, C, R, b, x);
  const bmpc_status st = last_error_status();
  if (st == BMPC_OK) p->factored = true;
  return st;
}

bmpc_status bmpc_set_refine_stop(bmpc_plan p, int32_t stop) {
  if (!p || (stop != BMPC_STOP_CORRECTION && stop != BMPC_STOP_BACKWARD_ERROR))
    return BMPC_ERR_INVALID;
  p->refine_stop = stop;
  return BMPC_OK;
}

bmpc_status bmpc_query_structure(bmpc_plan p, int32_t* rows, int32_t* cols, int64_t cap,
                                 int64_t* count) {
  if (!p || p->ragged) return BMPC_ERR_INVALID;
  return bmpc_structure(p->d.N, rows, cols, cap, count);
}

bmpc_status bmpc_grad_blocks(bmpc_plan p, const double* x, const double* lam, double* dD,
                             double* dE, double* dC, double* dR) {
  if (!p || !x || !lam || p->ragged) return BMPC_ERR_INVALID;
  GradArgs g{};
  g.S = p->d.S;
  g.B = p->B;
  g.N = p->d.N;
  g.n = p->d.n;
  g.nrhs = p->d.nrhs;
  g.x = x;
  g.lam = lam;
  g.dD = dD;
  g.dE = p->d.N > 1 ? dE : nullptr;
  g.dC = dC;
  g.dR = dR;
  timed(p, KC_GRAD_BLOCKS, [&] { launch_grad_blocks(g, p->stream); });
  return last_error_status();
}

bmpc_status bmpc_get_info(bmpc_plan p, int64_t* info) {
  if (!p || !info) return BMPC_ERR_INVALID;
  if (p->ragged) return ragged_info(p, info);
  unsigned long long v = 0;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return BMPC_ERR_DEVICE;
  if (hipMemcpy(&v, p->d_info, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
    return BMPC_ERR_DEVICE;
  if (v == ~0ull || !p->factored) {
    *info = 0;
    return BMPC_OK;
  }
  // recorded: system base + tail base + permuted position * n + row (1-based);
  // reported: the same row in natural stage order
  const int64_t Nn = (int64_t)p->d.N * p->d.n, n = p->d.n;
  const int64_t sys_rows = (int64_t)p->d.S * Nn + n;
  const int64_t p0 = (int64_t)v - 1;
  const int64_t sys = p0 / sys_rows, r0 = p0 % sys_rows;
  if (r0 < (int64_t)p->d.S * Nn) {
    const int64_t s = r0 / Nn, rem = r0 % Nn, pos = rem / n, i = rem % n;
    *info = sys * sys_rows + s * Nn + (int64_t)p->perm[pos] * n + i + 1;
  } else {
    *info = (int64_t)v;
  }
  return BMPC_ERR_NOT_SPD;
}

bmpc_status bmpc_get_stats(bmpc_plan p, int32_t* iters, double* rel_correction) {
  if (!p) return BMPC_ERR_INVALID;
  int flags[2] = {0, 0};
  double rel = 0.0;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return BMPC_ERR_DEVICE;
  if (hipMemcpy(flags, p->flags, sizeof(flags), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&rel, p->relcorr, sizeof(rel), hipMemcpyDeviceToHost) != hipSuccess)
    return BMPC_ERR_DEVICE;
  if (iters) *iters = flags[1];
  if (rel_correction) *rel_correction = rel;
  if (p->last_max_iters > 0 && !flags[0]) return BMPC_ERR_NOT_CONVERGED;
  return BMPC_OK;
}

bmpc_status bmpc_query_perm(bmpc_plan p, int32_t* perm) {
  if (!p || !perm || p->ragged) return BMPC_ERR_INVALID;
  for (int i = 0; i < p->d.N; ++i) perm[i] = p->perm[i];
  return BMPC_OK;
}

bmpc_status bmpc_query_cost(bmpc_plan p, bmpc_cost* cost) {
  if (!p || !cost) return BMPC_ERR_INVALID;
  std::memset(cost, 0, sizeof(*cost));
  if (p->ragged) {  // sums over the systems; levels and passes of the deepest one
    for (bmpc_plan s : ragged_subs(p)) {
      cost->factor_flops += s->costs.factor_flops;
      cost->solve_flops += s->costs.solve_flops;
      cost->factor_bytes += s->costs.factor_bytes;
      cost->solve_bytes += s->costs.solve_bytes;
      cost->residual_bytes += s->costs.residual_bytes;
      cost->levels = std::max(cost->levels, s->costs.levels);
      cost->passes = std::max(cost->passes, (int32_t)s->costs.passes.size());
      cost->window_depth = std::max(cost->window_depth, s->Tw);
      cost->later_depth = std::max(cost->later_depth, s->Tw2);
    }
    cost->workspace_bytes = p->workspace_bytes;
    return BMPC_OK;
  }
  cost->factor_flops = p->costs.factor_flops;
  cost->solve_flops = p->costs.solve_flops;
  cost->factor_bytes = p->costs.factor_bytes;
  cost->solve_bytes = p->costs.solve_bytes;
  cost->residual_bytes = p->costs.residual_bytes;
  cost->levels = p->costs.levels;
  cost->passes = (int32_t)p->costs.passes.size();
  cost->window_depth = p->Tw;
  cost->later_depth = p->Tw2;
  cost->workspace_bytes = p->workspace_bytes;
  return BMPC_OK;
}

bmpc_status bmpc_query_kernel_cost(bmpc_plan p, int32_t cls, double* bytes, double* flops,
                                   int32_t* launches) {
  if (!p || cls < 0 || cls >= KC_COUNT) return BMPC_ERR_INVALID;
  if (p->ragged) {  // sums over the systems; launches: not defined per system
    double by = 0, fl = 0;
    for (bmpc_plan s : ragged_subs(p)) {
      by += s->costs.pass_bytes[cls];
      fl += s->costs.pass_flops[cls];
    }
    if (bytes) *bytes = by;
    if (flops) *flops = fl;
    if (launches) *launches = 0;
    return BMPC_OK;
  }
  if (bytes) *bytes = p->costs.pass_bytes[cls];
  if (flops) *flops = p->costs.pass_flops[cls];
  if (launches) *launches = p->costs.launches[cls];
  return BMPC_OK;
}

bmpc_status bmpc_export_tail_factor(bmpc_plan p, int32_t s, double* L, double* F) {
  if (p && p->ragged) {  // chain s of the concatenated systems
    if (!p->factored) return BMPC_ERR_STATE;
    (void)hipStreamSynchronize(p->stream);
    for (bmpc_plan sub : ragged_subs(p)) {
      if (s < sub->d.S) return bmpc_export_tail_factor(sub, s, L, F);
      s -= sub->d.S;
    }
    return BMPC_ERR_INVALID;
  }
  if (!p || !L || !F || s < 0 || s >= p->B * p->d.S) return BMPC_ERR_INVALID;
  if (!p->factored) return BMPC_ERR_STATE;
  const int N = p->d.N, n = p->d.n, m = p->m;
  const size_t nn = (size_t)n * n, tb = p->fp64 ? 8 : 4;
  const size_t gblocks = (size_t)(N > 1 ? N - 1 : 1);  // blocks copied per chain
  std::vector<unsigned char> li(N * nn * tb), gl(gblocks * nn * tb), gr(gblocks * nn * tb),
      f(nn * tb);
  if (hipStreamSynchronize(p->stream) != hipSuccess) return BMPC_ERR_DEVICE;
  auto cp = [&](void* dst, const void* src, size_t off, size_t bytes) {
    return hipMemcpy(dst, (const unsigned char*)src + off, bytes, hipMemcpyDeviceToHost) ==
           hipSuccess;
  };
  if (!cp(li.data(), p->Linv, (size_t)s * N * nn * tb, li.size()) ||
      !cp(gl.data(), p->Gl, (size_t)s * g_chain_blocks(N) * nn * tb, gl.size()) ||
      !cp(gr.data(), p->Gr, (size_t)s * g_chain_blocks(N) * nn * tb, gr.size()) ||
      !cp(f.data(), p->F, (size_t)s * nn * tb, f.size()))
    return BMPC_ERR_DEVICE;
  auto val = [&](const std::vector<unsigned char>& buf, size_t idx) -> double {
    if (p->fp64) return reinterpret_cast<const double*>(buf.data())[idx];
    return (double)reinterpret_cast<const float*>(buf.data())[idx];
  };
  const size_t Nn = (size_t)N * n;
  std::memset(L, 0, sizeof(double) * Nn * Nn);
  auto put = [&](int rowpos, int colpos, const std::vector<unsigned char>& buf, size_t blk) {
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c)
        L[((size_t)rowpos * n + r) * Nn + (size_t)colpos * n + c] = val(buf, blk * nn + r * n + c);
  };
  const std::vector<int>& pp = p->permpos;
  // diagonal blocks (inverted) are stored packed by rows
  for (int j = 1; j <= N; ++j)
    for (int r = 0; r < n; ++r)
      for (int c = 0; c <= r; ++c)
        L[((size_t)pp[j - 1] * n + r) * Nn + (size_t)pp[j - 1] * n + c] =
            val(li, (size_t)(j - 1) * nn + (size_t)r * (r + 1) / 2 + c);
  for (int j = 1; j <= m; ++j) {
    const int v = ctz_host((unsigned)j);
    const int jl = j - (1 << v), jr = j + (1 << v);
    if (jl >= 1) put(pp[jl - 1], pp[j - 1], gl, j - 1);
    put(jr <= m ? pp[jr - 1] : pp[N - 1], pp[j - 1], gr, j - 1);
  }
  for (size_t e = 0; e < nn; ++e) F[e] = val(f, e);
  return BMPC_OK;
}

bmpc_status bmpc_export_root_factor(bmpc_plan p, double* LR) {
  if (!p || !LR) return BMPC_ERR_INVALID;
  if (!p->factored) return BMPC_ERR_STATE;
  if (p->ragged) {  // the systems' n_i x n_i root factors one after the other
    if (hipStreamSynchronize(p->stream) != hipSuccess) return BMPC_ERR_DEVICE;
    for (bmpc_plan sub : ragged_subs(p)) {
      const size_t nn = (size_t)sub->d.n * sub->d.n;
      if (hipMemcpy(LR, sub->LR, nn * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return BMPC_ERR_DEVICE;
      LR += nn;
    }
    return BMPC_OK;
  }
  if (hipStreamSynchronize(p->stream) != hipSuccess) return BMPC_ERR_DEVICE;
  if (hipMemcpy(LR, p->LR, (size_t)p->B * p->d.n * p->d.n * 8, hipMemcpyDeviceToHost) !=
      hipSuccess)
    return BMPC_ERR_DEVICE;
  return BMPC_OK;
}

bmpc_status bmpc_set_profiling(bmpc_plan p, int32_t enable) {
  if (!p) return BMPC_ERR_INVALID;
  if (!enable) collect_timings(p);
  p->profiling = enable != 0;
  return BMPC_OK;
}

bmpc_status bmpc_get_kernel_times(bmpc_plan p, int32_t max_classes, int64_t* launches,
                                  double* total_ms) {
  if (!p || max_classes < 0 || (max_classes > 0 && (!launches || !total_ms)))
    return BMPC_ERR_INVALID;
  collect_timings(p);
  for (int c = 0; c < std::min<int>(max_classes, KC_COUNT); ++c) {
    launches[c] = p->launches[c];
    total_ms[c] = p->total_ms[c];
  }
  return BMPC_OK;
}

bmpc_status bmpc_reset_kernel_times(bmpc_plan p) {
  if (!p) return BMPC_ERR_INVALID;
  collect_timings(p);
  for (int c = 0; c < KC_COUNT; ++c) {
    p->launches[c] = 0;
    p->total_ms[c] = 0.0;
  }
  return BMPC_OK;
}

int32_t bmpc_kernel_class_count(void) { return KC_COUNT; }

const char* bmpc_kernel_class_name(int32_t cls) {
  static const char* names[KC_COUNT] = {
      "factor_init",  "factor_first_pass", "factor_mid_pass", "factor_final_pass",
      "root_reduce",  "root_potrf",        "solve_fwd",       "solve_x_fwd",
      "solve_root",   "solve_x_bwd",       "solve_bwd",       "residual",
      "residual_root", "refine_misc",     "grad_blocks",     "factor_level1_inverse"};
  if (cls < 0 || cls >= KC_COUNT) return "";
  return names[cls];
}

bmpc_status bmpc_destroy(bmpc_plan p) {
  if (!p) return BMPC_ERR_INVALID;
  (void)hipStreamSynchronize(p->stream);
  ragged_destroy(p);
  free_plan_memory(p);
  delete p;
  return BMPC_OK;
}

}  // extern "C"
