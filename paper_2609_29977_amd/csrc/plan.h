// The plan object behind the C ABI and the host helpers its entry points share
// (api.hip: one system or a uniform batch; ragged.hip: systems of different shapes).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "bmpc.h"
#include "bmpc_internal.h"
#include "multi.h"

namespace bmpc {

constexpr int kLdsBudget = 160 * 1024;

struct PassPlan {
  int mk, shift, windows, is_final, tw;  // tw: levels of this pass
  double flops, bytes;  // algorithmic flops / HBM bytes of the pass
};

struct Timing {
  int cls;
  hipEvent_t a, b;
};

struct Costs {
  std::vector<PassPlan> passes;
  double factor_flops = 0, solve_flops = 0, factor_bytes = 0, solve_bytes = 0,
         residual_bytes = 0, L_bytes = 0;
  double pass_flops[KC_COUNT] = {0}, pass_bytes[KC_COUNT] = {0};
  int launches[KC_COUNT] = {0};
  int levels = 0, Tw = 0, Tw2 = 0;
};

struct RaggedState;  // ragged.hip

}  // namespace bmpc

struct bmpc_plan_s {
  // a ragged batch: one uniform plan per system, launched together (ragged.hip)
  bmpc::RaggedState* ragged = nullptr;
  bmpc_dims d{};
  bmpc_precision prec = BMPC_FP64;
  bool fp64 = true;
  int m = 0, nmax = 8, Tw = 1, Tw2 = 1, groups = 1;
  int B = 1;      // systems in the batch
  int opt_flags = 0;  // BMPC_FLAG_*
  int chunk = bmpc::kMaxRhs;  // right-hand sides per launch
  int refine_stop = BMPC_STOP_CORRECTION;
  hipStream_t stream = nullptr;
  bmpc::Costs costs;
  std::vector<int> perm, permpos;
  int stride = 1;
  // device buffers
  void* Linv = nullptr;
  void* Gl = nullptr;
  void* Gr = nullptr;
  void* F = nullptr;
  double* U = nullptr;
  double* Upart = nullptr;
  double* LR = nullptr;
  void* acc[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  void* accX = nullptr;
  void* vacc[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // fused forward: R, L
  void* vaccX = nullptr;
  int* d_permpos = nullptr;
  unsigned long long* d_info = nullptr;
  void* y = nullptr;
  double* w = nullptr;
  double* x0 = nullptr;
  double* rbuf = nullptr;
  double* norms = nullptr;  // rnorm, dnorm, xnorm: 3 * nrhs
  double* npart = nullptr;  // partial maxima: 2 * nrhs * kNormBlocks
  int* flags = nullptr;     // done, iterations
  double* relcorr = nullptr;
  // backward-error stop: |b| per segment, |K| per system, the residual's row-sum
  // partials (per tail workgroup), root-row maxima and per-chain |C_s| row sums
  double* bnorm = nullptr;
  double* knorm = nullptr;
  double* kpart = nullptr;
  double* kroot = nullptr;
  double* crow = nullptr;
  int kper = 0;  // residual workgroups per system
  int* hflag = nullptr;  // pinned host copy of the refinement's stop flag
  // Workspace placement: measure (only add up the sizes), or carve from an arena owned
  // by a ragged parent; otherwise each buffer is its own allocation.
  bool measure = false;
  char* arena = nullptr;
  size_t arena_used = 0;
  bmpc_plan_s* parent = nullptr;  // ragged batch this plan is one system of
  std::vector<void*> allocs;
  double workspace_bytes = 0;
  bool factored = false;
  int last_max_iters = 0;
  // profiling
  bool profiling = false;
  std::vector<bmpc::Timing> timings;
  std::vector<hipEvent_t> event_pool;
  int64_t launches[bmpc::KC_COUNT] = {0};
  double total_ms[bmpc::KC_COUNT] = {0};
};

namespace bmpc {

size_t factor_pass_lds_bytes(bool fp64, int nmax, int Tw, int nrhs_fused);
int pick_later_depth(bool fp64, int nmax, int nrhs, int Tw, const bmpc_options* o);
int nmax_for(int n);
Costs make_costs(const bmpc_dims& d, bool fp64, int Tw, int Tw2, int B, bool no_top_merge);
std::vector<int> make_permpos(int N);
std::vector<int> make_perm(int N);
bool dims_ok(const bmpc_dims* d, int B = 1);
int flags_of(const bmpc_options* o);
bool no_top_merge_of(const bmpc_options* o);
int pick_window_depth(bool fp64, int nmax, int nrhs, const bmpc_options* o);
bool dalloc(bmpc_plan p, void** ptr, size_t bytes);
void free_plan_memory(bmpc_plan p);
bmpc_status last_error_status();
size_t vec_len(bmpc_plan p);
int chunks_of(bmpc_plan p);
int chunk_rhs(bmpc_plan p, int c);
SolveArgs solve_args(bmpc_plan p, const double* b, double* x, int q0, int nq);
FactorPassArgs factor_pass_args(bmpc_plan p, int k, const double* D, const double* E,
                                const double* C, const double* b, int nq);
ResidualArgs residual_args(bmpc_plan p, int c, const double* D, const double* E,
                           const double* C, const double* R, const double* b, const double* x,
                           double* r, bool knorm);
// Builds a plan's analysis and workspaces (everything bmpc_analyze_ex does after the
// argument checks); with a ragged parent the workspaces come from its arena.
bmpc_status init_plan(bmpc_plan p, const bmpc_dims* dims, bmpc_precision prec, void* stream,
                      const bmpc_options* opts);
bool stop_reached(bmpc_plan p);

// ragged.hip
bmpc_status ragged_factor(bmpc_plan p, const double* D, const double* E, const double* C,
                          const double* R, const double* b, double* x);
bmpc_status ragged_solve(bmpc_plan p, const double* b, double* x);
bmpc_status ragged_refine(bmpc_plan p, const double* D, const double* E, const double* C,
                          const double* R, const double* b, double* x, double tol,
                          int max_iters, bool fused);
void ragged_destroy(bmpc_plan p);
bmpc_status ragged_info(bmpc_plan p, int64_t* info);
const std::vector<bmpc_plan>& ragged_subs(bmpc_plan p);

inline hipEvent_t take_event(bmpc_plan p) {
  if (!p->event_pool.empty()) {
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Bracket a launch with events when profiling is on.
template <typename F>
void timed(bmpc_plan p, int cls, F&& launch) {
  if (!p->profiling) {
    launch();
    return;
  }
  Timing t{cls, take_event(p), take_event(p)};
  (void)hipEventRecord(t.a, p->stream);
  launch();
  (void)hipEventRecord(t.b, p->stream);
  p->timings.push_back(t);
}

inline void collect_timings(bmpc_plan p) {
  if (p->timings.empty()) return;
  (void)hipEventSynchronize(p->timings.back().b);
  for (const Timing& t : p->timings) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      p->launches[t.cls] += 1;
      p->total_ms[t.cls] += ms;
    }
    p->event_pool.push_back(t.a);
    p->event_pool.push_back(t.b);
  }
  p->timings.clear();
}

// Right-hand sides per plan: no limit of the method; this bound keeps the per-segment
// norm arrays and index arithmetic small.
constexpr int kMaxPlanRhs = 4096;

}  // namespace bmpc
