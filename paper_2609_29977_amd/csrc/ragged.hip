// Ragged batches: independent systems of different shapes (S, N, n) in one plan.
//
// Each system is analysed as its own one-system plan (ordering Pi_i, level table,
// passes, workspaces carved from one allocation), and every step of the factor, solve
// and refinement sequences becomes one launch over all the systems that take part in
// it (per block-size class and kernel variant): the work items of a launch are the
// systems' chain windows, chain positions or root blocks, the largest systems first
// (see multi.h).  The per-system argument tables are built here once; a call only
// passes the caller's base pointers, so calls can be captured into a HIP graph.
// Systems with more stages simply take part in more pass and level launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "plan.h"

namespace bmpc {

enum RaggedOp {
  RO_INFO_RESET = 0,
  RO_FACTOR,
  RO_ROOT_REDUCE,
  RO_ROOT_POTRF,
  RO_SOLVE,
  RO_RESIDUAL,
  RO_RESIDUAL_ROOT,
  RO_L1INV
};

struct LaunchRec {
  int op = 0, cls = 0;
  int nmax = 32, kind = 0;
  bool first = false, final = false, fwd = false, full = false;
  size_t table = 0;  // byte offset of the item table in the device table buffer
  int nitems = 0;
  unsigned blocks = 0, threads = 0;
  size_t lds = 0;
};
typedef std::vector<LaunchRec> Seq;

struct RaggedState {
  std::vector<bmpc_plan> subs;
  std::vector<int> rank;  // position of each system in the item order (largest work first)
  std::vector<size_t> offD, offE, offC, offR, offV, rows;  // element offsets (B + 1 each)
  int nrhs = 1, chunk = kMaxRhs, chunks = 1;
  char* arena = nullptr;
  char* dtab = nullptr;
  std::vector<unsigned char> htab;
  Seq factor[2];               // [forward substitution of the first chunk inside]
  Seq back0;                   // after a fused factor: root step and backward sweep, chunk 0
  std::vector<Seq> solve, corr;  // per chunk: plain solve, refinement correction
  std::vector<Seq> resid[2];   // per chunk [with the row sums of |K|]
  unsigned long long* info = nullptr;  // per system
  double* rbuf = nullptr;      // residual / correction vectors, the callers' vector layout
  int nseg = 0;
  SegRec* segs = nullptr;
  int* seg_sys = nullptr;
  int* kp_off = nullptr;
  double *rnorm = nullptr, *dnorm = nullptr, *xnorm = nullptr, *bnorm = nullptr;
  double *knorm = nullptr, *kpart = nullptr, *kroot = nullptr, *worst = nullptr;
  int* ok = nullptr;
  std::vector<void*> allocs;
};

namespace {

template <class Args>
struct Pending {
  int sys;
  Args a;
  int p0, p1;
  unsigned gx, gy, gz;
};

// Appends a launch whose items are the given systems' entries, largest work first.
template <class Args>
void emit(RaggedState& R, Seq& seq, LaunchRec rec, std::vector<Pending<Args>> items) {
  if (items.empty()) return;
  std::sort(items.begin(), items.end(),
            [&](const Pending<Args>& x, const Pending<Args>& y) { return R.rank[x.sys] < R.rank[y.sys]; });
  size_t off = (R.htab.size() + 255) & ~(size_t)255;
  R.htab.resize(off + items.size() * sizeof(MultiItem<Args>));
  MultiItem<Args>* t = reinterpret_cast<MultiItem<Args>*>(R.htab.data() + off);
  unsigned start = 0;
  for (size_t k = 0; k < items.size(); ++k) {
    MultiItem<Args> it{};
    it.a = items[k].a;
    it.p0 = items[k].p0;
    it.p1 = items[k].p1;
    it.start = start;
    it.gx = items[k].gx;
    it.gy = items[k].gy;
    std::memcpy(&t[k], &it, sizeof(it));
    start += items[k].gx * items[k].gy * items[k].gz;
  }
  rec.table = off;
  rec.nitems = (int)items.size();
  rec.blocks = start;
  if (start > 0) seq.push_back(rec);
}

int nclass(int n) { return n <= 8 ? 8 : (n <= 16 ? 16 : 32); }

const double* fake(size_t el) { return rel_field<const double>(el); }
double* fake_w(size_t el) { return rel_field<double>(el); }

// The steps of one solve chunk from the root step on (root step, x_1 backward step,
// merged top backward levels, backward levels).
void build_back(RaggedState& R, Seq& seq, const std::vector<SolveArgs>& args, int q0) {
  (void)q0;
  const int B = (int)R.subs.size();
  {
    std::vector<Pending<SolveArgs>> items;
    for (int i = 0; i < B; ++i) items.push_back({i, args[i], 0, 0, 1u, 1u, 1u});
    LaunchRec rec;
    rec.op = RO_SOLVE;
    rec.cls = KC_SOLVE_ROOT;
    rec.kind = SK_ROOT;
    rec.threads = 1024;
    emit(R, seq, rec, items);
  }
  std::map<int, std::vector<Pending<SolveArgs>>> xb, top;
  int maxL = 0;
  std::vector<int> topl(B), L(B);
  for (int i = 0; i < B; ++i) {
    bmpc_plan s = R.subs[i];
    xb[s->nmax].push_back({i, args[i], 0, 0, (unsigned)s->d.S, 1u, 1u});
    L[i] = chain_levels(s->m);
    topl[i] = (s->opt_flags & BMPC_FLAG_NO_BWD_TOP_MERGE)
                  ? L[i] + 1
                  : bwd_top_level(s->m, s->d.n, args[i].nrhs, s->d.S, 1);
    if (topl[i] <= L[i]) top[s->nmax].push_back({i, args[i], topl[i], 0, (unsigned)s->d.S, 1u, 1u});
    maxL = std::max(maxL, L[i]);
  }
  for (auto& g : xb) {
    LaunchRec rec;
    rec.op = RO_SOLVE;
    rec.cls = KC_SOLVE_X_BWD;
    rec.kind = SK_X_BWD;
    rec.nmax = g.first;
    rec.threads = kSolveThreads;
    emit(R, seq, rec, g.second);
  }
  for (auto& g : top) {
    LaunchRec rec;
    rec.op = RO_SOLVE;
    rec.cls = KC_SOLVE_BWD;
    rec.kind = SK_BWD_TOP;
    rec.nmax = g.first;
    rec.threads = 64 * kBwdTopWaves;
    emit(R, seq, rec, g.second);
  }
  for (int l = maxL; l >= 1; --l) {
    std::map<std::tuple<int, int, bool>, std::vector<Pending<SolveArgs>>> groups;
    std::map<std::tuple<int, int, bool>, LaunchRec> recs;
    for (int i = 0; i < B; ++i) {
      bmpc_plan s = R.subs[i];
      if (l > L[i] || l >= topl[i]) continue;
      const LevelCfg c = solve_level_config(args[i], l, false, s->nmax, s->fp64);
      if (c.count <= 0) continue;
      const auto key = std::make_tuple(s->nmax, c.kind, c.full);
      groups[key].push_back({i, args[i], l, c.count, c.gx, c.gy, c.gz});
      LaunchRec& rec = recs[key];
      rec.op = RO_SOLVE;
      rec.cls = KC_SOLVE_BWD;
      rec.kind = c.kind;
      rec.nmax = s->nmax;
      rec.fwd = false;
      rec.full = c.full;
      rec.threads = c.threads;
      rec.lds = std::max(rec.lds, c.lds);
    }
    for (auto& g : groups) emit(R, seq, recs[g.first], g.second);
  }
}

// Forward sweep and x_1 forward step of one chunk.
void build_fwd(RaggedState& R, Seq& seq, const std::vector<SolveArgs>& args) {
  const int B = (int)R.subs.size();
  int maxL = 0;
  for (int i = 0; i < B; ++i) maxL = std::max(maxL, chain_levels(R.subs[i]->m));
  for (int l = 1; l <= maxL; ++l) {
    std::map<std::tuple<int, int, bool>, std::vector<Pending<SolveArgs>>> groups;
    std::map<std::tuple<int, int, bool>, LaunchRec> recs;
    for (int i = 0; i < B; ++i) {
      bmpc_plan s = R.subs[i];
      if (l > chain_levels(s->m)) continue;
      const LevelCfg c = solve_level_config(args[i], l, true, s->nmax, s->fp64);
      if (c.count <= 0) continue;
      const auto key = std::make_tuple(s->nmax, c.kind, c.full);
      groups[key].push_back({i, args[i], l, c.count, c.gx, c.gy, c.gz});
      LaunchRec& rec = recs[key];
      rec.op = RO_SOLVE;
      rec.cls = KC_SOLVE_FWD;
      rec.kind = c.kind;
      rec.nmax = s->nmax;
      rec.fwd = true;
      rec.full = c.full;
      rec.threads = std::max(rec.threads, c.threads);
      rec.lds = std::max(rec.lds, c.lds);
    }
    for (auto& g : groups) emit(R, seq, recs[g.first], g.second);
  }
  std::map<int, std::vector<Pending<SolveArgs>>> xf;
  for (int i = 0; i < B; ++i)
    xf[R.subs[i]->nmax].push_back({i, args[i], 0, 0, (unsigned)R.subs[i]->d.S, 1u, 1u});
  for (auto& g : xf) {
    LaunchRec rec;
    rec.op = RO_SOLVE;
    rec.cls = KC_SOLVE_X_FWD;
    rec.kind = SK_X_FWD;
    rec.nmax = g.first;
    rec.threads = kSolveThreads;
    emit(R, seq, rec, g.second);
  }
}

// Solve arguments of chunk c for every system (correction: the refinement's scaled
// solve that adds its result to x).
std::vector<SolveArgs> chunk_args(bmpc_plan p, int c, bool correction) {
  RaggedState& R = *p->ragged;
  std::vector<SolveArgs> args;
  for (size_t i = 0; i < R.subs.size(); ++i) {
    bmpc_plan s = R.subs[i];
    SolveArgs a = solve_args(s, fake(R.offV[i]), fake_w(R.offV[i]), c * R.chunk,
                             chunk_rhs(s, c));
    if (correction) {
      a.rnorm = R.rnorm + i * R.nrhs + c * R.chunk;
      a.dstore = fake_w(R.offV[i] + (size_t)c * R.chunk * vec_len(s));
      a.done = p->flags;
      a.accumulate = 1;
    }
    args.push_back(a);
  }
  return args;
}

void build_factor(bmpc_plan p, Seq& seq, bool fused) {
  RaggedState& R = *p->ragged;
  const int B = (int)R.subs.size();
  {
    LaunchRec rec;
    rec.op = RO_INFO_RESET;
    rec.cls = KC_FACTOR_INIT;
    seq.push_back(rec);
  }
  {
    // level-1 inverses of every system's first pass, one launch per tile size and
    // n == NMAX (level1_blocks_per_wave blocks per wave, four waves per workgroup)
    std::map<std::tuple<int, bool>, std::vector<Pending<FactorPassArgs>>> groups;
    for (int i = 0; i < B; ++i) {
      bmpc_plan s = R.subs[i];
      const int nodd = s->d.N / 2;  // odd positions 1, 3, .. of the N - 1 chain positions
      if (nodd == 0) continue;
      const FactorPassArgs a = factor_pass_args(s, 0, fake(R.offD[i]), fake(R.offE[i]),
                                                fake(R.offC[i]), nullptr, 0);
      const unsigned total = (unsigned)(s->B * s->d.S) * (unsigned)nodd;
      const unsigned per_wg =
          4u * (unsigned)level1_blocks_per_wave(s->nmax, p->prec == BMPC_FP64);
      groups[std::make_tuple(s->nmax, s->d.n == s->nmax)].push_back(
          {i, a, nodd, (int)total, (total + per_wg - 1) / per_wg, 1u, 1u});
    }
    for (auto& g : groups) {
      LaunchRec rec;
      rec.op = RO_L1INV;
      rec.cls = KC_FACTOR_L1INV;
      rec.nmax = std::get<0>(g.first);
      rec.full = std::get<1>(g.first);
      emit(R, seq, rec, g.second);
    }
  }
  int maxpass = 0;
  for (bmpc_plan s : R.subs) maxpass = std::max(maxpass, (int)s->costs.passes.size());
  for (int k = 0; k < maxpass; ++k) {
    std::map<std::tuple<int, bool, bool>, std::vector<Pending<FactorPassArgs>>> groups;
    std::map<std::tuple<int, bool, bool>, LaunchRec> recs;
    for (int i = 0; i < B; ++i) {
      bmpc_plan s = R.subs[i];
      const int np = (int)s->costs.passes.size();
      if (k >= np) continue;
      const int nq = fused ? chunk_rhs(s, 0) : 0;
      const FactorPassArgs a = factor_pass_args(s, k, fake(R.offD[i]), fake(R.offE[i]),
                                                fake(R.offC[i]), fused ? fake(R.offV[i]) : nullptr,
                                                nq);
      const bool fin = k == np - 1;
      const bool full = s->d.n == s->nmax;
      const auto key = std::make_tuple(s->nmax, fin, full);
      groups[key].push_back({i, a, 0, 0, (unsigned)(s->d.S * s->costs.passes[k].windows), 1u, 1u});
      LaunchRec& rec = recs[key];
      rec.op = RO_FACTOR;
      rec.full = full;
      rec.cls = fin ? KC_FACTOR_FINAL : (k == 0 ? KC_FACTOR_FIRST : KC_FACTOR_MID);
      rec.nmax = s->nmax;
      rec.first = k == 0;
      rec.final = fin;
      rec.fwd = fused;
      rec.lds = std::max(rec.lds,
                         factor_pass_lds_bytes(s->fp64, s->nmax, s->costs.passes[k].tw, nq));
    }
    for (auto& g : groups) emit(R, seq, recs[g.first], g.second);
  }
  std::vector<Pending<RootArgs>> red;
  std::map<int, std::vector<Pending<RootArgs>>> pot;
  for (int i = 0; i < B; ++i) {
    bmpc_plan s = R.subs[i];
    RootArgs ra{};
    ra.U = s->U;
    ra.part = s->Upart;
    ra.R = fake(R.offR[i]);
    ra.LR = s->LR;
    ra.info = s->d_info;
    ra.S = s->d.S;
    ra.n = s->d.n;
    ra.groups = s->groups;
    ra.root_row = (unsigned long long)s->d.S * s->d.N * s->d.n;
    ra.sys_rows = ra.root_row + s->d.n;
    red.push_back({i, ra, 0, 0, (unsigned)s->groups, 1u, 1u});
    pot[s->d.n <= 16 ? 16 : 32].push_back({i, ra, 0, 0, 1u, 1u, 1u});
  }
  LaunchRec rr;
  rr.op = RO_ROOT_REDUCE;
  rr.cls = KC_ROOT_REDUCE;
  emit(R, seq, rr, red);
  for (auto& g : pot) {
    LaunchRec rp;
    rp.op = RO_ROOT_POTRF;
    rp.cls = KC_ROOT_POTRF;
    rp.nmax = g.first;
    emit(R, seq, rp, g.second);
  }
}

void build_residual(bmpc_plan p, Seq& seq, int c, bool knorm) {
  RaggedState& R = *p->ragged;
  const int B = (int)R.subs.size();
  std::map<std::tuple<int, bool>, std::vector<Pending<ResidualArgs>>> groups;
  std::map<std::tuple<int, bool>, LaunchRec> recs;
  std::vector<Pending<ResidualArgs>> roots;
  for (int i = 0; i < B; ++i) {
    bmpc_plan s = R.subs[i];
    ResidualArgs ra = residual_args(s, c, fake(R.offD[i]), fake(R.offE[i]), fake(R.offC[i]),
                                    fake(R.offR[i]), fake(R.offV[i]), fake(R.offV[i]),
                                    fake_w(R.offV[i]), knorm && c == 0);
    ra.done = p->flags;
    const int chunks = (s->d.N + ra.chunk - 1) / ra.chunk;
    const auto key = std::make_tuple(s->nmax, s->d.n == s->nmax);
    groups[key].push_back({i, ra, chunks, 0, (unsigned)(s->d.S * chunks), 1u, 1u});
    LaunchRec& rec = recs[key];
    rec.op = RO_RESIDUAL;
    rec.cls = KC_RESIDUAL;
    rec.nmax = s->nmax;
    rec.full = s->d.n == s->nmax;
    rec.lds = std::max(rec.lds, residual_lds(s->nmax, ra.nrhs));
    roots.push_back({i, ra, 0, 0, 1u, 1u, 1u});
  }
  for (auto& g : groups) emit(R, seq, recs[g.first], g.second);
  LaunchRec rr;
  rr.op = RO_RESIDUAL_ROOT;
  rr.cls = KC_RESIDUAL_ROOT;
  emit(R, seq, rr, roots);
}

template <typename T>
void run(bmpc_plan p, const Seq& seq, const Reloc& r) {
  RaggedState& R = *p->ragged;
  hipStream_t st = p->stream;
  for (const LaunchRec& rec : seq) {
    const void* tab = R.dtab + rec.table;
    timed(p, rec.cls, [&] {
      switch (rec.op) {
        case RO_INFO_RESET:
          launch_info_reset(R.info, (int)R.subs.size(), st);
          break;
        case RO_L1INV:
          launch_level1_inverse_multi<T>(static_cast<const MultiItem<FactorPassArgs>*>(tab),
                                         rec.nitems, rec.blocks, rec.nmax, rec.full, r, st);
          break;
        case RO_FACTOR:
          launch_factor_pass_multi<T>(static_cast<const MultiItem<FactorPassArgs>*>(tab),
                                      rec.nitems, rec.blocks, rec.nmax, rec.first, rec.final,
                                      rec.fwd, rec.full, rec.lds, r, st);
          break;
        case RO_ROOT_REDUCE:
          launch_root_reduce_multi(static_cast<const MultiItem<RootArgs>*>(tab), rec.nitems,
                                   rec.blocks, st);
          break;
        case RO_ROOT_POTRF:
          launch_root_potrf_multi(static_cast<const MultiItem<RootArgs>*>(tab), rec.nitems,
                                  rec.blocks, rec.nmax, r, st);
          break;
        case RO_SOLVE:
          launch_solve_multi<T>(rec.kind, rec.fwd, rec.full, rec.nmax,
                                static_cast<const MultiItem<SolveArgs>*>(tab), rec.nitems,
                                rec.blocks, rec.threads, rec.lds, r, st);
          break;
        case RO_RESIDUAL:
          launch_residual_multi(rec.nmax, rec.full,
                                static_cast<const MultiItem<ResidualArgs>*>(tab), rec.nitems,
                                rec.blocks, rec.lds, r, st);
          break;
        case RO_RESIDUAL_ROOT:
          launch_residual_root_multi(static_cast<const MultiItem<ResidualArgs>*>(tab),
                                     rec.nitems, rec.blocks, r, st);
          break;
      }
    });
  }
}

bool ralloc(RaggedState& R, void** ptr, size_t bytes) {
  if (hipMalloc(ptr, std::max<size_t>(bytes, 256)) != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return false;
  }
  R.allocs.push_back(*ptr);
  return true;
}

template <typename T>
void solve_all(bmpc_plan p, const Reloc& r, int first_chunk) {
  RaggedState& R = *p->ragged;
  for (int c = first_chunk; c < R.chunks; ++c) run<T>(p, R.solve[c], r);
}

}  // namespace

const std::vector<bmpc_plan>& ragged_subs(bmpc_plan p) { return p->ragged->subs; }

// info of the first system (in system order) whose factorization failed, as the
// 1-based natural row in the concatenated systems (each numbered as in bmpc_get_info).
bmpc_status ragged_info(bmpc_plan p, int64_t* info) {
  RaggedState& R = *p->ragged;
  const int B = (int)R.subs.size();
  std::vector<unsigned long long> v(B);
  if (hipStreamSynchronize(p->stream) != hipSuccess ||
      hipMemcpy(v.data(), R.info, (size_t)B * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return BMPC_ERR_DEVICE;
  *info = 0;
  if (!p->factored) return BMPC_OK;
  for (int i = 0; i < B; ++i) {
    if (v[i] == ~0ull) continue;
    int64_t local = 0;
    bmpc_get_info(R.subs[i], &local);
    *info = (int64_t)R.rows[i] + local;
    return BMPC_ERR_NOT_SPD;
  }
  return BMPC_OK;
}

void ragged_destroy(bmpc_plan p) {
  RaggedState* R = p->ragged;
  if (!R) return;
  for (bmpc_plan s : R->subs) {
    free_plan_memory(s);
    delete s;
  }
  for (void* a : R->allocs) (void)hipFree(a);
  delete R;
  p->ragged = nullptr;
}

bmpc_status ragged_factor(bmpc_plan p, const double* D, const double* E, const double* C,
                          const double* R_, const double* b, double* x) {
  RaggedState& R = *p->ragged;
  const Reloc r{D, E, C, R_, b, x, nullptr};
  const bool fused = b != nullptr;
  if (p->fp64)
    run<double>(p, R.factor[fused ? 1 : 0], r);
  else
    run<float>(p, R.factor[fused ? 1 : 0], r);
  if (fused) {
    if (p->fp64) {
      run<double>(p, R.back0, r);
      solve_all<double>(p, r, 1);
    } else {
      run<float>(p, R.back0, r);
      solve_all<float>(p, r, 1);
    }
  }
  const bmpc_status st = last_error_status();
  if (st == BMPC_OK) {
    p->factored = true;
    for (bmpc_plan s : R.subs) s->factored = true;
  }
  return st;
}

bmpc_status ragged_solve(bmpc_plan p, const double* b, double* x) {
  const Reloc r{nullptr, nullptr, nullptr, nullptr, b, x, nullptr};
  if (p->fp64)
    solve_all<double>(p, r, 0);
  else
    solve_all<float>(p, r, 0);
  return last_error_status();
}

bmpc_status ragged_refine(bmpc_plan p, const double* D, const double* E, const double* C,
                          const double* R_, const double* b, double* x, double tol,
                          int max_iters, bool fused) {
  RaggedState& R = *p->ragged;
  hipStream_t st = p->stream;
  const bool be = p->refine_stop == BMPC_STOP_BACKWARD_ERROR;
  const int B = (int)R.subs.size();
  timed(p, KC_REFINE_MISC, [&] { launch_refine_reset(p->flags, st); });
  if (fused) {
    if (ragged_factor(p, D, E, C, R_, b, x) != BMPC_OK) return BMPC_ERR_DEVICE;
  } else {
    if (ragged_solve(p, b, x) != BMPC_OK) return BMPC_ERR_DEVICE;
  }
  const Reloc rr{D, E, C, R_, b, x, R.rbuf};        // residual into rbuf
  const Reloc rc{nullptr, nullptr, nullptr, nullptr, R.rbuf, x, R.rbuf};  // correction
  auto residual = [&](bool knorm) {
    for (int c = 0; c < R.chunks; ++c) {
      if (p->fp64)
        run<double>(p, R.resid[knorm ? 1 : 0][c], rr);
      else
        run<float>(p, R.resid[knorm ? 1 : 0][c], rr);
    }
  };
  auto correction = [&] {
    for (int c = 0; c < R.chunks; ++c) {
      if (p->fp64)
        run<double>(p, R.corr[c], rc);
      else
        run<float>(p, R.corr[c], rc);
    }
  };
  auto check = [&](int mode, const double* v1, bool knorm, int count) {
    timed(p, KC_REFINE_MISC, [&] {
      launch_seg_maxabs(mode == 1 ? R.rbuf : v1, x, R.segs, R.nseg,
                        mode == 1 ? R.rnorm : R.dnorm, R.xnorm, p->flags, st);
      launch_ragged_check(mode, mode == 1 ? R.rnorm : R.dnorm, R.xnorm, R.bnorm, R.seg_sys,
                          R.nseg, B, knorm ? R.kpart : nullptr, R.kp_off, R.kroot, R.knorm, tol,
                          count, p->flags, p->relcorr, R.ok, R.worst, st);
    });
  };
  if (be)
    timed(p, KC_REFINE_MISC, [&] {
      launch_seg_maxabs(b, nullptr, R.segs, R.nseg, R.bnorm, nullptr, nullptr, st);
    });
  bool stopped = false;
  for (int it = 0; it < max_iters; ++it) {
    residual(be && it == 0);
    if (be) {
      check(1, nullptr, it == 0, 1);
      // as in the one-system loop: no host wait on an FP32 first solve's check
      const bool hopeless = it == 0 && !p->fp64 && tol < 0x1p-30;
      if (!hopeless && (stopped = stop_reached(p))) break;
    } else {
      timed(p, KC_REFINE_MISC, [&] {
        launch_seg_maxabs(R.rbuf, nullptr, R.segs, R.nseg, R.rnorm, nullptr, p->flags, st);
      });
    }
    correction();
    if (!be) {
      check(0, R.rbuf, false, 2);
      if (it + 1 < max_iters && (stopped = stop_reached(p))) break;
    }
  }
  if (be && !stopped) {
    residual(max_iters == 0);
    check(1, nullptr, max_iters == 0, 0);
  }
  p->last_max_iters = be ? std::max(max_iters, 1) : max_iters;
  return last_error_status();
}

}  // namespace bmpc

using namespace bmpc;

extern "C" {

bmpc_status bmpc_analyze_ragged(int32_t B, const bmpc_dims* dims, bmpc_precision prec,
                                void* stream, const bmpc_options* opts, bmpc_plan* out) {
  if (!out) return BMPC_ERR_INVALID;
  *out = nullptr;
  if (B < 1 || !dims || (prec != BMPC_FP64 && prec != BMPC_FP32_REFINE)) return BMPC_ERR_INVALID;
  for (int i = 0; i < B; ++i)
    if (!dims_ok(&dims[i], 1) || dims[i].n > 32 || dims[i].nrhs != dims[0].nrhs ||
        (opts && opts[i].num_systems > 1))
      return BMPC_ERR_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return BMPC_ERR_DEVICE;
  bmpc_plan p = new (std::nothrow) bmpc_plan_s();
  if (!p) return BMPC_ERR_ALLOC;
  p->ragged = new (std::nothrow) RaggedState();
  if (!p->ragged) {
    delete p;
    return BMPC_ERR_ALLOC;
  }
  RaggedState& R = *p->ragged;
  auto fail = [&](bmpc_status st) {
    ragged_destroy(p);
    free_plan_memory(p);
    delete p;
    return st;
  };
  p->prec = prec;
  p->fp64 = prec == BMPC_FP64;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  p->opt_flags = opts ? opts[0].flags : 0;
  p->B = B;
  p->d = dims[0];
  R.nrhs = dims[0].nrhs;
  auto sys_opts = [&](int i) {
    bmpc_options so{};
    if (opts) so = opts[i];
    so.num_systems = 1;
    return so;
  };
  // per-system plans: sizes first, then one allocation carved in system order
  size_t total = 0;
  std::vector<size_t> base(B);
  for (int i = 0; i < B; ++i) {
    bmpc_plan s = new (std::nothrow) bmpc_plan_s();
    if (!s) return fail(BMPC_ERR_ALLOC);
    R.subs.push_back(s);
    s->parent = p;
    s->measure = true;
    const bmpc_options so = sys_opts(i);
    if (init_plan(s, &dims[i], prec, stream, &so) != BMPC_OK) return fail(BMPC_ERR_INVALID);
    base[i] = total;
    total += (s->arena_used + 255) & ~(size_t)255;
  }
  if (!ralloc(R, (void**)&R.arena, total)) return fail(BMPC_ERR_ALLOC);
  for (int i = 0; i < B; ++i) {
    bmpc_plan s = R.subs[i];
    s->measure = false;
    s->arena = R.arena + base[i];
    s->arena_used = 0;
    s->workspace_bytes = 0;
    const bmpc_options so = sys_opts(i);
    const bmpc_status st = init_plan(s, &dims[i], prec, stream, &so);
    if (st != BMPC_OK) return fail(st);
    p->workspace_bytes += s->workspace_bytes;
  }
  // layout of the callers' arrays and the shared buffers
  R.offD.assign(B + 1, 0);
  R.offE.assign(B + 1, 0);
  R.offC.assign(B + 1, 0);
  R.offR.assign(B + 1, 0);
  R.offV.assign(B + 1, 0);
  R.rows.assign(B + 1, 0);
  std::vector<int> kp(B + 1, 0);
  R.chunk = kMaxRhs;
  R.chunks = (R.nrhs + R.chunk - 1) / R.chunk;
  for (int i = 0; i < B; ++i) {
    const bmpc_dims& d = dims[i];
    const size_t nn = (size_t)d.n * d.n;
    R.offD[i + 1] = R.offD[i] + (size_t)d.S * d.N * nn;
    R.offE[i + 1] = R.offE[i] + (size_t)d.S * (d.N - 1) * nn;
    R.offC[i + 1] = R.offC[i] + (size_t)d.S * nn;
    R.offR[i + 1] = R.offR[i] + nn;
    R.rows[i + 1] = R.rows[i] + ((size_t)d.S * d.N + 1) * d.n;
    R.offV[i + 1] = R.offV[i] + (size_t)R.nrhs * ((size_t)d.S * d.N + 1) * d.n;
    kp[i + 1] = kp[i] + R.subs[i]->kper;
  }
  R.nseg = B * R.nrhs;
  std::vector<SegRec> segs(R.nseg);
  std::vector<int> seg_sys(R.nseg);
  for (int i = 0; i < B; ++i)
    for (int q = 0; q < R.nrhs; ++q) {
      const size_t len = R.rows[i + 1] - R.rows[i];
      segs[i * R.nrhs + q] = {R.offV[i] + (size_t)q * len, len};
      seg_sys[i * R.nrhs + q] = i;
    }
  const size_t ns = (size_t)R.nseg;
  bool ok = ralloc(R, (void**)&R.info, (size_t)B * 8) &&
            ralloc(R, (void**)&R.rbuf, R.offV[B] * 8) &&
            ralloc(R, (void**)&p->flags, 2 * sizeof(int)) &&
            ralloc(R, (void**)&p->relcorr, sizeof(double)) &&
            ralloc(R, (void**)&R.segs, ns * sizeof(SegRec)) &&
            ralloc(R, (void**)&R.seg_sys, ns * sizeof(int)) &&
            ralloc(R, (void**)&R.kp_off, (size_t)(B + 1) * sizeof(int)) &&
            ralloc(R, (void**)&R.rnorm, ns * 8) && ralloc(R, (void**)&R.dnorm, ns * 8) &&
            ralloc(R, (void**)&R.xnorm, ns * 8) && ralloc(R, (void**)&R.bnorm, ns * 8) &&
            ralloc(R, (void**)&R.knorm, (size_t)B * 8) &&
            ralloc(R, (void**)&R.kpart, (size_t)kp[B] * 8) &&
            ralloc(R, (void**)&R.kroot, (size_t)B * 8) &&
            ralloc(R, (void**)&R.worst, (size_t)B * 8) &&
            ralloc(R, (void**)&R.ok, (size_t)B * sizeof(int));
  if (!ok) return fail(BMPC_ERR_ALLOC);
  if (hipHostMalloc((void**)&p->hflag, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    p->hflag = nullptr;
    (void)hipGetLastError();
    return fail(BMPC_ERR_ALLOC);
  }
  for (int i = 0; i < B; ++i) {
    bmpc_plan s = R.subs[i];
    s->flags = p->flags;
    s->rbuf = R.rbuf + R.offV[i];
    s->d_info = R.info + i;
    s->kpart = R.kpart + kp[i];
    s->kroot = R.kroot + i;
    s->stream = p->stream;
  }
  // item order: largest work (tail blocks x block volume) first
  std::vector<int> order(B);
  for (int i = 0; i < B; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b2) {
    auto work = [&](int k) { return (double)dims[k].S * dims[k].N * dims[k].n * dims[k].n * dims[k].n; };
    return work(a) > work(b2);
  });
  R.rank.assign(B, 0);
  for (int k = 0; k < B; ++k) R.rank[order[k]] = k;
  // launch tables
  build_factor(p, R.factor[0], false);
  build_factor(p, R.factor[1], true);
  R.solve.resize(R.chunks);
  R.corr.resize(R.chunks);
  R.resid[0].resize(R.chunks);
  R.resid[1].resize(R.chunks);
  for (int c = 0; c < R.chunks; ++c) {
    const std::vector<SolveArgs> a = chunk_args(p, c, false);
    build_fwd(R, R.solve[c], a);
    build_back(R, R.solve[c], a, c * R.chunk);
    if (c == 0) build_back(R, R.back0, a, 0);
    const std::vector<SolveArgs> ca = chunk_args(p, c, true);
    build_fwd(R, R.corr[c], ca);
    build_back(R, R.corr[c], ca, c * R.chunk);
    build_residual(p, R.resid[0][c], c, false);
    build_residual(p, R.resid[1][c], c, true);
  }
  if (!ralloc(R, (void**)&R.dtab, R.htab.size())) return fail(BMPC_ERR_ALLOC);
  if (hipMemcpy(R.dtab, R.htab.data(), R.htab.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(R.segs, segs.data(), ns * sizeof(SegRec), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(R.seg_sys, seg_sys.data(), ns * sizeof(int), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(R.kp_off, kp.data(), (size_t)(B + 1) * sizeof(int), hipMemcpyHostToDevice) !=
          hipSuccess) {
    (void)hipGetLastError();
    return fail(BMPC_ERR_DEVICE);
  }
  *out = p;
  return BMPC_OK;
}

bmpc_status bmpc_ragged_layout(bmpc_plan p, int32_t i, bmpc_dims* dims, int64_t* offsets) {
  if (!p || !p->ragged || i < 0 || i >= (int)p->ragged->subs.size()) return BMPC_ERR_INVALID;
  const RaggedState& R = *p->ragged;
  if (dims) *dims = R.subs[i]->d;
  if (offsets) {
    offsets[0] = (int64_t)R.offD[i];
    offsets[1] = (int64_t)R.offE[i];
    offsets[2] = (int64_t)R.offC[i];
    offsets[3] = (int64_t)R.offR[i];
    offsets[4] = (int64_t)R.offV[i];
  }
  return BMPC_OK;
}

}  // extern "C"
