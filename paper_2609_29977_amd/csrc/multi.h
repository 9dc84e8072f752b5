// One launch over many systems of different shapes (gfx950).
//
// A ragged batch keeps, for every kernel of the factor, solve and refinement
// sequences, a table of work items: one per system that takes part in that launch,
// with the system's kernel arguments and the extent of its grid.  The launch's grid is
// the concatenation of the systems' grids in table order (largest work first); a
// workgroup finds its item by binary search on the first-block offsets and runs the
// same body as the one-system kernel on its local block coordinates.  Fields of the
// arguments that point into the caller's arrays hold offsets (in elements) from the
// array's start; the caller's base pointers come with each launch (Reloc), so the
// tables are built once per plan and every call, captured or not, uses them as they
// are.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bmpc_internal.h"

namespace bmpc {

// Base pointers of one call: the caller's blocks and vectors (vectors of every system
// concatenated, see include/bmpc.h), and the vector the correction solve reads and
// stores its update into.
struct Reloc {
  const double* D;
  const double* E;
  const double* C;
  const double* R;
  const double* b;
  double* x;
  double* r;
};

template <class Args>
struct MultiItem {
  Args a;          // caller-array fields: element offsets
  int p0, p1;      // kernel parameters (level, count, ...)
  unsigned start;  // first block of this system in the launch
  unsigned gx, gy; // grid extents of the system in x and y (z follows)
};

template <class Args>
__device__ inline int multi_find(const MultiItem<Args>* items, int n, unsigned b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {  // largest p with items[p].start <= b
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].start <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Local block coordinates of this workgroup within its item's grid.
struct LocalBlock {
  unsigned x, y, z;
};
template <class Args>
__device__ inline LocalBlock multi_local(const MultiItem<Args>& it) {
  const unsigned l = blockIdx.x - it.start;
  const unsigned xy = it.gx * it.gy;
  return {l % it.gx, (l % xy) / it.gx, l / xy};
}

// A caller-array field relocated to this call: the field holds kRelBias plus a byte
// offset (the bias keeps every such field non-null, so host code that tests a pointer
// for presence sees it as set).
constexpr uintptr_t kRelBias = 256;
template <typename P>
__device__ inline P* rel(P* base, const void* off) {
  return (base && off) ? reinterpret_cast<P*>(reinterpret_cast<uintptr_t>(base) +
                                              (reinterpret_cast<uintptr_t>(off) - kRelBias))
                       : nullptr;
}
template <typename P>
inline P* rel_field(size_t elements) {
  return reinterpret_cast<P*>(elements * sizeof(double) + kRelBias);
}

// Arguments of the root reduction (U, part) and the root Cholesky (R relative, the
// rest absolute) of one system.
struct RootArgs {
  const double* U;
  double* part;
  const double* R;
  double* LR;
  unsigned long long* info;
  int S, n, groups;
  unsigned long long sys_rows, root_row;
};

// One (system, right-hand side) vector of a ragged batch: its element offset in the
// concatenated vectors and its length.
struct SegRec {
  size_t off;
  size_t len;
};

// Launchers (next to the kernels they wrap).  items: device table of nitems items in
// launch order; blocks: the sum of their grids.
// full: every item has n == nmax.
template <typename T>
void launch_factor_pass_multi(const MultiItem<FactorPassArgs>* items, int nitems,
                              unsigned blocks, int nmax, bool first, bool final, bool fwd,
                              bool full, size_t lds, const Reloc& r, hipStream_t st);
// Blocks per wave of the level-1 inverse kernels for tile size nmax: FP64 32 x 32 blocks
// in pairs (one per 32-lane half of the wave in the diagonal leaves), the others alone
// (in FP32 a pair measured no faster).  A workgroup holds four waves.
constexpr int level1_blocks_per_wave(int nmax, bool fp64) { return fp64 && nmax > 16 ? 2 : 1; }
// Level-1 inverses of a ragged batch: item p0 = odd positions per chain, p1 = blocks
// (level1_blocks_per_wave per wave, four waves per workgroup) of the system.
template <typename T>
void launch_level1_inverse_multi(const MultiItem<FactorPassArgs>* items, int nitems,
                                 unsigned blocks, int nmax, bool full, const Reloc& r,
                                 hipStream_t st);
void launch_root_reduce_multi(const MultiItem<RootArgs>* items, int nitems, unsigned blocks,
                              hipStream_t st);
void launch_root_potrf_multi(const MultiItem<RootArgs>* items, int nitems, unsigned blocks,
                             int nmax, const Reloc& r, hipStream_t st);
void launch_info_reset(unsigned long long* info, int count, hipStream_t st);

enum SolveKind {
  SK_LEVEL = 0,   // solve_level_kernel (general; full = n == NMAX)
  SK_LEVEL_ONE,   // solve_level_one_kernel (one right-hand side, n == NMAX)
  SK_BWD_ROWS,    // solve_bwd_rows_kernel (backward level, n = 32, one right-hand side)
  SK_BWD_TOP,     // solve_bwd_top_kernel (merged top backward levels)
  SK_X_FWD,
  SK_X_BWD,
  SK_ROOT
};
struct LevelCfg {
  int kind;        // SolveKind
  bool full;       // n == NMAX (general level kernel)
  int count;       // positions of the level per chain
  unsigned gx, gy, gz, threads;
  size_t lds;
};
LevelCfg solve_level_config(const SolveArgs& a, int level, bool fwd, int nmax, bool fp64);

template <typename T>
void launch_solve_multi(int kind, bool fwd, bool full, int nmax,
                        const MultiItem<SolveArgs>* items, int nitems, unsigned blocks,
                        unsigned threads, size_t lds, const Reloc& r, hipStream_t st);

// Dynamic LDS of a level launch (waves per position, right-hand sides of the chunk) and
// of a residual launch.
size_t solve_level_lds(bool fp64, int nmax, int waves, int nrhs);
size_t residual_lds(int nmax, int nrhs);

void launch_residual_multi(int nmax, bool full, const MultiItem<ResidualArgs>* items,
                           int nitems, unsigned blocks, size_t lds, const Reloc& r,
                           hipStream_t st);
void launch_residual_root_multi(const MultiItem<ResidualArgs>* items, int nitems,
                                unsigned blocks, const Reloc& r, hipStream_t st);

// Ragged refinement bookkeeping over the (system, right-hand side) segments.
// out[k] = max |v[seg k]| (and out2[k] = max |v2[seg k]| if v2), one workgroup per
// segment; skipped when *done is set (done may be null).
void launch_seg_maxabs(const double* v, const double* v2, const SegRec* segs, int nseg,
                       double* out, double* out2, const int* done, hipStream_t st);
// Stop tests of a ragged batch (flags[0] = done, flags[1] = corrections, relcorr = the
// largest test quantity), after launch_seg_maxabs:
//   correction size: dn[k] <= tol * xn[k] for every segment;
//   backward error: rn[k] <= tol * (knorm[sys(k)] * xn[k] + bn[k]), knorm[sys] reduced
//   here from kpart[kp_off[sys] .. kp_off[sys + 1]) and kroot[sys] when kpart is set.
void launch_ragged_check(int mode, const double* dn_or_rn, const double* xn, const double* bn,
                         const int* seg_sys, int nseg, int B, const double* kpart,
                         const int* kp_off, const double* kroot, double* knorm, double tol,
                         int count, int* flags, double* relcorr, int* sys_ok,
                         double* sys_worst, hipStream_t st);

}  // namespace bmpc
