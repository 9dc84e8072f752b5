// Vector indexing shared by the solve kernels (solve.hip, solve64.hip).
#pragma once

#include "bmpc_internal.h"

namespace bmpc {

// Vectors b, x, r are [B][nrhs][len], len = (S*N+1)*n: system sys, right-hand side q
// of the launch's chunk starts at sys*vsys + q*len (the pointers are offset to the
// chunk), its tails in stage order, its root last.  Chain g of the batch
// (0 <= g < B*S) is scenario g % S of system g / S.  vec_off gives the offset of
// (chain g, q = 0, stage); seg_of the first norm index of g's system in the chunk.
__device__ inline size_t vec_len(const SolveArgs& a) { return ((size_t)a.S * a.N + 1) * a.n; }
__device__ inline size_t vec_off(const SolveArgs& a, int g, int stage) {
  const int sys = g / a.S, sl = g - sys * a.S;
  return (size_t)sys * a.vsys + ((size_t)sl * a.N + stage) * a.n;
}
__device__ inline int seg_of(const SolveArgs& a, int g) { return (g / a.S) * a.seg_sys; }

// x[off + q*len] = d  or  x += rnorm * d with rnorm * d kept in dstore.
__device__ inline void scatter_value(const SolveArgs& a, int q, size_t off, int seg0, double d) {
  const size_t idx = (size_t)q * vec_len(a) + off;
  if (a.accumulate) {
    const double dd = a.rnorm[seg0 + q] * d;
    a.x[idx] += dd;
    a.dstore[idx] = dd;
  } else {
    a.x[idx] = d;
  }
}

}  // namespace bmpc
