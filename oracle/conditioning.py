"""Spectral condition number of the synthetic branch systems (TEST INFRASTRUCTURE).

Measures kappa(K) = lambda_max / lambda_min of the SPD matrix of eq.
(root_coupled_matrix) (tails of eq. (tail_block_tridiagonal), root border, natural
order of Section III-B), to report how hard each workload is for the FP32 factor
with refinement.  Neither the library nor the oracle's solver uses it.

  lambda_max: Lanczos on K (ARPACK via scipy.sparse.linalg.eigsh, largest algebraic).
  lambda_min: Lanczos in shift-invert mode about 0 (eigsh with sigma = 0, a sparse LU
              of K), which returns the eigenvalue of K nearest to zero.

Both act on a sparse assembly of K that reads only the lower triangles of D and R,
as the solver does.  Run as ``python -m oracle.conditioning c2`` (optionally with a
stage count that replaces N, for the largest workloads).
"""
from __future__ import annotations

import sys

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def sparse_K(D, E, C, R) -> sp.csc_matrix:
    """K in natural order (tails in forward stage order, root last) as a sparse matrix."""
    S, N, n, _ = D.shape
    r0 = S * N * n
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    rows, cols, vals = [], [], []

    def put(r, c, blk):
        rows.append((r + ii).ravel())
        cols.append((c + jj).ravel())
        vals.append(blk.ravel())

    def sym_lower(a):  # the symmetric block whose lower triangle is that of a
        return np.tril(a) + np.tril(a, -1).T

    for s in range(S):
        o = s * N * n
        for k in range(N):
            put(o + k * n, o + k * n, sym_lower(D[s, k]))
        for k in range(N - 1):
            put(o + (k + 1) * n, o + k * n, E[s, k])  # block (k+1, k)
            put(o + k * n, o + (k + 1) * n, E[s, k].T)
        put(r0, o, C[s])  # block (root, stage 0)
        put(o, r0, C[s].T)
    put(r0, r0, sym_lower(R))
    tot = (S * N + 1) * n
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(tot, tot))
    return K.tocsc()


def extreme_eigenvalues(D, E, C, R, tol: float = 1e-10):
    """(lambda_min, lambda_max) of K."""
    K = sparse_K(D, E, C, R)
    lmax = spla.eigsh(K, k=1, which="LA", tol=tol, return_eigenvectors=False)[0]
    lmin = spla.eigsh(K, k=1, sigma=0.0, which="LM", tol=tol, return_eigenvectors=False)[0]
    return float(lmin), float(lmax)


def condition_number(D, E, C, R, tol: float = 1e-10) -> float:
    lmin, lmax = extreme_eigenvalues(D, E, C, R, tol)
    return lmax / lmin


def main(argv) -> None:
    from synth.branch_system import CONFIGS, make_system
    name = argv[0] if argv else "c1"
    S, N, n, nrhs, delta = CONFIGS[name]
    if len(argv) > 1:
        N = int(argv[1])
    s = make_system(S, N, n, 1, delta, 0)
    lmin, lmax = extreme_eigenvalues(s.D, s.E, s.C, s.R)
    print(f"{name}: S={S} N={N} n={n} delta={delta}: lambda_min={lmin:.6g} "
          f"lambda_max={lmax:.6g} kappa={lmax / lmin:.4g}")


if __name__ == "__main__":
    main(sys.argv[1:])
