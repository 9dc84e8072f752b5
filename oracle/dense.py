"""Dense assembly of the branch system for tiny brute-force checks (TEST INFRASTRUCTURE).

``assemble_K`` writes out eq. (root_coupled_matrix) with the tails of
eq. (tail_block_tridiagonal) in the paper's natural order (Section III-B: tails in
forward stage order, root last), reading only the lower triangles of D and R as the
GPU library does.  ``perm_matrix`` builds Pi of Section IV-A as a dense scalar
permutation.  Only sizes of a few hundred unknowns are meant.
"""
from __future__ import annotations

import numpy as np

from . import symbolic


def _sym_from_lower(A: np.ndarray) -> np.ndarray:
    L = np.tril(A)
    return L + np.tril(A, -1).T


def assemble_K(D, E, C, R) -> np.ndarray:
    S, N, n, _ = D.shape
    tot = (S * N + 1) * n
    K = np.zeros((tot, tot))
    r0 = S * N * n
    for s in range(S):
        o = s * N * n
        for k in range(N):
            K[o + k * n:o + (k + 1) * n, o + k * n:o + (k + 1) * n] = _sym_from_lower(D[s, k])
        for k in range(N - 1):
            blk = E[s, k]  # block (k+1, k)
            K[o + (k + 1) * n:o + (k + 2) * n, o + k * n:o + (k + 1) * n] = blk
            K[o + k * n:o + (k + 1) * n, o + (k + 1) * n:o + (k + 2) * n] = blk.T
        K[r0:r0 + n, o:o + n] = C[s]
        K[o:o + n, r0:r0 + n] = C[s].T
    K[r0:, r0:] = _sym_from_lower(R)
    return K


def perm_index(S: int, N: int, n: int, kind: str = "d") -> np.ndarray:
    """Scalar index vector p of Pi: the i-th variable of the permuted order is natural
    variable p[i], so (Pi K Pi^T) = K[p][:, p]."""
    order = symbolic.ordering(N, kind)
    idx = []
    for s in range(S):
        for k in order:
            base = (s * N + k) * n
            idx.extend(range(base, base + n))
    idx.extend(range(S * N * n, (S * N + 1) * n))
    return np.array(idx)


def perm_matrix(S: int, N: int, n: int, kind: str = "d") -> np.ndarray:
    """Scalar permutation matrix P with (P K P^T) the block-permuted matrix: row i of
    P selects the i-th scalar variable of the permuted order."""
    idx = perm_index(S, N, n, kind)
    P = np.zeros((idx.size, idx.size))
    P[np.arange(idx.size), idx] = 1.0
    return P
