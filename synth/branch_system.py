"""Seeded synthetic root-coupled branch systems (inputs only, no solver arithmetic).

The paper's experiments use quadrotor branch-MPC systems (Section V-A) that are not
available here; these synthetic systems stand in for them.  They keep the structure
of the system the paper solves (eq. (root_coupled_matrix) and
eq. (tail_block_tridiagonal)): S scenario tails of N stages with n x n blocks,
block-tridiagonal inside each tail, and one coupling block C_s between the root and
the first stage of every tail.

Recipe (all draws from one numpy PCG64 stream, in this order):
  E  (S, N-1, n, n)  entries 0.5 * N(0, 1/n)      E[s,k] sits at block (k+1, k)
  C  (S, n, n)       entries 0.5 * N(0, 1/n)      C[s] sits at block (root, stage 0)
  MD (S, N, n, n)    N(0, 1)
  MR (n, n)          N(0, 1)
  b  (nrhs, (S*N+1)*n) N(0, 1)
  D[s,k] = MD MD^T / n + (|E[s,k-1]|_2 + |E[s,k]|_2 + [k=0] |C[s]|_2 + delta) I
  R      = MR MR^T / n + (sum_s |C[s]|_2 + delta) I
with |.|_2 the spectral norm and E[s,-1] = E[s,N-1] = 0.  D and R are symmetrised
bitwise as (A + A^T)/2.  Block diagonal dominance makes the matrix SPD with
lambda_min >= delta.

Stage indices here are 0-based: generator stage k is the paper's stage k+1.

This module is shared by the oracle and the GPU path as the single source of
inputs; it holds none of the factorization or solve arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class BranchSystem:
    S: int
    N: int
    n: int
    nrhs: int
    delta: float
    seed: int
    D: np.ndarray  # (S, N, n, n) float64, symmetric
    E: np.ndarray  # (S, N-1, n, n) float64
    C: np.ndarray  # (S, n, n) float64
    R: np.ndarray  # (n, n) float64, symmetric
    b: np.ndarray  # (nrhs, (S*N+1)*n) float64

    @property
    def unknowns(self) -> int:
        return (self.S * self.N + 1) * self.n


# Workloads of the benchmark and parity suite: name -> (S, N, n, nrhs, delta).
CONFIGS = {
    "c1": (4, 16, 8, 1, 1.0),          # plain FP64, tiny
    "c2": (256, 128, 16, 4, 1e-2),     # plain FP64, paper-scale block size n=16
    "c3": (512, 256, 32, 1, 1e-5),     # precision workload: FP32 + refinement vs FP64
}


def _spectral_norms(blocks: np.ndarray) -> np.ndarray:
    """Largest singular value of every n x n block in a stacked array."""
    if blocks.size == 0:
        return np.zeros(blocks.shape[:-2])
    return np.linalg.svd(blocks, compute_uv=False)[..., 0]


def _sym(a: np.ndarray) -> np.ndarray:
    return (a + np.swapaxes(a, -1, -2)) * 0.5


def make_system(S: int, N: int, n: int, nrhs: int = 1, delta: float = 1.0,
                seed: int = 0, zero_coupling: bool = False,
                zero_chain: bool = False) -> BranchSystem:
    """Draw one seeded system.

    zero_coupling sets every C[s] to 0 (decoupled tails); zero_chain sets every
    E[s,k] to 0 (block-diagonal tails).  Both are special cases used by tests; the
    draw order is unchanged so the remaining arrays are identical to the default.
    """
    if S < 1 or N < 1 or n < 1 or nrhs < 1:
        raise ValueError("S, N, n, nrhs must be >= 1")
    rng = np.random.default_rng(seed)
    scale = 0.5 / np.sqrt(n)
    E = rng.standard_normal((S, N - 1, n, n)) * scale
    C = rng.standard_normal((S, n, n)) * scale
    if zero_chain:
        E[...] = 0.0
    if zero_coupling:
        C[...] = 0.0
    D = rng.standard_normal((S, N, n, n))
    MR = rng.standard_normal((n, n))
    b = rng.standard_normal((nrhs, (S * N + 1) * n))

    D = np.matmul(D, np.swapaxes(D, -1, -2)) / n
    shift = np.full((S, N), float(delta))
    if N > 1:
        en = _spectral_norms(E)  # (S, N-1)
        shift[:, 1:] += en       # |E[s,k-1]|
        shift[:, :-1] += en      # |E[s,k]|
    cn = _spectral_norms(C)      # (S,)
    shift[:, 0] += cn
    idx = np.arange(n)
    D[:, :, idx, idx] += shift[:, :, None]
    D = _sym(D)

    R = MR @ MR.T / n
    R[idx, idx] += float(np.sum(cn)) + float(delta)
    R = _sym(R)
    return BranchSystem(S, N, n, nrhs, float(delta), seed,
                        np.ascontiguousarray(D), np.ascontiguousarray(E),
                        np.ascontiguousarray(C), np.ascontiguousarray(R),
                        np.ascontiguousarray(b))


def make_config(name: str, seed: int = 0) -> BranchSystem:
    S, N, n, nrhs, delta = CONFIGS[name]
    return make_system(S, N, n, nrhs, delta, seed)
