"""Gradients of a loss through the solve x = K^{-1} b (FP64 oracle, TEST INFRASTRUCTURE).

Only the tests and the benchmark use this module; it shares nothing with the GPU
library.  It is the plain definition, written out:

Differentiating K x = b for a loss l(x) with g = dl/dx gives the adjoint system
K^T lam = g; K is symmetric, so lam = K^{-1} g is a second solve with the same K.
Then dl/db = lam and, as a dense matrix, dl/dK = -lam x^T (summed over the
right-hand sides).  Each block array collects the entries of K it fills
(eq. (root_coupled_matrix), eq. (tail_block_tridiagonal)):

  D[s,k]  fills block (k, k) symmetrically:  dD[s,k] = sym(-lam_{s,k} x_{s,k}^T)
  E[s,k]  fills (k+1, k) and, transposed, (k, k+1):
          dE[s,k] = -(lam_{s,k+1} x_{s,k}^T + x_{s,k+1} lam_{s,k}^T)
  C[s]    fills (root, stage 0) and, transposed, (stage 0, root):
          dC[s] = -(lam_0 x_{s,0}^T + x_0 lam_{s,0}^T)
  R       fills the root block symmetrically:  dR = sym(-lam_0 x_0^T)

with sym(A) = (A + A^T) / 2 (the gradient of a symmetric argument, so that a
symmetric perturbation dD changes the loss by <dD, dD_pert>).  The layout is the
generator's: D[S][N][n][n], E[S][N-1][n][n], C[S][n][n], R[n][n],
b, x, lam [nrhs][(S*N+1)*n].  The pin of these formulas is central finite differences
of the loss through `oracle.solve` (tests/test_gradients_oracle.py).
"""
from __future__ import annotations

import numpy as np

from . import oracle


def _split(v, S, N, n):
    """[nrhs][(S*N+1)*n] -> tails [nrhs][S][N][n], root [nrhs][n]."""
    nrhs = v.shape[0]
    tails = v[:, :S * N * n].reshape(nrhs, S, N, n)
    root = v[:, S * N * n:]
    return tails, root


def _sym(a):
    return 0.5 * (a + np.swapaxes(a, -1, -2))


def block_gradients(x, lam, S, N, n):
    """(dD, dE, dC, dR) from the solution x and the adjoint lam, summed over rhs."""
    xt, x0 = _split(np.asarray(x, dtype=np.float64), S, N, n)
    lt, l0 = _split(np.asarray(lam, dtype=np.float64), S, N, n)
    dD = -_sym(np.einsum("qski,qskj->skij", lt, xt))
    if N > 1:
        dE = -(np.einsum("qski,qskj->skij", lt[:, :, 1:], xt[:, :, :-1]) +
               np.einsum("qski,qskj->skij", xt[:, :, 1:], lt[:, :, :-1]))
    else:
        dE = np.zeros((S, 0, n, n))
    dC = -(np.einsum("qi,qsj->sij", l0, xt[:, :, 0]) + np.einsum("qi,qsj->sij", x0, lt[:, :, 0]))
    dR = -_sym(np.einsum("qi,qj->ij", l0, x0))
    return dD, dE, dC, dR


def loss(D, E, C, R, b):
    """l = 0.5 * sum of squares of x = K^{-1} b (all right-hand sides)."""
    x, info = oracle.solve(D, E, C, R, b)
    assert info == 0
    return 0.5 * float(np.sum(x * x)), x


def loss_gradients(D, E, C, R, b):
    """x, lam and (db, dD, dE, dC, dR) for l = 0.5 ||x||^2 (g = x)."""
    S, N, n = D.shape[0], D.shape[1], D.shape[2]
    _, x = loss(D, E, C, R, b)
    lam, info = oracle.solve(D, E, C, R, x)
    assert info == 0
    dD, dE, dC, dR = block_gradients(x, lam, S, N, n)
    return x, lam, (lam, dD, dE, dC, dR)
