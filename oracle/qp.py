"""Reduced IPM system of a branch-MPC QP, densely (FP64 oracle, TEST INFRASTRUCTURE).

Plain definition, written out (appendix on the linear systems of IPM and ADMM): with
the QP data assembled into dense P, A, G and W over all variables in the natural
order (tails in stage order, root last, as the right-hand side b), the regularized
IPM KKT matrix is [[P + tau I, A^T, G^T], [A, -delta I, 0], [G, 0, -(W + delta I)]]
and eliminating its second and third block rows gives the SPD matrix
K = P + tau I + delta^{-1} A^T A + G^T (W + delta I)^{-1} G.
The ADMM matrix of the same appendix (the OSQP form) is written out the same way:
[[P + sigma I, A^T, G^T], [A, -rho^{-1} I, 0], [G, 0, -rho^{-1} I]], and eliminating
its second and third block rows gives P + sigma I + rho A^T A + rho G^T G.
`blocks` reads D, E, C, R out of the dense K in the layout of synth.branch_system.
"""
from __future__ import annotations

import numpy as np


def _var(S, N, n, s, k):
    """Offset of stage k of scenario s (k = -1: the root) in the natural order."""
    return S * N * n if k < 0 else (s * N + k) * n


def dense_qp(qp):
    """Dense P, A, G (rows stacked link by link) and the diagonal of W."""
    S, N, n = qp.S, qp.N, qp.n
    nv = (S * N + 1) * n
    me, mi = qp.A.shape[2], qp.G.shape[2]
    P = np.zeros((nv, nv))
    A = np.zeros((S * (N + 1) * me, nv))
    G = np.zeros((S * (N + 1) * mi, nv))
    W = np.zeros(S * (N + 1) * mi)
    for s in range(S):
        for j in range(N + 1):
            u = _var(S, N, n, s, j - 1)
            v = _var(S, N, n, s, j) if j < N else None
            cols = [(u, slice(0, n))] + ([(v, slice(n, 2 * n))] if v is not None else [])
            re = (s * (N + 1) + j) * me
            ri = (s * (N + 1) + j) * mi
            for ca, sa in cols:
                for cb, sb in cols:
                    P[ca:ca + n, cb:cb + n] += qp.Q[s, j][sa, sb]
                A[re:re + me, ca:ca + n] = qp.A[s, j][:, sa]
                G[ri:ri + mi, ca:ca + n] = qp.G[s, j][:, sa]
            W[ri:ri + mi] = qp.w[s, j]
    return P, A, G, W


def reduced_K(qp):
    P, A, G, W = dense_qp(qp)
    K = P + qp.tau * np.eye(P.shape[0]) + (A.T @ A) / qp.delta + G.T @ (G / (W + qp.delta)[:, None])
    return 0.5 * (K + K.T)


def kkt(qp):
    """The regularized IPM KKT matrix (before the reduction)."""
    P, A, G, W = dense_qp(qp)
    nv, ne, ni = P.shape[0], A.shape[0], G.shape[0]
    M = np.zeros((nv + ne + ni, nv + ne + ni))
    M[:nv, :nv] = P + qp.tau * np.eye(nv)
    M[:nv, nv:nv + ne] = A.T
    M[nv:nv + ne, :nv] = A
    M[:nv, nv + ne:] = G.T
    M[nv + ne:, :nv] = G
    M[nv:nv + ne, nv:nv + ne] = -qp.delta * np.eye(ne)
    M[nv + ne:, nv + ne:] = -np.diag(W + qp.delta)
    return M


def blocks(K, S, N, n):
    """D [S][N][n][n], E [S][N-1][n][n] (block (k+1, k)), C [S][n][n] (block (root,
    stage 0)) and R [n][n] read out of a dense K in the natural order."""
    D = np.zeros((S, N, n, n))
    E = np.zeros((S, max(N - 1, 0), n, n))
    C = np.zeros((S, n, n))
    r = S * N * n
    for s in range(S):
        for k in range(N):
            o = (s * N + k) * n
            D[s, k] = K[o:o + n, o:o + n]
            if k + 1 < N:
                E[s, k] = K[o + n:o + 2 * n, o:o + n]
        o = s * N * n
        C[s] = K[r:r + n, o:o + n]
    return D, E, C, K[r:, r:].copy()


def admm_kkt(qp, sigma: float, rho: float):
    """The ADMM KKT matrix of the appendix (OSQP form) for the QP data of ``qp``
    (its IPM weights and regularization are not used)."""
    P, A, G, _ = dense_qp(qp)
    nv, ne, ni = P.shape[0], A.shape[0], G.shape[0]
    M = np.zeros((nv + ne + ni, nv + ne + ni))
    M[:nv, :nv] = P + sigma * np.eye(nv)
    M[:nv, nv:nv + ne] = A.T
    M[nv:nv + ne, :nv] = A
    M[:nv, nv + ne:] = G.T
    M[nv + ne:, :nv] = G
    M[nv:, nv:] = -np.eye(ne + ni) / rho
    return M


def admm_reduced_K(qp, sigma: float, rho: float):
    """The reduced ADMM matrix P + sigma I + rho (A^T A + G^T G)."""
    P, A, G, _ = dense_qp(qp)
    K = P + sigma * np.eye(P.shape[0]) + rho * (A.T @ A + G.T @ G)
    return 0.5 * (K + K.T)
