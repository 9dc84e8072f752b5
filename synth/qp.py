"""Seeded synthetic linear branch-MPC QP data (inputs only, no solver arithmetic).

Variables: the root x_0 and, per scenario s, stages x_{s,0..N-1}, each of size
n = nx + nu (state and input, Assumption 1).  Every term of the QP (appendix on the
linear systems of IPM and ADMM) touches at most two neighbouring blocks and is stored
per "link": link 0 of scenario s couples (u, v) = (x_0, x_{s,0}), link k (1 <= k < N)
couples (x_{s,k-1}, x_{s,k}), link N is the terminal term on u = x_{s,N-1} (its v part
is unused and zero).  Per link j:
  Q[s][j]  (2n x 2n)  cost Hessian, PSD            (P = sum of the links' Q)
  A[s][j]  (me x 2n)  equality rows: dynamics  x^state_v = Ad x^state_u + Bd x^input_u
                      written as [Ad Bd | -I 0]; zero for the terminal link
  G[s][j]  (mi x 2n)  inequality rows: box constraints on v (+I and -I rows);
                      zero for the terminal link
  w[s][j]  (mi)       IPM weights (the diagonal of W), positive
Dynamics are scenario dependent (a nominal stable Ad, Bd plus a per-scenario
perturbation), as in branch MPC with uncertain models.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class BranchQP:
    S: int
    N: int
    nx: int
    nu: int
    Q: np.ndarray   # (S, N+1, 2n, 2n)
    A: np.ndarray   # (S, N+1, nx, 2n)
    G: np.ndarray   # (S, N+1, 2n, 2n)  mi = 2n
    w: np.ndarray   # (S, N+1, 2n)
    tau: float
    delta: float

    @property
    def n(self):
        return self.nx + self.nu


def make_qp(S, N, nx, nu, tau=1e-6, delta=1e-2, seed=0) -> BranchQP:
    rng = np.random.default_rng(seed)
    n = nx + nu
    Ad0 = np.eye(nx) + 0.1 * rng.standard_normal((nx, nx)) / np.sqrt(nx)
    Bd0 = 0.1 * rng.standard_normal((nx, nu))
    Q = np.zeros((S, N + 1, 2 * n, 2 * n))
    A = np.zeros((S, N + 1, nx, 2 * n))
    G = np.zeros((S, N + 1, 2 * n, 2 * n))
    w = np.ones((S, N + 1, 2 * n))
    for s in range(S):
        Ad = Ad0 + 0.02 * rng.standard_normal((nx, nx))
        Bd = Bd0 + 0.02 * rng.standard_normal((nx, nu))
        for j in range(N + 1):
            M = rng.standard_normal((2 * n, 2 * n))
            Q[s, j] = M @ M.T / (2 * n)
            if j == N:
                Q[s, j][n:, :] = 0.0
                Q[s, j][:, n:] = 0.0
                continue
            A[s, j][:, :nx] = Ad
            A[s, j][:, nx:n] = Bd
            A[s, j][:, n:n + nx] = -np.eye(nx)
            G[s, j][:n, n:] = np.eye(n)
            G[s, j][n:, n:] = -np.eye(n)
            w[s, j] = 10.0 ** rng.uniform(-3, 1, 2 * n)
    return BranchQP(S, N, nx, nu, Q, A, G, w, tau, delta)
