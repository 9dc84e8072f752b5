"""The algebra of sharding the method by scenario (CPU, no GPUs or processes).

Sharded, each GPU would own a subset of the scenario tails with their D, E, C and b.
It factors its tails, and contributes to the root only two partial sums: its tails'
Schur complements sum_s C~_s K_s^{-1} C~_s^T (the U_s of Algorithm 1, summed) and its
tails' reduced right-hand sides sum_s C~_s K_s^{-1} b_s (the w_s of Algorithm 2, summed),
where C~_s places C_s on the first stage of tail s.  One all-reduce of those two n x n and
n-sized sums gives every GPU the root system; each solves it and back-substitutes
x_s = K_s^{-1} (b_s - C~_s^T x_0) locally.  This test carries out exactly that split with
dense per-tail solves and checks that every way of splitting the scenarios gives the
unsharded oracle's solution."""
import numpy as np
import pytest

from oracle import oracle
from synth.branch_system import make_system


def _tail_matrix(D, E):
    N, n, _ = D.shape
    K = np.zeros((N * n, N * n))
    for k in range(N):
        d = np.tril(D[k]) + np.tril(D[k], -1).T
        K[k * n:(k + 1) * n, k * n:(k + 1) * n] = d
    for k in range(N - 1):
        K[(k + 1) * n:(k + 2) * n, k * n:(k + 1) * n] = E[k]
        K[k * n:(k + 1) * n, (k + 1) * n:(k + 2) * n] = E[k].T
    return K


def _shard_partials(s, tails):
    """(sum of Schur complements, sum of reduced right-hand sides, per-tail solvers) of
    one shard."""
    N, n = s.N, s.n
    U = np.zeros((n, n))
    w = np.zeros((s.b.shape[0], n))
    solvers = {}
    for t in tails:
        K = _tail_matrix(s.D[t], s.E[t] if N > 1 else np.zeros((0, n, n)))
        Ct = np.zeros((n, N * n))
        Ct[:, :n] = s.C[t]  # C_s couples the root to the tail's first stage
        bt = s.b[:, t * N * n:(t + 1) * N * n]
        KinvCt = np.linalg.solve(K, Ct.T)
        U += Ct @ KinvCt
        w += (Ct @ np.linalg.solve(K, bt.T)).T
        solvers[t] = (K, Ct, bt)
    return U, w, solvers


@pytest.mark.parametrize("shards", [1, 2, 3, 5])
def test_sharded_solution_equals_unsharded(shards):
    s = make_system(7, 6, 3, 2, 1e-2, 41)
    ref, info = oracle.solve(s.D, s.E, s.C, s.R, s.b)
    assert info == 0
    split = np.array_split(np.arange(s.S), shards)
    parts = [_shard_partials(s, list(g)) for g in split]
    # the one collective: sums of the per-shard partials (in shard order)
    U = sum(p[0] for p in parts)
    w = sum(p[1] for p in parts)
    n, SNn = s.n, s.S * s.N * s.n
    R = np.tril(s.R) + np.tril(s.R, -1).T
    x0 = np.linalg.solve(R - U, (s.b[:, SNn:] - w).T).T
    x = np.zeros_like(s.b)
    x[:, SNn:] = x0
    for p in parts:
        for t, (K, Ct, bt) in p[2].items():
            x[:, t * s.N * n:(t + 1) * s.N * n] = np.linalg.solve(K, (bt - x0 @ Ct).T).T
    assert np.max(np.abs(x - ref)) <= 1e-12 * np.max(np.abs(ref))
