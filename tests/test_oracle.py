"""Pins of the FP64 CPU oracle against brute force, closed forms and invariants."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense, oracle
from synth.branch_system import make_system

U64 = np.finfo(np.float64).eps


def rel_inf(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def block_matvec(D, E, C, R, x):
    """K x straight from the block definition (eq. (root_coupled_matrix),
    eq. (tail_block_tridiagonal)); x is (nrhs, (S*N+1)*n)."""
    S, N, n, _ = D.shape
    Ds = np.tril(D) + np.swapaxes(np.tril(D, -1), -1, -2)
    Rs = np.tril(R) + np.tril(R, -1).T
    xt = x[:, :S * N * n].reshape(x.shape[0], S, N, n)
    x0 = x[:, S * N * n:]
    y = np.einsum("skij,qskj->qski", Ds, xt)
    if N > 1:
        y[:, :, 1:] += np.einsum("skij,qskj->qski", E, xt[:, :, :-1])
        y[:, :, :-1] += np.einsum("skji,qskj->qski", E, xt[:, :, 1:])
    y[:, :, 0] += np.einsum("sji,qj->qsi", C, x0)
    y0 = x0 @ Rs.T + np.einsum("sij,qsj->qi", C, xt[:, :, 0])
    return np.concatenate([y.reshape(x.shape[0], -1), y0], axis=1)


TINY = [(1, 1, 1, 0), (1, 1, 3, 1), (2, 1, 2, 2), (1, 2, 2, 3), (3, 2, 1, 4),
        (2, 3, 2, 5), (3, 9, 4, 6), (2, 9, 3, 7), (1, 16, 2, 8), (3, 5, 4, 9)]


@pytest.mark.parametrize("S,N,n,seed", TINY)
def test_oracle_matches_dense_brute_force(S, N, n, seed):
    s = make_system(S, N, n, 2, 1e-2, seed)
    K = dense.assemble_K(s.D, s.E, s.C, s.R)
    ref = np.linalg.solve(K, s.b.T).T
    x, info = oracle.solve(s.D, s.E, s.C, s.R, s.b)
    assert info == 0
    assert rel_inf(x, ref) <= 1e-12


@pytest.mark.parametrize("S,N,n,seed", TINY[3:])
def test_oracle_factor_reconstructs_K(S, N, n, seed):
    s = make_system(S, N, n, 1, 1.0, seed)
    K = dense.assemble_K(s.D, s.E, s.C, s.R)
    L, info = oracle.factor_dense(s.D, s.E, s.C, s.R)
    assert info == 0
    assert np.allclose(L, np.tril(L))
    err = np.linalg.norm(L @ L.T - K) / np.linalg.norm(K)
    assert err <= 10 * n * U64
    # Natural order: the root border fills in along each tail (ordering (a)).
    if N > 1:
        Nn = N * n
        assert np.any(L[S * Nn:, (N - 1) * n:Nn] != 0.0)


@pytest.mark.parametrize("S,N,n,nrhs", [(4, 16, 8, 1), (16, 33, 5, 3), (7, 64, 16, 2)])
def test_oracle_backward_error(S, N, n, nrhs):
    s = make_system(S, N, n, nrhs, 1e-2, 11)
    x, info = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=4)
    assert info == 0
    r = s.b - block_matvec(s.D, s.E, s.C, s.R, x)
    Knorm = np.max(block_matvec(np.abs(s.D), np.abs(s.E), np.abs(s.C), np.abs(s.R),
                                np.ones((1, s.b.shape[1]))))  # ||K||_inf
    be = np.max(np.abs(r)) / (Knorm * np.max(np.abs(x)) + np.max(np.abs(s.b)))
    assert be <= 10 * U64


def test_decoupled_tails_reduce_to_banded_and_root_solves():
    """C = 0: every tail is a block-tridiagonal SPD solve (scipy solveh_banded) and the
    root is an independent Cholesky solve."""
    S, N, n = 3, 12, 4
    s = make_system(S, N, n, 1, 1e-1, 21, zero_coupling=True)
    x, info = oracle.solve(s.D, s.E, s.C, s.R, s.b)
    assert info == 0
    p = 2 * n - 1
    for t in range(S):
        K = dense.assemble_K(s.D[t:t + 1], s.E[t:t + 1], s.C[t:t + 1], s.R)[:N * n, :N * n]
        ab = np.zeros((p + 1, N * n))
        for d in range(p + 1):
            ab[d, :N * n - d] = np.diagonal(K, -d)
        ref = sla.solveh_banded(ab, s.b[0, t * N * n:(t + 1) * N * n], lower=True)
        assert rel_inf(x[0, t * N * n:(t + 1) * N * n], ref) <= 1e-12
    R = np.tril(s.R) + np.tril(s.R, -1).T
    ref0 = sla.cho_solve(sla.cho_factor(R), s.b[0, S * N * n:])
    assert rel_inf(x[0, S * N * n:], ref0) <= 1e-12


def test_single_stage_closed_form():
    """N = 1: x_0 = (R - sum C D^-1 C^T)^{-1}(r_0 - sum C D^-1 r_s),
    x_s = D_s^{-1}(r_s - C_s^T x_0)."""
    S, n = 5, 6
    s = make_system(S, 1, n, 1, 1e-1, 22)
    x, info = oracle.solve(s.D, s.E, s.C, s.R, s.b)
    assert info == 0
    b = s.b[0]
    Dm = [np.tril(s.D[t, 0]) + np.tril(s.D[t, 0], -1).T for t in range(S)]
    R = np.tril(s.R) + np.tril(s.R, -1).T
    Sc = R - sum(s.C[t] @ np.linalg.solve(Dm[t], s.C[t].T) for t in range(S))
    rhs = b[S * n:] - sum(s.C[t] @ np.linalg.solve(Dm[t], b[t * n:(t + 1) * n]) for t in range(S))
    x0 = np.linalg.solve(Sc, rhs)
    assert rel_inf(x[0, S * n:], x0) <= 1e-12
    for t in range(S):
        xt = np.linalg.solve(Dm[t], b[t * n:(t + 1) * n] - s.C[t].T @ x0)
        assert rel_inf(x[0, t * n:(t + 1) * n], xt) <= 1e-11


def test_block_diagonal_tails_decouple_stages():
    """E = 0: stages k >= 1 are independent D-solves; stage 0 and the root form an
    arrow system (the N = 1 closed form)."""
    S, N, n = 3, 5, 3
    s = make_system(S, N, n, 1, 1e-1, 23, zero_chain=True)
    x, info = oracle.solve(s.D, s.E, s.C, s.R, s.b)
    assert info == 0
    b = s.b[0]
    for t in range(S):
        for k in range(1, N):
            Dk = np.tril(s.D[t, k]) + np.tril(s.D[t, k], -1).T
            o = (t * N + k) * n
            assert rel_inf(x[0, o:o + n], np.linalg.solve(Dk, b[o:o + n])) <= 1e-12


def test_scalar_tail_is_tridiagonal_plus_border():
    """S = 1, n = 1: a scalar tridiagonal system with one border row, solved by
    scipy's banded LU on the bordered matrix reordered root-first."""
    N = 40
    s = make_system(1, N, 1, 1, 1e-1, 24)
    x, info = oracle.solve(s.D, s.E, s.C, s.R, s.b)
    assert info == 0
    # Put the root first: then the matrix is tridiagonal (root couples stage 0 only).
    a = np.zeros((3, N + 1))
    diag = np.concatenate([[s.R[0, 0]], s.D[0, :, 0, 0]])
    off = np.concatenate([[s.C[0, 0, 0]], s.E[0, :, 0, 0]])
    a[1] = diag
    a[0, 1:] = off
    a[2, :-1] = off
    rhs = np.concatenate([s.b[0, N:], s.b[0, :N]])
    ref = sla.solve_banded((1, 1), a, rhs)
    got = np.concatenate([x[0, N:], x[0, :N]])
    assert rel_inf(got, ref) <= 1e-12


def test_thread_count_does_not_change_bits():
    s = make_system(9, 20, 4, 2, 1e-2, 25)
    x1, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=1)
    x4, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=4)
    assert np.array_equal(x1, x4)


@pytest.mark.parametrize("stage,shift", [(3, -40.0), (0, -40.0), (6, -2.5)])
def test_info_reports_first_failing_leading_minor(stage, shift):
    """A non-SPD input: info is the order of the first leading minor of K (natural
    order) that is not positive definite, found here by brute-force eigenvalues."""
    S, N, n = 2, 7, 3
    s = make_system(S, N, n, 1, 1e-1, 26)
    D = s.D.copy()
    D[1, stage] += shift * np.eye(n)
    K = dense.assemble_K(D, s.E, s.C, s.R)
    first = next(i for i in range(1, K.shape[0] + 1)
                 if np.linalg.eigvalsh(K[:i, :i])[0] <= 0.0)
    _, info = oracle.solve(D, s.E, s.C, s.R, s.b)
    assert info == first
