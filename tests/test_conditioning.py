"""Condition-number measurement of the synthetic systems (CPU).

The sparse K used for the measurement must equal the dense assembly entry by entry,
the Lanczos extreme eigenvalues must match LAPACK's dense symmetric eigensolver, and
the generator's block diagonal dominance must give lambda_min >= delta (block
Gershgorin: every diagonal block exceeds the spectral norms of its row's off-diagonal
blocks by delta)."""
import numpy as np
import pytest

from oracle.conditioning import extreme_eigenvalues, sparse_K
from oracle.dense import assemble_K
from synth.branch_system import make_config, make_system

SMALL = [(1, 1, 1, 1.0, 0), (2, 1, 3, 1e-2, 1), (3, 2, 2, 1.0, 2), (4, 9, 4, 1e-2, 3),
         (2, 17, 5, 1e-5, 4), (5, 8, 6, 1.0, 5)]


@pytest.mark.parametrize("S,N,n,delta,seed", SMALL)
def test_sparse_assembly_equals_dense(S, N, n, delta, seed):
    s = make_system(S, N, n, 1, delta, seed)
    assert np.array_equal(sparse_K(s.D, s.E, s.C, s.R).toarray(),
                          assemble_K(s.D, s.E, s.C, s.R))


@pytest.mark.parametrize("S,N,n,delta,seed", [c for c in SMALL if (c[0] * c[1] + 1) * c[2] > 8])
def test_extreme_eigenvalues_match_dense_eigensolver(S, N, n, delta, seed):
    s = make_system(S, N, n, 1, delta, seed)
    w = np.linalg.eigvalsh(assemble_K(s.D, s.E, s.C, s.R))
    lmin, lmax = extreme_eigenvalues(s.D, s.E, s.C, s.R)
    assert abs(lmin - w[0]) <= 1e-8 * w[-1]
    assert abs(lmax - w[-1]) <= 1e-8 * w[-1]


def test_c1_condition_number():
    s = make_config("c1", seed=0)
    w = np.linalg.eigvalsh(assemble_K(s.D, s.E, s.C, s.R))
    lmin, lmax = extreme_eigenvalues(s.D, s.E, s.C, s.R)
    assert lmax / lmin == pytest.approx(w[-1] / w[0], rel=1e-8)


@pytest.mark.parametrize("delta", [1.0, 1e-2, 1e-5])
def test_generator_lambda_min_at_least_delta(delta):
    for seed in range(3):
        s = make_system(3, 7, 4, 1, delta, seed)
        w = np.linalg.eigvalsh(assemble_K(s.D, s.E, s.C, s.R))
        assert w[0] >= delta * (1 - 1e-12)


def test_condition_number_of_a_diagonal_system():
    # E = 0, C = 0 and diagonal D, R: K is diagonal, so kappa is the ratio of its
    # largest to its smallest diagonal entry (a closed form).
    from oracle.conditioning import condition_number
    S, N, n = 3, 4, 3
    rng = np.random.default_rng(7)
    diag = rng.uniform(0.5, 40.0, size=(S * N + 1) * n)
    D = np.zeros((S, N, n, n))
    for s in range(S):
        for k in range(N):
            o = (s * N + k) * n
            D[s, k] = np.diag(diag[o:o + n])
    E = np.zeros((S, N - 1, n, n))
    C = np.zeros((S, n, n))
    R = np.diag(diag[S * N * n:])
    assert condition_number(D, E, C, R) == pytest.approx(diag.max() / diag.min(), rel=1e-9)


@pytest.mark.parametrize("S,N,n,delta,seed", [(2, 5, 3, 1e-2, 11), (3, 4, 4, 1.0, 12)])
def test_condition_number_matches_svd_ratio(S, N, n, delta, seed):
    # For SPD K the 2-norm condition number is also the ratio of the extreme singular
    # values (LAPACK's SVD, a different route from the Lanczos iterations).
    from oracle.conditioning import condition_number
    s = make_system(S, N, n, 1, delta, seed)
    assert condition_number(s.D, s.E, s.C, s.R) == pytest.approx(
        np.linalg.cond(assemble_K(s.D, s.E, s.C, s.R), 2), rel=1e-8)
