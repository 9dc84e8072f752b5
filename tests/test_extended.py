"""Pins of the extended-precision reference (CPU): exact arithmetic with Python
fractions on small inputs."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import dense, oracle
from oracle.conditioning import sparse_K
from oracle.extended import dd_residual, refine_reference, stress_system, two_prod, two_sum
from synth.branch_system import make_system

U64 = np.finfo(np.float64).eps / 2  # unit roundoff


def _rng_doubles(rng, k):
    return rng.standard_normal(k) * np.exp2(rng.integers(-40, 40, k))


def test_two_prod_and_two_sum_are_exact():
    rng = np.random.default_rng(0)
    a, b = _rng_doubles(rng, 400), _rng_doubles(rng, 400)
    p, e = two_prod(a, b)
    s, f = two_sum(a, b)
    for i in range(a.size):
        assert Fraction(p[i]) + Fraction(e[i]) == Fraction(a[i]) * Fraction(b[i])
        assert Fraction(s[i]) + Fraction(f[i]) == Fraction(a[i]) + Fraction(b[i])


def _exact_residual(K, x, b):
    Kd = K.toarray()
    m = Kd.shape[0]
    out = []
    for i in range(m):
        acc = Fraction(b[i])
        for j in np.nonzero(Kd[i])[0]:
            acc -= Fraction(Kd[i, j]) * Fraction(x[j])
        out.append(acc)
    return out


def test_dd_residual_within_dot2_bound():
    """Dot2 returns the residual as if computed in twice the precision: |r - r*| <=
    u |r*| + gamma_k^2 sum |terms| (Ogita, Rump, Oishi), with k terms per row."""
    s = make_system(2, 4, 3, 1, 1e-2, 3)
    K = sparse_K(s.D, s.E, s.C, s.R)
    x, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b)  # near solution: heavy cancellation
    r = dd_residual(K, x, s.b)[0]
    exact = _exact_residual(K, x[0], s.b[0])
    Kd = np.abs(K.toarray())
    k = int((Kd != 0).sum(axis=1).max()) + 1
    gamma = k * U64 / (1 - k * U64)
    for i, ex in enumerate(exact):
        terms = abs(s.b[0, i]) + float(Kd[i] @ np.abs(x[0]))
        assert abs(Fraction(r[i]) - ex) <= U64 * abs(ex) + Fraction(gamma * gamma * terms)


def _exact_solve(K, b):
    """Gaussian elimination in rationals (partial pivoting is unnecessary for SPD K)."""
    m = K.shape[0]
    A = [[Fraction(v) for v in row] + [Fraction(bv)] for row, bv in zip(K, b)]
    for c in range(m):
        piv = A[c][c]
        for r in range(c + 1, m):
            if A[r][c] != 0:
                f = A[r][c] / piv
                for j in range(c, m + 1):
                    A[r][j] -= f * A[c][j]
    x = [Fraction(0)] * m
    for r in range(m - 1, -1, -1):
        acc = A[r][m] - sum(A[r][j] * x[j] for j in range(r + 1, m))
        x[r] = acc / A[r][r]
    return x


def test_refined_reference_matches_exact_solution_at_kappa_1e6():
    s = make_system(2, 4, 3, 1, 1e-2, 5)
    D, E, C, R, sigma = stress_system(s.D, s.E, s.C, s.R, 1e6)
    K = dense.assemble_K(D, E, C, R)
    w = np.linalg.eigvalsh(K)
    assert w[-1] / w[0] == pytest.approx(1e6, rel=1e-3)
    exact = np.array([float(v) for v in _exact_solve(K, s.b[0])])
    plain, _ = oracle.solve(D, E, C, R, s.b)
    ref = refine_reference(D, E, C, R, s.b, steps=2)
    scale = np.max(np.abs(exact))
    err_ref = np.max(np.abs(ref[0] - exact)) / scale
    err_plain = np.max(np.abs(plain[0] - exact)) / scale
    assert err_ref <= 4 * U64
    assert err_plain <= 1e6 * 1e3 * U64  # the FP64 oracle alone: about kappa * u


@pytest.mark.parametrize("kappa", [1e3, 1e5, 1e6])
def test_stress_system_reaches_requested_condition_number(kappa):
    s = make_system(3, 7, 4, 1, 1e-2, 9)
    D, E, C, R, sigma = stress_system(s.D, s.E, s.C, s.R, kappa)
    assert np.array_equal(D, np.swapaxes(D, -1, -2))
    w = np.linalg.eigvalsh(dense.assemble_K(D, E, C, R))
    assert w[0] > 0
    assert w[-1] / w[0] == pytest.approx(kappa, rel=1e-3)
