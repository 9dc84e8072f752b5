"""Pins of the oracle's solve gradients (oracle/gradients.py) by central finite
differences of the loss l = 0.5 ||K^{-1} b||^2 through the oracle solve.

Symmetric arguments (D, R) are perturbed symmetrically (entries (i, j) and (j, i)
together), matching the symmetric-gradient convention; E and C entries singly."""
import numpy as np
import pytest

from oracle import gradients
from synth.branch_system import make_system

H = 1e-6


def fd(fun, arr, idx, sym=False):
    """Central difference of fun() when arr[idx] (and its mirror) moves; arr is
    perturbed in place and restored."""
    a = arr
    i, j = idx[-2], idx[-1]
    def pert(delta):
        a[idx] += delta
        if sym and i != j:
            a[idx[:-2] + (j, i)] += delta
    pert(H)
    lp = fun()
    pert(-2 * H)
    lm = fun()
    pert(H)
    return (lp - lm) / (2 * H), a


@pytest.mark.parametrize("S,N,n,nrhs,zero_c", [(2, 4, 4, 1, False), (3, 5, 3, 2, False),
                                               (2, 1, 4, 1, False), (2, 4, 3, 1, True)])
def test_gradients_match_central_differences(S, N, n, nrhs, zero_c):
    s = make_system(S, N, n, nrhs, 1e-1, 21, zero_coupling=zero_c)
    D, E, C, R, b = (s.D.copy(), s.E.copy(), s.C.copy(), s.R.copy(), s.b.copy())
    _, _, (db, dD, dE, dC, dR) = gradients.loss_gradients(D, E, C, R, b)
    rng = np.random.default_rng(5)
    arrays = {"D": D, "E": E, "C": C, "R": R, "b": b}
    grads = {"D": dD, "E": dE, "C": dC, "R": dR, "b": db}
    worst = 0.0
    for name in ("D", "E", "C", "R", "b"):
        arr = arrays[name]
        if arr.size == 0:
            continue
        for _ in range(6):
            idx = tuple(int(rng.integers(0, d)) for d in arr.shape)
            sym = name in ("D", "R")

            def fun():
                return gradients.loss(arrays["D"], arrays["E"], arrays["C"], arrays["R"],
                                      arrays["b"])[0]
            num, _ = fd(fun, arr, idx, sym)
            g = grads[name]
            i, j = idx[-2], idx[-1]
            ana = g[idx] + (g[idx[:-2] + (j, i)] if sym and i != j else 0.0)
            scale = max(1.0, abs(num))
            worst = max(worst, abs(num - ana) / scale)
            assert abs(num - ana) <= 1e-6 * scale, (name, idx, num, ana)
    assert worst < 1e-6


def test_adjoint_is_a_solve_with_the_same_matrix():
    """lam = K^{-1} x: K lam reproduces x (dense check on a tiny system)."""
    from oracle import dense
    s = make_system(2, 3, 3, 2, 1e-1, 22)
    x, lam, _ = gradients.loss_gradients(s.D, s.E, s.C, s.R, s.b)
    K = dense.assemble_K(s.D, s.E, s.C, s.R)
    assert np.allclose(K @ lam.T, x.T, rtol=1e-12, atol=1e-12)


def test_symmetric_gradients_are_symmetric():
    s = make_system(2, 4, 4, 1, 1e-1, 23)
    _, _, (_, dD, _, _, dR) = gradients.loss_gradients(s.D, s.E, s.C, s.R, s.b)
    assert np.array_equal(dD, np.swapaxes(dD, -1, -2))
    assert np.array_equal(dR, dR.T)
