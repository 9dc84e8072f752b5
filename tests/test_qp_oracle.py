"""Pins of the reduced IPM system oracle (oracle/qp.py): the reduction against the full
KKT solve, SPD-ness, and the root-coupled block pattern of the reduced matrix."""
import numpy as np
import pytest

from oracle import dense, qp as oqp
from synth.qp import make_qp


@pytest.mark.parametrize("S,N,nx,nu", [(2, 4, 2, 1), (3, 5, 3, 2), (2, 1, 2, 2)])
def test_reduced_system_solves_the_kkt_system(S, N, nx, nu):
    q = make_qp(S, N, nx, nu, tau=1e-3, delta=1e-1, seed=1)
    K = oqp.reduced_K(q)
    M = oqp.kkt(q)
    nv = K.shape[0]
    rng = np.random.default_rng(2)
    rhs = np.zeros(M.shape[0])
    rhs[:nv] = rng.standard_normal(nv)
    full = np.linalg.solve(M, rhs)
    red = np.linalg.solve(K, rhs[:nv])
    assert np.allclose(red, full[:nv], rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("S,N,nx,nu", [(2, 6, 2, 1), (3, 3, 3, 2)])
def test_reduced_matrix_is_spd_with_the_root_coupled_pattern(S, N, nx, nu):
    q = make_qp(S, N, nx, nu, seed=3)
    n = nx + nu
    K = oqp.reduced_K(q)
    assert np.linalg.eigvalsh(K)[0] > 0
    D, E, C, R = oqp.blocks(K, S, N, n)
    rebuilt = dense.assemble_K(D, E, C, R)
    assert np.array_equal(rebuilt, K)  # nothing outside D, E, C, R
