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


@pytest.mark.parametrize("S,N,nx,nu,sigma,rho", [(2, 4, 2, 1, 1e-6, 0.1), (3, 5, 3, 2, 1e-3, 10.0),
                                                 (2, 1, 2, 2, 1e-6, 1.0)])
def test_admm_reduced_system_solves_the_admm_kkt_system(S, N, nx, nu, sigma, rho):
    # ADMM paragraph of the appendix: eliminating the second and third block rows of
    # the OSQP matrix leaves P + sigma I + rho A^T A + rho G^T G; its solve must give
    # the x part of the full KKT solve for a right-hand side that is zero below x.
    q = make_qp(S, N, nx, nu, seed=4)
    K = oqp.admm_reduced_K(q, sigma, rho)
    M = oqp.admm_kkt(q, sigma, rho)
    nv = K.shape[0]
    rng = np.random.default_rng(5)
    rhs = np.zeros(M.shape[0])
    rhs[:nv] = rng.standard_normal(nv)
    full = np.linalg.solve(M, rhs)
    red = np.linalg.solve(K, rhs[:nv])
    assert np.allclose(red, full[:nv], rtol=1e-9, atol=1e-11)
    assert np.linalg.eigvalsh(K)[0] > 0


def test_admm_system_is_the_ipm_reduction_with_zero_weights():
    # The two appendix matrices differ only in their weights: the IPM reduction with
    # tau = sigma, delta = 1/rho and W = 0 is the ADMM reduction.
    import dataclasses
    q = make_qp(3, 6, 3, 2, seed=6)
    sigma, rho = 1e-4, 3.0
    qz = dataclasses.replace(q, w=np.zeros_like(q.w), tau=sigma, delta=1.0 / rho)
    assert np.allclose(oqp.reduced_K(qz), oqp.admm_reduced_K(q, sigma, rho), rtol=1e-13,
                       atol=1e-13 * np.max(np.abs(oqp.admm_reduced_K(q, sigma, rho))))
    D, E, C, R = oqp.blocks(oqp.admm_reduced_K(q, sigma, rho), 3, 6, q.n)
    assert np.array_equal(dense.assemble_K(D, E, C, R), oqp.admm_reduced_K(q, sigma, rho))
