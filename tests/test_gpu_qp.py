"""GPU: assembly of the reduced IPM system (bmpc_assemble_qp) against the dense oracle
(oracle/qp.py), and the IPM step solved through the library against the full KKT
solve."""
import numpy as np
import pytest

from oracle import qp as oqp
from synth.qp import make_qp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("S,N,nx,nu", [(2, 4, 2, 1), (3, 9, 3, 2), (2, 1, 2, 2), (4, 17, 12, 4),
                                       (2, 5, 24, 8)])
def test_assembly_matches_dense_reduction(S, N, nx, nu):
    from paper_2609_29977_amd import bmpc
    q = make_qp(S, N, nx, nu, tau=1e-4, delta=1e-2, seed=7)
    n = q.n
    ref = oqp.blocks(oqp.reduced_K(q), S, N, n)
    got = bmpc.assemble_qp(_dev(q.Q), _dev(q.A), _dev(q.G), _dev(q.w), q.tau, q.delta)
    torch.cuda.synchronize()
    scale = max(np.max(np.abs(r)) for r in ref if r.size)
    for g, r, name in zip(got, ref, "DECR"):
        if r.size == 0:
            continue
        assert np.max(np.abs(g.cpu().numpy() - r)) <= 1e-13 * scale, name


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ipm_step_matches_full_kkt_solve(precision):
    from paper_2609_29977_amd import bmpc
    S, N, nx, nu = 3, 12, 4, 2
    q = make_qp(S, N, nx, nu, tau=1e-4, delta=1e-1, seed=8)
    n = q.n
    M = oqp.kkt(q)
    nv = (S * N + 1) * n
    rng = np.random.default_rng(9)
    rhs = np.zeros(M.shape[0])
    rhs[:nv] = rng.standard_normal(nv)
    full = np.linalg.solve(M, rhs)[:nv]
    D, E, C, R = bmpc.assemble_qp(_dev(q.Q), _dev(q.A), _dev(q.G), _dev(q.w), q.tau, q.delta)
    plan = bmpc.Plan(S, N, n, 1, precision)
    plan.factor(D, E, C, R)
    b = _dev(rhs[:nv][None, :])
    x = plan.solve(b) if precision == "fp64" else plan.refine(D, E, C, R, b, tol=1e-14,
                                                             max_iters=20)
    x = x.cpu().numpy()[0]
    assert np.max(np.abs(x - full)) <= 1e-9 * np.max(np.abs(full))
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_admm_system_through_the_ipm_assembly(precision):
    # ADMM paragraph of the appendix: with W = 0, tau = sigma and delta = 1/rho the
    # assembly builds P + sigma I + rho (A^T A + G^T G); checked block by block against
    # the dense ADMM reduction and, solved through the library, against the full ADMM
    # KKT solve.
    from paper_2609_29977_amd import bmpc
    S, N, nx, nu = 3, 10, 4, 2
    sigma, rho = 1e-6, 0.5
    q = make_qp(S, N, nx, nu, seed=10)
    n = q.n
    ref = oqp.blocks(oqp.admm_reduced_K(q, sigma, rho), S, N, n)
    w0 = np.zeros_like(q.w)
    D, E, C, R = bmpc.assemble_qp(_dev(q.Q), _dev(q.A), _dev(q.G), _dev(w0), sigma, 1.0 / rho)
    torch.cuda.synchronize()
    scale = max(np.max(np.abs(r)) for r in ref)
    for g, r, name in zip((D, E, C, R), ref, "DECR"):
        assert np.max(np.abs(g.cpu().numpy() - r)) <= 1e-13 * scale, name
    M = oqp.admm_kkt(q, sigma, rho)
    nv = (S * N + 1) * n
    rng = np.random.default_rng(11)
    rhs = np.zeros(M.shape[0])
    rhs[:nv] = rng.standard_normal(nv)
    full = np.linalg.solve(M, rhs)[:nv]
    plan = bmpc.Plan(S, N, n, 1, precision)
    plan.factor(D, E, C, R)
    b = _dev(rhs[:nv][None, :])
    x = plan.solve(b) if precision == "fp64" else plan.refine(D, E, C, R, b, tol=1e-14,
                                                             max_iters=20)
    assert plan.info() == 0
    x = x.cpu().numpy()[0]
    assert np.max(np.abs(x - full)) <= 1e-9 * np.max(np.abs(full))
    plan.close()
