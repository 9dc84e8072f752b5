"""GPU: the oracle's self-checks applied to the HIP path (through the C ABI).

* Normwise backward error of the solution, ||K x - b||_inf / (||K||_inf ||x||_inf +
  ||b||_inf), at the level of FP64 rounding: the FP64 path, and the FP32 factor with
  refinement run until the correction stops changing x (the FP64 residual makes its
  fixed point the FP64 solution).
* Reconstruction: the factor blocks the plan stores, pulled back into one lower
  triangular L in the elimination order Pi, give ||L L^T - Pi K Pi^T||_F / ||K||_F at
  the rounding level of the factor's precision (10 n u).
K x is formed with the sparse assembly of K that reads only the lower triangles of D
and R, as the library does."""
import numpy as np
import pytest

from oracle import dense
from oracle.conditioning import sparse_K
from synth.branch_system import make_config, make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps
U32 = float(np.finfo(np.float32).eps)


def _bm():
    from paper_2609_29977_amd import bmpc
    return bmpc


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def blocks(s):
    return _dev(s.D), _dev(s.E) if s.N > 1 else None, _dev(s.C), _dev(s.R)


def backward_error(s, x):
    K = sparse_K(s.D, s.E, s.C, s.R)
    r = s.b - (K @ x.T).T
    knorm = float(np.max(np.asarray(abs(K).sum(axis=1))))
    return float(np.max(np.abs(r)) / (knorm * np.max(np.abs(x)) + np.max(np.abs(s.b))))


SYSTEMS = [("c1", None), ("c2", None), ((16, 33, 5, 3, 1e-2), 11), ((7, 64, 16, 2, 1e-5), 12),
           ((3, 100, 32, 1, 1e-5), 13)]


def _system(spec, seed):
    if isinstance(spec, str):
        return make_config(spec, seed=0)
    S, N, n, nrhs, delta = spec
    return make_system(S, N, n, nrhs, delta, seed)


@pytest.mark.parametrize("spec,seed", SYSTEMS)
def test_fp64_backward_error(spec, seed):
    s = _system(spec, seed)
    p = _bm().Plan(s.S, s.N, s.n, s.nrhs, "fp64")
    p.factor(*blocks(s))
    x = p.solve(_dev(s.b)).cpu().numpy()
    assert p.info() == 0
    p.close()
    be = backward_error(s, x)
    print(f"fp64 backward error {be / U64:.2f} u")
    assert be <= 10 * U64


@pytest.mark.parametrize("spec,seed", SYSTEMS)
def test_fp32_refined_backward_error(spec, seed):
    s = _system(spec, seed)
    p = _bm().Plan(s.S, s.N, s.n, s.nrhs, "fp32")
    p.factor(*blocks(s))
    x = p.refine(*blocks(s), _dev(s.b), tol=0.0, max_iters=4).cpu().numpy()
    assert p.info() == 0
    p.close()
    be = backward_error(s, x)
    print(f"fp32+ir backward error {be / U64:.2f} u")
    assert be <= 10 * U64


@pytest.mark.parametrize("S,N,n", [(2, 9, 4), (3, 17, 8), (2, 33, 5), (1, 16, 32), (2, 5, 16)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_factor_reconstructs_permuted_K(S, N, n, precision):
    bm = _bm()
    s = make_system(S, N, n, 1, 1e-2, 21)
    K = dense.assemble_K(s.D, s.E, s.C, s.R)
    perm = dense.perm_index(S, N, n, "d")
    PKP = K[np.ix_(perm, perm)]
    p = bm.Plan(S, N, n, 1, precision)
    p.factor(*blocks(s))
    assert p.info() == 0
    Nn, tot = N * n, (S * N + 1) * n
    L = np.zeros((tot, tot))
    for t in range(S):
        Lt, F = p.export_tail_factor(t)
        for k in range(N):  # the plan stores the diagonal blocks inverted
            blk = slice(k * n, (k + 1) * n)
            Lt[blk, blk] = np.linalg.inv(Lt[blk, blk])
        L[t * Nn:(t + 1) * Nn, t * Nn:(t + 1) * Nn] = np.tril(Lt)
        L[S * Nn:, t * Nn + (N - 1) * n:(t + 1) * Nn] = F  # root row: x_1 column only
    L[S * Nn:, S * Nn:] = np.tril(p.export_root_factor())
    p.close()
    err = np.linalg.norm(L @ L.T - PKP) / np.linalg.norm(K)
    u = U64 if precision == "fp64" else U32
    print(f"{precision} reconstruction {err / u:.3f} n u-units={err / (n * u):.3f}")
    assert err <= 10 * n * u
