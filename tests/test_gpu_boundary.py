"""GPU: the boundary's right-hand sides, structure query, stop tests and sweep options.

* nrhs beyond one kernel chunk (Section III-B partitions every right-hand side like the
  unknowns and puts no bound on their number): 9, 12 and 17 right-hand sides through
  every entry point, both precisions, one system and a batch, against the oracle.
* bmpc_query_structure equals the host structure (and so the elimination game).
* the backward-error stop of the refinement: x is returned only with
  |b - K x| <= tol (|K| |x| + |b|); checked on c1, c2, c3 and ill-conditioned systems,
  where the returned x must also meet the forward-error bars.
* the merged top backward levels give bitwise the results of one launch per level.
"""
import numpy as np
import pytest

from oracle import oracle
from oracle.extended import refine_reference, stress_system
from synth.branch_system import make_config, make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _bm():
    from paper_2609_29977_amd import bmpc
    return bmpc


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_inf(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def backward_error(s, x):
    """Normwise backward error of every right-hand side, max over them (FP64 residual
    by the oracle's dense-free block product, numpy)."""
    from oracle.conditioning import sparse_K
    K = sparse_K(s.D, s.E, s.C, s.R)
    knorm = abs(K).sum(axis=1).max()
    worst = 0.0
    for q in range(x.shape[0]):
        r = s.b[q] - K @ x[q]
        worst = max(worst, np.max(np.abs(r)) / (knorm * np.max(np.abs(x[q])) +
                                                np.max(np.abs(s.b[q]))))
    return worst


@pytest.mark.parametrize("S,N,n,nrhs", [(3, 17, 8, 12), (2, 9, 16, 9), (2, 33, 32, 17),
                                        (4, 1, 5, 12), (2, 2, 3, 10)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_many_right_hand_sides(S, N, n, nrhs, precision):
    bm = _bm()
    s = make_system(S, N, n, nrhs, 1e-2, 60 + n)
    ref, info = oracle.solve(s.D, s.E, s.C, s.R, s.b)
    assert info == 0
    D, E, C, R, b = (_dev(a) for a in (s.D, s.E, s.C, s.R, s.b))
    E = E if N > 1 else None
    tol = 1e-11 if precision == "fp64" else 1e-10
    p = bm.Plan(S, N, n, nrhs, precision)
    if precision == "fp64":
        outs = [p.factor_solve(D, E, C, R, b), p.solve(b)]
        p.factor(D, E, C, R)
        outs.append(p.solve(b))
        bb = b.clone()
        p.solve(bb, bb)  # in place
        outs.append(bb)
    else:
        outs = [p.factor_refine(D, E, C, R, b, tol=1e-13, max_iters=10),
                p.refine(D, E, C, R, b, tol=1e-13, max_iters=10)]
        assert p.stats()[2]
    assert p.info() == 0
    for x in outs:
        assert rel_inf(x.cpu().numpy(), ref) <= tol
    # every right-hand side on its own meets the bar (no chunk mixes another's values)
    X = outs[0].cpu().numpy()
    for q in range(nrhs):
        assert np.max(np.abs(X[q] - ref[q])) <= tol * np.max(np.abs(ref))
    p.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_many_right_hand_sides_in_a_batch(precision):
    bm = _bm()
    B, S, N, n, nrhs = 3, 4, 20, 8, 12
    systems = [make_system(S, N, n, nrhs, 1e-2, 70 + i) for i in range(B)]
    st = lambda name: _dev(np.stack([getattr(x, name) for x in systems]))
    D = st("D").reshape(B * S, N, n, n)
    E = st("E").reshape(B * S, N - 1, n, n)
    C = st("C").reshape(B * S, n, n)
    R, b = st("R"), st("b")
    p = bm.Plan(S, N, n, nrhs, precision, num_systems=B)
    if precision == "fp64":
        x = p.factor_solve(D, E, C, R, b)
    else:
        x = p.factor_refine(D, E, C, R, b, tol=1e-13, max_iters=10)
        assert p.stats()[2]
    X = x.cpu().numpy()
    for i, s in enumerate(systems):
        ref, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b)
        assert rel_inf(X[i], ref) <= (1e-11 if precision == "fp64" else 1e-10)
    p.close()


@pytest.mark.parametrize("N", [1, 2, 9, 17, 100, 256])
def test_query_structure_matches_host_structure(N):
    bm = _bm()
    p = bm.Plan(2, N, 4, 1, "fp64")
    assert p.structure() == bm.structure(N)
    p.close()


_C3 = {}


def _system(name):
    if name not in _C3:
        s = make_config(name, seed=0)
        ref, info = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=16)
        assert info == 0
        _C3[name] = (s, ref)
    return _C3[name]


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
@pytest.mark.parametrize("fused", [True, False])
def test_backward_error_stop(name, fused):
    """FP32 factor, refinement until the normwise backward error is <= 16 u: the library
    certifies x by its own FP64 residual; the result meets the 1e-10 forward bar."""
    bm = _bm()
    s, ref = _system(name)
    D, E, C, R, b = (_dev(a) for a in (s.D, s.E, s.C, s.R, s.b))
    p = bm.Plan(s.S, s.N, s.n, s.nrhs, "fp32")
    p.set_refine_stop("backward_error")
    tol = 16 * U64
    if fused:
        x = p.factor_refine(D, E, C, R, b, tol=tol, max_iters=10)
    else:
        p.factor(D, E, C, R)
        x = p.refine(D, E, C, R, b, tol=tol, max_iters=10)
    iters, eta, ok = p.stats()
    X = x.cpu().numpy()
    assert ok and 1 <= iters <= 3, (iters, eta)
    assert eta <= tol
    assert rel_inf(X, ref) <= 1e-10
    if s.S * s.N <= 40000:
        # the reported backward error is the one of the returned x
        assert backward_error(s, X) <= 2 * tol
    p.close()


def test_backward_error_stop_reports_failure():
    """max_iters = 0 certifies the plain FP32 solve, whose backward error is about the
    single-precision unit: not converged, and the reported value says so."""
    bm = _bm()
    s = make_system(3, 17, 8, 1, 1e-2, 5)
    D, E, C, R, b = (_dev(a) for a in (s.D, s.E, s.C, s.R, s.b))
    p = bm.Plan(3, 17, 8, 1, "fp32")
    p.set_refine_stop("backward_error")
    p.factor(D, E, C, R)
    p.refine(D, E, C, R, b, tol=16 * U64, max_iters=0)
    iters, eta, ok = p.stats()
    assert not ok and iters == 0 and eta > 1e-10
    p.close()


@pytest.mark.parametrize("kappa", [1e4, 1e6])
def test_backward_error_stop_on_ill_conditioned_systems(kappa):
    bm = _bm()
    s = make_system(4, 64, 32, 1, 1e-5, 32)
    D, E, C, R, _ = stress_system(s.D, s.E, s.C, s.R, kappa)
    ref = refine_reference(D, E, C, R, s.b, steps=2, nthreads=4)
    blocks = [_dev(a) for a in (D, E, C, R)]
    p = bm.Plan(4, 64, 32, 1, "fp32")
    p.set_refine_stop("backward_error")
    tol = 32 * U64
    x = p.factor_refine(*blocks, _dev(s.b), tol=tol, max_iters=20).cpu().numpy()
    iters, eta, ok = p.stats()
    assert ok and eta <= tol
    err = rel_inf(x, ref)
    # forward error <= kappa * backward error, with a factor 10 for the max norm
    assert err <= 10 * kappa * tol
    if kappa <= 1e4:
        assert err <= 1e-10
    p.close()


@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("N", [17, 129, 257])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_merged_top_backward_levels_are_bitwise_the_level_launches(n, N, precision):
    bm = _bm()
    S = 6
    s = make_system(S, N, n, 1, 1e-2, 80 + n)
    D, E, C, R, b = (_dev(a) for a in (s.D, s.E, s.C, s.R, s.b))
    outs = []
    for flags in (0, bm.FLAG_NO_BWD_TOP_MERGE):
        p = bm.Plan(S, N, n, 1, precision, flags=flags)
        p.factor(D, E, C, R)
        xs = p.solve(b).cpu().numpy()
        xr = p.refine(D, E, C, R, b, tol=0.0, max_iters=2).cpu().numpy()
        outs.append((xs, xr))
        p.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
