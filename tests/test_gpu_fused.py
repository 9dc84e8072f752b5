"""GPU: factorization with the tail forward substitution inside it (bmpc_factor_solve,
bmpc_factor_refine), through the C ABI.

The fused path computes the same y = L^{-1} Pi b as the forward sweep of the solve, in
the elimination order instead of the level order, so it matches the separate factor +
solve calls up to rounding order, and the FP64 oracle at the usual bars (1e-11 FP64,
1e-10 FP32 + refinement).  The matrix arithmetic of the factorization is untouched, so
a later plain solve with the same plan reproduces the separate path bit for bit.
Window depths 1 and 2 force several passes (the right-hand-side updates of window
boundaries are carried between passes like the block updates)."""
import numpy as np
import pytest

from oracle import oracle
from synth.branch_system import make_config, make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _bm():
    from paper_2609_29977_amd import bmpc
    return bmpc


def _dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def blocks(s):
    return _dev(s.D), _dev(s.E) if s.N > 1 else None, _dev(s.C), _dev(s.R)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


SHAPES = [(1, 1, 1, 1), (3, 1, 5, 2), (2, 2, 3, 1), (1, 3, 8, 1), (2, 5, 4, 3), (3, 9, 3, 1),
          (2, 16, 8, 2), (4, 17, 16, 1), (2, 33, 5, 1), (3, 64, 17, 2), (2, 100, 31, 1),
          (2, 129, 32, 1), (1, 256, 32, 1)]


@pytest.mark.parametrize("S,N,n,nrhs", SHAPES)
def test_fp64_fused_matches_oracle_and_separate_path(S, N, n, nrhs):
    bm = _bm()
    s = make_system(S, N, n, nrhs, 1e-2, 21)
    s2 = make_system(S, N, n, nrhs, 1e-2, 22)  # a second right-hand side
    ref, info = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=4)
    assert info == 0
    b, b2 = _dev(s.b), _dev(s2.b)
    for wd in (0, 1, 2):
        pf = bm.Plan(S, N, n, nrhs, "fp64", wd)
        xf = pf.factor_solve(*blocks(s), b).cpu().numpy()
        ps = bm.Plan(S, N, n, nrhs, "fp64", wd)
        ps.factor(*blocks(s))
        xs = ps.solve(b).cpu().numpy()
        assert pf.info() == 0
        assert rel(xf, ref) <= 1e-11, wd
        assert rel(xf, xs) <= 1e-12, wd
        # the factor left in the plan is the separate path's, bit for bit
        assert np.array_equal(pf.solve(b2).cpu().numpy(), ps.solve(b2).cpu().numpy()), wd
        pf.close()
        ps.close()


@pytest.mark.parametrize("S,N,n,nrhs", SHAPES)
def test_fp32_fused_solve_and_refine_match_oracle(S, N, n, nrhs):
    bm = _bm()
    s = make_system(S, N, n, nrhs, 1e-2, 23)
    ref, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=4)
    b = _dev(s.b)
    for wd in (0, 1):
        p = bm.Plan(S, N, n, nrhs, "fp32", wd)
        xf = p.factor_solve(*blocks(s), b).cpu().numpy()
        xs = p.solve(b).cpu().numpy()  # same factor, separate forward sweep
        assert rel(xf, ref) <= 1e-3, wd  # plain FP32 solve
        assert rel(xf, xs) <= 1e-4, wd
        x = p.factor_refine(*blocks(s), b, tol=1e-13, max_iters=10).cpu().numpy()
        iters, relc, conv = p.stats()
        assert p.info() == 0 and conv, wd
        assert 1 <= iters <= 6, wd
        assert rel(x, ref) <= 1e-10, wd
        p.close()


def test_fused_solve_may_overwrite_b():
    bm = _bm()
    s = make_system(3, 33, 16, 2, 1e-2, 24)
    ref, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=4)
    p = bm.Plan(3, 33, 16, 2, "fp64")
    bx = _dev(s.b)
    p.factor_solve(*blocks(s), bx, x=bx)
    assert rel(bx.cpu().numpy(), ref) <= 1e-11
    p.close()


@pytest.mark.parametrize("S,N,n,nrhs", [(5, 17, 16, 2), (3, 64, 32, 1), (2, 2, 3, 3)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_batch_matches_single_system_fused(S, N, n, nrhs, precision):
    """A batch runs every chain and root on the same code and data as a one-system
    plan, so the fused batch reproduces the one-system fused results bitwise."""
    bm = _bm()
    B = 3
    systems = [make_system(S, N, n, nrhs, 1e-2, 70 + i) for i in range(B)]
    D = _dev(np.concatenate([x.D for x in systems]))
    E = _dev(np.concatenate([x.E for x in systems])) if N > 1 else None
    C = _dev(np.concatenate([x.C for x in systems]))
    R = _dev(np.stack([x.R for x in systems]))
    b = _dev(np.stack([x.b for x in systems]))
    pb = bm.Plan(S, N, n, nrhs, precision, num_systems=B)
    xb = pb.factor_solve(D, E, C, R, b).cpu().numpy()
    assert pb.info() == 0
    pb.close()
    for i, s in enumerate(systems):
        p1 = bm.Plan(S, N, n, nrhs, precision)
        x1 = p1.factor_solve(*blocks(s), _dev(s.b)).cpu().numpy()
        p1.close()
        assert np.array_equal(xb[i], x1), i


def test_fused_metric_workload_full_size():
    """S=512, N=256, n=32: the fused FP64 path and the fused FP32 + one refinement step
    against the oracle on the whole solution vector."""
    bm = _bm()
    s = make_config("c3", seed=0)
    ref, info = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=16)
    assert info == 0
    b = _dev(s.b)
    p64 = bm.Plan(s.S, s.N, s.n, s.nrhs, "fp64")
    x64 = p64.factor_solve(*blocks(s), b).cpu().numpy()
    assert p64.info() == 0 and rel(x64, ref) <= 1e-11
    p64.close()
    p32 = bm.Plan(s.S, s.N, s.n, s.nrhs, "fp32")
    x32 = p32.factor_refine(*blocks(s), b, tol=0.0, max_iters=1).cpu().numpy()
    iters, _, _ = p32.stats()
    assert p32.info() == 0 and iters == 1
    assert rel(x32, ref) <= 1e-10
    p32.close()


@pytest.mark.parametrize("S,N,n", [(3, 17, 16), (2, 33, 32), (2, 9, 7)])
def test_maximum_right_hand_sides(S, N, n):
    """kMaxRhs = 8 right-hand sides, the most a plan accepts (9 is rejected by the
    analysis), through the fused and the separate entry points in both precisions."""
    bm = _bm()
    s = make_system(S, N, n, 8, 1e-2, 25)
    ref, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=4)
    b = _dev(s.b)
    p64 = bm.Plan(S, N, n, 8, "fp64")
    assert rel(p64.factor_solve(*blocks(s), b).cpu().numpy(), ref) <= 1e-11
    assert rel(p64.solve(b).cpu().numpy(), ref) <= 1e-11
    p64.close()
    p32 = bm.Plan(S, N, n, 8, "fp32")
    x = p32.factor_refine(*blocks(s), b, tol=1e-13, max_iters=10).cpu().numpy()
    assert p32.info() == 0 and p32.stats()[2]
    assert rel(x, ref) <= 1e-10
    x = p32.refine(*blocks(s), b, tol=1e-13, max_iters=10).cpu().numpy()
    assert rel(x, ref) <= 1e-10
    p32.close()
