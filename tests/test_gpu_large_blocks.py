"""GPU: block sizes 33..64 (Assumption 1 fixes one block size n_b for all stages, with
no bound; the library's limit is 64).

Blocks of 33..64 run through their own factor passes (one level per pass, the Schur
updates of the two neighbours in MFMA accumulators) and solve kernels (four waves per
block).  Checked like the smaller sizes: every stored factor block against dense
chol(Pi K Pi^T) (unique, so element-wise comparable), solutions through every entry
point against the FP64 oracle (1e-11 FP64, 1e-10 FP32 + refinement), a batch, the
pivot report and the gradients."""
import numpy as np
import pytest

from oracle import dense, gradients, oracle
from synth.branch_system import make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _bm():
    from paper_2609_29977_amd import bmpc
    return bmpc


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_inf(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("S,N,n", [(2, 1, 64), (2, 2, 40), (1, 3, 64), (2, 5, 33), (2, 9, 48),
                                   (1, 17, 64), (2, 6, 57)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_factor_blocks_match_dense_reordered_cholesky(S, N, n, precision):
    bm = _bm()
    s = make_system(S, N, n, 1, 1e-1, 17)
    K = dense.assemble_K(s.D, s.E, s.C, s.R)
    p = dense.perm_index(S, N, n, "d")
    L = np.linalg.cholesky(K[np.ix_(p, p)])
    tol = 1e-12 if precision == "fp64" else 5e-5
    plan = bm.Plan(S, N, n, 1, precision)
    plan.factor(*(_dev(a) if a.size else None for a in (s.D, s.E, s.C, s.R)))
    Nn = N * n
    scale = np.max(np.abs(L))
    for t in range(S):
        Lt, F = plan.export_tail_factor(t)
        ref = L[t * Nn:(t + 1) * Nn, t * Nn:(t + 1) * Nn]
        got = Lt.copy()
        for k in range(N):  # diagonal blocks are stored inverted
            blk = slice(k * n, (k + 1) * n)
            got[blk, blk] = np.linalg.inv(Lt[blk, blk])
        assert np.max(np.abs(got - ref)) <= tol * scale, t
        Fref = L[S * Nn:, t * Nn + (N - 1) * n:t * Nn + Nn]
        assert np.max(np.abs(F - Fref)) <= tol * scale
    LR = plan.export_root_factor()
    assert np.max(np.abs(np.tril(LR) - L[S * Nn:, S * Nn:])) <= tol * scale
    assert plan.info() == 0
    plan.close()


@pytest.mark.parametrize("S,N,n,nrhs", [(4, 33, 64, 1), (8, 64, 48, 3), (3, 100, 33, 6),
                                        (5, 16, 64, 2), (2, 257, 40, 1)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solutions_match_oracle(S, N, n, nrhs, precision):
    bm = _bm()
    s = make_system(S, N, n, nrhs, 1e-2, 18)
    ref, info = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=8)
    assert info == 0
    D, E, C, R, b = (_dev(a) for a in (s.D, s.E, s.C, s.R, s.b))
    plan = bm.Plan(S, N, n, nrhs, precision)
    if precision == "fp64":
        outs = [plan.factor_solve(D, E, C, R, b), plan.solve(b)]
        tol = 1e-11
    else:
        outs = [plan.factor_refine(D, E, C, R, b, tol=1e-13, max_iters=10),
                plan.refine(D, E, C, R, b, tol=1e-13, max_iters=10)]
        assert plan.stats()[2]
        plan.set_refine_stop("backward_error")
        outs.append(plan.refine(D, E, C, R, b, tol=16 * 2.0 ** -53, max_iters=10))
        it, eta, ok = plan.stats()
        assert ok and eta <= 16 * 2.0 ** -53
        tol = 1e-10
    assert plan.info() == 0
    for x in outs:
        assert rel_inf(x.cpu().numpy(), ref) <= tol
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_of_large_blocks(precision):
    bm = _bm()
    B, S, N, n = 3, 3, 20, 64
    systems = [make_system(S, N, n, 1, 1e-2, 90 + i) for i in range(B)]
    st = lambda name: _dev(np.stack([getattr(x, name) for x in systems]))
    D = st("D").reshape(B * S, N, n, n)
    E = st("E").reshape(B * S, N - 1, n, n)
    C = st("C").reshape(B * S, n, n)
    R, b = st("R"), st("b")
    plan = bm.Plan(S, N, n, 1, precision, num_systems=B)
    x = (plan.factor_solve(D, E, C, R, b) if precision == "fp64"
         else plan.factor_refine(D, E, C, R, b, tol=1e-13, max_iters=10))
    X = x.cpu().numpy()
    for i, s in enumerate(systems):
        ref, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b)
        assert rel_inf(X[i], ref) <= (1e-11 if precision == "fp64" else 1e-10)
    plan.close()


@pytest.mark.parametrize("stage,shift", [(5, -60.0), (0, -60.0)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_info_names_first_failing_pivot(stage, shift, precision):
    bm = _bm()
    S, N, n = 2, 9, 40
    s = make_system(S, N, n, 1, 1e-1, 19)
    s.D[1, stage] += shift * np.eye(n)
    K = dense.assemble_K(s.D, s.E, s.C, s.R)
    p = dense.perm_index(S, N, n, "d")
    Kp = K[np.ix_(p, p)]
    # first leading minor of Pi K Pi^T that is not positive definite: bisect on the
    # Cholesky of leading blocks (the minors are nested)
    lo, hi = 1, Kp.shape[0]
    while lo < hi:
        mid = (lo + hi) // 2
        try:
            np.linalg.cholesky(Kp[:mid, :mid])
            lo = mid + 1
        except np.linalg.LinAlgError:
            hi = mid
    natural = int(p[lo - 1]) + 1
    plan = bm.Plan(S, N, n, 1, precision)
    plan.factor(*(_dev(a) for a in (s.D, s.E, s.C, s.R)))
    assert plan.info() == natural
    plan.close()


def test_gradients_with_large_blocks():
    from paper_2609_29977_amd.autograd import branch_solve
    s = make_system(2, 9, 48, 2, 1e-2, 20)
    _, _, (db, dD, dE, dC, dR) = gradients.loss_gradients(s.D, s.E, s.C, s.R, s.b)
    D, E, C, R, b = (_dev(a).requires_grad_() for a in (s.D, s.E, s.C, s.R, s.b))
    x = branch_solve(D, E, C, R, b, "fp64")
    (0.5 * (x * x).sum()).backward()
    torch.cuda.synchronize()
    for got, ref in ((b.grad, db), (D.grad, dD), (E.grad, dE), (C.grad, dC), (R.grad, dR)):
        assert rel_inf(got.cpu().numpy(), ref) <= 1e-9
