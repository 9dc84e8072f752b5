"""GPU: batches of independent systems of one shape in one plan (num_systems).

Every chain and every root runs the same code on the same data as in a one-system
plan, so a batch must reproduce the one-system results bitwise; and each system of a
batch against the FP64 oracle to the usual bars (1e-11 FP64, 1e-10 FP32 + IR)."""
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


def stacked(systems):
    D = np.concatenate([s.D for s in systems])
    E = np.concatenate([s.E for s in systems]) if systems[0].N > 1 else None
    C = np.concatenate([s.C for s in systems])
    R = np.stack([s.R for s in systems])
    b = np.stack([s.b for s in systems])
    return D, E, C, R, b


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


SHAPES = [(5, 17, 16, 2), (3, 64, 32, 1), (4, 1, 8, 1), (2, 2, 3, 3), (7, 33, 5, 1)]


@pytest.mark.parametrize("S,N,n,nrhs", SHAPES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_reproduces_single_system_plans_bitwise(S, N, n, nrhs, precision):
    bm = _bm()
    B = 3
    systems = [make_system(S, N, n, nrhs, 1e-2, 50 + i) for i in range(B)]
    D, E, C, R, b = (None if a is None else _dev(a) for a in stacked(systems))
    plan = bm.Plan(S, N, n, nrhs, precision, num_systems=B)
    plan.factor(D, E, C, R)
    xb = plan.solve(b).cpu().numpy()
    assert plan.info() == 0
    plan.close()
    for i, s in enumerate(systems):
        p1 = bm.Plan(S, N, n, nrhs, precision)
        p1.factor(*(None if a is None else _dev(a) for a in (s.D, s.E if N > 1 else None, s.C, s.R)))
        x1 = p1.solve(_dev(s.b)).cpu().numpy()
        p1.close()
        assert np.array_equal(xb[i], x1), i


@pytest.mark.parametrize("S,N,n,nrhs", SHAPES)
def test_batch_against_oracle(S, N, n, nrhs):
    bm = _bm()
    B = 4
    deltas = [1e-4, 1e-2, 1e-1, 1.0]
    systems = [make_system(S, N, n, nrhs, deltas[i], 60 + i) for i in range(B)]
    refs = [oracle.solve(s.D, s.E, s.C, s.R, s.b)[0] for s in systems]
    arrs = [None if a is None else _dev(a) for a in stacked(systems)]
    D, E, C, R, b = arrs
    p64 = bm.Plan(S, N, n, nrhs, "fp64", num_systems=B)
    p64.factor(D, E, C, R)
    x64 = p64.solve(b).cpu().numpy()
    p32 = bm.Plan(S, N, n, nrhs, "fp32", num_systems=B)
    p32.factor(D, E, C, R)
    x32 = p32.refine(D, E, C, R, b, tol=1e-13, max_iters=10).cpu().numpy()
    iters, relc, conv = p32.stats()
    assert conv and 1 <= iters <= 6
    for i in range(B):
        assert rel(x64[i], refs[i]) <= 1e-11, i
        assert rel(x32[i], refs[i]) <= 1e-10, i
    p64.close()
    p32.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_info_names_the_failing_system_row(precision):
    bm = _bm()
    S, N, n, B = 2, 9, 3, 3
    systems = [make_system(S, N, n, 1, 1e-1, 70 + i) for i in range(B)]
    systems[1].D[0, 4] += -60.0 * np.eye(n)
    s = systems[1]
    K = dense.assemble_K(s.D, s.E, s.C, s.R)
    p = dense.perm_index(S, N, n, "d")
    Kp = K[np.ix_(p, p)]
    first = next(i for i in range(1, Kp.shape[0] + 1) if np.linalg.eigvalsh(Kp[:i, :i])[0] <= 0)
    natural = int(p[first - 1]) + 1
    D, E, C, R, b = (_dev(a) for a in stacked(systems))
    plan = bm.Plan(S, N, n, 1, precision, num_systems=B)
    plan.factor(D, E, C, R)
    assert plan.info() == 1 * (S * N + 1) * n + natural
    plan.close()


def test_batch_gradients_match_oracle():
    bm = _bm()
    S, N, n, nrhs, B = 4, 9, 6, 2, 3
    systems = [make_system(S, N, n, nrhs, 1e-1, 80 + i) for i in range(B)]
    xs, lams = [], []
    for s in systems:
        x, lam, _ = gradients.loss_gradients(s.D, s.E, s.C, s.R, s.b)
        xs.append(x)
        lams.append(lam)
    plan = bm.Plan(S, N, n, nrhs, "fp64", num_systems=B)
    dD, dE, dC, dR = plan.grad_blocks(_dev(np.stack(xs)), _dev(np.stack(lams)))
    dD, dE, dC, dR = (t.cpu().numpy() for t in (dD, dE, dC, dR))
    for i in range(B):
        ref = gradients.block_gradients(xs[i], lams[i], S, N, n)
        got = (dD[i * S:(i + 1) * S], dE[i * S:(i + 1) * S], dC[i * S:(i + 1) * S], dR[i])
        for g, r in zip(got, ref):
            assert rel(g, r) <= 1e-14
    plan.close()
