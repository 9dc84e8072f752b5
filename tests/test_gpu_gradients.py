"""GPU parity of the solve gradients (bmpc_grad_blocks and the autograd Function)
against the FP64 oracle gradients (oracle/gradients.py, pinned by finite differences).

Bars: the block-gradient kernel on the oracle's x and lam to 1e-14 (it is the same
outer products in FP64); the full FP64 autograd path to 1e-9 relative (two GPU solves
at ~1e-15 each, so the bar is loose); the FP32 + refinement path to 1e-9 as well."""
import numpy as np
import pytest

from oracle import gradients
from synth.branch_system import make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    b = np.asarray(b)
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


SHAPES = [(2, 4, 4, 1), (3, 5, 3, 2), (2, 1, 4, 1), (5, 33, 16, 1), (4, 64, 16, 1),
          (2, 17, 32, 3)]


@pytest.mark.parametrize("S,N,n,nrhs", SHAPES)
def test_grad_blocks_kernel_matches_oracle(S, N, n, nrhs):
    from paper_2609_29977_amd import bmpc
    s = make_system(S, N, n, nrhs, 1e-1, 31)
    x, lam, _ = gradients.loss_gradients(s.D, s.E, s.C, s.R, s.b)
    ref = gradients.block_gradients(x, lam, S, N, n)
    plan = bmpc.Plan(S, N, n, nrhs, "fp64")
    got = plan.grad_blocks(_dev(x), _dev(lam))
    torch.cuda.synchronize()
    for g, r, name in zip(got, ref, "DECR"):
        if r.size == 0:
            continue
        assert rel(g.cpu().numpy(), r) <= 1e-14, name
    plan.close()


@pytest.mark.parametrize("S,N,n,nrhs", SHAPES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autograd_matches_oracle(S, N, n, nrhs, precision):
    from paper_2609_29977_amd.autograd import branch_solve
    s = make_system(S, N, n, nrhs, 1e-2, 32)
    _, _, (db, dD, dE, dC, dR) = gradients.loss_gradients(s.D, s.E, s.C, s.R, s.b)
    D, C, R, b = (_dev(a).requires_grad_() for a in (s.D, s.C, s.R, s.b))
    E = _dev(s.E).requires_grad_() if N > 1 else None
    x = branch_solve(D, E, C, R, b, precision)
    (0.5 * (x * x).sum()).backward()
    torch.cuda.synchronize()
    assert rel(b.grad.cpu().numpy(), db) <= 1e-9
    assert rel(D.grad.cpu().numpy(), dD) <= 1e-9
    assert rel(C.grad.cpu().numpy(), dC) <= 1e-9
    assert rel(R.grad.cpu().numpy(), dR) <= 1e-9
    if N > 1:
        assert rel(E.grad.cpu().numpy(), dE) <= 1e-9


def test_batched_gradients_at_workload_shape():
    """Four independent systems at the gradient workload's shape (S=128, N=64, n=16)."""
    from paper_2609_29977_amd.autograd import batched_branch_solve
    systems = [make_system(128, 64, 16, 1, 1e-2, 40 + i) for i in range(4)]
    st = lambda name: _dev(np.stack([getattr(s, name) for s in systems])).requires_grad_()
    D, E, C, R, b = st("D"), st("E"), st("C"), st("R"), st("b")
    x = batched_branch_solve(D, E, C, R, b, "fp64")
    (0.5 * (x * x).sum()).backward()
    torch.cuda.synchronize()
    for i, s in enumerate(systems):
        _, _, (db, dD, dE, dC, dR) = gradients.loss_gradients(s.D, s.E, s.C, s.R, s.b)
        assert rel(b.grad[i].cpu().numpy(), db) <= 1e-9
        assert rel(D.grad[i].cpu().numpy(), dD) <= 1e-9
        assert rel(E.grad[i].cpu().numpy(), dE) <= 1e-9
        assert rel(C.grad[i].cpu().numpy(), dC) <= 1e-9
        assert rel(R.grad[i].cpu().numpy(), dR) <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_pooled_plan_follows_the_current_stream(precision):
    """A plan pooled on the default stream, reused by a forward and backward issued on
    a side stream: its kernels must run on that stream (ordered after the inputs are
    produced there and before the outputs are read there)."""
    from paper_2609_29977_amd.autograd import branch_solve
    s = make_system(3, 9, 8, 1, 1e-2, 33)
    _, _, (db, dD, dE, dC, dR) = gradients.loss_gradients(s.D, s.E, s.C, s.R, s.b)
    # warm the pool on the default stream
    args = [_dev(a).requires_grad_() for a in (s.D, s.E, s.C, s.R, s.b)]
    x = branch_solve(*args, precision)
    (0.5 * (x * x).sum()).backward()
    del x
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        # inputs produced on the side stream right before the solve
        D, E, C, R, b = (_dev(np.zeros_like(a)) for a in (s.D, s.E, s.C, s.R, s.b))
        for t, a in zip((D, E, C, R, b), (s.D, s.E, s.C, s.R, s.b)):
            t.add_(torch.from_numpy(a).to("cuda", non_blocking=True))
        for t in (D, E, C, R, b):
            t.requires_grad_()
        x = branch_solve(D, E, C, R, b, precision)
        (0.5 * (x * x).sum()).backward()
    side.synchronize()
    assert rel(b.grad.cpu().numpy(), db) <= 1e-9
    assert rel(D.grad.cpu().numpy(), dD) <= 1e-9
    assert rel(E.grad.cpu().numpy(), dE) <= 1e-9
    assert rel(C.grad.cpu().numpy(), dC) <= 1e-9
    assert rel(R.grad.cpu().numpy(), dR) <= 1e-9


def test_second_backward_with_retained_graph():
    """retain_graph=True: the plan (and its factor) stays with the graph, so a second
    backward gives the same gradients (accumulated twice)."""
    from paper_2609_29977_amd.autograd import branch_solve
    s = make_system(2, 7, 4, 1, 1e-2, 34)
    _, _, (db, dD, dE, dC, dR) = gradients.loss_gradients(s.D, s.E, s.C, s.R, s.b)
    D, E, C, R, b = (_dev(a).requires_grad_() for a in (s.D, s.E, s.C, s.R, s.b))
    x = branch_solve(D, E, C, R, b, "fp64")
    loss = 0.5 * (x * x).sum()
    loss.backward(retain_graph=True)
    # another solve of the same shape in between must not take the retained plan
    y = branch_solve(*(_dev(a) for a in (s.D, s.E, s.C, s.R, s.b)), "fp64")
    loss.backward()
    torch.cuda.synchronize()
    assert rel(b.grad.cpu().numpy(), 2 * db) <= 1e-9
    assert rel(D.grad.cpu().numpy(), 2 * dD) <= 1e-9
    assert rel(E.grad.cpu().numpy(), 2 * dE) <= 1e-9
    del y
