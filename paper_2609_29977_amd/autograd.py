"""torch.autograd support: x = K^{-1} b differentiable in D, E, C, R and b.

Forward: factor and solve through the C ABI (FP64, or FP32 with iterative
refinement).  Backward: the adjoint lam = K^{-1} g is one more solve with the same
factor (K is symmetric; refined like the forward solve in FP32 plans), db = lam, and
the block gradients come from bmpc_grad_blocks (dD and dR symmetric, see
include/bmpc.h).  All arithmetic runs in the HIP library; this module only moves
tensors.

Streams: every call runs on the stream that is current when it is made; a pooled plan
is moved to that stream before use, so its kernels are ordered after the producers of
the inputs and before the consumers of the outputs, which torch allocates on the same
stream.
"""
from __future__ import annotations

import warnings
import weakref

import torch

from . import bmpc

# Plans are reused across calls of the same shape.  A forward takes a plan from the
# pool; its factor must survive every backward through that forward, so the plan goes
# back to the pool only when the autograd context is freed (after the last backward,
# or when the graph is dropped), which also allows retain_graph=True.
_POOL: dict = {}

# Check, after every FP32 refinement, that the stop test was met (one stream
# synchronization per check); a refinement that hit its iteration limit warns.
check_convergence = True


def _on_current_stream(plan):
    st = torch.cuda.current_stream()
    if plan._stream is None or plan._stream.cuda_stream != st.cuda_stream:
        plan.set_stream(st)
    return plan


def _acquire(S, N, n, nrhs, precision, num_systems=1):
    key = (S, N, n, nrhs, bmpc._prec(precision), torch.cuda.current_device(), num_systems)
    free = _POOL.get(key)
    if free:
        plan = free.pop()
    else:
        plan = bmpc.Plan(S, N, n, nrhs, precision, num_systems=num_systems)
    return key, _on_current_stream(plan)


def _release(key, plan):
    _POOL.setdefault(key, []).append(plan)


def _hold_until_freed(ctx, key, plan):
    """Keep plan with ctx; return it to the pool when ctx is freed."""
    ctx.plan = plan
    weakref.finalize(ctx, _release, key, plan)


def _refined(plan, D, E, C, R, b, tol, iters, what):
    x = plan.refine(D, E, C, R, b, tol=tol, max_iters=iters)
    if check_convergence:
        it, rel, ok = plan.stats()
        if not ok:
            warnings.warn(f"{what}: FP32 refinement did not meet its stop test in {it} "
                          f"corrections (last relative correction {rel:.2e})",
                          RuntimeWarning, stacklevel=3)
    return x


def clear_plan_pool():
    """Destroy the pooled plans (frees their device workspaces)."""
    for plans in _POOL.values():
        for p in plans:
            p.close()
    _POOL.clear()


class BranchSolve(torch.autograd.Function):
    """x = K(D, E, C, R)^{-1} b for one system; tensors in the layout of include/bmpc.h
    with b of shape [nrhs, (S*N+1)*n]."""

    @staticmethod
    def forward(ctx, D, E, C, R, b, precision="fp64", refine_tol=1e-12, refine_iters=10):
        S, N, n = D.shape[0], D.shape[1], D.shape[2]
        nrhs = b.shape[0]
        key, plan = _acquire(S, N, n, nrhs, precision)
        D, C, R, b = D.contiguous(), C.contiguous(), R.contiguous(), b.contiguous()
        E = E.contiguous() if N > 1 else None
        plan.factor(D, E, C, R)
        if plan.precision == bmpc.FP64:
            x = plan.solve(b)
        else:
            x = _refined(plan, D, E, C, R, b, refine_tol, refine_iters, "branch_solve forward")
        _hold_until_freed(ctx, key, plan)
        ctx.refine = (refine_tol, refine_iters)
        if plan.precision == bmpc.FP64:
            ctx.save_for_backward(x)
        else:
            ctx.save_for_backward(x, D, E if N > 1 else torch.empty(0, device=D.device), C, R)
        ctx.N = N
        return x

    @staticmethod
    def backward(ctx, gx):
        plan = _on_current_stream(ctx.plan)
        if plan.precision == bmpc.FP64:
            (x,) = ctx.saved_tensors
            lam = plan.solve(gx.contiguous())
        else:
            # the adjoint is refined like the forward solve (FP64 residuals)
            x, D, E, C, R = ctx.saved_tensors
            tol, iters = ctx.refine
            lam = _refined(plan, D, E if ctx.N > 1 else None, C, R, gx.contiguous(), tol, iters,
                           "branch_solve backward")
        dD, dE, dC, dR = plan.grad_blocks(x, lam)
        return dD, (dE if ctx.N > 1 else None), dC, dR, lam, None, None, None


def branch_solve(D, E, C, R, b, precision="fp64"):
    """Differentiable solve of one root-coupled branch system."""
    return BranchSolve.apply(D, E, C, R, b, precision)


class BatchedBranchSolve(torch.autograd.Function):
    """Independent systems of one shape stacked on a leading batch dimension
    (D [B][S][N][n][n], E [B][S][N-1][n][n], C [B][S][n][n], R [B][n][n],
    b [B][nrhs][(S*N+1)*n]), factored and solved together in one batch plan."""

    @staticmethod
    def forward(ctx, D, E, C, R, b, precision="fp64", refine_tol=1e-12, refine_iters=10):
        B, S, N, n = D.shape[0], D.shape[1], D.shape[2], D.shape[3]
        nrhs = b.shape[1]
        key, plan = _acquire(S, N, n, nrhs, precision, num_systems=B)
        D, C, R, b = D.contiguous(), C.contiguous(), R.contiguous(), b.contiguous()
        E = E.contiguous() if N > 1 else None
        plan.factor(D, E, C, R)
        if plan.precision == bmpc.FP64:
            x = plan.solve(b)
            ctx.save_for_backward(x)
        else:
            x = _refined(plan, D, E, C, R, b, refine_tol, refine_iters,
                         "batched_branch_solve forward")
            ctx.save_for_backward(x, D, E if N > 1 else torch.empty(0, device=D.device), C, R)
        _hold_until_freed(ctx, key, plan)
        ctx.N = N
        ctx.refine = (refine_tol, refine_iters)
        ctx.shapes = (B, S, N, n)
        return x

    @staticmethod
    def backward(ctx, gx):
        plan = _on_current_stream(ctx.plan)
        if plan.precision == bmpc.FP64:
            (x,) = ctx.saved_tensors
            lam = plan.solve(gx.contiguous())
        else:
            x, D, E, C, R = ctx.saved_tensors
            tol, iters = ctx.refine
            lam = _refined(plan, D, E if ctx.N > 1 else None, C, R, gx.contiguous(), tol, iters,
                           "batched_branch_solve backward")
        dD, dE, dC, dR = plan.grad_blocks(x, lam)
        B, S, N, n = ctx.shapes
        dE = dE.view(B, S, N - 1, n, n) if N > 1 else None
        return (dD.view(B, S, N, n, n), dE, dC.view(B, S, n, n), dR.view(B, n, n), lam,
                None, None, None)


def batched_branch_solve(D, E, C, R, b, precision="fp64"):
    """Independent systems of one shape stacked on a leading batch dimension, solved in
    one batch plan (one factor and one solve for all of them)."""
    return BatchedBranchSolve.apply(D, E, C, R, b, precision)
