"""Many independent systems of different shapes, solved together in one ragged plan.

A thin holder around bmpc.RaggedPlan (bmpc_analyze_ragged): the systems' arrays live
in the plan's concatenated layout, every step of the factorization and solves is one
launch over all systems, and nothing is padded.  PyTorch only moves data here (copies
into and out of the concatenated arrays); the factorization and solves run in the HIP
library.
"""
from __future__ import annotations

import torch

from . import bmpc


class HeteroBatch:
    """Storage and a ragged plan for systems of shapes shapes[i] = (S, N, n, nrhs)
    (one nrhs for all)."""

    def __init__(self, shapes, precision="fp32", device="cuda", stream=None):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.plan = bmpc.RaggedPlan(self.shapes, precision, stream=self.stream)
        f64 = torch.float64
        sz = self.plan.sizes
        with torch.cuda.stream(self.stream):
            self.D, self.E, self.C, self.R = (torch.zeros(max(k, 1), dtype=f64, device=self.device)
                                              for k in sz[:4])
            self.b = torch.zeros(sz[4], dtype=f64, device=self.device)
            self.x = torch.zeros_like(self.b)
        self.graph = None

    @property
    def padded_work(self) -> float:
        """Computed / real tail blocks: 1 (the ragged plan pads nothing)."""
        return 1.0

    def put(self, i, D, E, C, R, b):
        """Copy system i (arrays in the one-system layout, any device) into its slices."""
        S, N, n, nrhs = self.shapes[i]
        p = self.plan
        with torch.cuda.stream(self.stream):
            p.unpack(0, self.D, i).copy_(torch.as_tensor(D).reshape(-1))
            if N > 1:
                p.unpack(1, self.E, i).copy_(torch.as_tensor(E).reshape(-1))
            p.unpack(2, self.C, i).copy_(torch.as_tensor(C).reshape(-1))
            p.unpack(3, self.R, i).copy_(torch.as_tensor(R).reshape(-1))
            p.unpack(4, self.b, i).copy_(torch.as_tensor(b).reshape(-1))

    def system(self, i):
        """Views of system i's D, E, C, R, b in the concatenated arrays."""
        S, N, n, nrhs = self.shapes[i]
        p = self.plan
        return (p.unpack(0, self.D, i).view(S, N, n, n),
                p.unpack(1, self.E, i).view(S, max(N - 1, 0), n, n),
                p.unpack(2, self.C, i).view(S, n, n), p.unpack(3, self.R, i).view(n, n),
                p.unpack(4, self.b, i).view(nrhs, (S * N + 1) * n))

    def solution(self, i):
        """x of system i in the one-system layout [nrhs][(S*N+1)*n] (a copy)."""
        S, N, n, nrhs = self.shapes[i]
        self.stream.synchronize()
        return self.plan.unpack(4, self.x, i).view(nrhs, (S * N + 1) * n).clone()

    def solve(self, refine_tol=0.0, refine_iters=1):
        """Factor and solve every system (FP32: refined; FP64: plain solve) on the batch's
        stream, ordered after the current stream's earlier work; the current stream
        waits for it."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
        p = self.plan
        if p.precision == bmpc.FP64:
            p.factor_solve(self.D, self.E, self.C, self.R, self.b, self.x)
        else:
            p.factor_refine(self.D, self.E, self.C, self.R, self.b, self.x, tol=refine_tol,
                            max_iters=refine_iters)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def capture(self, refine_tol=0.0, refine_iters=1):
        """Record solve() once into a HIP graph (torch.cuda.CUDAGraph) on the batch's
        stream; the plan's launch tables are built at analysis, so the replay needs no
        host work beyond the graph launch."""
        with torch.cuda.stream(self.stream):
            self.solve(refine_tol, refine_iters)  # warm-up
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self.solve(refine_tol, refine_iters)
        torch.cuda.synchronize()
        return self.graph

    def replay(self):
        self.graph.replay()

    def info(self):
        """0 if every factorization succeeded, else the failing row (see bmpc_get_info)."""
        return self.plan.info()

    def close(self):
        self.plan.close()
