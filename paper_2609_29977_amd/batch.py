"""Many independent systems of different shapes, solved as a few uniform batches.

Systems are grouped into buckets of one shape: n exact, S and N rounded up to a
ladder of sizes (at most 1.5x each).  Each bucket is one batch plan (num_systems),
so every bucket is factored and solved with the same launches as one system.  The
padding is exact: a padded scenario has D = I, E = 0, C = 0 and b = 0 (it does not
couple to the root, so its Schur update is zero); padded stages are appended after
the last stage of a tail with zero coupling, D = I and b = 0.  Both decouple, their
unknowns come out as 0 and the real unknowns are those of the unpadded system.
PyTorch only moves data here (packing into the bucket arrays, views of the
results); the factorization and solves run in the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import bmpc

LADDER = (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024)


def bucket(v: int) -> int:
    for b in LADDER:
        if b >= v:
            return b
    return ((v + 255) // 256) * 256


@dataclass
class _Group:
    n: int
    S: int
    N: int
    nrhs: int
    members: list = field(default_factory=list)  # indices of systems
    plan: object = None
    stream: object = None
    D: object = None
    E: object = None
    C: object = None
    R: object = None
    b: object = None
    x: object = None


class HeteroBatch:
    """Bucketed storage and plans for systems of shapes shapes[i] = (S, N, n, nrhs)."""

    def __init__(self, shapes, precision="fp32", device="cuda", streams: int = 4):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.precision = precision
        self.device = torch.device(device)
        groups = {}
        self.slot = []
        for i, (S, N, n, nrhs) in enumerate(self.shapes):
            key = (n, bucket(S), bucket(N) if N > 1 else 1, nrhs)
            g = groups.setdefault(key, _Group(n=key[0], S=key[1], N=key[2], nrhs=key[3]))
            self.slot.append((key, len(g.members)))
            g.members.append(i)
        self.groups = groups
        # Buckets are independent: they run on `streams` streams (default priority),
        # longest first onto the least loaded stream, so that small buckets fill the
        # device together.
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, streams))]
        load = [0.0] * len(self.streams)
        for g in sorted(groups.values(), key=lambda g: -len(g.members) * g.S * g.N * g.n ** 3):
            k = min(range(len(load)), key=load.__getitem__)
            g.stream = self.streams[k]
            load[k] += len(g.members) * g.S * g.N * g.n ** 3
        f64 = torch.float64
        for g in groups.values():
            B, S, N, n = len(g.members), g.S, g.N, g.n
            eye = torch.eye(n, dtype=f64, device=self.device)
            g.D = eye.expand(B * S, N, n, n).contiguous()
            g.E = torch.zeros((B * S, max(N - 1, 0), n, n), dtype=f64, device=self.device)
            g.C = torch.zeros((B * S, n, n), dtype=f64, device=self.device)
            g.R = eye.expand(B, n, n).contiguous()
            g.b = torch.zeros((B, g.nrhs, (S * N + 1) * n), dtype=f64, device=self.device)
            g.x = torch.zeros_like(g.b)
            g.plan = bmpc.Plan(S, N, n, g.nrhs, precision, num_systems=B, stream=g.stream)

    @property
    def padded_work(self) -> float:
        """Padded / real tail blocks (the padding overhead)."""
        real = sum(S * N * n * n for S, N, n, _ in self.shapes)
        pad = sum(len(g.members) * g.S * g.N * g.n * g.n for g in self.groups.values())
        return pad / real

    def _views(self, i):
        key, k = self.slot[i]
        g = self.groups[key]
        S, N, n, nrhs = self.shapes[i]
        s0 = k * g.S
        return g, k, s0, S, N, n, nrhs

    def put(self, i, D, E, C, R, b):
        """Copy system i (arrays in the one-system layout, any device) into its slot."""
        g, k, s0, S, N, n, nrhs = self._views(i)
        g.D[s0:s0 + S, :N] = torch.as_tensor(D, device=self.device).reshape(S, N, n, n)
        if N > 1:
            g.E[s0:s0 + S, :N - 1] = torch.as_tensor(E, device=self.device).reshape(S, N - 1, n, n)
        g.C[s0:s0 + S] = torch.as_tensor(C, device=self.device).reshape(S, n, n)
        g.R[k] = torch.as_tensor(R, device=self.device).reshape(n, n)
        bb = torch.as_tensor(b, device=self.device).reshape(nrhs, S * N * n + n)
        dst = g.b[k, :, :g.S * g.N * n].view(nrhs, g.S, g.N, n)
        dst[:, :S, :N] = bb[:, :S * N * n].view(nrhs, S, N, n)
        g.b[k, :, g.S * g.N * n:] = bb[:, S * N * n:]

    def solution(self, i):
        """x of system i in the one-system layout [nrhs][(S*N+1)*n] (a copy)."""
        g, k, s0, S, N, n, nrhs = self._views(i)
        xt = g.x[k, :, :g.S * g.N * n].view(nrhs, g.S, g.N, n)[:, :S, :N].reshape(nrhs, S * N * n)
        return torch.cat([xt, g.x[k, :, g.S * g.N * n:]], dim=1)

    def solve(self, refine_tol=0.0, refine_iters=1):
        """Factor and solve every bucket (FP32 plans: refined; FP64: plain solve).
        Ordered after the current stream's earlier work; the current stream waits for
        all buckets."""
        cur = torch.cuda.current_stream(self.device)
        for st in self.streams:
            st.wait_stream(cur)
        for g in self.groups.values():
            E = g.E if g.N > 1 else None
            g.plan.factor(g.D, E, g.C, g.R)
            if g.plan.precision == bmpc.FP64:
                g.plan.solve(g.b, g.x)
            else:
                g.plan.refine(g.D, E, g.C, g.R, g.b, g.x, tol=refine_tol,
                              max_iters=refine_iters)
        for st in self.streams:
            cur.wait_stream(st)

    def capture(self, refine_tol=0.0, refine_iters=1):
        """Record solve() once into a HIP graph (torch.cuda.CUDAGraph): the library
        allocates nothing and records no memset in factor/refine, so the launches of
        every bucket, forked over the bucket streams and joined, replay as one graph."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.solve(refine_tol, refine_iters)  # warm-up
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=side):
            self.solve(refine_tol, refine_iters)
        torch.cuda.synchronize()
        return self.graph

    def replay(self):
        self.graph.replay()

    def info(self):
        """Per bucket: (key, info) for buckets whose factorization failed."""
        return [(k, g.plan.info()) for k, g in self.groups.items() if g.plan.info() != 0]

    def close(self):
        for g in self.groups.values():
            g.plan.close()
