"""Seeded synthetic branch systems generated on the GPU (inputs only, no solver
arithmetic), for workloads too large for the host generator.

Same recipe as synth.branch_system (E and C entries 0.5 * N(0, 1/n), D = M M^T / n +
(|E_{k-1}| + |E_k| + [k=0] |C| + delta) I, R = M M^T / n + (sum_s |C_s| + delta) I,
b ~ N(0, 1), D and R symmetrised bitwise), with two differences: the random numbers
come from torch's device generator (so the values differ from the host generator's
for the same seed), and the block norms are Frobenius norms, which bound the
spectral norms from above, so block diagonal dominance, SPD-ness and lambda_min >=
delta still hold.
"""
from __future__ import annotations

import torch


def make_system_gpu(S, N, n, nrhs, delta, seed, device="cuda"):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    kw = dict(dtype=f64, device=device, generator=g)
    sd = 0.5 / n ** 0.5
    E = torch.randn((S, max(N - 1, 0), n, n), **kw) * sd
    C = torch.randn((S, n, n), **kw) * sd
    MD = torch.randn((S, N, n, n), **kw)
    MR = torch.randn((n, n), **kw)
    b = torch.randn((nrhs, (S * N + 1) * n), **kw)
    nE = torch.linalg.matrix_norm(E) if N > 1 else torch.zeros((S, 0), dtype=f64, device=device)
    nC = torch.linalg.matrix_norm(C)
    shift = torch.full((S, N), float(delta), dtype=f64, device=device)
    if N > 1:
        shift[:, 1:] += nE
        shift[:, :-1] += nE
    shift[:, 0] += nC
    eye = torch.eye(n, dtype=f64, device=device)
    D = MD @ MD.transpose(-1, -2).contiguous() / n + shift[..., None, None] * eye
    D = (D + D.transpose(-1, -2)) * 0.5
    R = MR @ MR.T.contiguous() / n + (nC.sum() + delta) * eye
    R = (R + R.T) * 0.5
    return D, E, C, R, b
