"""GPU: the allocation-free QP assembly (bmpc_assemble_qp_noalloc) against
bmpc_assemble_qp, which takes its scratch from the caller: the same kernels, so the
outputs must be bitwise equal.  Two calls in a row, the second with a smaller input
(the static scratch keeps the first call's contents), and an input beyond the scratch
is refused."""
import numpy as np
import pytest

from synth.qp import make_qp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _outputs(S, N, n):
    f64 = torch.float64
    return (torch.full((S, N, n, n), np.nan, dtype=f64, device="cuda"),
            torch.full((S, max(N - 1, 0), n, n), np.nan, dtype=f64, device="cuda"),
            torch.full((S, n, n), np.nan, dtype=f64, device="cuda"),
            torch.full((n, n), np.nan, dtype=f64, device="cuda"))


def test_noalloc_assembly_matches_the_workspace_entry_point():
    from paper_2609_29977_amd import bmpc
    for (S, N, nx, nu, seed) in ((24, 17, 12, 4, 1), (5, 9, 6, 2, 2)):
        q = make_qp(S, N, nx, nu, tau=1e-4, delta=1e-2, seed=seed)
        n = q.n
        args = (_dev(q.Q), _dev(q.A), _dev(q.G), _dev(q.w), q.tau, q.delta)
        ref = bmpc.assemble_qp(*args)
        got = bmpc.assemble_qp(*args, out=_outputs(S, N, n), noalloc=True)
        torch.cuda.synchronize()
        for g, r, name in zip(got, ref, "DECR"):
            assert torch.equal(g, r), (S, N, name)


def test_noalloc_assembly_refuses_inputs_beyond_its_scratch():
    from paper_2609_29977_amd import bmpc
    S, N, nx, nu = 513, 2, 24, 8  # S * n * n = 513 * 32 * 32 > 512 * 32 * 32
    q = make_qp(S, N, nx, nu, seed=3)
    with pytest.raises(bmpc.BmpcError) as e:
        bmpc.assemble_qp(_dev(q.Q), _dev(q.A), _dev(q.G), _dev(q.w), q.tau, q.delta,
                         out=_outputs(S, N, q.n), noalloc=True)
    assert e.value.status == bmpc.ERR_INVALID
