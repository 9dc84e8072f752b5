"""GPU: a plan's factor and solve captured as HIP graphs (one graph each, on a side
stream) and replayed, as the timing of the paper-grid workload does.  Every replay,
with eager work of the program between replays, must reproduce the eager result bit
for bit, also after new inputs are copied into the captured buffers."""
import numpy as np
import pytest

from synth.branch_system import make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("S,N,n,precision", [(20, 30, 16, "fp64"), (7, 33, 16, "fp32"),
                                             (3, 9, 32, "fp64")])
def test_factor_and_solve_graph_replays_match_eager(S, N, n, precision):
    from paper_2609_29977_amd import bmpc
    dev = torch.device("cuda:0")
    sys_a = make_system(S, N, n, 1, 1e-2, 501)
    sys_b = make_system(S, N, n, 1, 1e-2, 502)
    to = lambda a: torch.from_numpy(a).to(dev)
    D, E, C, R, b = (to(a) for a in (sys_a.D, sys_a.E, sys_a.C, sys_a.R, sys_a.b))
    x = torch.empty_like(b)

    def eager(s):
        p = bmpc.Plan(S, N, n, 1, precision)
        p.factor(to(s.D), to(s.E), to(s.C), to(s.R))
        out = p.solve(to(s.b)).cpu().numpy()
        p.close()
        return out

    ref_a, ref_b = eager(sys_a), eager(sys_b)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    p = bmpc.Plan(S, N, n, 1, precision, stream=side)
    with torch.cuda.stream(side):
        p.factor(D, E, C, R)
        p.solve(b, x)
    torch.cuda.synchronize()
    gf, gs = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(gf, stream=side):
        p.factor(D, E, C, R)
    with torch.cuda.graph(gs, stream=side):
        p.solve(b, x)
    torch.cuda.synchronize()
    for rep in range(3):
        x.zero_()
        junk = torch.randn(1 << 20, device=dev).sum()  # eager work between replays
        gf.replay()
        gs.replay()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), ref_a), rep
        assert float(junk) == float(junk)
    # new inputs in the captured buffers
    for t, a in zip((D, E, C, R, b), (sys_b.D, sys_b.E, sys_b.C, sys_b.R, sys_b.b)):
        t.copy_(torch.from_numpy(a))
    for rep in range(2):
        x.zero_()
        gf.replay()
        gs.replay()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), ref_b), rep
    assert p.info() == 0
    p.close()
