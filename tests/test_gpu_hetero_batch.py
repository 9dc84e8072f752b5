"""GPU: systems of different shapes through paper_2609_29977_amd.batch (one ragged plan)
against the FP64 oracle, per system (1e-11 FP64, 1e-10 FP32 + refinement)."""
import numpy as np
import pytest

from oracle import oracle
from synth.branch_system import make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_hetero_batch_against_oracle(precision):
    from paper_2609_29977_amd.batch import HeteroBatch
    rng = np.random.default_rng(3)
    shapes, systems = [], []
    for i in range(14):
        S = int(rng.integers(2, 10))
        N = int(rng.integers(3, 41))
        n = int(rng.choice([3, 8, 16]))
        delta = float(10 ** rng.uniform(-4, 0))
        systems.append(make_system(S, N, n, 1, delta, 200 + i))
        shapes.append((S, N, n, 1))
    hb = HeteroBatch(shapes, precision)
    assert hb.padded_work == 1.0
    for i, s in enumerate(systems):
        hb.put(i, s.D, s.E, s.C, s.R, s.b)
    if precision == "fp64":
        hb.solve()
    else:
        hb.solve(refine_tol=1e-13, refine_iters=10)
    torch.cuda.synchronize()
    assert hb.info() == 0
    bar = 1e-11 if precision == "fp64" else 1e-10
    for i, s in enumerate(systems):
        ref, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b)
        x = hb.solution(i).cpu().numpy()
        assert np.max(np.abs(x - ref)) <= bar * np.max(np.abs(ref)), i
    hb.close()


def test_gpu_generator_recipe_properties():
    """The device generator keeps the recipe's structure: symmetric D and R, and block
    diagonal dominance with margin delta (so lambda_min >= delta)."""
    from synth.branch_system_gpu import make_system_gpu
    D, E, C, R, b = make_system_gpu(3, 6, 4, 1, 1e-2, 5)
    D, E, C, R = (t.cpu().numpy() for t in (D, E, C, R))
    assert np.array_equal(D, np.swapaxes(D, -1, -2)) and np.array_equal(R, R.T)
    from oracle import dense
    K = dense.assemble_K(D, E, C, R)
    assert np.linalg.eigvalsh(K)[0] >= 1e-2 * (1 - 1e-9)


def test_graph_replays_match_eager():
    """The captured batch solve replays to the eager result, bitwise, every time, with
    eager work of the program between the replays."""
    from paper_2609_29977_amd.batch import HeteroBatch
    shapes = [(3, 9, 8, 1), (5, 17, 8, 1), (2, 33, 16, 1), (4, 12, 3, 1)]
    systems = [make_system(S, N, n, 1, 1e-2, 300 + i) for i, (S, N, n, _) in enumerate(shapes)]
    hb = HeteroBatch(shapes, "fp32")
    for i, s in enumerate(systems):
        hb.put(i, s.D, s.E, s.C, s.R, s.b)
    hb.solve(refine_tol=0.0, refine_iters=1)
    torch.cuda.synchronize()
    eager = [hb.solution(i).cpu().numpy() for i in range(len(shapes))]
    hb.capture(refine_tol=0.0, refine_iters=1)
    for rep in range(3):
        hb.x.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        hb.replay()
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            assert np.array_equal(hb.solution(i).cpu().numpy(), eager[i]), (rep, i)
        assert float(junk) == float(junk)
    hb.close()
