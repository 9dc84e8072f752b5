"""GPU: the autotuner (bmpc_autotune) and the launch configurations it chooses among.

Every configuration must give the same solution up to rounding: each candidate mapping
is checked against the oracle, and the tuner's choice applied per system in a ragged
batch."""
import numpy as np
import pytest

from oracle import oracle
from synth.branch_system import make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("S,N,n,precision", [(16, 33, 16, "fp32"), (8, 64, 32, "fp64"),
                                             (12, 17, 8, "fp32")])
def test_autotune_returns_a_candidate(S, N, n, precision):
    from paper_2609_29977_amd import bmpc
    wd, flags, best, times = bmpc.autotune(S, N, n, 1, precision, reps=3)
    assert 1 <= wd <= 6 and flags in (0, 1, 2, 3)
    assert len(times) >= 4 and best == pytest.approx(min(times))
    assert len(times) % 4 == 0  # four sweep mappings per window depth


@pytest.mark.parametrize("flags", [0, 1, 2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_mapping_matches_the_oracle(flags, precision):
    from paper_2609_29977_amd import bmpc
    s = make_system(6, 129, 32, 1, 1e-2, 44)
    ref, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=8)
    D, E, C, R, b = (_dev(a) for a in (s.D, s.E, s.C, s.R, s.b))
    for wd in (2, 4):
        p = bmpc.Plan(6, 129, 32, 1, precision, wd, flags=flags)
        x = (p.factor_solve(D, E, C, R, b) if precision == "fp64"
             else p.factor_refine(D, E, C, R, b, tol=1e-13, max_iters=10))
        bar = 1e-11 if precision == "fp64" else 1e-10
        assert np.max(np.abs(x.cpu().numpy() - ref)) <= bar * np.max(np.abs(ref)), (wd, flags)
        p.close()


def test_tuned_options_in_a_ragged_batch():
    from paper_2609_29977_amd import bmpc
    shapes = [(20, 40, 8), (9, 130, 16), (30, 70, 32), (4, 200, 32)]
    systems = [make_system(S, N, n, 1, 1e-2, 50 + i) for i, (S, N, n) in enumerate(shapes)]
    opts = []
    for S, N, n in shapes:
        wd, flags, _, _ = bmpc.autotune(S, N, n, 1, "fp32", reps=2)
        opts.append((wd, flags))
    rp = bmpc.RaggedPlan([(S, N, n, 1) for S, N, n in shapes], "fp32", options=opts)
    dev = lambda name: [_dev(getattr(s, name)) for s in systems]
    D, E, C, R, b = (rp.pack(w, dev(name)) for w, name in enumerate("DECRb"))
    x = rp.factor_refine(D, E, C, R, b, tol=1e-13, max_iters=10)
    for i, s in enumerate(systems):
        ref, _ = oracle.solve(s.D, s.E, s.C, s.R, s.b)
        xi = rp.unpack(4, x, i).cpu().numpy().reshape(1, -1)
        assert np.max(np.abs(xi - ref)) <= 1e-10 * np.max(np.abs(ref))
    rp.close()


def test_autotune_on_a_batch():
    """Tuned on a batch of systems (throughput): the choice is still a candidate, and a
    batch is timed slower than one of its systems."""
    from paper_2609_29977_amd import bmpc
    wd1, _, one, _ = bmpc.autotune(16, 40, 16, 1, "fp32", reps=3)
    wd, flags, many, times = bmpc.autotune(16, 40, 16, 1, "fp32", reps=3, num_systems=64)
    assert 1 <= wd <= 6 and flags in (0, 1, 2, 3)
    assert many == pytest.approx(min(times)) and many > one
