"""GPU: ragged batches -- independent systems of different S, N and n in one plan
(bmpc_analyze_ragged), each step one launch over all systems.

* every system against the FP64 oracle (1e-11 FP64, 1e-10 FP32 + refinement), block
  sizes 3..32 (the batching workload's 8, 16, 32 among them), S up to 70, N up to 160,
  fused and separate entry points, one and three right-hand sides;
* every system bitwise equal to its own one-system plan (the launches run the same
  kernel bodies on the same arguments);
* a captured graph replays to the eager result bitwise;
* the backward-error stop, and info naming the failing system's row.
"""
import numpy as np
import pytest

from oracle import oracle
from synth.branch_system import make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _bm():
    from paper_2609_29977_amd import bmpc
    return bmpc


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


SHAPES = [(70, 129, 32), (3, 160, 16), (64, 17, 8), (5, 1, 32), (9, 2, 13), (2, 77, 24),
          (33, 40, 16), (4, 64, 3), (1, 256, 8), (12, 33, 32), (7, 9, 5), (20, 100, 8)]


def _systems(nrhs, seed=500):
    rng = np.random.default_rng(seed)
    out = []
    for i, (S, N, n) in enumerate(SHAPES):
        delta = float(10 ** rng.uniform(-4, 0))
        out.append(make_system(S, N, n, nrhs, delta, seed + i))
    return out


def _pack(rp, systems):
    parts = lambda name: [_dev(getattr(s, name)) for s in systems]
    D = rp.pack(0, parts("D"))
    E = rp.pack(1, [_dev(s.E) if s.N > 1 else None for s in systems])
    C = rp.pack(2, parts("C"))
    R = rp.pack(3, parts("R"))
    b = rp.pack(4, parts("b"))
    return D, E, C, R, b


_REFS = {}


def _refs(systems, key):
    if key not in _REFS:
        _REFS[key] = [oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=8)[0] for s in systems]
    return _REFS[key]


@pytest.mark.parametrize("nrhs", [1, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("fused", [True, False])
def test_every_system_matches_the_oracle(nrhs, precision, fused):
    bm = _bm()
    systems = _systems(nrhs)
    refs = _refs(systems, nrhs)
    rp = bm.RaggedPlan([(s.S, s.N, s.n, nrhs) for s in systems], precision)
    D, E, C, R, b = _pack(rp, systems)
    if precision == "fp64":
        if fused:
            x = rp.factor_solve(D, E, C, R, b)
        else:
            rp.factor(D, E, C, R)
            x = rp.solve(b)
        bar = 1e-11
    else:
        if fused:
            x = rp.factor_refine(D, E, C, R, b, tol=1e-13, max_iters=10)
        else:
            rp.factor(D, E, C, R)
            x = rp.refine(D, E, C, R, b, tol=1e-13, max_iters=10)
        it, rel, ok = rp.stats()
        assert ok and it >= 1
        bar = 1e-10
    assert rp.info() == 0
    for i, (s, ref) in enumerate(zip(systems, refs)):
        xi = rp.unpack(4, x, i).cpu().numpy().reshape(nrhs, -1)
        err = np.max(np.abs(xi - ref)) / np.max(np.abs(ref))
        assert err <= bar, (i, s.S, s.N, s.n, err)
    rp.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bitwise_equal_to_one_system_plans(precision):
    bm = _bm()
    systems = _systems(1, seed=600)
    rp = bm.RaggedPlan([(s.S, s.N, s.n, 1) for s in systems], precision)
    D, E, C, R, b = _pack(rp, systems)
    if precision == "fp64":
        x = rp.factor_solve(D, E, C, R, b)
    else:
        x = rp.factor_refine(D, E, C, R, b, tol=0.0, max_iters=2)
    torch.cuda.synchronize()
    chain = 0
    for i, s in enumerate(systems):
        p = bm.Plan(s.S, s.N, s.n, 1, precision)
        args = [_dev(a) if a.size else None for a in (s.D, s.E, s.C, s.R)]
        bi = _dev(s.b)
        xi = (p.factor_solve(*args, bi) if precision == "fp64"
              else p.factor_refine(*args, bi, tol=0.0, max_iters=2))
        assert torch.equal(rp.unpack(4, x, i), xi.reshape(-1)), i
        # stored factor of the first chain of the system
        Lr, Fr = rp.export_tail_factor(chain)
        Lp, Fp = p.export_tail_factor(0)
        assert np.array_equal(Lr[:Lp.shape[0], :Lp.shape[1]], Lp) and np.array_equal(Fr[:Fp.shape[0], :Fp.shape[1]], Fp)
        chain += s.S
        p.close()
    rp.close()


def test_graph_replays_match_eager():
    bm = _bm()
    systems = _systems(1, seed=700)[:8]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    rp = bm.RaggedPlan([(s.S, s.N, s.n, 1) for s in systems], "fp32", stream=side)
    with torch.cuda.stream(side):
        D, E, C, R, b = _pack(rp, systems)
        x = torch.zeros_like(b)
        rp.factor_refine(D, E, C, R, b, x, tol=0.0, max_iters=1)
    side.synchronize()
    eager = x.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        rp.factor_refine(D, E, C, R, b, x, tol=0.0, max_iters=1)
    torch.cuda.synchronize()
    for rep in range(3):
        x.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, eager), rep
        assert float(junk) == float(junk)
    rp.close()


def test_backward_error_stop():
    bm = _bm()
    systems = _systems(1, seed=800)
    refs = [oracle.solve(s.D, s.E, s.C, s.R, s.b, nthreads=8)[0] for s in systems]
    rp = bm.RaggedPlan([(s.S, s.N, s.n, 1) for s in systems], "fp32")
    rp.set_refine_stop("backward_error")
    D, E, C, R, b = _pack(rp, systems)
    tol = 16 * 2.0 ** -53
    x = rp.factor_refine(D, E, C, R, b, tol=tol, max_iters=10)
    it, eta, ok = rp.stats()
    assert ok and eta <= tol and 1 <= it <= 3
    for i, ref in enumerate(refs):
        xi = rp.unpack(4, x, i).cpu().numpy().reshape(1, -1)
        assert np.max(np.abs(xi - ref)) <= 1e-10 * np.max(np.abs(ref))
    rp.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["x1", "odd"])
def test_info_names_the_failing_system(precision, which):
    bm = _bm()
    systems = _systems(1, seed=900)[:6]
    bad = 3
    # stage 0 = x_1, eliminated last; stage N-1 = chain position 1, a level-1 block
    # factored by the level-1 inverse launch before the first pass
    stage = 0 if which == "x1" else systems[bad].N - 1
    systems[bad].D[1, stage] -= 80.0 * np.eye(systems[bad].n)
    rp = bm.RaggedPlan([(s.S, s.N, s.n, 1) for s in systems], precision)
    D, E, C, R, b = _pack(rp, systems)
    rp.factor(D, E, C, R)
    got = rp.info()
    p = bm.Plan(systems[bad].S, systems[bad].N, systems[bad].n, 1, precision)
    p.factor(*(_dev(a) if a.size else None for a in (systems[bad].D, systems[bad].E,
                                                     systems[bad].C, systems[bad].R)))
    local = p.info()
    assert local > 0
    rows_before = sum((s.S * s.N + 1) * s.n for s in systems[:bad])
    assert got == rows_before + local
    p.close()
    rp.close()
