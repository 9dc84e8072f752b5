"""Property tests (hypothesis) over small random shapes, CPU only.

* The library's host analysis against the oracle's independent symbolic module: the
  ordering Pi_i of Section IV-A and the factor block structure of the elimination game,
  bit for bit, with x_1 last and one root-row block per tail (Theorem 1).
* The ordering's level count: floor(log2(N - 1)) + 1 chain levels plus the x_1 level.
* The oracle against a dense LAPACK solve of the assembled K.
* The cost model's flop count against a count taken from the symbolic structure."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

from oracle import dense, oracle, symbolic
from paper_2609_29977_amd import bmpc
from synth.branch_system import make_system

FAST = settings(max_examples=40, deadline=None)


@FAST
@given(st.integers(1, 700))
def test_ordering_and_structure_match_the_symbolic_module(N):
    perm = bmpc.ordering(N)
    assert perm == symbolic.tail_perm(N)
    assert sorted(perm) == list(range(N)) and perm[-1] == 0  # x_1 (stage 0) last
    if N <= 80:
        struct = bmpc.structure(N)
        assert struct == symbolic.tail_structure(N, "d")
        assert symbolic.root_row_blocks(N, "d") == 1


@FAST
@given(st.integers(2, 5000))
def test_level_count(N):
    c = bmpc.cost_model(1, N, 1, 1, "fp64")
    assert c.levels == (N - 1).bit_length() + 1


@settings(max_examples=25, deadline=None)
@given(st.integers(1, 3), st.integers(1, 9), st.integers(1, 4), st.integers(0, 2 ** 31 - 1),
       st.sampled_from([1.0, 1e-2]), st.integers(1, 3))
def test_oracle_matches_dense_solve(S, N, n, seed, delta, nrhs):
    s = make_system(S, N, n, nrhs, delta, seed)
    K = dense.assemble_K(s.D, s.E, s.C, s.R)
    ref = np.linalg.solve(K, s.b.T).T
    x, info = oracle.solve(s.D, s.E, s.C, s.R, s.b)
    assert info == 0
    assert np.max(np.abs(x - ref)) <= 1e-10 * np.max(np.abs(ref))


def _flops_from_structure(S, N, n):
    potrf = n ** 3 / 3 + n ** 2 / 2 + n / 6
    trsm, syrk, gemm = n ** 3, n ** 3 + n ** 2, 2 * n ** 3
    order = [(0, k) for k in symbolic.tail_perm(N)]
    adj = {v: set(nb) for v, nb in symbolic.block_graph(1, N).items()}
    done, per_tail = set(), 0.0
    for v in order:
        later = [u for u in adj[v] if u not in done]
        per_tail += potrf + len(later) * (trsm + syrk) + gemm * len(later) * (len(later) - 1) / 2
        for a in later:
            for c in later:
                if a != c:
                    adj[a].add(c)
        done.add(v)
    return S * per_tail + S * n * n + potrf


@FAST
@given(st.integers(1, 40), st.integers(1, 60), st.integers(1, 32))
def test_cost_model_flops_match_structure(S, N, n):
    c = bmpc.cost_model(S, N, n, 1, "fp64")
    assert abs(c.factor_flops - _flops_from_structure(S, N, n)) <= 1e-12 * c.factor_flops
