"""Pins of the oracle's symbolic module (orderings, fill, levels) -- CPU only."""
import math
import os

import numpy as np
import pytest

from oracle import dense, symbolic
from synth.branch_system import make_system

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gamma7_pattern.txt")


def _read_golden():
    order_line, rows = None, []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("order:"):
                order_line = line[len("order:"):].split()
            else:
                rows.append(line.split())
    return order_line, rows


def test_gamma7_matches_printed_example():
    order_tokens, _ = _read_golden()
    groups, cur = [], []
    for t in order_tokens:
        if t == "|":
            groups.append(cur)
            cur = []
        else:
            cur.append(int(t))
    groups.append(cur)
    seq = list(range(1, 8))
    assert symbolic.gamma(seq) == [x for g in groups for x in g]
    assert symbolic.gamma_groups(seq) == groups


def test_gamma7_block_pattern_matches_printed_matrix():
    """Gamma_7 Psi Gamma_7^T, eq. (seven_block_permutation)."""
    _, rows = _read_golden()
    N = 7

    def psi(i, j):  # 1-based block labels of Psi
        if i == j:
            return f"D{i}"
        if i == j + 1:
            return f"E{j}"
        if j == i + 1:
            return f"E{i}^T"
        return "."

    perm = symbolic.gamma(list(range(1, N + 1)))
    got = [[psi(perm[a], perm[b]) for b in range(N)] for a in range(N)]
    assert got == rows


def test_tail_perm_is_gamma_of_reversed_tail():
    # For N = 8 the chain (x_8, ..., x_2) has 7 blocks, so Pi_i applies the printed
    # Gamma_7 with xi_j = x_{9-j}; x_1 (0-based stage 0) stays last.
    order_tokens, _ = _read_golden()
    g7 = [int(t) for t in order_tokens if t != "|"]
    expect = [(9 - j) - 1 for j in g7] + [0]
    assert symbolic.tail_perm(8) == expect
    assert symbolic.tail_perm(1) == [0]
    assert symbolic.tail_perm(2) == [1, 0]
    assert symbolic.tail_perm(9) == [8, 6, 4, 2, 7, 3, 5, 1, 0]


@pytest.mark.parametrize("N", [1, 2, 3, 4, 7, 8, 9, 16, 31, 100, 255, 256])
def test_tail_perm_is_a_permutation_with_stage0_last(N):
    p = symbolic.tail_perm(N)
    assert sorted(p) == list(range(N))
    assert p[-1] == 0


@pytest.mark.parametrize("N", [2, 3, 4, 5, 8, 9, 17, 64, 128, 255, 256])
def test_level_count_is_logarithmic(N):
    # Each recursion of Gamma halves the chain (Section II): floor(log2(N-1)) + 1
    # chain levels, then the root-coupled block x_1.
    lv = symbolic.tail_levels(N)
    assert max(lv) == math.floor(math.log2(N - 1)) + 2
    assert lv[-1] == max(lv)
    # Blocks of one Gamma group share a level, and levels rise group by group.
    groups = symbolic.gamma_groups(list(range(N - 1)))
    pos = 0
    for g_i, g in enumerate(groups):
        assert lv[pos:pos + len(g)] == [g_i + 1] * len(g)
        pos += len(g)


@pytest.mark.parametrize("N", [2, 3, 5, 9, 16, 33])
def test_theorem1_single_root_coupling_block(N):
    # Appendix B: under Pi_i the root row of the factor holds only the terminal
    # block of the tail.  Ordering (a) fills the whole border, (b) keeps one block.
    assert symbolic.root_row_blocks(N, "d") == 1
    assert symbolic.root_row_blocks(N, "a") == N
    assert symbolic.root_row_blocks(N, "b") == 1
    s = symbolic.tail_structure(N, "d")
    assert (N, N - 1) in s


def test_ordering_c_spreads_the_coupling():
    # Fig. 2(c): Gamma on the whole reversed tail lets x_1 enter an early level.
    for N in (3, 5, 9, 17):
        assert symbolic.root_row_blocks(N, "c") > 1


@pytest.mark.parametrize("N", [1, 2, 3, 9, 16, 256])
def test_offdiagonal_block_count(N):
    # Each eliminated chain block couples to its right neighbour (or x_1) and, except
    # the first survivor of each level, to its left neighbour: per level 2e-1 blocks.
    s = symbolic.tail_structure(N, "d")
    off = sum(1 for r, c in s if r != c and r < N)
    m, expect = N - 1, 0
    while m > 0:
        e = (m + 1) // 2
        expect += 2 * e - 1
        m //= 2
    assert off == expect
    if N == 256:
        assert off == 502


@pytest.mark.parametrize("S,N,n,seed", [(2, 9, 3, 0), (1, 1, 2, 1), (1, 2, 3, 2),
                                        (3, 4, 2, 3), (2, 7, 1, 4), (1, 16, 2, 5),
                                        (2, 13, 2, 6)])
def test_fill_invariant_of_dense_reordered_cholesky(S, N, n, seed):
    """LAPACK's dense chol(Pi K Pi^T) is exactly zero outside the symbolically
    predicted blocks and nonzero inside them (the Fig. 2 case is S=2, N=9, n=3)."""
    sys_ = make_system(S, N, n, 1, 1.0, seed)
    K = dense.assemble_K(sys_.D, sys_.E, sys_.C, sys_.R)
    P = dense.perm_matrix(S, N, n, "d")
    L = np.linalg.cholesky(P @ K @ P.T)
    struct = set(symbolic.tail_structure(N, "d"))
    nb = S * N + 1
    for I in range(nb):
        for J in range(I + 1):
            blk = L[I * n:(I + 1) * n, J * n:(J + 1) * n]
            sI, pI = (I // N, I % N) if I < S * N else (None, N)
            sJ, pJ = (J // N, J % N) if J < S * N else (None, N)
            if sI is not None and sJ is not None and sI != sJ:
                expected = False
            else:
                expected = (pI, pJ) in struct
            if expected:
                assert np.any(blk != 0.0), (I, J)
            else:
                assert np.all(blk == 0.0), (I, J)


def test_global_perm_written_out_for_two_tails():
    # Pi = blkdiag(Pi_1, ..., Pi_M, I) (Section IV-A) for S = 2, N = 3: each tail is
    # reversed, Gamma_2 leaves (x_3, x_2) in place, x_1 stays last, the root follows.
    assert symbolic.global_perm(2, 3) == [(0, 2), (0, 1), (0, 0), (1, 2), (1, 1), (1, 0),
                                         symbolic.ROOT]
    assert symbolic.global_perm(1, 1) == [(0, 0), symbolic.ROOT]


@pytest.mark.parametrize("S,N,n", [(1, 1, 2), (2, 9, 3), (3, 5, 1), (2, 16, 2)])
def test_global_perm_is_blockwise_the_scalar_permutation(S, N, n):
    # Expanding every block variable of Pi into its n scalars gives the permutation
    # that puts K into the factored order; checked against an independent expansion
    # (the scalar index vector built from each tail's ordering).
    gp = symbolic.global_perm(S, N)
    assert len(gp) == S * N + 1 and len(set(gp)) == len(gp)
    idx = []
    for v in gp:
        base = S * N * n if v == symbolic.ROOT else (v[0] * N + v[1]) * n
        idx.extend(range(base, base + n))
    assert idx == dense.perm_index(S, N, n, "d").tolist()


@pytest.mark.parametrize("S,N", [(2, 9), (3, 4), (1, 17)])
def test_global_perm_keeps_one_root_block_per_tail(S, N):
    # Theorem 1 on the whole system: eliminating the block graph of K in the order of
    # Pi leaves exactly one root-row block per tail, the tail's last (x_1) variable;
    # the forward order of Fig. 2(a) fills the whole border.
    blocks, _ = symbolic.elimination_game(symbolic.block_graph(S, N),
                                          symbolic.global_perm(S, N))
    root_row = sorted(c for r, c in blocks if r == symbolic.ROOT and c != symbolic.ROOT)
    assert root_row == [(s, 0) for s in range(S)]
    fwd = [(s, k) for s in range(S) for k in range(N)] + [symbolic.ROOT]
    blocks_a, _ = symbolic.elimination_game(symbolic.block_graph(S, N), fwd)
    assert sum(1 for r, c in blocks_a if r == symbolic.ROOT and c != symbolic.ROOT) == S * N
