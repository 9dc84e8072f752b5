"""Symbolic side of the oracle: orderings and block fill (TEST INFRASTRUCTURE).

Pure-Python integer code, independent of the GPU library.  It provides
  * Gamma_N, the recursive odd-even block permutation (Section II);
  * Omega, the block reversal of a tail, and Pi_i = blkdiag(Gamma_{N-1}, I) Omega_i
    (Section IV-A), plus the contrasting orderings (a)-(c) of Fig. 2;
  * the block graph of K (eq. (root_coupled_matrix), eq. (tail_block_tridiagonal))
    and the elimination game on it, which predicts which blocks of the Cholesky
    factor are nonzero under a given ordering and at which elimination level each
    block variable can be eliminated.

Stages are 0-based generator stages: generator stage k is the paper's stage k+1,
so the root-coupled stage (the paper's x_1) is stage 0.
"""
from __future__ import annotations

from typing import Hashable, Iterable, List, Sequence, Tuple

ROOT = "root"


def gamma(seq: Sequence) -> list:
    """Gamma applied to an ordered sequence: its 1st, 3rd, 5th, ... items in order,
    followed by Gamma of the remaining (2nd, 4th, ...) items (Section II)."""
    seq = list(seq)
    if not seq:
        return []
    return seq[0::2] + gamma(seq[1::2])


def gamma_groups(seq: Sequence) -> List[list]:
    """The groups produced by the recursive calls of Gamma (the vertical bars of the
    Gamma_7 example in Section II); blocks inside one group are mutually uncoupled."""
    seq = list(seq)
    groups = []
    while seq:
        groups.append(seq[0::2])
        seq = seq[1::2]
    return groups


def omega(N: int) -> List[int]:
    """Block reversal of one tail: paper stages (N, ..., 1) as 0-based stages."""
    return list(range(N - 1, -1, -1))


def tail_perm(N: int) -> List[int]:
    """Pi_i of Section IV-A as 0-based stages in permuted order: reverse the tail,
    apply Gamma_{N-1} to (x_N, ..., x_2) and keep x_1 (stage 0) last."""
    if N < 1:
        raise ValueError("N >= 1")
    rev = omega(N)
    return gamma(rev[:-1]) + [rev[-1]]


def ordering(N: int, kind: str) -> List[int]:
    """Tail orderings of Fig. 2: 'a' forward, 'b' reversed sequential, 'c' Gamma on
    the whole reversed tail, 'd' the proposed Pi_i."""
    if kind == "a":
        return list(range(N))
    if kind == "b":
        return omega(N)
    if kind == "c":
        return gamma(omega(N))
    if kind == "d":
        return tail_perm(N)
    raise ValueError(kind)


def global_perm(S: int, N: int) -> List[Tuple[int, int]]:
    """Pi = blkdiag(Pi_1, ..., Pi_M, I): the block variables (s, stage) of all tails in
    permuted order, each tail with the same pattern, the root last."""
    p = tail_perm(N)
    return [(s, k) for s in range(S) for k in p] + [ROOT]


def block_graph(S: int, N: int):
    """Adjacency of the block variables of K: (s,k)-(s,k+1) inside a tail and
    (s,0)-root for every scenario."""
    adj = {ROOT: set()}
    for s in range(S):
        for k in range(N):
            adj[(s, k)] = set()
        for k in range(N - 1):
            adj[(s, k)].add((s, k + 1))
            adj[(s, k + 1)].add((s, k))
        adj[(s, 0)].add(ROOT)
        adj[ROOT].add((s, 0))
    return adj


def elimination_game(adj, order: Iterable[Hashable]):
    """Symbolic block Cholesky: eliminate vertices in ``order``; each elimination
    connects all not-yet-eliminated neighbours (fill).  Returns
    (blocks, level) where blocks is the set of (row_var, col_var) pairs of nonzero
    factor blocks (diagonal included) and level[v] is the elimination level of v
    (1 + the largest level of an earlier vertex that updates v)."""
    adj = {v: set(nb) for v, nb in adj.items()}
    order = list(order)
    done = set()
    blocks = set()
    level = {v: 1 for v in order}
    for v in order:
        later = [u for u in adj[v] if u not in done]
        blocks.add((v, v))
        for u in later:
            blocks.add((u, v))
            level[u] = max(level[u], level[v] + 1)
        for a in later:
            for c in later:
                if a != c:
                    adj[a].add(c)
        done.add(v)
    return blocks, level


def tail_structure(N: int, kind: str = "d") -> List[Tuple[int, int]]:
    """Nonzero factor blocks of one tail plus the root under the tail ordering
    ``kind``, as sorted (row, col) pairs of permuted positions: tail positions
    0..N-1 in the ordering, the root at position N.  The structure is the same for
    every tail, so one tail with the root describes it."""
    order = ordering(N, kind)
    pos = {(0, k): i for i, k in enumerate(order)}
    pos[ROOT] = N
    blocks, _ = elimination_game(block_graph(1, N), [(0, k) for k in order] + [ROOT])
    return sorted((pos[r], pos[c]) for r, c in blocks)


def tail_levels(N: int) -> List[int]:
    """Elimination level of every permuted position of a tail under Pi_i (the root
    excluded)."""
    order = tail_perm(N)
    _, level = elimination_game(block_graph(1, N), [(0, k) for k in order] + [ROOT])
    return [level[(0, k)] for k in order]


def root_row_blocks(N: int, kind: str = "d") -> int:
    """How many tail blocks the root row of the factor holds for one tail."""
    return sum(1 for r, c in tail_structure(N, kind) if r == N and c < N)
