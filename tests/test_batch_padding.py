"""The padding used to put systems of different shapes into one bucket is exact
(CPU, oracle): a padded system's solution restricted to the real unknowns equals the
unpadded solution, and the padded unknowns are 0.  Padded scenarios: D = I, E = 0,
C = 0, b = 0; padded stages appended after the last stage with zero coupling."""
import numpy as np
import pytest

from oracle import oracle
from synth.branch_system import make_system


def pad(s, Sb, Nb):
    S, N, n = s.S, s.N, s.n
    D = np.broadcast_to(np.eye(n), (Sb, Nb, n, n)).copy()
    E = np.zeros((Sb, Nb - 1, n, n))
    C = np.zeros((Sb, n, n))
    D[:S, :N] = s.D
    E[:S, :N - 1] = s.E
    C[:S] = s.C
    b = np.zeros((s.nrhs, (Sb * Nb + 1) * n))
    bt = b[:, :Sb * Nb * n].reshape(s.nrhs, Sb, Nb, n)
    bt[:, :S, :N] = s.b[:, :S * N * n].reshape(s.nrhs, S, N, n)
    b[:, Sb * Nb * n:] = s.b[:, S * N * n:]
    return D, E, C, s.R, b


@pytest.mark.parametrize("S,N,n,Sb,Nb", [(3, 5, 4, 4, 8), (2, 16, 3, 3, 16), (5, 9, 2, 8, 12)])
def test_padding_is_exact(S, N, n, Sb, Nb):
    s = make_system(S, N, n, 2, 1e-2, 90)
    ref, info = oracle.solve(s.D, s.E, s.C, s.R, s.b)
    assert info == 0
    D, E, C, R, b = pad(s, Sb, Nb)
    x, info = oracle.solve(D, E, C, R, b)
    assert info == 0
    xt = x[:, :Sb * Nb * n].reshape(2, Sb, Nb, n)
    got = np.concatenate([xt[:, :S, :N].reshape(2, -1), x[:, Sb * Nb * n:]], axis=1)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    mask = np.ones((Sb, Nb), bool)
    mask[:S, :N] = False
    assert np.all(xt[:, mask] == 0.0)


def test_bucket_ladder():
    from paper_2609_29977_amd.batch import bucket
    for v in range(1, 1100):
        bv = bucket(v)
        assert bv >= v and (bv <= max(8, 1.5 * v) or v > 1024)
