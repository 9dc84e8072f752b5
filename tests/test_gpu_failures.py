"""GPU: NaN inputs are reported, not hidden.

A NaN anywhere in the matrix reaches a pivot of the factorization (the NaN-aware pivot
test !(p > 0) fails on it), so the factor sets info and bmpc_get_info returns NOT_SPD; a
NaN in the right-hand side propagates into the solution; and refinement, whose norms
propagate NaN, never meets its stop test and reports no convergence after max_iters."""
import math

import numpy as np
import pytest

from synth.branch_system import make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

S, N, n = 3, 17, 8


def _bm():
    from paper_2609_29977_amd import bmpc
    return bmpc


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("where", ["D diagonal", "D off-diagonal", "E", "C", "R"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nan_in_matrix_sets_info(where, precision):
    s = make_system(S, N, n, 1, 1e-2, 61)
    D, E, C, R = s.D.copy(), s.E.copy(), s.C.copy(), s.R.copy()
    if where == "D diagonal":
        D[1, 5, 3, 3] = np.nan
    elif where == "D off-diagonal":
        D[2, 9, 6, 2] = np.nan  # lower triangle: read
    elif where == "E":
        E[0, 4, 1, 7] = np.nan
    elif where == "C":
        C[2, 0, 5] = np.nan
    else:
        R[4, 2] = np.nan
    p = _bm().Plan(S, N, n, 1, precision)
    p.factor(_dev(D), _dev(E), _dev(C), _dev(R))
    assert p.info() != 0, where
    p.close()


def test_nan_in_rhs_propagates_and_refinement_does_not_converge():
    bm = _bm()
    s = make_system(S, N, n, 1, 1e-2, 62)
    b = s.b.copy()
    b[0, 37] = np.nan
    blocks = (_dev(s.D), _dev(s.E), _dev(s.C), _dev(s.R))
    p64 = bm.Plan(S, N, n, 1, "fp64")
    p64.factor(*blocks)
    x = p64.solve(_dev(b)).cpu().numpy()
    assert p64.info() == 0 and np.isnan(x).any()
    p64.close()
    p32 = bm.Plan(S, N, n, 1, "fp32")
    p32.factor(*blocks)
    p32.refine(*blocks, _dev(b), tol=1e-12, max_iters=3)
    iters, relc, conv = p32.stats()
    assert not conv and iters == 3
    assert math.isnan(relc) or relc > 1e-12
    p32.close()


def test_allocation_failure_is_reported_and_leaves_no_error_behind():
    """A plan within the dimension limits whose workspaces cannot fit in HBM (S = 31000,
    N = 1000, n = 32 in FP64: three factor arrays of 254 GB each) fails with
    BMPC_ERR_ALLOC and frees what it had allocated; the failure does not surface as an
    error of later, valid calls."""
    bm = _bm()
    with pytest.raises(bm.BmpcError) as e:
        bm.Plan(31000, 1000, 32, 1, "fp64")
    assert e.value.status == bm.ERR_ALLOC
    s = make_system(S, N, n, 1, 1e-2, 63)
    p = bm.Plan(S, N, n, 1, "fp64")
    p.factor(_dev(s.D), _dev(s.E), _dev(s.C), _dev(s.R))
    x = p.solve(_dev(s.b)).cpu().numpy()
    assert p.info() == 0 and np.isfinite(x).all()
    p.close()
