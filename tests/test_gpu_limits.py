"""GPU: more scenarios than a grid's y dimension holds.

The one-right-hand-side solve kernels put the scenario index on the grid's y dimension
(at most 65535); beyond that the plan falls back to the kernels with one flattened grid
dimension.  Both precisions, fused and separate entry points, against the oracle."""
import numpy as np
import pytest

from oracle import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("S,N,n", [(70000, 2, 32), (66000, 5, 8)])
def test_more_scenarios_than_a_grid_dimension(S, N, n):
    from paper_2609_29977_amd import bmpc
    from synth.branch_system_gpu import make_system_gpu
    D, E, C, R, b = make_system_gpu(S, N, n, 1, 1e-2, 91)
    host = [t.cpu().numpy() for t in (D, E, C, R, b)]
    ref, info = oracle.solve(*host, nthreads=16)
    assert info == 0
    scale = np.max(np.abs(ref))
    for precision, tol in (("fp64", 1e-11), ("fp32", 1e-10)):
        p = bmpc.Plan(S, N, n, 1, precision)
        if precision == "fp64":
            xf = p.factor_solve(D, E, C, R, b)
            xs = p.solve(b)
        else:
            xf = p.factor_refine(D, E, C, R, b, tol=1e-13, max_iters=10)
            xs = p.refine(D, E, C, R, b, tol=1e-13, max_iters=10)
        assert p.info() == 0
        for x in (xf, xs):
            assert np.max(np.abs(x.cpu().numpy() - ref)) <= tol * scale, precision
        p.close()
