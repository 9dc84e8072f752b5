"""GPU: ill-conditioned systems (K shifted towards singularity, kappa = 1e4 and 1e6).

Reference: the oracle's solution refined with double-double residuals (accurate to
about u, pinned against exact rational solves in test_extended.py).  Bound on the
relative max-norm forward error: kappa * (backward error), with the backward error of
both GPU paths at most 10 u (test_gpu_backward.py) and a factor 10 for the max-norm
condition number against the 2-norm kappa: 100 kappa u.  At kappa = 1e4 this is under
the 1e-10 bar of the FP32 + refinement path; at kappa = 1e6 no FP64-residual method can
promise 1e-10, and the bound is what is checked.

The FP32 factor with refinement converges while kappa * u_32 < 1: the correction shrinks
by about kappa * u_32 per step (6e-4 at kappa = 1e4, 6e-2 at 1e6), so the stop test
||d|| <= tol ||x|| is met within a step count that grows with kappa, and at its fixed
point the FP64 residual limits the correction to about kappa * u."""
import numpy as np
import pytest

from oracle.extended import refine_reference, stress_system
from synth.branch_system import make_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2


def _bm():
    from paper_2609_29977_amd import bmpc
    return bmpc


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


CASES = [((8, 33, 16, 1e-2), 31), ((4, 64, 32, 1e-5), 32)]


@pytest.mark.parametrize("kappa", [1e4, 1e6])
@pytest.mark.parametrize("shape,seed", CASES)
def test_ill_conditioned_fp64_and_refined_fp32(shape, seed, kappa):
    S, N, n, delta = shape
    s = make_system(S, N, n, 1, delta, seed)
    D, E, C, R, _ = stress_system(s.D, s.E, s.C, s.R, kappa)
    ref = refine_reference(D, E, C, R, s.b, steps=2, nthreads=4)
    scale = np.max(np.abs(ref))
    blocks = (_dev(D), _dev(E), _dev(C), _dev(R))
    b = _dev(s.b)
    bound = 100 * kappa * U64

    p64 = _bm().Plan(S, N, n, 1, "fp64")
    p64.factor(*blocks)
    x64 = p64.solve(b).cpu().numpy()
    assert p64.info() == 0
    p64.close()
    e64 = np.max(np.abs(x64 - ref)) / scale

    p32 = _bm().Plan(S, N, n, 1, "fp32")
    p32.factor(*blocks)
    tol = max(1e-12, 10 * kappa * U64)
    x32 = p32.refine(*blocks, b, tol=tol, max_iters=20).cpu().numpy()
    iters, relc, conv = p32.stats()
    assert p32.info() == 0
    p32.close()
    e32 = np.max(np.abs(x32 - ref)) / scale
    print(f"kappa {kappa:.0e}: fp64 err {e64:.2e}, fp32+ir err {e32:.2e} after {iters} "
          f"corrections (last {relc:.1e}), bound {bound:.1e}")
    assert e64 <= bound
    assert conv and iters <= (4 if kappa <= 1e4 else 12)
    assert e32 <= bound
    if kappa <= 1e4:
        assert e32 <= 1e-10
