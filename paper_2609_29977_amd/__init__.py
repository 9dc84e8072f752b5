"""MI355X (gfx950) direct solver for root-coupled branch-MPC systems.

The HIP library ``libbmpc.so`` (built from ``csrc/``) implements the two-level
parallel Cholesky factorization and triangular solves of Algorithms 1 and 2 and
mixed-precision iterative refinement behind the C ABI of ``include/bmpc.h``;
``bmpc`` is its Python binding.
"""
from . import bmpc  # noqa: F401
from .bmpc import Plan, cost_model, ordering, structure  # noqa: F401
