"""Extended-precision reference solutions for ill-conditioned systems (TEST INFRASTRUCTURE).

The FP64 oracle's forward error grows like kappa(K) * u; at kappa ~ 1e6 that is about
1e-10, as large as the error bars the library is held to.  A reference accurate to
about u is obtained by classical iterative refinement of the oracle's solution in
which only the residual b - K x is evaluated in twice the working precision
(double-double): every product K_ij x_j is split exactly into a sum of two doubles
(Dekker 1971, splitting with 2^27 + 1) and the terms of a row are accumulated with
error-free two-sums (Knuth), as in Ogita, Rump and Oishi's Dot2 (2005).  The result is
as accurate as if the residual were computed in quadruple precision and then rounded,
so the refined x converges to the FP64 rounding of the exact solution while
kappa * u < 1.  Neither the library nor the oracle's solver uses this module.

``stress_system`` shifts a generated system towards singularity, K <- K - sigma I
(sigma subtracted from the diagonals of D and R), with sigma chosen from the measured
extreme eigenvalues so that kappa(K - sigma I) equals a requested value.
"""
from __future__ import annotations

import numpy as np

from . import oracle
from .conditioning import extreme_eigenvalues, sparse_K

_SPLIT = 134217729.0  # 2^27 + 1


def _split(a):
    c = _SPLIT * a
    hi = c - (c - a)
    return hi, a - hi


def two_prod(a, b):
    """p + e = a * b exactly (Dekker), elementwise."""
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def two_sum(a, b):
    """s + e = a + b exactly (Knuth), elementwise."""
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def dd_residual(K, x, b):
    """r = b - K x for the sparse K (CSR) and vectors x, b of shape (nrhs, m), each
    entry accumulated in double-double (Dot2 over the row's terms and b_i) and rounded
    once to double."""
    K = K.tocsr()
    K.sort_indices()
    x = np.atleast_2d(x)
    b = np.atleast_2d(b)
    m = K.shape[0]
    starts, ends = K.indptr[:-1], K.indptr[1:]
    lens = ends - starts
    out = np.empty_like(b)
    for q in range(b.shape[0]):
        s = b[q].copy()
        c = np.zeros(m)
        for t in range(int(lens.max()) if m else 0):
            rows = np.nonzero(lens > t)[0]
            idx = starts[rows] + t
            p, e = two_prod(-K.data[idx], x[q, K.indices[idx]])
            s_new, e2 = two_sum(s[rows], p)
            s[rows] = s_new
            c[rows] += e2 + e
        out[q] = s + c
    return out


def refine_reference(D, E, C, R, b, steps: int = 2, nthreads: int = 1):
    """The oracle's solution refined with double-double residuals; returns x."""
    K = sparse_K(D, E, C, R)
    x, info = oracle.solve(D, E, C, R, b, nthreads=nthreads)
    if info != 0:
        raise RuntimeError(f"oracle factorization failed (info {info})")
    for _ in range(steps):
        r = dd_residual(K, x, b)
        d, _ = oracle.solve(D, E, C, R, r, nthreads=nthreads)
        x = x + d
    return x


def stress_system(D, E, C, R, kappa: float):
    """Copies of the blocks with sigma I subtracted from every diagonal block (D and R),
    sigma = lambda_min - lambda_max / kappa, so that kappa(K - sigma I) = kappa up to the
    eigenvalue tolerance.  Returns (D, E, C, R, sigma)."""
    lmin, lmax = extreme_eigenvalues(D, E, C, R)
    # lambda_max - sigma differs from lambda_max; solve (lmax - s) / (lmin - s) = kappa
    sigma = (kappa * lmin - lmax) / (kappa - 1.0)
    n = D.shape[-1]
    eye = np.eye(n)
    return D - sigma * eye, E.copy(), C.copy(), R - sigma * eye, sigma
