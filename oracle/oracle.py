"""Python front end of the FP64 CPU oracle (TEST INFRASTRUCTURE).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg use
this module.  It loads ``liboracle.so`` built from ``bmpc_oracle.c`` (plain C, gcc,
OpenMP over scenarios) and shares nothing with the GPU library.

Every function takes the block arrays in the layout of the synthetic generator
(``synth.branch_system``): D[S][N][n][n], E[S][N-1][n][n] (E[s,k] at block
(k+1, k)), C[S][n][n] (at block (root, stage 0)), R[n][n] and b[nrhs][(S*N+1)*n].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bmpc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the oracle library with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-Wall", "-Wextra", _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"oracle library missing: {_LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    ci = ctypes.c_int
    lib.oracle_solve.argtypes = [ci, ci, ci, ci, dp, dp, dp, dp, dp, dp, ci, dp, i64p]
    lib.oracle_solve.restype = ci
    lib.oracle_factor_export.argtypes = [ci, ci, ci, dp, dp, dp, dp, dp, dp, dp, i64p]
    lib.oracle_factor_export.restype = ci
    lib.oracle_threads.argtypes = [ci]
    lib.oracle_threads.restype = ci
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prep(D, E, C, R):
    D = np.ascontiguousarray(D, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    C = np.ascontiguousarray(C, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    S, N, n, _ = D.shape
    if E.size == 0:
        E = np.zeros((S, 1, n, n))  # never read when N == 1
    return D, E, C, R, S, N, n


def threads_used(nthreads: int) -> int:
    return int(_load().oracle_threads(int(nthreads)))


def solve(D, E, C, R, b, nthreads: int = 1, return_times: bool = False):
    """x = K^{-1} b in FP64 (natural-order band Cholesky).  Returns (x, info)
    or (x, info, (t_factor_s, t_solve_s))."""
    lib = _load()
    D, E, C, R, S, N, n = _prep(D, E, C, R)
    b = np.ascontiguousarray(b, dtype=np.float64)
    if b.ndim == 1:
        b = b[None, :]
    nrhs = b.shape[0]
    if b.shape[1] != (S * N + 1) * n:
        raise ValueError("b has the wrong length")
    x = np.zeros_like(b)
    times = np.zeros(2)
    info = ctypes.c_int64(0)
    rc = lib.oracle_solve(S, N, n, nrhs, _ptr(D), _ptr(E), _ptr(C), _ptr(R), _ptr(b),
                          _ptr(x), int(nthreads), _ptr(times), ctypes.byref(info))
    if rc != 0:
        raise RuntimeError("oracle_solve failed (bad arguments or out of memory)")
    if return_times:
        return x, int(info.value), (float(times[0]), float(times[1]))
    return x, int(info.value)


def factor_dense(D, E, C, R):
    """Dense lower factor L (natural order, root last) with L L^T = K, for small
    systems; returns (L, info)."""
    lib = _load()
    D, E, C, R, S, N, n = _prep(D, E, C, R)
    p = 2 * n - 1
    Nn = N * n
    AB = np.zeros((S, Nn, p + 1))
    W = np.zeros((S, n, Nn))
    LR = np.zeros((n, n))
    info = ctypes.c_int64(0)
    rc = lib.oracle_factor_export(S, N, n, _ptr(D), _ptr(E), _ptr(C), _ptr(R),
                                  _ptr(AB), _ptr(W), _ptr(LR), ctypes.byref(info))
    if rc != 0:
        raise RuntimeError("oracle_factor_export failed")
    tot = S * Nn + n
    L = np.zeros((tot, tot))
    for s in range(S):
        o = s * Nn
        for j in range(Nn):
            last = min(j + p, Nn - 1)
            L[o + j:o + last + 1, o + j] = AB[s, j, :last - j + 1]
        L[S * Nn:, o:o + Nn] = W[s]
    L[S * Nn:, S * Nn:] = np.tril(LR)
    return L, int(info.value)
