"""Thin Python binding of the bmpc C ABI (include/bmpc.h).

Argument marshalling only: torch tensors provide device memory and the current HIP
stream; every step of the factorization and solves runs in the HIP kernels of
``libbmpc.so``.  There is no CPU fallback: a missing library or GPU raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbmpc.so")

OK, ERR_INVALID, ERR_NOT_SPD, ERR_ALLOC, ERR_DEVICE, ERR_STATE, ERR_NOT_CONVERGED = \
    0, -1, -2, -3, -4, -5, -6
FP64, FP32_REFINE = 0, 1
FLAG_NO_BWD_TOP_MERGE = 0x1
FLAG_FWD_ONE_WAVE = 0x2
STOP_CORRECTION, STOP_BACKWARD_ERROR = 0, 1
UNIT_ROUNDOFF = 2.0 ** -53

EXPORTED = [
    "bmpc_analyze", "bmpc_analyze_ex", "bmpc_set_stream", "bmpc_factor", "bmpc_solve",
    "bmpc_refine", "bmpc_get_info", "bmpc_get_stats", "bmpc_query_perm",
    "bmpc_query_cost", "bmpc_query_kernel_cost", "bmpc_export_tail_factor",
    "bmpc_export_root_factor", "bmpc_set_profiling", "bmpc_get_kernel_times",
    "bmpc_reset_kernel_times", "bmpc_kernel_class_name", "bmpc_kernel_class_count",
    "bmpc_destroy", "bmpc_status_string", "bmpc_ordering", "bmpc_structure",
    "bmpc_cost_model", "bmpc_grad_blocks", "bmpc_assemble_qp", "bmpc_factor_solve",
    "bmpc_factor_refine", "bmpc_set_refine_stop", "bmpc_query_structure",
    "bmpc_assemble_qp_noalloc", "bmpc_analyze_ragged", "bmpc_ragged_layout", "bmpc_autotune",
]


class BmpcError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


class _Dims(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("N", ctypes.c_int32), ("n", ctypes.c_int32),
                ("nrhs", ctypes.c_int32)]


class _QpDims(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("N", ctypes.c_int32), ("n", ctypes.c_int32),
                ("me", ctypes.c_int32), ("mi", ctypes.c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("window_depth", ctypes.c_int32), ("num_systems", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("later_depth", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class _Cost(ctypes.Structure):
    _fields_ = [("factor_flops", ctypes.c_double), ("solve_flops", ctypes.c_double),
                ("factor_bytes", ctypes.c_double), ("solve_bytes", ctypes.c_double),
                ("residual_bytes", ctypes.c_double), ("levels", ctypes.c_int32),
                ("passes", ctypes.c_int32), ("window_depth", ctypes.c_int32),
                ("later_depth", ctypes.c_int32), ("workspace_bytes", ctypes.c_double)]


@dataclass
class Cost:
    factor_flops: float
    solve_flops: float
    factor_bytes: float
    solve_bytes: float
    residual_bytes: float
    levels: int
    passes: int
    window_depth: int
    workspace_bytes: float
    later_depth: int = 0


_lib = None


def lib():
    """Load libbmpc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"bmpc HIP library not built: {LIB_PATH} "
                           "(run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "bmpc_analyze": [P(_Dims), i32, vp, P(vp)],
        "bmpc_analyze_ex": [P(_Dims), i32, vp, P(_Options), P(vp)],
        "bmpc_set_stream": [vp, vp],
        "bmpc_set_refine_stop": [vp, i32],
        "bmpc_analyze_ragged": [i32, P(_Dims), i32, vp, P(_Options), P(vp)],
        "bmpc_ragged_layout": [vp, i32, P(_Dims), P(i64)],
        "bmpc_autotune": [P(_Dims), i32, i32, vp, i32, P(_Options), P(dbl), P(dbl), i32,
                          P(i32)],
        "bmpc_query_structure": [vp, P(i32), P(i32), i64, P(i64)],
        "bmpc_factor": [vp, vp, vp, vp, vp],
        "bmpc_solve": [vp, vp, vp],
        "bmpc_refine": [vp, vp, vp, vp, vp, vp, vp, dbl, i32],
        "bmpc_factor_solve": [vp, vp, vp, vp, vp, vp, vp],
        "bmpc_factor_refine": [vp, vp, vp, vp, vp, vp, vp, dbl, i32],
        "bmpc_get_info": [vp, P(i64)],
        "bmpc_get_stats": [vp, P(i32), P(dbl)],
        "bmpc_query_perm": [vp, P(i32)],
        "bmpc_query_cost": [vp, P(_Cost)],
        "bmpc_query_kernel_cost": [vp, i32, P(dbl), P(dbl), P(i32)],
        "bmpc_export_tail_factor": [vp, i32, P(dbl), P(dbl)],
        "bmpc_export_root_factor": [vp, P(dbl)],
        "bmpc_set_profiling": [vp, i32],
        "bmpc_get_kernel_times": [vp, i32, P(i64), P(dbl)],
        "bmpc_reset_kernel_times": [vp],
        "bmpc_destroy": [vp],
        "bmpc_ordering": [i32, P(i32)],
        "bmpc_structure": [i32, P(i32), P(i32), i64, P(i64)],
        "bmpc_cost_model": [P(_Dims), i32, P(_Options), P(_Cost)],
        "bmpc_grad_blocks": [vp, vp, vp, vp, vp, vp, vp],
        "bmpc_assemble_qp": [P(_QpDims), vp, vp, vp, vp, dbl, dbl, vp, vp, vp, vp, vp, vp],
        "bmpc_assemble_qp_noalloc": [P(_QpDims), vp, vp, vp, vp, dbl, dbl, vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.bmpc_status_string.argtypes = [ctypes.c_int]
    L.bmpc_status_string.restype = ctypes.c_char_p
    L.bmpc_kernel_class_name.argtypes = [i32]
    L.bmpc_kernel_class_name.restype = ctypes.c_char_p
    L.bmpc_kernel_class_count.argtypes = []
    L.bmpc_kernel_class_count.restype = i32
    _lib = L
    return L


def status_string(st: int) -> str:
    return lib().bmpc_status_string(int(st)).decode()


def _check(st: int, what: str):
    if st != OK:
        raise BmpcError(st, what)


def _prec(precision) -> int:
    if precision in (FP64, "fp64", "f64"):
        return FP64
    if precision in (FP32_REFINE, "fp32", "fp32_refine", "f32"):
        return FP32_REFINE
    raise ValueError(f"unknown precision {precision!r}")


def _cost(c: _Cost) -> Cost:
    return Cost(c.factor_flops, c.solve_flops, c.factor_bytes, c.solve_bytes,
                c.residual_bytes, c.levels, c.passes, c.window_depth, c.workspace_bytes,
                c.later_depth)


# ---- host-only helpers -------------------------------------------------------------

def ordering(N: int) -> list:
    buf = (ctypes.c_int32 * N)()
    _check(lib().bmpc_ordering(N, buf), "bmpc_ordering")
    return list(buf)


def structure(N: int) -> list:
    cnt = ctypes.c_int64(0)
    _check(lib().bmpc_structure(N, None, None, 0, ctypes.byref(cnt)), "bmpc_structure")
    k = cnt.value
    rows, cols = (ctypes.c_int32 * k)(), (ctypes.c_int32 * k)()
    _check(lib().bmpc_structure(N, rows, cols, k, ctypes.byref(cnt)), "bmpc_structure")
    return list(zip(rows, cols))


def cost_model(S: int, N: int, n: int, nrhs: int = 1, precision="fp64",
               window_depth: int = 0, num_systems: int = 1, flags: int = 0,
               later_depth: int = 0) -> Cost:
    d = _Dims(S, N, n, nrhs)
    o = _Options(window_depth, num_systems, flags, later_depth)
    c = _Cost()
    _check(lib().bmpc_cost_model(ctypes.byref(d), _prec(precision), ctypes.byref(o),
                                 ctypes.byref(c)), "bmpc_cost_model")
    return _cost(c)


def autotune(S: int, N: int, n: int, nrhs: int = 1, precision="fp32", reps: int = 5,
             stream=None, num_systems: int = 1):
    """Fastest launch configuration for the shape (bmpc_autotune), timed on one system
    or on a batch of num_systems of them: returns (window_depth, flags, best_ms,
    candidate_ms)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    d = _Dims(S, N, n, nrhs)
    best = _Options()
    best_ms = ctypes.c_double(0.0)
    times = (ctypes.c_double * 64)()
    cnt = ctypes.c_int32(0)
    _check(lib().bmpc_autotune(ctypes.byref(d), int(num_systems), _prec(precision),
                               ctypes.c_void_p(stream.cuda_stream), int(reps),
                               ctypes.byref(best), ctypes.byref(best_ms), times, 64,
                               ctypes.byref(cnt)), "bmpc_autotune")
    return best.window_depth, best.flags, best_ms.value, list(times[:min(cnt.value, 64)])


def kernel_class_names() -> list:
    L = lib()
    return [L.bmpc_kernel_class_name(i).decode() for i in range(L.bmpc_kernel_class_count())]


# ---- device plan -----------------------------------------------------------------

def _ptr(t, what, dtype=None, numel=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def assemble_qp(Q, A, G, w, tau: float, delta: float, stream=None, out=None,
                noalloc: bool = False):
    """Reduced IPM system K = P + tau I + A^T A / delta + G^T (W + delta I)^{-1} G of a
    branch-MPC QP given per link (see bmpc_assemble_qp): returns D, E, C, R (device
    tensors, FP64) ready for Plan.factor.  out = (D, E, C, R) writes into given tensors;
    noalloc uses bmpc_assemble_qp_noalloc (the library's static scratch, no work array)."""
    import torch
    S, L, n2, _ = Q.shape
    N, n = L - 1, n2 // 2
    me, mi = A.shape[2], G.shape[2]
    f64 = torch.float64
    dev = Q.device
    d = _QpDims(S, N, n, me, mi)
    if out is None:
        D = torch.empty((S, N, n, n), dtype=f64, device=dev)
        E = torch.empty((S, max(N - 1, 0), n, n), dtype=f64, device=dev)
        C = torch.empty((S, n, n), dtype=f64, device=dev)
        R = torch.empty((n, n), dtype=f64, device=dev)
    else:
        D, E, C, R = out
    if stream is None:
        stream = torch.cuda.current_stream()
    args = [_ptr(Q, "Q", f64, S * L * n2 * n2), _ptr(A, "A", f64, S * L * me * n2) if me else None,
            _ptr(G, "G", f64, S * L * mi * n2) if mi else None,
            _ptr(w, "w", f64, S * L * mi) if mi else None]
    outs = [_ptr(D, "D", f64, S * N * n * n),
            _ptr(E, "E", f64, S * (N - 1) * n * n) if N > 1 else None,
            _ptr(C, "C", f64, S * n * n), _ptr(R, "R", f64, n * n)]
    st = ctypes.c_void_p(stream.cuda_stream)
    if noalloc:
        _check(lib().bmpc_assemble_qp_noalloc(ctypes.byref(d), *args, float(tau), float(delta),
                                              *outs, st), "bmpc_assemble_qp_noalloc")
    else:
        work = torch.empty((S, n, n), dtype=f64, device=dev)
        _check(lib().bmpc_assemble_qp(ctypes.byref(d), *args, float(tau), float(delta), *outs,
                                      ctypes.c_void_p(work.data_ptr()), st), "bmpc_assemble_qp")
    return D, E, C, R


class Plan:
    """A bmpc plan: analysis + persistent device workspaces for one (S, N, n, nrhs),
    or for a batch of num_systems independent systems of that shape (arrays stacked
    along the leading dimension, see include/bmpc.h).  RaggedPlan holds systems of
    different shapes."""

    def __init__(self, S: int, N: int, n: int, nrhs: int = 1, precision="fp64",
                 window_depth: int = 0, stream=None, num_systems: int = 1, flags: int = 0,
                 later_depth: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("bmpc needs a HIP device (torch.cuda.is_available() is False)")
        self.S, self.N, self.n, self.nrhs = int(S), int(N), int(n), int(nrhs)
        self.B = int(num_systems)
        self.precision = _prec(precision)
        self._h = ctypes.c_void_p()
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        d = _Dims(self.S, self.N, self.n, self.nrhs)
        o = _Options(int(window_depth), self.B, int(flags), int(later_depth))
        _check(lib().bmpc_analyze_ex(ctypes.byref(d), self.precision,
                                     ctypes.c_void_p(stream.cuda_stream), ctypes.byref(o),
                                     ctypes.byref(self._h)), "bmpc_analyze")

    @property
    def length(self) -> int:
        return (self.S * self.N + 1) * self.n

    def close(self):
        if self._h and self._h.value:
            lib().bmpc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._stream = stream
        _check(lib().bmpc_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)),
               "bmpc_set_stream")

    def set_refine_stop(self, stop):
        """Stop test of later refine / factor_refine calls: "correction"
        (|d| <= tol |x|, the default) or "backward_error"
        (|b - K x| <= tol (|K| |x| + |b|), infinity norms)."""
        code = {"correction": STOP_CORRECTION, "backward_error": STOP_BACKWARD_ERROR}.get(stop, stop)
        _check(lib().bmpc_set_refine_stop(self._h, int(code)), "bmpc_set_refine_stop")

    def _blocks(self, D, E, C, R):
        import torch
        S, N, n, B = self.S, self.N, self.n, self.B
        f64 = torch.float64
        return (_ptr(D, "D", f64, B * S * N * n * n),
                _ptr(E, "E", f64, B * S * (N - 1) * n * n) if N > 1 else None,
                _ptr(C, "C", f64, B * S * n * n), _ptr(R, "R", f64, B * n * n))

    def factor(self, D, E, C, R):
        _check(lib().bmpc_factor(self._h, *self._blocks(D, E, C, R)), "bmpc_factor")

    def _rhs(self, b, x):
        import torch
        if x is None:
            x = torch.empty_like(b)
        return (_ptr(b, "b", torch.float64, self.B * self.nrhs * self.length),
                _ptr(x, "x", torch.float64, self.B * self.nrhs * self.length), x)

    def solve(self, b, x=None):
        pb, px, x = self._rhs(b, x)
        _check(lib().bmpc_solve(self._h, pb, px), "bmpc_solve")
        return x

    def refine(self, D, E, C, R, b, x=None, tol: float = 1e-12, max_iters: int = 10):
        blocks = self._blocks(D, E, C, R)
        pb, px, x = self._rhs(b, x)
        _check(lib().bmpc_refine(self._h, *blocks, pb, px, float(tol), int(max_iters)),
               "bmpc_refine")
        return x

    def factor_solve(self, D, E, C, R, b, x=None):
        """factor + solve with the forward substitution inside the factorization."""
        blocks = self._blocks(D, E, C, R)
        pb, px, x = self._rhs(b, x)
        _check(lib().bmpc_factor_solve(self._h, *blocks, pb, px), "bmpc_factor_solve")
        return x

    def factor_refine(self, D, E, C, R, b, x=None, tol: float = 1e-12, max_iters: int = 10):
        """factor + refine, the first solve's forward part inside the factorization."""
        blocks = self._blocks(D, E, C, R)
        pb, px, x = self._rhs(b, x)
        _check(lib().bmpc_factor_refine(self._h, *blocks, pb, px, float(tol), int(max_iters)),
               "bmpc_factor_refine")
        return x

    def grad_blocks(self, x, lam):
        """(dD, dE, dC, dR) of a loss through x = K^{-1} b, from the solution x and the
        adjoint lam = K^{-1} dloss/dx (see bmpc_grad_blocks)."""
        import torch
        S, N, n, B = self.S, self.N, self.n, self.B
        f64 = torch.float64
        px = _ptr(x, "x", f64, B * self.nrhs * self.length)
        pl = _ptr(lam, "lam", f64, B * self.nrhs * self.length)
        dev = x.device
        dD = torch.empty((B * S, N, n, n), dtype=f64, device=dev)
        dE = torch.empty((B * S, max(N - 1, 0), n, n), dtype=f64, device=dev)
        dC = torch.empty((B * S, n, n), dtype=f64, device=dev)
        dR = torch.empty((B, n, n) if B > 1 else (n, n), dtype=f64, device=dev)
        _check(lib().bmpc_grad_blocks(self._h, px, pl, ctypes.c_void_p(dD.data_ptr()),
                                      ctypes.c_void_p(dE.data_ptr()) if N > 1 else None,
                                      ctypes.c_void_p(dC.data_ptr()),
                                      ctypes.c_void_p(dR.data_ptr())), "bmpc_grad_blocks")
        return dD, dE, dC, dR

    def info(self) -> int:
        v = ctypes.c_int64(0)
        st = lib().bmpc_get_info(self._h, ctypes.byref(v))
        if st not in (OK, ERR_NOT_SPD):
            _check(st, "bmpc_get_info")
        return int(v.value)

    def stats(self):
        it, rel = ctypes.c_int32(0), ctypes.c_double(0.0)
        st = lib().bmpc_get_stats(self._h, ctypes.byref(it), ctypes.byref(rel))
        if st not in (OK, ERR_NOT_CONVERGED):
            _check(st, "bmpc_get_stats")
        return int(it.value), float(rel.value), st == OK

    def perm(self) -> list:
        buf = (ctypes.c_int32 * self.N)()
        _check(lib().bmpc_query_perm(self._h, buf), "bmpc_query_perm")
        return list(buf)

    def structure(self) -> list:
        """(row, col) permuted block pairs of one tail's factor plus the root row."""
        cnt = ctypes.c_int64(0)
        _check(lib().bmpc_query_structure(self._h, None, None, 0, ctypes.byref(cnt)),
               "bmpc_query_structure")
        k = cnt.value
        rows, cols = (ctypes.c_int32 * k)(), (ctypes.c_int32 * k)()
        _check(lib().bmpc_query_structure(self._h, rows, cols, k, ctypes.byref(cnt)),
               "bmpc_query_structure")
        return list(zip(rows, cols))

    def cost(self) -> Cost:
        c = _Cost()
        _check(lib().bmpc_query_cost(self._h, ctypes.byref(c)), "bmpc_query_cost")
        return _cost(c)

    def kernel_cost(self, cls: int):
        """(bytes, flops, launches) of kernel class cls per call of its entry point."""
        b, f, k = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_int32(0)
        _check(lib().bmpc_query_kernel_cost(self._h, int(cls), ctypes.byref(b),
                                            ctypes.byref(f), ctypes.byref(k)),
               "bmpc_query_kernel_cost")
        return float(b.value), float(f.value), int(k.value)

    def export_tail_factor(self, s: int):
        import numpy as np
        Nn = self.N * self.n
        L = np.zeros((Nn, Nn))
        F = np.zeros((self.n, self.n))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().bmpc_export_tail_factor(self._h, int(s), L.ctypes.data_as(dp),
                                             F.ctypes.data_as(dp)), "bmpc_export_tail_factor")
        return L, F

    def export_root_factor(self):
        import numpy as np
        LR = np.zeros((self.B, self.n, self.n))
        _check(lib().bmpc_export_root_factor(
            self._h, LR.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
            "bmpc_export_root_factor")
        return LR[0] if self.B == 1 else LR

    def set_profiling(self, enable: bool):
        _check(lib().bmpc_set_profiling(self._h, int(bool(enable))), "bmpc_set_profiling")

    def reset_kernel_times(self):
        _check(lib().bmpc_reset_kernel_times(self._h), "bmpc_reset_kernel_times")

    def kernel_times(self) -> dict:
        L = lib()
        k = L.bmpc_kernel_class_count()
        launches = (ctypes.c_int64 * k)()
        ms = (ctypes.c_double * k)()
        _check(L.bmpc_get_kernel_times(self._h, k, launches, ms), "bmpc_get_kernel_times")
        names = kernel_class_names()
        return {names[i]: (int(launches[i]), float(ms[i])) for i in range(k)}


class RaggedPlan(Plan):
    """Independent systems of different shapes (S_i, N_i, n_i) with one nrhs, factored
    and solved together (bmpc_analyze_ragged).  The arrays are the systems' own arrays
    concatenated in system order (flat FP64 device tensors); layout(i) gives each
    system's element offsets, and pack() / unpack() move per-system tensors in and out.
    factor / solve / refine / factor_solve / factor_refine / info / stats take and
    return the concatenated arrays."""

    def __init__(self, shapes, precision="fp32", window_depth: int = 0, stream=None,
                 flags: int = 0, options=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("bmpc needs a HIP device (torch.cuda.is_available() is False)")
        shapes = [tuple(int(v) for v in sh) for sh in shapes]
        self.shapes = shapes
        self.B = len(shapes)
        self.nrhs = shapes[0][3]
        self.precision = _prec(precision)
        self._h = ctypes.c_void_p()
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        dims = (_Dims * self.B)(*[_Dims(*sh) for sh in shapes])
        if options is None:
            options = [(window_depth, flags)] * self.B
        # (window_depth, flags) or (window_depth, flags, later_depth) per system
        opts = (_Options * self.B)(*[_Options(int(o[0]), 0, int(o[1]),
                                              int(o[2]) if len(o) > 2 else 0)
                                     for o in options])
        _check(lib().bmpc_analyze_ragged(self.B, dims, self.precision,
                                         ctypes.c_void_p(stream.cuda_stream), opts,
                                         ctypes.byref(self._h)), "bmpc_analyze_ragged")
        self.offsets = [self.layout(i)[1] for i in range(self.B)] + [self._totals()]

    def layout(self, i):
        d = _Dims()
        off = (ctypes.c_int64 * 5)()
        _check(lib().bmpc_ragged_layout(self._h, int(i), ctypes.byref(d), off),
               "bmpc_ragged_layout")
        return (d.S, d.N, d.n, d.nrhs), list(off)

    def _totals(self):
        S, N, n, q = self.shapes[-1]
        last = self.layout(self.B - 1)[1]
        return [last[0] + S * N * n * n, last[1] + S * (N - 1) * n * n, last[2] + S * n * n,
                last[3] + n * n, last[4] + q * (S * N + 1) * n]

    @property
    def sizes(self):
        """Element counts of the concatenated D, E, C, R and vectors."""
        return self.offsets[-1]

    def pack(self, which: int, parts, out=None):
        """Concatenate per-system tensors (which: 0 D, 1 E, 2 C, 3 R, 4 vectors)."""
        import torch
        dev = next(t for t in parts if t is not None).device
        if out is None:
            out = torch.empty(max(self.sizes[which], 1), dtype=torch.float64, device=dev)
        for i, t in enumerate(parts):
            a, b = self.offsets[i][which], self.offsets[i + 1][which]
            if b > a:
                out[a:b] = t.reshape(-1)
        return out

    def unpack(self, which: int, flat, i: int):
        a, b = self.offsets[i][which], self.offsets[i + 1][which]
        return flat[a:b]

    def _blocks(self, D, E, C, R):
        import torch
        f64 = torch.float64
        s = self.sizes
        return (_ptr(D, "D", f64, s[0]), _ptr(E, "E", f64, max(s[1], 1)),
                _ptr(C, "C", f64, s[2]), _ptr(R, "R", f64, s[3]))

    def _rhs(self, b, x):
        import torch
        if x is None:
            x = torch.empty_like(b)
        return (_ptr(b, "b", torch.float64, self.sizes[4]),
                _ptr(x, "x", torch.float64, self.sizes[4]), x)

    def export_tail_factor(self, chain: int):
        """Stored factor of chain `chain` of the concatenated systems (see
        Plan.export_tail_factor), sized for its system."""
        import numpy as np
        s = int(chain)
        for S, N, n, _ in self.shapes:
            if s < S:
                break
            s -= S
        L = np.zeros((N * n, N * n))
        F = np.zeros((n, n))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().bmpc_export_tail_factor(self._h, int(chain), L.ctypes.data_as(dp),
                                             F.ctypes.data_as(dp)), "bmpc_export_tail_factor")
        return L, F
