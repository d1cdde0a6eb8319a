"""Python binding of libchfsi (residual-based Chebyshev filtered subspace iteration on MI355X).

This module only marshals arguments into the C ABI declared in
``include/chfsi.h``; every numerical step runs in the library's HIP kernels.
PyTorch is used for device memory and streams only: tensors are passed by
``data_ptr()`` and streams by their HIP handle.

There is no CPU fallback: if ``libchfsi.so`` is not built (``python -m
paper_2503_22652_amd.build``) every entry point raises ``RuntimeError``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchfsi.so")

# status codes (chfsi_status)
OK, ERR_ARG, ERR_NOMEM, ERR_DEVICE, ERR_NOT_SPD, ERR_NOCONV, ERR_NUMERIC, ERR_BUSY, \
    ERR_CANCELLED, ERR_TIMEOUT = range(10)
STATUS_NAMES = ["OK", "ERR_ARG", "ERR_NOMEM", "ERR_DEVICE", "ERR_NOT_SPD", "ERR_NOCONV",
                "ERR_NUMERIC", "ERR_BUSY", "ERR_CANCELLED", "ERR_TIMEOUT"]
OP_IDENTITY, OP_DENSE, OP_STENCIL27, OP_DENSE_HERMITIAN, OP_STENCIL27_BLOCH, OP_CSR = range(6)
PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2
METHOD_CHFSI, METHOD_RCHFSI = 0, 1
MAX_HISTORY = 512


class chfsi_operator(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int64), ("dense", C.c_void_p), ("ld", C.c_int64),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("coef", C.c_double * 27), ("coef_mass", C.c_double * 27),
                ("field", C.c_void_p), ("field_mode", C.c_int32), ("bloch", C.c_double * 3),
                ("rowptr", C.c_void_p), ("colind", C.c_void_p), ("val", C.c_void_p),
                ("nnz", C.c_int64)]


class chfsi_params(C.Structure):
    _fields_ = [("n_wanted", C.c_int64), ("block", C.c_int64), ("degree", C.c_int32),
                ("max_iter", C.c_int32), ("tol", C.c_double), ("method", C.c_int32),
                ("filter_prec", C.c_int32), ("lambda_min", C.c_double),
                ("lambda_max", C.c_double), ("lambda_T", C.c_double), ("seed", C.c_uint64),
                ("init_random", C.c_int32), ("profile", C.c_int32),
                ("memory_mode", C.c_int32), ("binv_exact", C.c_int32),
                ("lanczos_steps", C.c_int32), ("stall_iters", C.c_int32),
                ("keep_best", C.c_int32), ("escalate", C.c_int32),
                ("amp_cap", C.c_double)]


class chfsi_report(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32),
                ("max_residual", C.c_double), ("time_total_ms", C.c_double),
                ("time_filter_ms", C.c_double), ("time_rr_ms", C.c_double),
                ("filter_flops", C.c_double), ("jacobi_sweeps", C.c_int32),
                ("kernel_launches", C.c_int32), ("kernel_ms", C.c_double),
                ("flags", C.c_int32), ("history", C.c_double * MAX_HISTORY),
                ("svqb_events", C.c_int32), ("svqb_dropped", C.c_int32),
                ("lambda_max_used", C.c_double), ("time_bounds_ms", C.c_double),
                ("best_iteration", C.c_int32), ("best_residual", C.c_double),
                ("escalation_iteration", C.c_int32),
                ("max_amplification", C.c_double), ("min_degree_used", C.c_int32)]


class chfsi_server_config(C.Structure):
    _fields_ = [("slots", C.c_int32), ("queue_capacity", C.c_int32),
                ("memory_budget", C.c_size_t)]


class chfsi_server_stats_t(C.Structure):
    _fields_ = [("budget", C.c_size_t), ("used", C.c_size_t), ("sequence_bytes", C.c_size_t),
                ("device_pool_chunks", C.c_int32), ("host_pool_chunks", C.c_int32)]


class chfsi_request(C.Structure):
    _fields_ = [("A", chfsi_operator), ("B", chfsi_operator), ("d_inv", C.c_void_p),
                ("params", chfsi_params), ("seq_id", C.c_int64), ("X0", C.c_void_p),
                ("X_out", C.c_void_p)]


class chfsi_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("max_residual", C.c_double),
                ("submit_ms", C.c_double), ("start_ms", C.c_double), ("finish_ms", C.c_double),
                ("n", C.c_int64), ("block", C.c_int64), ("evals", C.POINTER(C.c_double)),
                ("resnorms", C.POINTER(C.c_double))]


# exported symbols and their signatures (mirrors include/chfsi.h)
_SIGNATURES = {
    "chfsi_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(chfsi_operator),
                               C.POINTER(chfsi_operator), C.c_void_p, C.POINTER(chfsi_params),
                               C.c_void_p]),
    "chfsi_workspace_bytes": (C.c_size_t, [C.POINTER(chfsi_operator), C.POINTER(chfsi_operator),
                                           C.POINTER(chfsi_params)]),
    "chfsi_filter": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_double),
                               C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_double,
                               C.c_double, C.c_double, C.c_int32]),
    "chfsi_rayleigh_ritz": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                      C.c_void_p, C.c_int64, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]),
    "chfsi_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_double),
                              C.POINTER(C.c_double), C.POINTER(chfsi_report)]),
    "chfsi_destroy": (None, [C.c_void_p]),
    "chfsi_estimate_bounds": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]),
    "chfsi_filter_static_bytes": (C.c_size_t, [C.c_int64, C.c_int64, C.c_int32]),
    "chfsi_filter_static": (C.c_int, [C.POINTER(chfsi_operator), C.c_void_p, C.c_int64,
                                      C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                      C.c_void_p, C.c_int64, C.c_double, C.c_double, C.c_double,
                                      C.c_int32, C.c_void_p]),
    "chfsi_filter_kernel_time": (C.c_int, [C.c_void_p, C.POINTER(C.c_double),
                                           C.POINTER(C.c_int32)]),
    "chfsi_last_error": (C.c_char_p, []),
    "chfsi_version": (C.c_char_p, []),
    "chfsi_server_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(chfsi_server_config)]),
    "chfsi_submit": (C.c_int, [C.c_void_p, C.POINTER(chfsi_request), C.POINTER(C.c_uint64)]),
    "chfsi_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(chfsi_result)]),
    "chfsi_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "chfsi_result_free": (None, [C.POINTER(chfsi_result)]),
    "chfsi_server_destroy": (None, [C.c_void_p]),
    "chfsi_server_stats": (C.c_int, [C.c_void_p, C.POINTER(chfsi_server_stats_t)]),
}

_lib = None


def lib():
    """Load libchfsi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2503_22652_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class ChfsiError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().chfsi_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES[status] if 0 <= status < 10 else status}: {msg}")
        self.status = status


def _check(status: int, where: str, allow=(OK,)):
    if status not in allow:
        raise ChfsiError(status, where)
    return status


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(getattr(stream, "cuda_stream", stream))


def dense_operator(A) -> chfsi_operator:
    """Operator struct for a symmetric float64 CUDA tensor (column-major = its transpose-free view)."""
    op = chfsi_operator()
    op.kind = OP_DENSE
    op.n = A.shape[0]
    op.dense = _ptr(A)
    op.ld = A.stride(1) if A.stride(0) == 1 else A.stride(0)
    return op


def hermitian_operator(A) -> chfsi_operator:
    """Operator struct for a complex Hermitian complex128 CUDA tensor (column-major:
    a transposed view of a contiguous buffer); ld in complex elements."""
    op = chfsi_operator()
    op.kind = OP_DENSE_HERMITIAN
    op.n = A.shape[0]
    op.dense = _ptr(A)
    op.ld = A.stride(1) if A.stride(0) == 1 else A.stride(0)
    return op


def to_colmajor_complex(a, device="cuda"):
    """Copy a host complex array to a column-major complex128 device tensor."""
    import numpy as np
    import torch
    arr = np.asarray(a, dtype=np.complex128)
    return torch.from_numpy(np.ascontiguousarray(arr.T)).to(device).t()


def colmajor_empty_complex(n: int, b: int, device="cuda"):
    """Uninitialised column-major complex128 n x b tensor."""
    import torch
    return torch.empty((b, n), dtype=torch.complex128, device=device).t()


def csr_operator(n: int, rowptr, colind, val) -> chfsi_operator:
    """Operator struct for a symmetric CSR matrix given as CUDA tensors
    (rowptr int64 [n + 1], colind int32 [nnz], val float64 [nnz])."""
    op = chfsi_operator()
    op.kind = OP_CSR
    op.n = n
    op.rowptr, op.colind, op.val = _ptr(rowptr), _ptr(colind), _ptr(val)
    op.nnz = int(val.numel())
    return op


def identity_operator(n: int) -> chfsi_operator:
    op = chfsi_operator()
    op.kind = OP_IDENTITY
    op.n = n
    return op


def stencil_operator(shape, coef, coef_mass=None, field=None, field_mode: int = 0,
                     bloch=None) -> chfsi_operator:
    """Periodic 27-point operator; shape = (nz, ny, nx); coef indexed [dz+1][dy+1][dx+1].
    With bloch = (kx, ky, kz) the operator acts on complex vectors with the
    Bloch phase exp(i k.o) on every offset o (kind OP_STENCIL27_BLOCH)."""
    nz, ny, nx = shape
    op = chfsi_operator()
    op.kind = OP_STENCIL27 if bloch is None else OP_STENCIL27_BLOCH
    if bloch is not None:
        for i in range(3):
            op.bloch[i] = float(bloch[i])
    op.n = nx * ny * nz
    op.nx, op.ny, op.nz = nx, ny, nz
    flat = [float(v) for v in _flat27(coef)]
    for i in range(27):
        op.coef[i] = flat[i]
    if coef_mass is not None:
        fm = [float(v) for v in _flat27(coef_mass)]
        for i in range(27):
            op.coef_mass[i] = fm[i]
    op.field = _ptr(field)
    op.field_mode = field_mode
    return op


def _flat27(c):
    try:
        import numpy as np
        return np.asarray(c, dtype=float).reshape(27).tolist()
    except Exception:
        return list(c)


def make_params(n_wanted: int, block: int, degree: int, max_iter: int = 100, tol: float = 1e-10,
                method: int = METHOD_RCHFSI, filter_prec: int = PREC_FP64,
                lambda_min: float = math.nan, lambda_max: float = math.nan,
                lambda_T: float = math.nan, seed: int = 0, init_random: int = 0,
                profile: int = 0, memory_mode: int = 0, binv_exact: int = 0,
                lanczos_steps: int = 0, stall_iters: int = 0,
                keep_best: int = 0, escalate: int = 0, amp_cap: float = 0.0) -> chfsi_params:
    p = chfsi_params()
    p.n_wanted, p.block, p.degree, p.max_iter, p.tol = n_wanted, block, degree, max_iter, tol
    p.method, p.filter_prec = method, filter_prec
    p.lambda_min, p.lambda_max, p.lambda_T = lambda_min, lambda_max, lambda_T
    p.seed, p.init_random, p.profile = seed, init_random, profile
    p.memory_mode = memory_mode
    p.binv_exact = binv_exact
    p.lanczos_steps = lanczos_steps
    p.stall_iters = stall_iters
    p.keep_best = keep_best
    p.escalate = escalate
    p.amp_cap = amp_cap
    return p


def chfsi_version() -> str:
    return lib().chfsi_version().decode()


def chfsi_last_error() -> str:
    return lib().chfsi_last_error().decode(errors="replace")


def chfsi_workspace_bytes(A: chfsi_operator, B: Optional[chfsi_operator], params: chfsi_params) -> int:
    return int(lib().chfsi_workspace_bytes(C.byref(A), C.byref(B) if B is not None else None,
                                           C.byref(params)))


class Context:
    """Owns a chfsi_ctx*.  Keeps references to the borrowed device tensors."""

    def __init__(self, handle: int, keep):
        self.handle = handle
        self._keep = keep

    def close(self):
        if self.handle:
            lib().chfsi_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chfsi_create(A: chfsi_operator, B: Optional[chfsi_operator], d_inv, params: chfsi_params,
                 stream=None, keep=()) -> Context:
    h = C.c_void_p()
    st = lib().chfsi_create(C.byref(h), C.byref(A), C.byref(B) if B is not None else None,
                            _ptr(d_inv), C.byref(params), _stream_handle(stream))
    _check(st, "chfsi_create")
    return Context(h.value, (A, B, d_inv, params) + tuple(keep))


def chfsi_filter(ctx: Context, X, ritz, resid, Yp, lmin: float, lmax: float, lT: float,
                 degree: int = 0) -> None:
    """Asynchronous filter pass; X/resid/Yp are float64 CUDA tensors (n x b, column-major)."""
    n = X.shape[0]
    ritz_arr = None
    if ritz is not None:
        vals = [float(v) for v in ritz]
        ritz_arr = (C.c_double * len(vals))(*vals)
    st = lib().chfsi_filter(ctx.handle, _ptr(X), _ld(X), ritz_arr, _ptr(resid),
                            _ld(resid) if resid is not None else n, _ptr(Yp), _ld(Yp),
                            lmin, lmax, lT, degree)
    _check(st, "chfsi_filter")


STATIC_SCRATCH_BYTES = 128 << 20


def chfsi_filter_static_bytes(n: int, b: int, degree: int) -> int:
    return int(lib().chfsi_filter_static_bytes(n, b, degree))


def chfsi_filter_static(A: chfsi_operator, d_inv, X, ritz_d, resid, Yp, lmin: float, lmax: float,
                        lT: float, degree: int, stream=None) -> None:
    """FP64 residual filter that allocates nothing (a static device scratch array).
    X/resid/Yp: float64 CUDA tensors (n x b, column-major); ritz_d: float64 CUDA
    tensor of the b Ritz values.  X = None binds the scratch array only (b = 0)."""
    b = 0 if X is None else X.shape[1]
    n = A.n
    st = lib().chfsi_filter_static(C.byref(A), _ptr(d_inv), b, _ptr(X), _ld(X) if X is not None else n,
                                   _ptr(ritz_d), _ptr(resid), _ld(resid) if resid is not None else n,
                                   _ptr(Yp), _ld(Yp) if Yp is not None else n, lmin, lmax, lT,
                                   degree, _stream_handle(stream))
    _check(st, "chfsi_filter_static")


def chfsi_estimate_bounds(ctx: Context, v0=None, steps: int = 0):
    """Lanczos estimates (lower, upper, theta_min, theta_max) of the spectrum of B^{-1} A."""
    lo, hi = C.c_double(), C.c_double()
    th = (C.c_double * 2)()
    _check(lib().chfsi_estimate_bounds(ctx.handle, _ptr(v0), steps, C.byref(lo), C.byref(hi), th),
           "chfsi_estimate_bounds")
    return lo.value, hi.value, th[0], th[1]


def chfsi_rayleigh_ritz(ctx: Context, Y, X, R):
    b = Y.shape[1]
    ritz = (C.c_double * b)()
    norms = (C.c_double * b)()
    st = lib().chfsi_rayleigh_ritz(ctx.handle, _ptr(Y), _ld(Y), _ptr(X), _ld(X), _ptr(R), _ld(R),
                                   ritz, norms)
    _check(st, "chfsi_rayleigh_ritz")
    return list(ritz), list(norms)


def chfsi_filter_kernel_time(ctx: Context):
    """(total_ms, launches) of the filter's operator-product kernels since the last call."""
    ms = C.c_double()
    n = C.c_int32()
    _check(lib().chfsi_filter_kernel_time(ctx.handle, C.byref(ms), C.byref(n)),
           "chfsi_filter_kernel_time")
    return ms.value, n.value


def chfsi_solve(ctx: Context, X):
    """Synchronous solve; returns (status, evals, resnorms, report dict)."""
    b = X.shape[1]
    ev = (C.c_double * b)()
    rn = (C.c_double * b)()
    rep = chfsi_report()
    st = lib().chfsi_solve(ctx.handle, _ptr(X), _ld(X), ev, rn, C.byref(rep))
    _check(st, "chfsi_solve", allow=(OK, ERR_NOCONV))
    return st, list(ev), list(rn), report_dict(rep)


def report_dict(rep: chfsi_report) -> dict:
    it = rep.iterations
    return {"iterations": it, "converged": bool(rep.converged), "max_residual": rep.max_residual,
            "time_total_ms": rep.time_total_ms, "time_filter_ms": rep.time_filter_ms,
            "time_rr_ms": rep.time_rr_ms, "filter_flops": rep.filter_flops,
            "jacobi_sweeps": rep.jacobi_sweeps, "flags": rep.flags,
            "svqb_events": rep.svqb_events, "svqb_dropped": rep.svqb_dropped,
            "lambda_max_used": rep.lambda_max_used, "time_bounds_ms": rep.time_bounds_ms,
            "best_iteration": rep.best_iteration, "best_residual": rep.best_residual,
            "escalation_iteration": rep.escalation_iteration,
            "max_amplification": rep.max_amplification, "min_degree_used": rep.min_degree_used,
            "kernel_launches": rep.kernel_launches, "kernel_ms": rep.kernel_ms,
            "history": [rep.history[i] for i in range(min(it + 1, MAX_HISTORY))]}


def _ld(t) -> int:
    """Leading dimension of a column-major 2D tensor view (stride of dim 1).

    A single column is addressed without its leading dimension, and the stride
    that torch (or numpy, whose strides of size-1 dimensions are arbitrary)
    reports for it can be anything, so its leading dimension is its length."""
    if t.dim() == 1:
        return t.shape[0]
    if t.stride(0) != 1 and t.shape[0] > 1:
        raise ValueError("blocks must be column-major (stride(0) == 1); use X.t().contiguous().t()")
    return t.shape[0] if t.shape[1] == 1 else t.stride(1)


def colmajor_empty(n: int, b: int, dtype=None, device="cuda"):
    """Uninitialised column-major n x b tensor (a transposed view of a b x n buffer)."""
    import torch
    return torch.empty((b, n), dtype=dtype or torch.float64, device=device).t()


def to_colmajor(a, device="cuda"):
    """Copy a host array / tensor to a column-major float64 device tensor."""
    import numpy as np
    import torch
    arr = np.asarray(a, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(arr.T)).to(device).t()


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
class Server:
    def __init__(self, slots: int = 4, queue_capacity: int = 1024, memory_budget: int = 0):
        cfg = chfsi_server_config(slots, queue_capacity, memory_budget)
        h = C.c_void_p()
        _check(lib().chfsi_server_create(C.byref(h), C.byref(cfg)), "chfsi_server_create")
        self.handle = h.value
        self._keep = {}

    def submit(self, req: chfsi_request, keep=()) -> int:
        t = C.c_uint64()
        _check(lib().chfsi_submit(self.handle, C.byref(req), C.byref(t)), "chfsi_submit")
        self._keep[t.value] = (req,) + tuple(keep)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> dict:
        res = chfsi_result()
        st = lib().chfsi_wait(self.handle, ticket, timeout_ms, C.byref(res))
        if st == ERR_TIMEOUT:
            raise TimeoutError(f"ticket {ticket} still running")
        out = {"status": res.status, "iterations": res.iterations,
               "max_residual": res.max_residual, "submit_ms": res.submit_ms,
               "start_ms": res.start_ms, "finish_ms": res.finish_ms,
               "evals": [res.evals[i] for i in range(res.block)] if res.evals else [],
               "resnorms": [res.resnorms[i] for i in range(res.block)] if res.resnorms else []}
        lib().chfsi_result_free(C.byref(res))
        self._keep.pop(ticket, None)
        if st not in (OK, ERR_NOCONV, ERR_CANCELLED):
            raise ChfsiError(st, "chfsi_wait")
        return out

    def stats(self) -> dict:
        st = chfsi_server_stats_t()
        _check(lib().chfsi_server_stats(self.handle, C.byref(st)), "chfsi_server_stats")
        return {"budget": st.budget, "used": st.used, "sequence_bytes": st.sequence_bytes,
                "device_pool_chunks": st.device_pool_chunks,
                "host_pool_chunks": st.host_pool_chunks}

    def cancel(self, ticket: int) -> int:
        return lib().chfsi_cancel(self.handle, ticket)

    def close(self):
        if self.handle:
            lib().chfsi_server_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
