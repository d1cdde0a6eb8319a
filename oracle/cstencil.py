"""ctypes loader of the oracle's C grid kernels (oracle/stencil27.c).

Test infrastructure only (see the package docstring).  ``build()`` compiles
the C file with gcc (-O3, OpenMP, no machine-specific flags, so the library
runs on any x86-64 host) into oracle/libstencil27.so; ``__graft_entry__.build``
calls it.  ``rchfsi_filter`` runs Algorithm 3 in FP64 on a block of columns
of a grid pencil; ``pencil_apply`` applies A to one grid vector.

Pins: both agree with the NumPy oracle (``stencil.make_ops`` and
``filters.residual_filter``) to rounding on small grids
(tests/test_oracle_cstencil.py).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "stencil27.c")
LIB = os.path.join(HERE, "libstencil27.so")

_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c99", SRC, "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle C build failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.o_pencil_apply.argtypes = [dp, dp, dp, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp]
        L.o_pencil_apply.restype = None
        L.o_rchfsi_filter.argtypes = [dp, dp, dp, C.c_int, C.c_int, C.c_int, C.c_int, dp,
                                      C.c_int64, dp, C.c_int64, dp, dp, C.c_int64, dp, C.c_int64,
                                      C.c_double, C.c_double, C.c_double, C.c_int]
        L.o_rchfsi_filter.restype = C.c_int
        L.o_threads.argtypes = []
        L.o_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _col(a):
    """Column-major float64 copy of a block (n x b) and its leading dimension."""
    a = np.asfortranarray(np.asarray(a, dtype=np.float64))
    return a, a.shape[0]


def threads() -> int:
    return int(lib().o_threads())


def pencil_apply(coef_A, coef_mass, V, field_mode: int, shape, x) -> np.ndarray:
    nz, ny, nx = shape
    n = nx * ny * nz
    cA = np.ascontiguousarray(np.asarray(coef_A, dtype=np.float64).reshape(27))
    cM = np.ascontiguousarray(np.asarray(coef_mass, dtype=np.float64).reshape(27))
    v = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1))
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    y, t1, t2 = np.empty(n), np.empty(n), np.empty(n)
    lib().o_pencil_apply(_dp(cA), _dp(cM), _dp(v), field_mode, nx, ny, nz, _dp(x), _dp(y),
                         _dp(t1), _dp(t2))
    return y


def rchfsi_filter(coef_A, coef_mass, V, field_mode: int, shape, dinv, X, ritz, R, degree: int,
                  lmin: float, lmax: float, lT: float) -> np.ndarray:
    """Algorithm 3 (FP64) on the columns of X with residual block R."""
    nz, ny, nx = shape
    cA = np.ascontiguousarray(np.asarray(coef_A, dtype=np.float64).reshape(27))
    cM = np.ascontiguousarray(np.asarray(coef_mass, dtype=np.float64).reshape(27))
    v = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1))
    Xc, ldx = _col(X)
    Rc, ldr = _col(R)
    b = Xc.shape[1]
    lam = np.ascontiguousarray(np.asarray(ritz, dtype=np.float64))
    Y = np.empty((Xc.shape[0], b), order="F")
    d = None if dinv is None else np.ascontiguousarray(np.asarray(dinv, dtype=np.float64))
    st = lib().o_rchfsi_filter(_dp(cA), _dp(cM), _dp(v), field_mode, nx, ny, nz,
                               None if d is None else _dp(d), b, _dp(Xc), ldx, _dp(lam), _dp(Rc),
                               ldr, _dp(Y), Y.shape[0], lmin, lmax, lT, degree)
    if st != 0:
        raise MemoryError("o_rchfsi_filter: scratch allocation failed")
    return Y
