"""Periodic 27-point grid operators applied to blocks of vectors (oracle).

Test infrastructure only (see the package docstring).

A grid vector has N = nx*ny*nz entries indexed x + nx*(y + ny*z); a block is
N x b.  ``apply_stencil`` evaluates y(r) = sum_o c[o] u(r + o) over the 27
offsets o in {-1,0,1}^3 with periodic wrap, by plain array rolls.

The pencil of the grid workloads is A = S_A + (potential term), B = S_B where
S_A = 0.5 K (Q1 stiffness) and S_B = M (Q1 mass).  Two readings of the
potential term are supported: ``field_mode=1`` the lumped diagonal V (R1),
``field_mode=2`` the mass-weighted 1/2 (diag(V) M + M diag(V)) (R2), which has
M's 27-point pattern and reduces to diag(V) under the same row-sum lumping
that turns M into D = I (the paper's Section 4.2 uses a mass-lumped diagonal
approximation of B in the filter only).

Complex (k-point) problems of Section 4.3 on a grid: the Bloch-phase
operators act on cell-periodic vectors with every offset's coefficient times
exp(i k.o), k = (kx, ky, kz) in radians per grid step (``apply_stencil_bloch``,
``make_ops_bloch``); the potential terms keep their form with M(k) in place
of M.  They are Hermitian, and k = 0 gives the real operators.

Pins: the stencil against an explicit Kronecker product of 1D circulant
matrices; with V = 0 the pencil's eigenvalues equal the Fourier-symbol closed
form sum_d 3(1 - cos t_d)/(2 + cos t_d), t_d = 2 pi j_d / n_d
(tests/test_oracle_stencil.py); the Bloch operators against the same symbol
at t + k, Hermitian symmetry, k = 0, and an independent construction by
twisted periodic wraps (tests/test_oracle_stencil_bloch.py).
"""
from __future__ import annotations

import numpy as np


def apply_stencil(coef: np.ndarray, U: np.ndarray, shape) -> np.ndarray:
    nz, ny, nx = shape
    U = np.asarray(U, dtype=np.float64)
    squeeze = U.ndim == 1
    if squeeze:
        U = U[:, None]
    b = U.shape[1]
    u = U.reshape(nz, ny, nx, b, order="C") if U.flags.c_contiguous else \
        np.ascontiguousarray(U).reshape(nz, ny, nx, b)
    y = np.zeros_like(u)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                c = coef[dz + 1, dy + 1, dx + 1]
                if c == 0.0:
                    continue
                y += c * np.roll(u, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
    y = y.reshape(nz * ny * nx, b)
    return y[:, 0] if squeeze else y


def make_ops(coef_A: np.ndarray, coef_B: np.ndarray, V: np.ndarray, shape, field_mode: int):
    """Callables (apply_A, apply_B) for the grid pencil."""
    v = np.asarray(V, dtype=np.float64).reshape(-1)

    def apply_B(U):
        return apply_stencil(coef_B, U, shape)

    def apply_A(U):
        U = np.asarray(U, dtype=np.float64)
        vv = v[:, None] if U.ndim == 2 else v
        out = apply_stencil(coef_A, U, shape)
        if field_mode == 1:
            out = out + vv * U
        elif field_mode == 2:
            out = out + 0.5 * vv * apply_B(U) + 0.5 * apply_B(vv * U)
        elif field_mode != 0:
            raise ValueError(field_mode)
        return out

    return apply_A, apply_B


def circulant_1d(st: np.ndarray, n: int) -> np.ndarray:
    """Dense n x n periodic matrix of a 3-point stencil (offsets -1, 0, +1)."""
    C = np.zeros((n, n))
    for i in range(n):
        for o in (-1, 0, 1):
            C[i, (i + o) % n] += st[o + 1]
    return C


def apply_stencil_bloch(coef: np.ndarray, U: np.ndarray, shape, k) -> np.ndarray:
    """y(r) = sum_o c[o] exp(i k.o) u(r + o), periodic wrap; U complex N x b."""
    nz, ny, nx = shape
    kx, ky, kz = (float(v) for v in k)
    U = np.asarray(U, dtype=np.complex128)
    squeeze = U.ndim == 1
    if squeeze:
        U = U[:, None]
    b = U.shape[1]
    u = np.ascontiguousarray(U).reshape(nz, ny, nx, b)
    y = np.zeros_like(u)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                c = coef[dz + 1, dy + 1, dx + 1]
                if c == 0.0:
                    continue
                ph = np.exp(1j * (kx * dx + ky * dy + kz * dz))
                y += (c * ph) * np.roll(u, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
    y = y.reshape(nz * ny * nx, b)
    return y[:, 0] if squeeze else y


def make_ops_bloch(coef_A: np.ndarray, coef_B: np.ndarray, V: np.ndarray, shape,
                   field_mode: int, k):
    """Callables (apply_A, apply_B) of the Bloch-phase grid pencil at wave vector k."""
    v = np.asarray(V, dtype=np.float64).reshape(-1)

    def apply_B(U):
        return apply_stencil_bloch(coef_B, U, shape, k)

    def apply_A(U):
        U = np.asarray(U, dtype=np.complex128)
        vv = v[:, None] if U.ndim == 2 else v
        out = apply_stencil_bloch(coef_A, U, shape, k)
        if field_mode == 1:
            out = out + vv * U
        elif field_mode == 2:
            out = out + 0.5 * vv * apply_B(U) + 0.5 * apply_B(vv * U)
        elif field_mode != 0:
            raise ValueError(field_mode)
        return out

    return apply_A, apply_B
