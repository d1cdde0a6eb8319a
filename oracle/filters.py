"""Chebyshev filters of the paper, in float64 (oracle).

Test infrastructure only (see the package docstring).

``chebyshev_filter``  follows Algorithm 2 (two temporaries that swap, one
product with H per degree).  ``residual_filter`` follows Algorithm 3: it runs
the same three-term recurrence on the filtered residuals R_X, R_Y and on the
diagonal Chebyshev-filtered eigenvalues Lambda_X, Lambda_Y, and rebuilds
Y_p = D^{-1} R_Y + X Lambda_Y at the end (Proposition 3.3 and
eq. rChFSIrecurrenceMP).  Operators are passed as callables so that dense
matrices, perturbed filter matrices and grid stencils all work.

Blocks may be real or complex (Section 4.3's Hermitian problems): the
recurrences have real coefficients, so they act on complex blocks unchanged.

Pins: on a matrix with known eigenvectors the filter must equal
Q C_p(Lambda) Q^T X (exact up to rounding); Algorithm 3 with D^{-1} = B^{-1}
equals Algorithm 2 with H = B^{-1} A (Section 3.2, closing remark); the
Lambda recurrence equals the closed-form C_p (tests/test_oracle_filters.py).
"""
from __future__ import annotations

from typing import Callable

import numpy as np

from .chebyshev import affine

Op = Callable[[np.ndarray], np.ndarray]


def chebyshev_filter(apply_H: Op, X: np.ndarray, p: int, lmin: float, lmax: float,
                     lT: float) -> np.ndarray:
    """Y_p = C_p(H) X by the three-term recurrence (Algorithm 2).

    ``apply_H(V)`` returns H V; for the generalized problem H = B^{-1} A, or
    D^{-1} A when an approximate inverse is used (eq. ChFSIrecurrenceSEPMP).
    """
    e, c, sigma = affine(lmin, lmax, lT)
    sigma1 = sigma
    gamma = 2.0 / sigma1
    Xt = np.array(X, dtype=np.result_type(X, np.float64), copy=True)
    Yt = (sigma1 / e) * (apply_H(Xt) - c * Xt)
    for _k in range(2, p + 1):
        sigma2 = 1.0 / (gamma - sigma)
        Xt = (2.0 * sigma2 / e) * apply_H(Yt) - (2.0 * sigma2 / e) * c * Yt - sigma * sigma2 * Xt
        Xt, Yt = Yt, Xt
        sigma = sigma2
    return Yt


def residual_filter(apply_A: Op, apply_Dinv: Op, X: np.ndarray, lam: np.ndarray,
                    Yres: np.ndarray, p: int, lmin: float, lmax: float, lT: float,
                    return_parts: bool = False):
    """Residual-based Chebyshev filter (Algorithm 3).

    Inputs follow the algorithm's INPUTS line: the current Ritz vectors X, the
    Ritz values ``lam`` (diagonal of Lambda^{(i)}), the approximate inverse
    D^{-1} (as a callable) and the residual Y = A X - B X Lambda^{(i)}.
    Returns D^{-1} R_Y + X Lambda_Y.  With ``return_parts`` also returns
    (R_Y, Lambda_Y) of the last degree.
    """
    e, c, sigma = affine(lmin, lmax, lT)
    sigma1 = sigma
    gamma = 2.0 / sigma1
    lam = np.asarray(lam, dtype=np.float64)
    Y = np.asarray(Yres, dtype=np.result_type(Yres, np.float64))
    RX = np.zeros_like(Y)
    RY = (sigma1 / e) * Y
    LX = np.ones_like(lam)
    LY = (sigma1 / e) * (lam - c)
    for _k in range(2, p + 1):
        sigma2 = 1.0 / (gamma - sigma)
        a = 2.0 * sigma2 / e
        RX = a * apply_A(apply_Dinv(RY)) - a * c * RY - sigma * sigma2 * RX + a * (Y * LY[None, :])
        LX = a * LY * lam - a * c * LY - sigma * sigma2 * LX
        RX, RY = RY, RX
        LX, LY = LY, LX
        sigma = sigma2
    out = apply_Dinv(RY) + np.asarray(X, dtype=np.result_type(X, np.float64)) * LY[None, :]
    if return_parts:
        return out, RY, LY
    return out


def dense_op(M: np.ndarray) -> Op:
    return lambda V: M @ V


def diag_op(d: np.ndarray) -> Op:
    d = np.asarray(d, dtype=np.float64)
    return lambda V: d[:, None] * V


def identity_op() -> Op:
    return lambda V: V
