"""Scaled Chebyshev polynomials and the filter's recurrence coefficients (oracle).

Test infrastructure only (see the package docstring).

Paper, Section 2.1: the affine map L(x) = (x - c)/e with centre
c = (lambda_max + lambda_T)/2 and half-width e = (lambda_max - lambda_T)/2 sends
the unwanted interval [lambda_T, lambda_max] to [-1, 1]; the scaled polynomial
is C_k(x) = T_k(L(x)) / T_k(L(lambda_min)).  The scaling coefficients are
sigma_1 = e/(lambda_min - c) and sigma_{k+1} = 1/(2/sigma_1 - sigma_k)
(eq. ChFSIrecurrence and Algorithm 2).  Section 3.2 names the recurrence
coefficients a_k = 2 sigma_{k+1}/e, b_k = -2 sigma_{k+1} c/e,
c_k = -sigma_k sigma_{k+1}.

Pins (tests/test_oracle_chebyshev.py): T_k against numpy's Chebyshev series
and T_m(cos t) = cos(m t); sigma_k = T_{k-1}(L0)/T_k(L0); the scalar
recurrence driven by (a_k, b_k, c_k) against the closed form C_k.
"""
from __future__ import annotations

import numpy as np


def affine(lmin: float, lmax: float, lT: float):
    """Return (e, c, sigma_1) of Section 2.1 / Algorithm 2, first line."""
    e = (lmax - lT) / 2.0
    c = (lmax + lT) / 2.0
    sigma1 = e / (lmin - c)
    return e, c, sigma1


def cheb_T(k: int, x):
    """Chebyshev polynomial of the first kind T_k(x), closed form.

    T_k(x) = cos(k arccos x) on |x| <= 1 and sign(x)^k cosh(k arccosh |x|)
    outside (the fast growth used by the filter, Section 2.1).
    """
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(k * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** k * np.cosh(k * np.arccosh(np.abs(xo)))
    return out


def scaled_cheb(x, k: int, lmin: float, lmax: float, lT: float):
    """C_k(x) = T_k(L(x)) / T_k(L(lambda_min)) (Section 2.1)."""
    e, c, _ = affine(lmin, lmax, lT)
    L = lambda t: (np.asarray(t, dtype=np.float64) - c) / e
    return cheb_T(k, L(x)) / cheb_T(k, L(np.array([lmin])))[0]


def sigmas(sigma1: float, p: int) -> np.ndarray:
    """[sigma_1, ..., sigma_p] with sigma_{k+1} = 1/(2/sigma_1 - sigma_k)."""
    s = np.empty(p, dtype=np.float64)
    s[0] = sigma1
    gamma = 2.0 / sigma1
    for k in range(1, p):
        s[k] = 1.0 / (gamma - s[k - 1])
    return s


def recurrence_coeffs(lmin: float, lmax: float, lT: float, p: int):
    """Rows (a_k, b_k, c_k) for k = 1..p-1 (Section 3.2 notation).

    Row k-1 of the result advances degree k to degree k+1:
    Y_{k+1} = a_k H Y_k + b_k Y_k + c_k Y_{k-1}.
    """
    e, c, s1 = affine(lmin, lmax, lT)
    s = sigmas(s1, p)
    out = np.empty((max(p - 1, 0), 3), dtype=np.float64)
    for k in range(1, p):
        sk, sk1 = s[k - 1], s[k]
        out[k - 1] = (2.0 * sk1 / e, -2.0 * sk1 * c / e, -sk * sk1)
    return out


def scalar_recurrence(x, lmin: float, lmax: float, lT: float, p: int):
    """C_0..C_p at the points x via the three-term recurrence (eq. ChFSIrecurrenceEigval).

    Lambda_0 = 1, Lambda_1 = (sigma_1/e)(x - c),
    Lambda_{k+1} = a_k Lambda_k x + b_k Lambda_k + c_k Lambda_{k-1}.
    Returns an array of shape (p+1, len(x)).
    """
    x = np.asarray(x, dtype=np.float64)
    e, c, s1 = affine(lmin, lmax, lT)
    out = np.empty((p + 1,) + x.shape, dtype=np.float64)
    out[0] = 1.0
    if p >= 1:
        out[1] = (s1 / e) * (x - c)
    for k, (a, b, cc) in enumerate(recurrence_coeffs(lmin, lmax, lT, p), start=1):
        out[k + 1] = a * out[k] * x + b * out[k] + cc * out[k - 1]
    return out
