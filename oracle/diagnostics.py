"""Convergence-condition diagnostics (oracle), Section 3.1 and Section 4.1.3.

Test infrastructure only (see the package docstring).

The analysis of Section 3.1 compares the block a method actually filters,
Y~ (Algorithm 2 with the approximate inverse D^{-1}, or Algorithm 3 with
D^{-1}), with the exact filter C_p(H) X, H = B^{-1} A, applied to the same
current basis X = X^(i).  Its filtering error is

    Delta^_p = B^{1/2} (Y~ - C_p(H) X),          ||Delta^_p||_2,

and the angle between the current subspace S^(i) (the n wanted columns) and
the exact wanted eigenspace S decreases when (the sufficient condition of
Section 3.1, used again in Section 4.1.3)

    |C_p(lambda_n)| - ||C_p(Lambda_2)||  >  ||Delta^_p|| (sec theta + csc theta),

theta = angle(S^(i), S) in the B-inner product, C_p the scaled Chebyshev
polynomial of the filter's bounds, ||C_p(Lambda_2)|| its largest magnitude
over the unwanted eigenvalues (the paper writes |C_p(lambda_{n+1})|; see
``chebyshev_gap`` for when the two differ).  The condition comes from Theorem 3.1:
for an n-dimensional S^(i), the span S_^(i+1) of the filtered block obeys

    tan angle(S_^(i+1), S) <= (||C_p(Lambda_2)|| + ||Delta^_p|| csc theta)
                              / (|C_p(lambda_n)| - ||Delta^_p|| sec theta) * tan theta

whenever the denominator is positive.  ``diagnose`` evaluates these
quantities for one basis; ``run`` repeats Algorithm 1 and records them at
every outer iteration.

||B^{1/2} D||_2 is computed as sqrt(lambda_max(D^T B D)), the same number
without forming B^{1/2}.

Pins (tests/test_oracle_diagnostics.py): with D^{-1} = B^{-1} the error is
zero to rounding for both methods (Algorithm 3 is an identity rewrite of
Algorithm 2); the norm equals the one formed with an explicit B^{1/2}; the
angle of the filtered span never exceeds the bound of Theorem 3.1; for
zeta = 1e-3 the ChFSI error saturates at O(zeta) and the condition is
eventually violated, while the R-ChFSI error falls with the residual and the
condition holds at every iteration (the behaviour Section 4.1.3 reports).
"""
from __future__ import annotations

from typing import Callable, Optional

import numpy as np

from . import chebyshev, filters, rr
from .angles import max_principal_angle


def b_norm2(Dlt: np.ndarray, B: Optional[np.ndarray]) -> float:
    """||B^{1/2} Dlt||_2 = sqrt(lambda_max(Dlt^T B Dlt))."""
    G = Dlt.conj().T @ (Dlt if B is None else B @ Dlt)
    return float(np.sqrt(max(np.max(np.linalg.eigvalsh(0.5 * (G + G.conj().T))), 0.0)))


def chebyshev_gap(lam_exact: np.ndarray, n: int, p: int, bounds):
    """(||C_p(Lambda_1)^{-1}||^{-1}, ||C_p(Lambda_2)||, |C_p(lambda_{n+1})|).

    The proof of Theorem 3.1 bounds the unwanted block by the spectral norm of
    C_p(Lambda_2), the largest |C_p| over the unwanted eigenvalues; the
    wanted block by the smallest |C_p| over the wanted ones, |C_p(lambda_n)|
    (|C_p| decreases from lambda_min up to lambda_T).  The theorem writes the
    former as |C_p(lambda_{n+1})|, which is the same number only when
    lambda_{n+1} <= lambda_T; with lambda_T between lambda_n and lambda_{n+1}
    the Chebyshev oscillation on [lambda_T, lambda_max] can make other unwanted
    eigenvalues larger in |C_p|, so the norm is used and the literal value is
    returned third, for reference.
    """
    lmin, lmax, lT = bounds
    c = np.abs(chebyshev.scaled_cheb(np.asarray(lam_exact, dtype=np.float64), p, lmin, lmax, lT))
    return float(np.min(c[:n])), float(np.max(c[n:])), float(c[n])


def theorem31_tan_bound(cn: float, cn1: float, err: float, theta: float) -> float:
    """Right-hand side of Theorem 3.1's bound on tan angle(S_^(i+1), S), or inf
    when its premise |C_p(lambda_n)| cos theta > ||Delta^_p|| fails."""
    den = cn - err / np.cos(theta)
    if den <= 0.0 or theta <= 0.0:
        return np.inf
    return (cn1 + err / np.sin(theta)) / den * np.tan(theta)


def diagnose(method: str, A: np.ndarray, B: np.ndarray, Binv: np.ndarray, Dinv: np.ndarray,
             X: np.ndarray, lam: np.ndarray, R: np.ndarray, p: int, bounds, U: np.ndarray,
             lam_exact: np.ndarray, n: int):
    """Filtering error, angle and both sides of the condition for one basis X.

    X: B-orthonormal Ritz vectors (N x b), lam their Ritz values, R = A X - B X
    diag(lam); U: exact wanted eigenvectors (N x n); lam_exact: the pencil's
    eigenvalues in ascending order (lambda_n = lam_exact[n-1]).
    """
    Y = low_filter(method, A, Dinv, X, lam, R, p, bounds)
    return measure(Y, A, B, Binv, X, p, bounds, U, lam_exact, n)


def low_filter(method: str, A: np.ndarray, Dinv: np.ndarray, X: np.ndarray, lam: np.ndarray,
               R: np.ndarray, p: int, bounds) -> np.ndarray:
    """The block the method filters with the approximate inverse D^{-1}."""
    lmin, lmax, lT = bounds
    if method == "chfsi":
        return filters.chebyshev_filter(lambda V: Dinv @ (A @ V), X, p, lmin, lmax, lT)
    if method == "rchfsi":
        return filters.residual_filter(filters.dense_op(A), filters.dense_op(Dinv), X, lam, R, p,
                                       lmin, lmax, lT)
    raise ValueError(method)


def measure(Y: np.ndarray, A: np.ndarray, B: np.ndarray, Binv: np.ndarray, X: np.ndarray, p: int,
            bounds, U: np.ndarray, lam_exact: np.ndarray, n: int):
    """Diagnostics of a filtered block Y (computed by any means) of the basis X.

    Compares Y with the exact filter C_p(B^{-1} A) X; when Y has n columns also
    returns the angle of its span and Theorem 3.1's bound on it.
    """
    lmin, lmax, lT = bounds
    H_exact = lambda V: Binv @ (A @ V)
    Y_exact = filters.chebyshev_filter(H_exact, X, p, lmin, lmax, lT)
    err = b_norm2(Y - Y_exact, B)
    theta = max_principal_angle(U, X[:, :n], B)
    cn, cn1, cn1_lit = chebyshev_gap(lam_exact, n, p, bounds)
    lhs = cn - cn1
    rhs = err * (1.0 / np.cos(theta) + 1.0 / np.sin(theta)) if theta > 0 else np.inf
    out = {"filter_error": err, "angle": theta, "lhs": lhs, "rhs": rhs, "holds": lhs > rhs,
           "lhs_literal": cn - cn1_lit, "Y": Y, "angle_next": None,
           "tan_bound": theorem31_tan_bound(cn, cn1, err, theta)}
    if Y.shape[1] == n:
        out["angle_next"] = max_principal_angle(U, Y, B)
    return out


def run(method: str, A: np.ndarray, B: np.ndarray, Binv: np.ndarray, Dinv: np.ndarray,
        X0: np.ndarray, n: int, p: int, bounds, iters: int,
        lam_exact: Optional[np.ndarray] = None, U: Optional[np.ndarray] = None):
    """Algorithm 1 with the method's filter; per-iteration diagnostics.

    Returns a list of dicts: iter, max_res (over the n wanted pairs), residual
    block norm ||R^(i)||_2, filter_error, angle, lhs, rhs, holds, angle_next
    (of the filtered span, block of n columns only) and tan_bound.
    """
    import scipy.linalg as sla
    if lam_exact is None or U is None:
        w, V = sla.eigh(A, B)
        lam_exact = w if lam_exact is None else lam_exact
        U = V[:, :n] if U is None else U
    opA, opB = filters.dense_op(A), filters.dense_op(B)
    o = rr.rayleigh_ritz(X0, opA, opB)
    hist = []
    for it in range(iters):
        d = diagnose(method, A, B, Binv, Dinv, o["X"], o["lam"], o["R"], p, bounds, U,
                     lam_exact, n)
        hist.append({"iter": it, "max_res": float(np.max(o["resnorm"][:n])),
                     "res_norm": float(np.linalg.norm(o["R"], 2)),
                     "filter_error": d["filter_error"], "angle": d["angle"], "lhs": d["lhs"],
                     "rhs": d["rhs"], "holds": d["holds"], "angle_next": d["angle_next"],
                     "tan_bound": d["tan_bound"]})
        o = rr.rayleigh_ritz(d["Y"], opA, opB)
    return hist
