"""Outer loop of Chebyshev filtered subspace iteration (oracle).

Test infrastructure only (see the package docstring).

Algorithm 1: starting from X^(0), repeat filter -> Rayleigh-Ritz -> rotate
while max_j r_j >= tau, where r_j = ||A x_j - eps_j B x_j|| for the n wanted
pairs (the block may hold more columns than the n wanted; only j <= n enters
the stopping test).  The filter is Algorithm 2 (``method="chfsi"``, with the
operator H = D^{-1} A, or H = B^{-1} A when an exact inverse is supplied) or
Algorithm 3 (``method="rchfsi"``).

Readings (the paper is silent on these; the same readings are written
independently in the library's host code):

* Lambda^(0) for the first residual filter comes from a Rayleigh-Ritz step on
  the random X^(0) (Algorithm 3 needs Ritz values and a residual as input).
* Bounds: ``bounds`` is either a fixed (lmin, lmax, lT) triple -- the
  controlled experiments of Section 4.1 use lmin = lambda_1 - 0.05,
  lT = (lambda_n + lambda_{n+1})/2, lmax = lambda_m + 0.1 -- or the adaptive
  policy ``("ritz", lmax)``: lT = largest Ritz value of the block,
  lmin = eps_1 - 0.05 (eps_b - eps_1), lmax as given.
* The filter may use a different (perturbed) matrix than the projection:
  ``apply_A_filter`` (Section 3.2, closing remark; Section 4.1).
* Columns dropped by the SVQB fallback are refilled with N(0,1) columns drawn
  from ``refill_rng``.

Parity: the converged Ritz values are the eigenvalues of (A, B), pinned by
dense ``eigh`` and by prescribed spectra (tests/test_oracle_solver.py).
"""
from __future__ import annotations

from typing import Callable, Optional

import numpy as np

from . import filters, rr


def bounds_from_policy(bounds, lam: np.ndarray):
    """(lmin, lmax, lT) for the next filter from a fixed triple or the Ritz policy."""
    if isinstance(bounds, tuple) and len(bounds) == 2 and bounds[0] == "ritz":
        lmax = float(bounds[1])
        e1, eb = float(lam[0]), float(lam[-1])
        return e1 - 0.05 * (eb - e1), lmax, eb
    lmin, lmax, lT = bounds
    return float(lmin), float(lmax), float(lT)


def solve(apply_A: Callable, apply_B: Callable, apply_Dinv: Callable, X0: np.ndarray,
          n_wanted: int, degree: int, tol: float, max_iter: int, bounds,
          method: str = "rchfsi", apply_A_filter: Optional[Callable] = None,
          exact_U: Optional[np.ndarray] = None, B_for_angle: Optional[np.ndarray] = None,
          early_stop: bool = True, refill_seed: int = 7):
    """Run Algorithm 1 and return the final pairs and a per-iteration history.

    ``exact_U`` (B-orthonormal exact wanted eigenvectors, N x n) enables the
    subspace-angle diagnostic (Definition 2.1) in the history.
    """
    from .angles import max_principal_angle
    if apply_A_filter is None:
        apply_A_filter = apply_A
    refill_rng = np.random.default_rng(refill_seed)
    out = rr.rayleigh_ritz(X0, apply_A, apply_B)
    X, lam, R, r = out["X"], out["lam"], out["R"], out["resnorm"]
    history = []
    b = X0.shape[1]

    def record(i, bnd, o):
        h = {"iter": i, "max_res": float(np.max(r[:n_wanted])), "lam": lam.copy(),
             "bounds": bnd, "svqb": o["svqb"], "dropped": o["dropped"]}
        if exact_U is not None:
            h["angle"] = max_principal_angle(exact_U, X[:, :n_wanted], B_for_angle)
        history.append(h)

    record(0, None, out)
    for it in range(1, max_iter + 1):
        if early_stop and np.max(r[:n_wanted]) < tol:
            break
        lmin, lmax, lT = bounds_from_policy(bounds, lam)
        if method == "chfsi":
            H = lambda V: apply_Dinv(apply_A_filter(V))
            Y = filters.chebyshev_filter(H, X, degree, lmin, lmax, lT)
        elif method == "rchfsi":
            Y = filters.residual_filter(apply_A_filter, apply_Dinv, X, lam, R, degree,
                                        lmin, lmax, lT)
        else:
            raise ValueError(method)
        out = rr.rayleigh_ritz(Y, apply_A, apply_B)
        X, lam, R, r = out["X"], out["lam"], out["R"], out["resnorm"]
        if X.shape[1] < b:  # SVQB dropped directions: refill (reading above)
            extra = refill_rng.standard_normal((X.shape[0], b - X.shape[1]))
            out = rr.rayleigh_ritz(np.concatenate([X, extra], axis=1), apply_A, apply_B)
            X, lam, R, r = out["X"], out["lam"], out["R"], out["resnorm"]
        record(it, (lmin, lmax, lT), out)
    return {"X": X, "lam": lam, "resnorm": r, "history": history,
            "iters": history[-1]["iter"], "converged": bool(np.max(r[:n_wanted]) < tol)}
