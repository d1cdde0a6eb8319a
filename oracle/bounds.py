"""Spectrum-bound estimates of the pencil (A, B) by a k-step Lanczos process (oracle).

Test infrastructure only (see the package docstring).

The filter needs lambda_max above the whole spectrum of B^{-1} A and treats
the bounds as estimates (Section 2.1).  The estimate is a k-step Lanczos
process on B^{-1} A, which is self-adjoint in the B-inner product
<x, y>_B = x^H B y:

    v_1 = v_0 / ||v_0||_B
    for j = 1..k:
        u = B^{-1} A v_j                 (here: an exact solve with B)
        alpha_j = <v_j, u>_B = v_j^H A v_j
        u = u - alpha_j v_j - beta_{j-1} v_{j-1}
        beta_j = ||u||_B,  v_{j+1} = u / beta_j

T_k = tridiag(beta, alpha, beta) has eigenvalues theta_1 <= ... <= theta_k,
the Ritz values of the pencil on the Krylov space; they lie inside the
pencil's spectrum (Courant-Fischer).  The estimates add the safeguard |beta_k|
("Ritz value + |beta_k|", Zhou, Saad, Tiago and Chelikowsky, J. Comput. Phys.
219 (2006)): upper = theta_k + |beta_k|, lower = theta_1 - |beta_k|.

Complex Hermitian pencils use the Hermitian inner product (alpha_j is real).

Pins (tests/test_oracle_bounds.py): a full-length run on a diagonal pencil
returns its eigenvalues and beta_k = 0; theta_1 and theta_k lie inside the
spectrum from dense eigh and the estimates enclose it on the dense and grid
pencils; the grid pencil without a potential has lambda_max = 18 exactly
(Fourier symbols, reading of the 27-point Q1 stencils).
"""
from __future__ import annotations

from typing import Callable

import numpy as np


def lanczos_bounds(apply_A: Callable, apply_B: Callable, solve_B: Callable, v0: np.ndarray,
                   steps: int) -> dict:
    """Run `steps` Lanczos steps on B^{-1} A in the B-inner product from v0.

    apply_A, apply_B, solve_B act on 1-D vectors (real or complex); solve_B(y)
    returns B^{-1} y.  Returns alpha, beta, theta (ascending eigenvalues of
    T_k), beta_last, lower and upper."""
    v = np.asarray(v0).astype(np.result_type(v0, np.float64)).copy()
    Bv = apply_B(v)
    nrm = np.sqrt(np.real(np.vdot(v, Bv)))
    v, Bv = v / nrm, Bv / nrm
    v_prev = np.zeros_like(v)
    beta_prev = 0.0
    alpha, beta = [], []
    for j in range(steps):
        w = apply_A(v)
        u = solve_B(w)
        a = float(np.real(np.vdot(v, w)))
        alpha.append(a)
        u = u - a * v - beta_prev * v_prev
        Bu = apply_B(u)
        bj = float(np.sqrt(max(np.real(np.vdot(u, Bu)), 0.0)))
        beta.append(bj)
        if j + 1 == steps or not bj > 1e-14 * abs(a) + 1e-300:
            break
        v_prev, v = v, u / bj
        beta_prev = bj
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    theta = np.linalg.eigvalsh(T)
    bl = abs(beta[k - 1])
    return {"alpha": np.asarray(alpha), "beta": np.asarray(beta), "theta": theta,
            "beta_last": bl, "lower": float(theta[0] - bl), "upper": float(theta[-1] + bl),
            "steps": k}
