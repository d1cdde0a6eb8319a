"""Brute-force cyclic Jacobi eigensolver for tiny symmetric matrices (oracle).

Test infrastructure only (see the package docstring).

Classical row-cyclic Jacobi: for every off-diagonal pair (p, q) choose the
plane rotation that annihilates a_pq (Golub & Van Loan, Sec. 8.5), apply it on
both sides, accumulate the rotations, and sweep until the off-diagonal mass is
below ``tol`` relative to the Frobenius norm.  Pure Python loops over pairs:
meant for n <= ~64 only.  It serves as an independent check of the LAPACK
eigensolver that ``oracle.rr`` relies on.

Pins: reconstructs A = V diag(w) V^T, V^T V = I, and matches closed-form
spectra (tests/test_oracle_rr.py).
"""
from __future__ import annotations

import math

import numpy as np


def jacobi_eigh(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    fro = math.sqrt(float(np.sum(A * A))) or 1.0
    for _ in range(max_sweeps):
        off = float(np.linalg.norm(A - np.diag(np.diag(A))))
        if off <= tol * fro:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                diff = A[q, q] - A[p, p]
                if apq == 0.0 or abs(apq) <= 1e-18 * abs(diff):
                    continue
                theta = diff / (2.0 * apq)
                if abs(theta) > 1e150:
                    t = 0.5 / theta
                else:
                    t = math.copysign(1.0, theta) / (abs(theta) + math.sqrt(theta * theta + 1.0))
                c = 1.0 / math.sqrt(t * t + 1.0)
                s = t * c
                # A <- J^T A J with J = rotation in (p, q)
                Ap = A[:, p].copy()
                Aq = A[:, q].copy()
                A[:, p] = c * Ap - s * Aq
                A[:, q] = s * Ap + c * Aq
                Ap = A[p, :].copy()
                Aq = A[q, :].copy()
                A[p, :] = c * Ap - s * Aq
                A[q, :] = s * Ap + c * Aq
                Vp = V[:, p].copy()
                Vq = V[:, q].copy()
                V[:, p] = c * Vp - s * Vq
                V[:, q] = s * Vp + c * Vq
    w = np.diag(A).copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]
