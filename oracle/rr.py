"""Rayleigh-Ritz on the filtered block and residual norms (oracle).

Test infrastructure only (see the package docstring).

Algorithm 1, steps 2-3: solve the projected pencil
(Y^T A Y) E = (Y^T B Y) E Lambda on the *non-orthogonal* filtered basis Y and
rotate X = Y E; the Ritz vectors are then B-orthonormal.  Residual norms are
r_j = ||A x_j - eps_j B x_j||_2 (Algorithm 1, loop condition).

Reading for a numerically singular Gram matrix (the paper only mentions
"numerical instabilities" at high degree): scale the columns of Y to unit
B-norm first, and when the scaled Gram matrix Y^T B Y is not positive definite
fall back to SVQB -- keep the eigen-directions of the scaled Gram matrix whose
eigenvalue exceeds ``drop_tol`` times the largest, and solve the standard
problem in that basis.  The caller refills dropped columns.

Complex blocks (Section 4.3's Hermitian problems) take the same steps with
conjugate transposes: Y^H A Y, Y^H B Y and X^H B X = I.

Pins: Ritz values against scipy's dsygvd on the same pencil AND against the
brute-force Jacobi of ``oracle.jacobi`` (tiny sizes); X^T B X = I; on a block
that spans an invariant subspace the Ritz values are exact eigenvalues
(tests/test_oracle_rr.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def column_norms(R: np.ndarray) -> np.ndarray:
    """Euclidean norm of every column."""
    return np.sqrt(np.sum(np.abs(np.asarray(R)) ** 2, axis=0))


def rayleigh_ritz(Y: np.ndarray, apply_A, apply_B, drop_tol: float = 1e-14):
    """Ritz pairs of (A, B) on span(Y) by the generalized projected pencil.

    Returns a dict with X (B-orthonormal Ritz vectors, ascending Ritz values),
    lam, R = A X - B X diag(lam), resnorm (column norms of R), dropped (number
    of basis directions discarded by the SVQB fallback) and svqb (bool).
    """
    Y = np.asarray(Y, dtype=np.result_type(Y, np.float64))
    AY = apply_A(Y)
    BY = apply_B(Y)
    Ga = Y.conj().T @ AY
    Gb = Y.conj().T @ BY
    Ga = 0.5 * (Ga + Ga.conj().T)
    Gb = 0.5 * (Gb + Gb.conj().T)
    s = 1.0 / np.sqrt(np.diag(Gb).real)
    Gas = s[:, None] * Ga * s[None, :]
    Gbs = s[:, None] * Gb * s[None, :]
    svqb = False
    dropped = 0
    try:
        # breakdown: a Cholesky pivot of the unit-diagonal scaled Gram matrix at
        # or below drop_tol (its smallest eigenvalue is then below drop_tol
        # times the largest, so SVQB would drop a direction)
        piv = np.abs(np.diag(np.linalg.cholesky(Gbs))) ** 2
        if not np.min(piv) > drop_tol:
            raise np.linalg.LinAlgError("numerically singular Gram matrix")
        lam, E = sla.eigh(Gas, Gbs)
        W = s[:, None] * E
    except np.linalg.LinAlgError:
        svqb = True
        w, U = np.linalg.eigh(Gbs)
        keep = w > drop_tol * w[-1]
        dropped = int(np.count_nonzero(~keep))
        T = U[:, keep] / np.sqrt(w[keep])[None, :]
        Hp = T.conj().T @ Gas @ T
        Hp = 0.5 * (Hp + Hp.conj().T)
        lam, E = np.linalg.eigh(Hp)
        W = s[:, None] * (T @ E)
    X = Y @ W
    AX = AY @ W
    BX = BY @ W
    R = AX - BX * lam[None, :]
    return {"X": X, "lam": lam, "R": R, "resnorm": column_norms(R), "svqb": svqb,
            "dropped": dropped}


def residual_norms(apply_A, apply_B, X: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """r_j = ||A x_j - lam_j B x_j||_2 computed directly from (X, lam)."""
    R = apply_A(X) - apply_B(X) * np.asarray(lam)[None, :]
    return column_norms(R)


def pencil_eigenvalues(A: np.ndarray, B, keep: int) -> np.ndarray:
    """Lowest `keep` eigenvalues of (A, B): Rayleigh-Ritz on the whole space.

    With the full basis Y = I the projected pencil is (A, B) itself, so this is
    the plain definition (LAPACK dsygvd/dsygvx through SciPy).
    """
    return sla.eigh(A, B, eigvals_only=True, subset_by_index=(0, keep - 1))
