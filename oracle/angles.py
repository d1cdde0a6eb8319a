"""Maximum principal angle between subspaces (oracle diagnostic).

Test infrastructure only (see the package docstring).

Definition 2.1: with X orthonormal spanning a p-dimensional subspace, X_perp an
orthonormal basis of its complement and Y an orthogonal basis (q <= p columns)
of the second subspace, tan(angle) = ||X_perp^T Y (X^T Y)^+|| when X^T Y has
rank q.  For generalized problems the paper measures angles in the
B^{1/2}-transformed coordinates (Section 2.1), i.e. with B-orthonormal bases.

``tan_angle_def21`` is the definition written out; ``max_principal_angle``
computes the same angle through the singular values of U^T B X (cosines of the
principal angles).  Pin: the two agree (tests/test_oracle_filters.py).
"""
from __future__ import annotations

import numpy as np


def tan_angle_def21(Xo: np.ndarray, Xperp: np.ndarray, Y: np.ndarray) -> float:
    M = Xo.T @ Y
    if np.linalg.matrix_rank(M) < Y.shape[1]:
        return np.pi / 2
    return float(np.linalg.norm(Xperp.T @ Y @ np.linalg.pinv(M), 2))


def _b_orthonormalize(X: np.ndarray, B=None) -> np.ndarray:
    if B is None:
        Q, _ = np.linalg.qr(X)
        return Q
    G = X.conj().T @ (B @ X)
    L = np.linalg.cholesky(0.5 * (G + G.conj().T))
    return np.linalg.solve(L.conj(), X.T).T


def max_principal_angle(U: np.ndarray, X: np.ndarray, B=None) -> float:
    """Largest principal angle between span(U) (dim n) and span(X) (dim >= n), B-inner product.

    Computed from its sine, sin = ||(I - P_X) U||_B with P_X the B-orthogonal
    projector onto span(X) and U B-orthonormal, which stays accurate for tiny
    angles (the cosine route loses them below ~1e-8).
    """
    Uo = _b_orthonormalize(np.asarray(U, dtype=np.result_type(U, np.float64)), B)
    Xo = _b_orthonormalize(np.asarray(X, dtype=np.result_type(X, np.float64)), B)
    BU = Uo if B is None else B @ Uo
    W = Uo - Xo @ (Xo.conj().T @ BU)
    G = W.conj().T @ (W if B is None else B @ W)
    s2 = float(np.max(np.linalg.eigvalsh(0.5 * (G + G.conj().T))))
    return float(np.arcsin(min(max(s2, 0.0), 1.0) ** 0.5))
