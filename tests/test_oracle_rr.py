"""Pins for oracle.rr (Rayleigh-Ritz, Algorithm 1 steps 2-3) and oracle.jacobi.

* Brute-force cyclic Jacobi reproduces a prescribed spectrum and reconstructs A.
* Ritz values of the projected pencil equal (a) LAPACK's dsygvd on an explicit
  Cholesky-reduced problem and (b) the brute-force Jacobi on that reduction.
* X^T B X = I; a block spanning an invariant subspace gives exact eigenvalues.
* Lemma A.4: ||R|| <= 2 ||H|| sin(angle) for the standard problem.
* A rank-deficient block triggers the SVQB reading and still returns the
  correct Ritz values on the non-degenerate part.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import angles, filters, jacobi, rr


def _sym(rng, lam):
    Q, _ = np.linalg.qr(rng.standard_normal((len(lam), len(lam))))
    return Q, 0.5 * ((Q * lam) @ Q.T + ((Q * lam) @ Q.T).T)


@pytest.mark.parametrize("n", [2, 5, 17, 33])
def test_jacobi_prescribed_spectrum(rng, n):
    lam = np.sort(rng.uniform(-3, 7, n))
    _, A = _sym(rng, lam)
    w, V = jacobi.jacobi_eigh(A)
    np.testing.assert_allclose(w, lam, atol=1e-12 * max(1, np.abs(lam).max()))
    np.testing.assert_allclose(V.T @ V, np.eye(n), atol=1e-13)
    np.testing.assert_allclose((V * w) @ V.T, A, atol=1e-12)


def test_rr_matches_lapack_and_jacobi(rng):
    n, b = 90, 12
    _, A = _sym(rng, rng.uniform(-2, 9, n))
    G = rng.standard_normal((n, n))
    B = G @ G.T / n + np.eye(n)
    Y = rng.standard_normal((n, b))
    out = rr.rayleigh_ritz(Y, filters.dense_op(A), filters.dense_op(B))
    # (a) explicit reduction and LAPACK
    Ga, Gb = Y.T @ A @ Y, Y.T @ B @ Y
    L = np.linalg.cholesky(0.5 * (Gb + Gb.T))
    Hs = np.linalg.solve(L, np.linalg.solve(L, 0.5 * (Ga + Ga.T)).T)
    wl = sla.eigvalsh(0.5 * (Hs + Hs.T))
    # (b) brute-force Jacobi on the same reduction
    wj, _ = jacobi.jacobi_eigh(0.5 * (Hs + Hs.T))
    np.testing.assert_allclose(out["lam"], wl, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(out["lam"], wj, rtol=1e-10, atol=1e-12)
    X = out["X"]
    np.testing.assert_allclose(X.T @ B @ X, np.eye(b), atol=1e-10)
    R = A @ X - (B @ X) * out["lam"][None, :]
    np.testing.assert_allclose(out["resnorm"], np.linalg.norm(R, axis=0), rtol=1e-8, atol=1e-12)


def test_rr_invariant_subspace_exact(rng):
    n, b = 70, 9
    lam = np.sort(rng.uniform(-1, 5, n))
    Q, A = _sym(rng, lam)
    Y = Q[:, :b] @ rng.standard_normal((b, b))
    out = rr.rayleigh_ritz(Y, filters.dense_op(A), filters.identity_op())
    np.testing.assert_allclose(out["lam"], lam[:b], atol=1e-12)
    assert out["resnorm"].max() < 1e-11


def test_lemma_a4_residual_angle(rng):
    n, b = 120, 8
    lam = np.sort(rng.uniform(-1, 5, n))
    Q, A = _sym(rng, lam)
    normH = np.abs(lam).max()
    for delta in (1e-1, 1e-3, 1e-6):
        Y = Q[:, :b] + delta * rng.standard_normal((n, b))
        out = rr.rayleigh_ritz(Y, filters.dense_op(A), filters.identity_op())
        sin_t = np.sin(angles.max_principal_angle(Q[:, :b], out["X"]))
        assert np.linalg.norm(out["R"], 2) <= 2 * normH * sin_t * (1 + 1e-9) + 1e-13


def test_svqb_fallback_on_rank_deficient_block(rng):
    n, b = 60, 8
    lam = np.sort(rng.uniform(-1, 5, n))
    Q, A = _sym(rng, lam)
    Y = Q[:, :b].copy()
    Y[:, -1] = Y[:, 0]                     # exact duplicate column
    out = rr.rayleigh_ritz(Y, filters.dense_op(A), filters.identity_op())
    assert out["svqb"] and out["dropped"] == 1
    np.testing.assert_allclose(out["lam"], lam[: b - 1], atol=1e-11)


def test_svqb_fallback_on_numerically_singular_block(rng):
    """A column that differs from another by 1e-9 (relative): the scaled Gram
    matrix is positive definite in exact arithmetic, but its smallest
    eigenvalue (~1e-18) is below the 1e-14 drop tolerance, so the Cholesky
    pivot test takes the SVQB fallback, drops that one direction, and the kept
    span (an invariant subspace) gives the exact eigenvalues; a pivot above the
    tolerance keeps the Cholesky path."""
    n, b = 60, 8
    lam = np.sort(rng.uniform(-1, 5, n))
    Q, A = _sym(rng, lam)
    Y = Q[:, :b].copy()
    Y[:, -1] = Y[:, 0] + 1e-9 * Q[:, b]
    out = rr.rayleigh_ritz(Y, filters.dense_op(A), filters.identity_op())
    assert out["svqb"] and out["dropped"] == 1
    np.testing.assert_allclose(out["lam"], lam[: b - 1], atol=1e-11)
    Y[:, -1] = Y[:, 0] + 1e-5 * Q[:, b]      # smallest eigenvalue ~5e-11: Cholesky
    out = rr.rayleigh_ritz(Y, filters.dense_op(A), filters.identity_op())
    assert not out["svqb"] and out["dropped"] == 0


def test_pencil_eigenvalues_shared_basis_and_jacobi(rng):
    """Full-space Rayleigh-Ritz = the pencil's spectrum: exact lam_j / b_j for a
    shared eigenbasis (the paper's generalized toy construction) and the
    brute-force Jacobi on an explicit Cholesky reduction."""
    import workloads as wl
    t = wl.toy_generalized(m=60, n=5, zeta=0.0, seed=3)
    w = rr.pencil_eigenvalues(t["A"], t["B"], 12)
    np.testing.assert_allclose(w, np.sort(t["lam_gen"])[:12], rtol=1e-12)
    A = t["A"] + 0.01 * wl.unit_sym_perturbation(rng, 60)
    L = np.linalg.cholesky(t["B"])
    H = np.linalg.solve(L, np.linalg.solve(L, A).T)
    wj, _ = jacobi.jacobi_eigh(0.5 * (H + H.T))
    np.testing.assert_allclose(rr.pencil_eigenvalues(A, t["B"], 10), wj[:10], rtol=1e-11)
