"""Pins for the oracle on complex Hermitian problems (Section 4.3).

The complex code paths are tied to the already-pinned real oracle through the
real embedding of a Hermitian matrix, H = H_r + i H_i  <->  [[H_r, -H_i],
[H_i, H_r]] (real symmetric, twice the size): a complex block Z maps to
[Z_r; Z_i], complex products map to real products, and every eigenvalue of H
appears twice in the embedding.  Also: the generator's prescribed spectrum,
B-orthonormal Ritz vectors, exact Ritz values on an invariant subspace, and a
full R-ChFSI solve against LAPACK's Hermitian pencil solver.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import filters, rr, solver


def embed(H):
    return np.block([[H.real, -H.imag], [H.imag, H.real]])


def embed_block(Z):
    return np.concatenate([Z.real, Z.imag], axis=0)


@pytest.fixture(scope="module")
def herm():
    return wl.dense_hermitian(n=240, n_low=16, block=20, degree=10, seed=5)


def test_generator_spectrum_and_hermitian(herm):
    assert np.array_equal(herm.A, herm.A.conj().T)
    assert np.array_equal(herm.B, herm.B.conj().T)
    w = np.linalg.eigvalsh(herm.A)
    assert np.max(np.abs(w - np.sort(herm.lam_A))) <= 1e-12 * np.max(np.abs(herm.lam_A))


def test_filters_equal_real_embedding(herm):
    n, b = herm.n, herm.block
    rng = np.random.default_rng(2)
    X = wl.random_block_complex(n, b, 3)
    R = 1e-2 * wl.random_block_complex(n, b, 4)
    lam = np.sort(rng.uniform(-1.0, 0.0, b))
    bounds = (-1.2, 10.5, 0.3)
    Ae, de = embed(herm.A), np.concatenate([herm.dinv, herm.dinv])
    got = filters.residual_filter(filters.dense_op(herm.A), filters.diag_op(herm.dinv), X, lam, R,
                                  10, *bounds)
    ref = filters.residual_filter(filters.dense_op(Ae), filters.diag_op(de), embed_block(X), lam,
                                  embed_block(R), 10, *bounds)
    assert got.dtype == np.complex128
    assert np.linalg.norm(embed_block(got) - ref) <= 1e-13 * np.linalg.norm(ref)
    H = lambda V: herm.dinv[:, None] * (herm.A @ V)
    He = lambda V: de[:, None] * (Ae @ V)
    got = filters.chebyshev_filter(H, X, 10, *bounds)
    ref = filters.chebyshev_filter(He, embed_block(X), 10, *bounds)
    assert np.linalg.norm(embed_block(got) - ref) <= 1e-13 * np.linalg.norm(ref)


def test_rayleigh_ritz_complex(herm):
    n, b = herm.n, herm.block
    Y = wl.random_block_complex(n, b, 6)
    o = rr.rayleigh_ritz(Y, filters.dense_op(herm.A), filters.dense_op(herm.B))
    X = o["X"]
    assert np.linalg.norm(X.conj().T @ herm.B @ X - np.eye(b)) <= 1e-12
    assert np.allclose(o["R"], herm.A @ X - herm.B @ X * o["lam"][None, :], atol=1e-12)
    # the real embedding of span(Y) (2b real directions) has every Ritz value twice
    Ae, Be = embed(herm.A), embed(herm.B)
    Ye = np.concatenate([embed_block(Y), embed_block(1j * Y)], axis=1)
    oe = rr.rayleigh_ritz(Ye, filters.dense_op(Ae), filters.dense_op(Be))
    pairs = oe["lam"].reshape(-1, 2)
    assert np.max(np.abs(pairs[:, 0] - pairs[:, 1])) <= 1e-11
    assert np.max(np.abs(pairs[:, 0] - o["lam"])) <= 1e-11
    # invariant subspace: exact eigenvalues
    w, V = sla.eigh(herm.A, herm.B)
    Q = np.linalg.qr(np.random.default_rng(8).standard_normal((8, 8))
                     + 1j * np.random.default_rng(9).standard_normal((8, 8)))[0]
    o2 = rr.rayleigh_ritz(V[:, :8] @ Q, filters.dense_op(herm.A), filters.dense_op(herm.B))
    assert np.max(np.abs(o2["lam"] - w[:8])) <= 1e-12 * np.max(np.abs(w))


def test_rchfsi_solve_complex_generalized(herm):
    n, b, k = herm.n, herm.block, herm.n_wanted
    w = sla.eigh(herm.A, herm.B, eigvals_only=True)
    lmax = 10.0 / (0.95 * herm.meta["dmin"]) + 0.1
    out = solver.solve(filters.dense_op(herm.A), filters.dense_op(herm.B),
                       filters.diag_op(herm.dinv), wl.random_block_complex(n, b, 11), k,
                       herm.degree, 1e-10, 60, ("ritz", lmax))
    assert out["converged"]
    assert np.max(np.abs(out["lam"][:k] - w[:k])) <= 1e-10 * np.max(np.abs(w[:k]))
    assert out["X"].dtype == np.complex128
