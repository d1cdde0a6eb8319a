"""Pins for oracle.bounds (k-step Lanczos estimates of the spectrum of B^{-1} A).

* A full-length run on a diagonal pencil spans the whole space: the Ritz
  values are the pencil's eigenvalues d_i / m_i and the last beta vanishes.
* Courant-Fischer: the Ritz values lie inside [lambda_min, lambda_max] of the
  pencil (dense eigh), and the safeguarded estimates enclose the spectrum,
  on the dense generalized recipe, a complex Hermitian pencil and the grid
  pencil with and without wells.
* The grid pencil without a potential has lambda_max(B^{-1} A) = 18 exactly:
  the largest ratio of the Fourier symbols 0.5 K^ / M^ of the 27-point Q1
  stiffness and mass stencils, reached at theta = (pi, pi, pi) on even grids.
"""
import numpy as np
import scipy.linalg as sla

import workloads as wl
from oracle import bounds, stencil


def _dense_ops(A, B):
    cf = sla.cho_factor(B)
    return (lambda x: A @ x), (lambda x: B @ x), (lambda y: sla.cho_solve(cf, y))


def test_full_run_on_diagonal_pencil_returns_its_eigenvalues():
    rng = np.random.default_rng(3)
    a = np.array([-3.0, -1.0, 0.5, 2.0, 4.0, 7.5, 9.0, 12.0])
    m = rng.uniform(0.5, 2.0, 8)
    A, B = np.diag(a), np.diag(m)
    r = bounds.lanczos_bounds(*_dense_ops(A, B), np.ones(8), steps=8)
    np.testing.assert_allclose(r["theta"], np.sort(a / m), rtol=1e-12, atol=1e-12)
    assert r["beta_last"] < 1e-10 * np.abs(a / m).max()
    assert abs(r["upper"] - (a / m).max()) < 1e-10


def test_estimates_enclose_the_dense_generalized_spectrum():
    p = wl.dense_generalized(n=400, n_low=20, block=24, degree=12, seed=7)
    w = sla.eigvalsh(p.A, p.B)
    v0 = wl.random_block(p.n, 1, 11)[:, 0]
    for steps in (6, 12, 24):
        r = bounds.lanczos_bounds(*_dense_ops(p.A, p.B), v0, steps)
        tol = 1e-10 * np.abs(w).max()
        assert w[0] - tol <= r["theta"][0] and r["theta"][-1] <= w[-1] + tol
        assert r["upper"] >= w[-1] and r["lower"] <= w[0]
    # more steps bring the top Ritz value closer to lambda_max
    r6 = bounds.lanczos_bounds(*_dense_ops(p.A, p.B), v0, 6)
    r24 = bounds.lanczos_bounds(*_dense_ops(p.A, p.B), v0, 24)
    assert w[-1] - r24["theta"][-1] <= w[-1] - r6["theta"][-1] + 1e-12


def test_estimates_enclose_a_complex_hermitian_spectrum():
    rng = np.random.default_rng(5)
    n = 60
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = 0.5 * (G + G.conj().T)
    H = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = np.eye(n) + 0.02 * (H @ H.conj().T)
    w = sla.eigvalsh(A, B)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    r = bounds.lanczos_bounds(*_dense_ops(A, B), v0, 20)
    tol = 1e-10 * np.abs(w).max()
    assert w[0] - tol <= r["theta"][0] and r["theta"][-1] <= w[-1] + tol
    assert r["upper"] >= w[-1] and r["lower"] <= w[0]
    full = bounds.lanczos_bounds(*_dense_ops(A, B), v0, n)
    assert abs(full["theta"][-1] - w[-1]) < 1e-8 * np.abs(w).max()


def _grid(shape, wells, seed):
    rng = np.random.default_rng(seed)
    V = wl.gaussian_wells(shape, wells, rng)[0] if wells else np.zeros(shape)
    cA = 0.5 * wl.tensor_stencil_27("stiffness")
    cB = wl.tensor_stencil_27("mass")
    apply_A, apply_B = stencil.make_ops(cA, cB, V, shape, 2)
    n = int(np.prod(shape))
    I = np.eye(n)
    Am, Bm = apply_A(I), apply_B(I)
    return 0.5 * (Am + Am.T), 0.5 * (Bm + Bm.T)


def test_grid_pencil_without_potential_tops_out_at_18():
    A, B = _grid((8, 8, 8), 0, 1)
    w = sla.eigvalsh(A, B)
    assert abs(w[-1] - 18.0) < 1e-10
    v0 = wl.random_block(A.shape[0], 1, 12)[:, 0]
    r = bounds.lanczos_bounds(*_dense_ops(A, B), v0, 12)
    assert r["theta"][-1] <= 18.0 + 1e-10 and r["upper"] >= 18.0


def test_estimates_enclose_the_grid_pencil_with_wells():
    A, B = _grid((8, 6, 10), 2, 4)
    w = sla.eigvalsh(A, B)
    v0 = wl.random_block(A.shape[0], 1, 13)[:, 0]
    r = bounds.lanczos_bounds(*_dense_ops(A, B), v0, 12)
    tol = 1e-10 * np.abs(w).max()
    assert w[0] - tol <= r["theta"][0] and r["theta"][-1] <= w[-1] + tol
    assert r["upper"] >= w[-1] and r["lower"] <= w[0]
