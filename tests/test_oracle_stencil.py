"""Pins for oracle.stencil (periodic 27-point grid pencil).

* The rolled 27-point application equals the explicit Kronecker product of 1D
  periodic (circulant) stiffness and mass matrices.
* The generated class coefficients equal the closed forms in
  tests/golden/stencil_symbols.json.
* With V = 0 the pencil's eigenvalues equal the Fourier-symbol closed form
  sum_d 3 (1 - cos t_d) / (2 + cos t_d).
* The mass-weighted potential (reading R2) is symmetric and reduces to diag(V)
  when the mass matrix is lumped to its row sums.
"""
import json
import os

import numpy as np
import scipy.linalg as sla

import workloads as wl
from oracle import stencil

GOLD = os.path.join(os.path.dirname(__file__), "golden", "stencil_symbols.json")


def _kron_ops(shape):
    nz, ny, nx = shape
    K1, M1 = wl.stencil_coefficients_1d()
    Kx, Ky, Kz = (stencil.circulant_1d(K1, n) for n in (nx, ny, nz))
    Mx, My, Mz = (stencil.circulant_1d(M1, n) for n in (nx, ny, nz))
    # index x + nx*(y + ny*z): kron(z-part, y-part, x-part)
    K = np.kron(Kz, np.kron(My, Mx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Mz, np.kron(My, Kx))
    M = np.kron(Mz, np.kron(My, Mx))
    return K, M


def test_stencil_equals_kronecker(rng):
    shape = (4, 5, 6)
    K, M = _kron_ops(shape)
    U = rng.standard_normal((K.shape[0], 3))
    np.testing.assert_allclose(stencil.apply_stencil(wl.tensor_stencil_27("stiffness"), U, shape),
                               K @ U, atol=1e-13)
    np.testing.assert_allclose(stencil.apply_stencil(wl.tensor_stencil_27("mass"), U, shape),
                               M @ U, atol=1e-13)


def test_class_coefficients_golden():
    g = json.load(open(GOLD))
    for kind, key in (("mass", "mass_class_coefficients"), ("stiffness", "stiffness_class_coefficients")):
        c = wl.tensor_stencil_27(kind)
        for cls in range(4):
            for idx in np.ndindex(3, 3, 3):
                if sum(abs(i - 1) for i in idx) == cls:
                    assert abs(c[idx] - g[key][cls]) < 1e-15
    assert abs(wl.tensor_stencil_27("mass").sum() - g["mass_row_sum"]) < 1e-15
    assert abs(wl.tensor_stencil_27("stiffness").sum() - g["stiffness_row_sum"]) < 1e-14


def test_zero_potential_pencil_closed_form():
    shape = (6, 6, 6)
    N = 216
    cA = 0.5 * wl.tensor_stencil_27("stiffness")
    cB = wl.tensor_stencil_27("mass")
    apply_A, apply_B = stencil.make_ops(cA, cB, np.zeros(shape), shape, 2)
    I = np.eye(N)
    A = apply_A(I)
    B = apply_B(I)
    w = sla.eigvalsh(A, B)
    t = 2 * np.pi * np.arange(6) / 6
    f = 3 * (1 - np.cos(t)) / (2 + np.cos(t))
    ref = np.sort((f[:, None, None] + f[None, :, None] + f[None, None, :]).ravel())
    np.testing.assert_allclose(w, ref, atol=1e-11)
    g = json.load(open(GOLD))
    assert abs(ref.max() - g["pencil_max_half_stiffness_over_mass"]) < 1e-12


def test_mass_weighted_potential(rng):
    shape = (4, 4, 5)
    N = 80
    V = rng.uniform(-3, 0, shape)
    cB = wl.tensor_stencil_27("mass")
    zero = np.zeros((3, 3, 3))
    apply_A2, apply_B = stencil.make_ops(zero, cB, V, shape, 2)
    apply_A1, _ = stencil.make_ops(zero, cB, V, shape, 1)
    P2 = apply_A2(np.eye(N))
    np.testing.assert_allclose(P2, P2.T, atol=1e-14)
    # lumping M to its row sums (all ones) maps 1/2 (diag(V) M + M diag(V)) to diag(V)
    Mrow = apply_B(np.ones(N))
    np.testing.assert_allclose(Mrow, 1.0, atol=1e-14)
    P1 = apply_A1(np.eye(N))
    np.testing.assert_allclose(P1, np.diag(V.reshape(-1)), atol=1e-15)
    lumped = 0.5 * (np.diag(V.reshape(-1)) @ np.diag(Mrow) + np.diag(Mrow) @ np.diag(V.reshape(-1)))
    np.testing.assert_allclose(lumped, P1, atol=1e-14)
