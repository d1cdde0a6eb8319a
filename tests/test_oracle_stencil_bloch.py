"""Pins for the Bloch-phase (k-point) grid operators of the oracle (Section 4.3
applied to the grid pencil).

* k = 0 gives the real operators.
* The operators are Hermitian (v^H A u = (A v)^H u) for every field mode.
* With V = 0 the pencil (0.5 K(k), M(k)) has the closed-form eigenvalues
  sum_d 3 (1 - cos(t_d + k_d)) / (2 + cos(t_d + k_d)), t_d = 2 pi j_d / n_d:
  the Fourier symbol of the real pencil shifted by k.
* A(k) = D^* A_tw D with D = diag(exp(i k.r)) and A_tw the real stencil whose
  periodic wraps carry the twist exp(i s k_d n_d) (s = +-1 for a wrap up or
  down), built here independently by explicit index arithmetic.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import stencil


SHAPE = (5, 6, 7)          # (nz, ny, nx)
K = (0.3, -0.7, 1.1)       # (kx, ky, kz) radians per grid step


def _coefs():
    return 0.5 * wl.tensor_stencil_27("stiffness"), wl.tensor_stencil_27("mass")


def _field(seed=3):
    V, _ = wl.gaussian_wells(SHAPE, 2, np.random.default_rng(seed))
    return V


def _cvec(n, b, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal((n, b)) + 1j * r.standard_normal((n, b))


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_zero_k_is_the_real_operator(mode):
    cA, cB = _coefs()
    V = _field()
    n = int(np.prod(SHAPE))
    U = _cvec(n, 3, 1)
    A0, B0 = stencil.make_ops(cA, cB, V, SHAPE, mode)
    Ak, Bk = stencil.make_ops_bloch(cA, cB, V, SHAPE, mode, (0.0, 0.0, 0.0))
    ref = A0(U.real) + 1j * A0(U.imag)
    np.testing.assert_allclose(Ak(U), ref, rtol=0, atol=1e-13)
    np.testing.assert_allclose(Bk(U), B0(U.real) + 1j * B0(U.imag), rtol=0, atol=1e-13)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_bloch_operators_are_hermitian(mode):
    cA, cB = _coefs()
    Ak, Bk = stencil.make_ops_bloch(cA, cB, _field(), SHAPE, mode, K)
    n = int(np.prod(SHAPE))
    u, v = _cvec(n, 1, 2)[:, 0], _cvec(n, 1, 3)[:, 0]
    for op in (Ak, Bk):
        lhs = np.vdot(v, op(u))
        rhs = np.vdot(op(v), u)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_zero_potential_pencil_shifted_symbol():
    cA, cB = _coefs()
    nz, ny, nx = SHAPE
    n = nz * ny * nx
    Ak, Bk = stencil.make_ops_bloch(cA, cB, np.zeros(SHAPE), SHAPE, 2, K)
    I = np.eye(n)
    w = sla.eigvalsh(Ak(I), Bk(I))
    f = lambda t: 3 * (1 - np.cos(t)) / (2 + np.cos(t))
    fx = f(2 * np.pi * np.arange(nx) / nx + K[0])
    fy = f(2 * np.pi * np.arange(ny) / ny + K[1])
    fz = f(2 * np.pi * np.arange(nz) / nz + K[2])
    ref = np.sort((fz[:, None, None] + fy[None, :, None] + fx[None, None, :]).ravel())
    np.testing.assert_allclose(w, ref, atol=1e-11)


def _twisted(coef, u, shape, k):
    """Real stencil with twisted periodic wraps, by explicit index arithmetic."""
    nz, ny, nx = shape
    kv = {"x": k[0] * nx, "y": k[1] * ny, "z": k[2] * nz}
    out = np.zeros(nz * ny * nx, dtype=np.complex128)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                acc = 0.0
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            c = coef[dz + 1, dy + 1, dx + 1]
                            ph = 0.0
                            qx, qy, qz = x + dx, y + dy, z + dz
                            if qx < 0 or qx >= nx:
                                ph += (1 if qx >= nx else -1) * kv["x"]
                            if qy < 0 or qy >= ny:
                                ph += (1 if qy >= ny else -1) * kv["y"]
                            if qz < 0 or qz >= nz:
                                ph += (1 if qz >= nz else -1) * kv["z"]
                            q = (qx % nx) + nx * ((qy % ny) + ny * (qz % nz))
                            acc += c * np.exp(1j * ph) * u[q]
                out[x + nx * (y + ny * z)] = acc
    return out


def test_unitary_equivalence_to_twisted_wraps():
    cA, cB = _coefs()
    nz, ny, nx = SHAPE
    n = nz * ny * nx
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = np.exp(1j * (K[0] * x + K[1] * y + K[2] * z)).ravel()
    u = _cvec(n, 1, 4)[:, 0]
    for coef in (cA, cB):
        got = stencil.apply_stencil_bloch(coef, u, SHAPE, K)
        ref = phase.conj() * _twisted(coef, phase * u, SHAPE, K)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
