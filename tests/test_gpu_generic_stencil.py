"""GPU parity of the grid path for a 27-point stencil whose coefficients are
not class-symmetric, against the oracle.

The operator is an anisotropic tensor-product Laplacian (different weights
along x, y and z) with the mass-weighted Gaussian-well potential.  Its
coefficients do not depend on the number of non-zero offset components
alone, so the vectorised z-marching and separable kernels (which take that
four-class form) do not apply.  The products, the filter steps and, at a
wave vector k, the wrap correction after each step then run in the scalar
per-point kernels, which take every offset's own coefficient.  The oracle
applies the 27 coefficients as given, so a swapped axis or a mirrored offset
shows up as a mismatch.  Bars as for the class-symmetric grids: FP64 filters
to 1e-11, FP32 / BF16-stored residual filters within the residual part they
carry (Theorem 3.4), Rayleigh-Ritz Ritz values to 1e-11.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import filters, rr, stencil
from parity import GRID_TERMS, assert_columns, prec_name, residual_part

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402

LMAX = 18.5                       # above the spectrum of both pencils here
WEIGHTS = (1.3, 0.6, 1.0)         # stiffness weights along (z, y, x)
K = (0.3, -0.7, 1.1)              # (kx, ky, kz), radians per grid step
SHAPE = (5, 9, 12)                # (nz, ny, nx)


def _aniso_stiffness():
    K1, M1 = wl.stencil_coefficients_1d()
    t = lambda a, b, c: np.einsum("i,j,k->ijk", a, b, c)
    wz, wy, wx = WEIGHTS
    return 0.5 * (wz * t(K1, M1, M1) + wy * t(M1, K1, M1) + wx * t(M1, M1, K1))


def _problem(bloch=None, seed=8):
    V, _ = wl.gaussian_wells(SHAPE, 3, np.random.default_rng(seed))
    cA, cB = _aniso_stiffness(), wl.tensor_stencil_27("mass")
    if bloch is None:
        apply_A, apply_B = stencil.make_ops(cA, cB, V, SHAPE, 2)
    else:
        apply_A, apply_B = stencil.make_ops_bloch(cA, cB, V, SHAPE, 2, bloch)
    Vd = torch.from_numpy(np.ascontiguousarray(V).reshape(-1)).cuda()
    opA = P.stencil_operator(SHAPE, cA, coef_mass=cB, field=Vd, field_mode=2, bloch=bloch)
    opB = P.stencil_operator(SHAPE, cB, bloch=bloch)
    return apply_A, apply_B, opA, opB, Vd


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_stiffness_is_not_class_symmetric():
    """The case under test: offsets of one class carry different weights."""
    c = _aniso_stiffness()
    assert c[0, 1, 1] != c[1, 0, 1] != c[1, 1, 0]
    np.testing.assert_array_equal(c, c[::-1, ::-1, ::-1])      # c(o) = c(-o)


@pytest.mark.parametrize("bloch", [None, K], ids=["real", "bloch"])
@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_FP32, P.PREC_BF16])
def test_generic_residual_filter_matches_oracle(prec, bloch):
    apply_A, apply_B, opA, opB, Vd = _problem(bloch)
    n, b, deg = int(np.prod(SHAPE)), 8, 10
    cplx = bloch is not None
    prm = P.make_params(6, b, deg, method=P.METHOD_RCHFSI, filter_prec=prec, lambda_max=LMAX)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Y0 = wl.random_block_complex(n, b, 4) if cplx else wl.random_block(n, b, 4)
    o = rr.rayleigh_ritz(Y0, apply_A, apply_B)
    bounds = (o["lam"][0] - 0.5, LMAX, o["lam"][-1])
    to_cm = P.to_colmajor_complex if cplx else P.to_colmajor
    Y = P.colmajor_empty_complex(n, b) if cplx else P.colmajor_empty(n, b)
    print("generic stencil filter", "bloch" if cplx else "real", "prec", prec, flush=True)
    P.chfsi_filter(ctx, to_cm(o["X"]), o["lam"], to_cm(o["R"]), Y, *bounds, degree=deg)
    torch.cuda.synchronize()
    got = Y.cpu().numpy()
    ref, RYp, _ = filters.residual_filter(apply_A, filters.identity_op(), o["X"], o["lam"],
                                          o["R"], deg, *bounds, return_parts=True)
    assert np.all(np.isfinite(got))
    scale = np.linalg.norm(ref, axis=0) if prec == P.PREC_FP64 else residual_part(RYp)
    assert_columns(got, ref, scale, prec_name(prec), deg, GRID_TERMS, "generic stencil")


@pytest.mark.parametrize("bloch", [None, K], ids=["real", "bloch"])
def test_generic_rayleigh_ritz_matches_oracle(bloch):
    apply_A, apply_B, opA, opB, Vd = _problem(bloch, seed=9)
    n, b = int(np.prod(SHAPE)), 10
    cplx = bloch is not None
    prm = P.make_params(8, b, 4, method=P.METHOD_RCHFSI, lambda_max=LMAX)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Yh = wl.random_block_complex(n, b, 5) if cplx else wl.random_block(n, b, 5)
    empty = P.colmajor_empty_complex if cplx else P.colmajor_empty
    X, R = empty(n, b), empty(n, b)
    to_cm = P.to_colmajor_complex if cplx else P.to_colmajor
    print("generic stencil Rayleigh-Ritz", "bloch" if cplx else "real", flush=True)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, to_cm(Yh), X, R)
    o = rr.rayleigh_ritz(Yh, apply_A, apply_B)
    lam = np.array(ritz)
    assert np.max(np.abs(lam - o["lam"])) <= 1e-11 * np.max(np.abs(o["lam"]))
    Xg, Rg = X.cpu().numpy(), R.cpu().numpy()
    assert np.linalg.norm(Xg.conj().T @ apply_B(Xg) - np.eye(b)) <= 1e-10
    Rref = apply_A(Xg) - apply_B(Xg) * lam[None, :]
    assert np.linalg.norm(Rg - Rref) <= 1e-10 * LMAX
    np.testing.assert_allclose(norms, np.linalg.norm(Rref, axis=0), rtol=1e-7, atol=1e-12)
