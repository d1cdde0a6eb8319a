"""GPU parity of the grid path on the smallest grids the library accepts
(three points along every axis), real and at a Bloch wave vector, against
the oracle.

On such grids every wrap is also a nearest neighbour of the other face:
with n_d = 3 the points x - 1 and x + 1 of an edge point are the two other
points of the row.  The boundary of the twisted-frame correction is every
point but (n_x - 2)(n_y - 2)(n_z - 2) of them, and one inner row holds only
the two x-face points.  The shapes reach the separable kernel (n_x = 3, and
n_x = 4 for FP32 / BF16), the z-march with two threads per row (n_x = 4 in
FP64, n_x = 8) and two inner planes (n_z = 4).  Bars as for the other grids:
FP64 filters to 1e-11, FP32 / BF16-stored residual filters within the
residual part they carry (Theorem 3.4), Rayleigh-Ritz Ritz values to 1e-11.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import filters, rr, stencil
from parity import GRID_TERMS, assert_columns, prec_name, residual_part

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402

LMAX = 18.5
K = (0.3, -0.7, 1.1)              # (kx, ky, kz), radians per grid step
SHAPES = [(3, 3, 3), (3, 3, 4), (3, 3, 8), (4, 3, 8), (3, 4, 4)]     # (nz, ny, nx)


def _problem(shape, bloch, seed=8):
    V, _ = wl.gaussian_wells(shape, 1, np.random.default_rng(seed))
    cA, cB = 0.5 * wl.tensor_stencil_27("stiffness"), wl.tensor_stencil_27("mass")
    if bloch is None:
        apply_A, apply_B = stencil.make_ops(cA, cB, V, shape, 2)
    else:
        apply_A, apply_B = stencil.make_ops_bloch(cA, cB, V, shape, 2, bloch)
    Vd = torch.from_numpy(np.ascontiguousarray(V).reshape(-1)).cuda()
    opA = P.stencil_operator(shape, cA, coef_mass=cB, field=Vd, field_mode=2, bloch=bloch)
    opB = P.stencil_operator(shape, cB, bloch=bloch)
    return apply_A, apply_B, opA, opB, Vd


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bloch", [None, K], ids=["real", "bloch"])
@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_FP32, P.PREC_BF16])
def test_min_grid_residual_filter_matches_oracle(prec, bloch, shape):
    apply_A, apply_B, opA, opB, Vd = _problem(shape, bloch)
    n, b, deg = int(np.prod(shape)), 4, 10
    cplx = bloch is not None
    prm = P.make_params(3, b, deg, method=P.METHOD_RCHFSI, filter_prec=prec, lambda_max=LMAX)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Y0 = wl.random_block_complex(n, b, 4) if cplx else wl.random_block(n, b, 4)
    o = rr.rayleigh_ritz(Y0, apply_A, apply_B)
    bounds = (o["lam"][0] - 0.5, LMAX, o["lam"][-1])
    to_cm = P.to_colmajor_complex if cplx else P.to_colmajor
    Y = P.colmajor_empty_complex(n, b) if cplx else P.colmajor_empty(n, b)
    print("min grid filter", shape, "bloch" if cplx else "real", "prec", prec, flush=True)
    P.chfsi_filter(ctx, to_cm(o["X"]), o["lam"], to_cm(o["R"]), Y, *bounds, degree=deg)
    torch.cuda.synchronize()
    got = Y.cpu().numpy()
    ref, RYp, _ = filters.residual_filter(apply_A, filters.identity_op(), o["X"], o["lam"],
                                          o["R"], deg, *bounds, return_parts=True)
    assert np.all(np.isfinite(got))
    scale = np.linalg.norm(ref, axis=0) if prec == P.PREC_FP64 else residual_part(RYp)
    assert_columns(got, ref, scale, prec_name(prec), deg, GRID_TERMS, "min grid")


@pytest.mark.parametrize("shape", [(3, 3, 3), (3, 3, 8)])
@pytest.mark.parametrize("bloch", [None, K], ids=["real", "bloch"])
def test_min_grid_rayleigh_ritz_matches_oracle(bloch, shape):
    apply_A, apply_B, opA, opB, Vd = _problem(shape, bloch, seed=9)
    n, b = int(np.prod(shape)), 6
    cplx = bloch is not None
    prm = P.make_params(4, b, 4, method=P.METHOD_RCHFSI, lambda_max=LMAX)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Yh = wl.random_block_complex(n, b, 5) if cplx else wl.random_block(n, b, 5)
    empty = P.colmajor_empty_complex if cplx else P.colmajor_empty
    X, R = empty(n, b), empty(n, b)
    to_cm = P.to_colmajor_complex if cplx else P.to_colmajor
    print("min grid Rayleigh-Ritz", shape, "bloch" if cplx else "real", flush=True)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, to_cm(Yh), X, R)
    o = rr.rayleigh_ritz(Yh, apply_A, apply_B)
    lam = np.array(ritz)
    assert np.max(np.abs(lam - o["lam"])) <= 1e-11 * np.max(np.abs(o["lam"]))
    Xg, Rg = X.cpu().numpy(), R.cpu().numpy()
    assert np.linalg.norm(Xg.conj().T @ apply_B(Xg) - np.eye(b)) <= 1e-10
    Rref = apply_A(Xg) - apply_B(Xg) * lam[None, :]
    assert np.linalg.norm(Rg - Rref) <= 1e-10 * LMAX
    np.testing.assert_allclose(norms, np.linalg.norm(Rref, axis=0), rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("shape", [(3, 3, 8), (5, 20, 64)])
@pytest.mark.parametrize("bloch", [None, K], ids=["real", "bloch"])
@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_FP32, P.PREC_BF16])
def test_single_vector_filter_and_rayleigh_ritz(prec, bloch, shape):
    """A block of one vector (one column, or one planar pair at a wave vector):
    every column group of the kernels but the first is idle."""
    apply_A, apply_B, opA, opB, Vd = _problem(shape, bloch, seed=10)
    n, b, deg = int(np.prod(shape)), 1, 10
    cplx = bloch is not None
    prm = P.make_params(1, b, deg, method=P.METHOD_RCHFSI, filter_prec=prec, lambda_max=LMAX)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Y0 = wl.random_block_complex(n, b, 6) if cplx else wl.random_block(n, b, 6)
    to_cm = P.to_colmajor_complex if cplx else P.to_colmajor
    empty = P.colmajor_empty_complex if cplx else P.colmajor_empty
    print("single vector", shape, "bloch" if cplx else "real", "prec", prec, flush=True)
    X, R = empty(n, b), empty(n, b)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, to_cm(Y0), X, R)
    o = rr.rayleigh_ritz(Y0, apply_A, apply_B)
    assert abs(ritz[0] - o["lam"][0]) <= 1e-11 * max(abs(o["lam"][0]), 1.0)
    np.testing.assert_allclose(norms, o["resnorm"], rtol=1e-7)
    bounds = (o["lam"][0] - 0.5, LMAX, o["lam"][0] + 0.5)
    Y = empty(n, b)
    P.chfsi_filter(ctx, to_cm(o["X"]), o["lam"], to_cm(o["R"]), Y, *bounds, degree=deg)
    torch.cuda.synchronize()
    got = Y.cpu().numpy()
    ref, RYp, _ = filters.residual_filter(apply_A, filters.identity_op(), o["X"], o["lam"],
                                          o["R"], deg, *bounds, return_parts=True)
    scale = np.linalg.norm(ref, axis=0) if prec == P.PREC_FP64 else residual_part(RYp)
    assert_columns(got, ref, scale, prec_name(prec), deg, GRID_TERMS, "min grid")
