"""GPU parity of the periodic 27-point (grid pencil) path against the oracle.

The grids are ragged and carry the mass-weighted Gaussian-well potential.
Shapes (nz, ny, nx) cover the vectorised z-marching kernel with one y tile,
several y tiles with a ragged last one (ny = 20 over 16- and 8-row tiles),
rows that leave threads idle (nx = 40: 10 or 20 threads per row), block
widths that leave a partial column group, the filter-step kernels compiled
for rows of 128 and 160 points (with ragged last y tiles at every slab
height: 8/8/4 and 6/6/2 rows, or 4 and 3 rows for FP64), and the scalar
fallback (nx = 10, not a multiple of 4).  Filters are compared column by
column with the bounds of tests/parity.py: FP64 relative to the column,
FP32 / BF16-stored residual filters relative to the residual part each column
carries (Theorem 3.4); a small solve with BF16 storage reaches the eigenvalues
of the dense pencil.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import filters, rr, stencil
from parity import GRID_TERMS, assert_columns, prec_name, residual_part

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402


def _grid_problem(shape=(9, 10, 12), wells=3, seed=8, mode=2):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    V, _ = wl.gaussian_wells(shape, wells, rng)
    cA = 0.5 * wl.tensor_stencil_27("stiffness")
    cB = wl.tensor_stencil_27("mass")
    apply_A, apply_B = stencil.make_ops(cA, cB, V, shape, mode)
    return shape, cA, cB, V, apply_A, apply_B


def _ops(shape, cA, cB, V, mode=2):
    Vd = torch.from_numpy(np.ascontiguousarray(V).reshape(-1)).cuda()
    opA = P.stencil_operator(shape, cA, coef_mass=cB, field=Vd, field_mode=mode)
    opB = P.stencil_operator(shape, cB)
    return opA, opB, Vd


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


SHAPES = [(9, 10, 12), (5, 20, 64), (4, 30, 40), (6, 9, 10), (4, 20, 128), (3, 14, 160)]


@pytest.mark.parametrize("shape", SHAPES)
def test_plain_filter_fp64_matches_oracle(shape):
    shape, cA, cB, V, apply_A, apply_B = _grid_problem(shape=shape)
    n = int(np.prod(shape))
    b = 7
    opA, opB, Vd = _ops(shape, cA, cB, V)
    prm = P.make_params(5, b, 6, method=P.METHOD_CHFSI, filter_prec=P.PREC_FP64, lambda_max=18.5)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    X = wl.random_block(n, b, 3)
    Y = P.colmajor_empty(n, b)
    bounds = (-6.0, 18.5, 0.5)
    for deg in (1, 6):
        P.chfsi_filter(ctx, P.to_colmajor(X), None, None, Y, *bounds, degree=deg)
        torch.cuda.synchronize()
        ref = filters.chebyshev_filter(apply_A, X, deg, *bounds)   # D^{-1} = I
        assert_columns(Y.cpu().numpy(), ref, np.linalg.norm(ref, axis=0), "fp64", deg,
                       GRID_TERMS, f"grid {shape} chfsi")


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_FP32, P.PREC_BF16])
def test_residual_filter_matches_oracle(prec, shape):
    shape, cA, cB, V, apply_A, apply_B = _grid_problem(shape=shape)
    n = int(np.prod(shape))
    b = 9
    opA, opB, Vd = _ops(shape, cA, cB, V)
    prm = P.make_params(6, b, 10, method=P.METHOD_RCHFSI, filter_prec=prec, lambda_max=18.5)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    o = rr.rayleigh_ritz(wl.random_block(n, b, 4), apply_A, apply_B)
    bounds = (o["lam"][0] - 0.5, 18.5, o["lam"][-1])
    Y = P.colmajor_empty(n, b)
    P.chfsi_filter(ctx, P.to_colmajor(o["X"]), o["lam"], P.to_colmajor(o["R"]), Y, *bounds)
    torch.cuda.synchronize()
    ref, RYp, _ = filters.residual_filter(apply_A, filters.identity_op(), o["X"], o["lam"], o["R"],
                                          10, *bounds, return_parts=True)
    got = Y.cpu().numpy()
    scale = np.linalg.norm(ref, axis=0) if prec == P.PREC_FP64 else residual_part(RYp)
    assert_columns(got, ref, scale, prec_name(prec), 10, GRID_TERMS, f"grid {shape} rchfsi")


@pytest.mark.parametrize("shape", [(8, 9, 10), (5, 20, 64), (4, 30, 40)])
def test_rayleigh_ritz_with_mass_matrix(shape):
    shape, cA, cB, V, apply_A, apply_B = _grid_problem(shape=shape)
    n = int(np.prod(shape))
    b = 12
    opA, opB, Vd = _ops(shape, cA, cB, V)
    prm = P.make_params(8, b, 4, lambda_max=18.5)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Y = wl.random_block(n, b, 5)
    Xd, Rd = P.colmajor_empty(n, b), P.colmajor_empty(n, b)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, P.to_colmajor(Y), Xd, Rd)
    o = rr.rayleigh_ritz(Y, apply_A, apply_B)
    np.testing.assert_allclose(ritz, o["lam"], atol=1e-11 * np.abs(o["lam"]).max())
    np.testing.assert_allclose(norms, o["resnorm"], rtol=1e-7)
    X = Xd.cpu().numpy()
    np.testing.assert_allclose(X.T @ apply_B(X), np.eye(b), atol=1e-10)


@pytest.mark.parametrize("memory_mode", [0, 1])
def test_rayleigh_ritz_wide_block(memory_mode):
    """b = 300: lower-panel Gram products (several panels, ragged last one)
    and, for grid operators, the residual as one stencil pass over X."""
    shape, cA, cB, V, apply_A, apply_B = _grid_problem(shape=(5, 20, 64), wells=3, seed=11)
    n = int(np.prod(shape))
    b = 300
    opA, opB, Vd = _ops(shape, cA, cB, V)
    prm = P.make_params(200, b, 6, method=P.METHOD_RCHFSI, filter_prec=P.PREC_BF16,
                        lambda_max=18.5, memory_mode=memory_mode)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Y = wl.random_block(n, b, 12)
    Xd, Rd = P.colmajor_empty(n, b), P.colmajor_empty(n, b)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, P.to_colmajor(Y), Xd, Rd)
    o = rr.rayleigh_ritz(Y, apply_A, apply_B)
    np.testing.assert_allclose(ritz, o["lam"], atol=1e-11 * np.abs(o["lam"]).max())
    np.testing.assert_allclose(norms, o["resnorm"], rtol=1e-7)
    X = Xd.cpu().numpy()
    np.testing.assert_allclose(X.T @ apply_B(X), np.eye(b), atol=1e-10)
    np.testing.assert_allclose(Rd.cpu().numpy(), apply_A(X) - apply_B(X) * np.asarray(ritz)[None, :],
                               atol=1e-11)


def test_rayleigh_ritz_gram_kernel_block_1100():
    """b = 1100 on a 24 x 28 x 32 grid (n = 21504 = 168 x 128): the Gram
    matrices Y^T A Y and Y^T B Y take the 256 x 128 long-reduction kernel (29
    lower tiles, eight k-ranges, ragged last row and column of tiles); Ritz
    values, residual norms and X^T B X = I against the oracle."""
    shape, cA, cB, V, apply_A, apply_B = _grid_problem(shape=(24, 28, 32), wells=4, seed=13)
    n = int(np.prod(shape))
    b = 1100
    opA, opB, Vd = _ops(shape, cA, cB, V)
    prm = P.make_params(900, b, 6, method=P.METHOD_RCHFSI, filter_prec=P.PREC_BF16,
                        lambda_max=18.5)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Y = wl.random_block(n, b, 14)
    Xd, Rd = P.colmajor_empty(n, b), P.colmajor_empty(n, b)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, P.to_colmajor(Y), Xd, Rd)
    o = rr.rayleigh_ritz(Y, apply_A, apply_B)
    np.testing.assert_allclose(ritz, o["lam"], atol=1e-11 * np.abs(o["lam"]).max())
    np.testing.assert_allclose(norms, o["resnorm"], rtol=1e-7)
    X = Xd.cpu().numpy()
    cols = np.arange(0, b, 37)
    np.testing.assert_allclose(X[:, cols].T @ apply_B(X[:, cols]), np.eye(len(cols)), atol=1e-10)


@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_BF16])
def test_small_grid_solve(prec):
    shape, cA, cB, V, apply_A, apply_B = _grid_problem(shape=(8, 8, 8), wells=2, seed=5)
    n = 512
    I = np.eye(n)
    w = sla.eigvalsh(apply_A(I), apply_B(I))
    opA, opB, Vd = _ops(shape, cA, cB, V)
    prm = P.make_params(6, 8, 8, max_iter=200, tol=1e-9, method=P.METHOD_RCHFSI,
                        filter_prec=prec, lambda_max=18.1)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Xd = P.to_colmajor(wl.random_block(n, 8, 31))
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    print(prec, rep["iterations"], rep["max_residual"])
    assert st == P.OK
    np.testing.assert_allclose(ev[:6], w[:6], rtol=1e-9, atol=1e-10)
    X = Xd.cpu().numpy()
    res = np.linalg.norm(apply_A(X[:, :6]) - apply_B(X[:, :6]) * np.asarray(ev[:6])[None, :], axis=0)
    assert res.max() <= 1e-9 * 1.01


@pytest.mark.parametrize("shape", [(16, 10, 12), (6, 20, 64)])
def test_slab_wise_rayleigh_ritz_matches_oracle(shape):
    """memory_mode 1: Gram matrices accumulated over z-slabs, in-place rotation,
    fused residual -- same Ritz pairs as the oracle."""
    shape, cA, cB, V, apply_A, apply_B = _grid_problem(shape=shape, wells=3, seed=9)
    n = int(np.prod(shape))
    b = 10
    opA, opB, Vd = _ops(shape, cA, cB, V)
    prm = P.make_params(8, b, 6, method=P.METHOD_RCHFSI, filter_prec=P.PREC_BF16,
                        lambda_max=18.5, memory_mode=1)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Y = wl.random_block(n, b, 6)
    Xd, Rd = P.colmajor_empty(n, b), P.colmajor_empty(n, b)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, P.to_colmajor(Y), Xd, Rd)
    o = rr.rayleigh_ritz(Y, apply_A, apply_B)
    np.testing.assert_allclose(ritz, o["lam"], atol=1e-11 * np.abs(o["lam"]).max())
    np.testing.assert_allclose(norms, o["resnorm"], rtol=1e-7)
    X = Xd.cpu().numpy()
    np.testing.assert_allclose(Rd.cpu().numpy(), apply_A(X) - apply_B(X) * np.asarray(ritz)[None, :],
                               atol=1e-11)


def test_slab_wise_solve_bf16():
    shape, cA, cB, V, apply_A, apply_B = _grid_problem(shape=(8, 8, 8), wells=2, seed=5)
    n = 512
    I = np.eye(n)
    w = sla.eigvalsh(apply_A(I), apply_B(I))
    opA, opB, Vd = _ops(shape, cA, cB, V)
    prm = P.make_params(6, 8, 8, max_iter=200, tol=1e-9, method=P.METHOD_RCHFSI,
                        filter_prec=P.PREC_BF16, lambda_max=18.1, memory_mode=1)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Xd = P.to_colmajor(wl.random_block(n, 8, 31))
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    assert st == P.OK
    np.testing.assert_allclose(ev[:6], w[:6], rtol=1e-9, atol=1e-10)
