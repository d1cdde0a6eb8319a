"""GPU parity of sparse (CSR) operators (CHFSI_OP_CSR) against the oracle.

Pencils: the 27-point grid pencil with the mass-weighted potential assembled
as CSR (27 entries per row, a ragged last row tile), a random symmetric
sparse pencil with an SPD sparse B (irregular rows), and the same with rows
longer than the LDS-staged kernel takes (the plain kernel).  The oracle
applies the same CSR matrices with scipy.  Filters are compared column by
column with the bounds of tests/parity.py (K = the longest row), Rayleigh-Ritz
by its Ritz values and residuals, the CSR path against the grid (stencil)
path on the same pencil, and full solves against LAPACK's eigenvalues.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import filters, rr
from parity import assert_columns, prec_name, residual_part

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402


def _dev_csr(M):
    rp = torch.from_numpy(M.indptr.astype(np.int64)).cuda()
    ci = torch.from_numpy(M.indices.astype(np.int32)).cuda()
    va = torch.from_numpy(M.data.astype(np.float64)).cuda()
    return P.csr_operator(M.shape[0], rp, ci, va), (rp, ci, va)


def _grid(shape=(9, 10, 12), wells=3, seed=8):
    rng = np.random.default_rng(seed)
    V, _ = wl.gaussian_wells(shape, wells, rng)
    cA = 0.5 * wl.tensor_stencil_27("stiffness")
    cB = wl.tensor_stencil_27("mass")
    A, B = wl.grid_pencil_csr(shape, cA, cB, V, 2)
    return A, B, None, (shape, cA, cB, V)


def _problem(kind):
    if kind == "grid":
        return _grid()
    if kind == "random":
        A, B, dinv = wl.random_sparse_pencil(700, 8, 0, 0, 5)
        return A, B, dinv, None
    A, B, dinv = wl.random_sparse_pencil(700, 8, 4, 120, 6)      # rows > 80: plain kernel
    return A, B, dinv, None


def _ctx(A, B, dinv, params):
    opA, kA = _dev_csr(A)
    opB, kB = _dev_csr(B)
    d = torch.from_numpy(dinv).cuda() if dinv is not None else None
    return P.chfsi_create(opA, opB, d, params, keep=kA + kB + (d,))


def _spectrum(A, B):
    return sla.eigvalsh(A.toarray(), B.toarray())


KINDS = ["grid", "random", "long_rows"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_FP32, P.PREC_BF16])
def test_csr_residual_filter_matches_oracle(kind, prec):
    A, B, dinv, _ = _problem(kind)
    n, b, deg = A.shape[0], 12, 10
    w = _spectrum(A, B)
    bounds = (float(w[0]) - 0.1, float(w[-1]) + 0.5, float(w[b + 4]))
    prm = P.make_params(8, b, deg, method=P.METHOD_RCHFSI, filter_prec=prec,
                        lambda_max=bounds[1])
    ctx = _ctx(A, B, dinv, prm)
    opA = lambda V: A @ V                                        # noqa: E731
    opB = lambda V: B @ V                                        # noqa: E731
    Dop = filters.diag_op(dinv) if dinv is not None else filters.identity_op()
    o = rr.rayleigh_ritz(wl.random_block(n, b, 3), opA, opB)
    Y = P.colmajor_empty(n, b)
    P.chfsi_filter(ctx, P.to_colmajor(o["X"]), o["lam"], P.to_colmajor(o["R"]), Y, *bounds,
                   degree=deg)
    torch.cuda.synchronize()
    ref, RYp, _ = filters.residual_filter(opA, Dop, o["X"], o["lam"], o["R"], deg, *bounds,
                                          return_parts=True)
    kmax = int(np.diff(A.indptr).max())
    pn = prec_name(prec)
    scale = np.linalg.norm(ref, axis=0) if pn == "fp64" else residual_part(RYp, dinv)
    assert_columns(Y.cpu().numpy(), ref, scale, pn, deg, kmax, f"csr {kind}")


@pytest.mark.parametrize("kind", KINDS)
def test_csr_plain_filter_fp64_matches_oracle(kind):
    A, B, dinv, _ = _problem(kind)
    n, b = A.shape[0], 7
    w = _spectrum(A, B)
    bounds = (float(w[0]) - 0.1, float(w[-1]) + 0.5, float(w[b + 4]))
    prm = P.make_params(5, b, 6, method=P.METHOD_CHFSI, filter_prec=P.PREC_FP64,
                        lambda_max=bounds[1])
    ctx = _ctx(A, B, dinv, prm)
    X = wl.random_block(n, b, 4)
    Y = P.colmajor_empty(n, b)
    d = dinv if dinv is not None else np.ones(n)
    for deg in (1, 6):
        P.chfsi_filter(ctx, P.to_colmajor(X), None, None, Y, *bounds, degree=deg)
        torch.cuda.synchronize()
        ref = filters.chebyshev_filter(lambda V: d[:, None] * (A @ V), X, deg, *bounds)
        assert_columns(Y.cpu().numpy(), ref, np.linalg.norm(ref, axis=0), "fp64", deg,
                       int(np.diff(A.indptr).max()), f"csr {kind} plain")


@pytest.mark.parametrize("kind", KINDS)
def test_csr_rayleigh_ritz_matches_oracle(kind):
    A, B, dinv, _ = _problem(kind)
    n, b = A.shape[0], 16
    prm = P.make_params(10, b, 4, lambda_max=100.0)
    ctx = _ctx(A, B, dinv, prm)
    Yh = wl.random_block(n, b, 6)
    Xd, Rd = P.colmajor_empty(n, b), P.colmajor_empty(n, b)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, P.to_colmajor(Yh), Xd, Rd)
    o = rr.rayleigh_ritz(Yh, lambda V: A @ V, lambda V: B @ V)
    scale = np.abs(o["lam"]).max()
    np.testing.assert_allclose(ritz, o["lam"], atol=1e-11 * scale)
    np.testing.assert_allclose(norms, o["resnorm"], rtol=1e-8, atol=1e-11 * scale)
    X = Xd.cpu().numpy()
    np.testing.assert_allclose(X.T @ (B @ X), np.eye(b), atol=1e-10)


def test_csr_path_matches_grid_path():
    """The same grid pencil as a 27-point stencil operator and as CSR: the FP64
    residual filters agree column by column."""
    A, B, _, (shape, cA, cB, V) = _grid()
    n, b, deg = A.shape[0], 9, 8
    bounds = (-6.0, 18.5, 0.5)
    o = rr.rayleigh_ritz(wl.random_block(n, b, 5), lambda X: A @ X, lambda X: B @ X)
    Vd = torch.from_numpy(np.ascontiguousarray(V).reshape(-1)).cuda()
    prm = P.make_params(6, b, deg, method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP64,
                        lambda_max=18.5)
    cs = P.chfsi_create(P.stencil_operator(shape, cA, coef_mass=cB, field=Vd, field_mode=2),
                        P.stencil_operator(shape, cB), None, prm, keep=(Vd,))
    cc = _ctx(A, B, None, prm)
    Xd, Rd = P.to_colmajor(o["X"]), P.to_colmajor(o["R"])
    Ys, Yc = P.colmajor_empty(n, b), P.colmajor_empty(n, b)
    P.chfsi_filter(cs, Xd, o["lam"], Rd, Ys, *bounds, degree=deg)
    P.chfsi_filter(cc, Xd, o["lam"], Rd, Yc, *bounds, degree=deg)
    torch.cuda.synchronize()
    ref = Ys.cpu().numpy()
    assert_columns(Yc.cpu().numpy(), ref, np.linalg.norm(ref, axis=0), "fp64", deg, 81,
                   "csr vs stencil")


@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_FP32, P.PREC_BF16])
def test_csr_grid_solve(prec):
    A, B, _, _ = _grid(shape=(8, 8, 8), wells=2, seed=5)
    w = _spectrum(A, B)
    prm = P.make_params(6, 8, 8, max_iter=200, tol=1e-9, method=P.METHOD_RCHFSI,
                        filter_prec=prec)               # lambda_max estimated
    ctx = _ctx(A, B, None, prm)
    Xd = P.to_colmajor(wl.random_block(512, 8, 31))
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    print(prec, rep["iterations"], rep["max_residual"], rep["lambda_max_used"])
    assert st == P.OK
    np.testing.assert_allclose(ev[:6], w[:6], rtol=1e-9, atol=1e-10)
    X = Xd.cpu().numpy()[:, :6]
    res = np.linalg.norm(A @ X - (B @ X) * np.asarray(ev[:6])[None, :], axis=0)
    assert res.max() <= 1e-9 * 1.01


@pytest.mark.parametrize("kind", ["random", "long_rows"])
def test_csr_generalized_solve(kind):
    A, B, dinv, _ = _problem(kind)
    n = A.shape[0]
    w = _spectrum(A, B)
    prm = P.make_params(16, 24, 12, max_iter=300, tol=1e-9, method=P.METHOD_RCHFSI,
                        filter_prec=P.PREC_FP32)
    ctx = _ctx(A, B, dinv, prm)
    Xd = P.to_colmajor(wl.random_block(n, 24, 8))
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    print(kind, rep["iterations"], rep["max_residual"], rep["lambda_max_used"], w[-1])
    assert st == P.OK
    scale = 1e-3 * np.abs(w).max()
    rel = np.abs(np.asarray(ev[:16]) - w[:16]) / np.maximum(np.abs(w[:16]), scale)
    assert rel.max() <= 1e-10


def test_csr_invalid_structure_rejected():
    A, B, dinv, _ = _problem("random")
    bad = A.copy()
    bad.indices = bad.indices.copy()
    bad.indices[5] = A.shape[0] + 3                     # column index out of range
    prm = P.make_params(8, 12, 6, lambda_max=100.0)
    with pytest.raises(P.ChfsiError) as e:
        _ctx(bad, B, dinv, prm)
    assert e.value.status == P.ERR_ARG and "CSR A" in str(e.value)
    bad2 = A.copy()
    bad2.indptr = bad2.indptr.copy()
    bad2.indptr[10] = bad2.indptr[12] + 1               # decreasing rowptr
    with pytest.raises(P.ChfsiError) as e:
        _ctx(bad2, B, dinv, prm)
    assert e.value.status == P.ERR_ARG
