"""GPU parity of the dense path at small and degenerate sizes, real symmetric
and complex Hermitian, against the oracle.

N below one 64-row tile (N = 37), one row past two tiles (N = 129), a block
of one vector, and a block that spans the whole space (b = N = 64).  Every
product then runs on partial tiles, and the eigensolver of the projected
pencil works on a padded problem.  Bars as for the other dense tests: filters
column by column within the bounds of tests/parity.py (FP64 relative to the
column, FP32 / BF16 residual filters relative to the residual part they carry,
Theorem 3.4), Ritz values to 1e-11 of the spectrum's scale.
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

SIZES = [(37, 1), (37, 5), (129, 3), (64, 64)]          # (N, b)


def _problem(n, b, cplx):
    gen = wl.dense_hermitian if cplx else wl.dense_generalized
    p = gen(n=n, n_low=b, block=b, degree=8, seed=77)
    return p, float(sla.eigvalsh(p.A, p.B)[-1]) + 0.5


def _ctx(p, prec, lmax, cplx):
    to_cm = P.to_colmajor_complex if cplx else P.to_colmajor
    A, B = to_cm(p.A), to_cm(p.B)
    d = torch.from_numpy(p.dinv).cuda()
    mk = P.hermitian_operator if cplx else P.dense_operator
    prm = P.make_params(p.n_wanted, p.block, 8, method=P.METHOD_RCHFSI, filter_prec=prec,
                        lambda_max=lmax)
    return P.chfsi_create(mk(A), mk(B), d, prm, keep=(A, B, d))


def _start(p, cplx, seed=5):
    Y0 = (wl.random_block_complex if cplx else wl.random_block)(p.n, p.block, seed)
    return rr.rayleigh_ritz(Y0, filters.dense_op(p.A), filters.dense_op(p.B))


@pytest.mark.parametrize("n,b", SIZES)
@pytest.mark.parametrize("cplx", [False, True], ids=["real", "complex"])
@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_FP32, P.PREC_BF16])
def test_small_dense_residual_filter_matches_oracle(prec, cplx, n, b):
    p, lmax = _problem(n, b, cplx)
    o = _start(p, cplx)
    lam = o["lam"]
    bounds = (lam[0] - 0.05 * (lam[-1] - lam[0] + 1.0), lmax, lam[-1])
    ctx = _ctx(p, prec, lmax, cplx)
    to_cm = P.to_colmajor_complex if cplx else P.to_colmajor
    Y = (P.colmajor_empty_complex if cplx else P.colmajor_empty)(n, b)
    print("small dense filter", "complex" if cplx else "real", "n", n, "b", b, "prec", prec,
          flush=True)
    P.chfsi_filter(ctx, to_cm(o["X"]), lam, to_cm(o["R"]), Y, *bounds, degree=8)
    torch.cuda.synchronize()
    got = Y.cpu().numpy()
    ref, RYp, _ = filters.residual_filter(filters.dense_op(p.A), filters.diag_op(p.dinv), o["X"],
                                          lam, o["R"], 8, *bounds, return_parts=True)
    assert np.all(np.isfinite(got))
    terms = 2 * n if cplx else n
    if prec == P.PREC_FP64:
        assert_columns(got, ref, np.linalg.norm(ref, axis=0), "fp64", 8, terms, "small dense")
    else:
        # (b = N: the start block spans the space, its residual part is at
        # the FP64 rounding level, so the FP64 bound on the column is added)
        assert_columns(got, ref, residual_part(RYp, p.dinv), prec_name(prec), 8, terms,
                       "small dense", fp64_floor=True)


@pytest.mark.parametrize("n,b", SIZES)
@pytest.mark.parametrize("cplx", [False, True], ids=["real", "complex"])
def test_small_dense_rayleigh_ritz_matches_oracle(cplx, n, b):
    p, lmax = _problem(n, b, cplx)
    ctx = _ctx(p, P.PREC_FP64, lmax, cplx)
    Yh = (wl.random_block_complex if cplx else wl.random_block)(n, b, 9)
    to_cm = P.to_colmajor_complex if cplx else P.to_colmajor
    empty = P.colmajor_empty_complex if cplx else P.colmajor_empty
    X, R = empty(n, b), empty(n, b)
    print("small dense Rayleigh-Ritz", "complex" if cplx else "real", "n", n, "b", b, flush=True)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, to_cm(Yh), X, R)
    o = rr.rayleigh_ritz(Yh, filters.dense_op(p.A), filters.dense_op(p.B))
    lam = np.asarray(ritz)
    scale = np.abs(o["lam"]).max()
    np.testing.assert_allclose(lam, o["lam"], rtol=0, atol=1e-11 * scale)
    Xg, Rg = X.cpu().numpy(), R.cpu().numpy()
    assert np.linalg.norm(Xg.conj().T @ p.B @ Xg - np.eye(b)) <= 1e-10
    Rref = p.A @ Xg - (p.B @ Xg) * lam[None, :]
    assert np.linalg.norm(Rg - Rref) <= 1e-10 * scale * np.sqrt(b)
    np.testing.assert_allclose(norms, np.linalg.norm(Rref, axis=0), rtol=1e-6, atol=1e-11 * scale)
