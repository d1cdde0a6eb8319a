"""Parity at the benchmark's full size (dense generalized, N = 8192, block 320,
256 wanted, degree 20), in the launch configuration bench.py times, for the
FP32 filter (the bench's) and the BF16-product filter.

* The FP32 residual filter on column samples: the filter is column-independent
  (Lambda is diagonal), so the oracle filters a sample of columns exactly and
  the GPU block must agree on those columns (error bounded by the residual
  part, Theorem 3.4).
* A full FP32 R-ChFSI solve to 1e-8: eigenvalues against the stored oracle
  values (tests/golden/dense_generalized_n8192_eigs.json), residuals and
  B-orthonormality recomputed on the CPU, Sylvester inertia (exactly 256
  negative eigenvalues).
* The complex Hermitian counterpart of the same workload (device-built pencil,
  320 complex vectors) on column samples, in FP64, FP32 and BF16.
"""
import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle import filters, rr
from parity import assert_columns, prec_name, residual_part

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden", "dense_generalized_n8192_eigs.json")


@pytest.fixture(scope="module")
def big():
    p = wl.dense_generalized(n=8192, n_low=256, block=320, degree=20, seed=1001)
    lmax = 10.0 / (0.95 * p.meta["dmin"]) + 0.1
    A, B = P.to_colmajor(p.A), P.to_colmajor(p.B)
    d = torch.from_numpy(p.dinv).cuda()
    return p, lmax, A, B, d


@pytest.mark.parametrize("prec", [P.PREC_FP32, P.PREC_BF16])
def test_filter_column_samples(big, prec):
    """FP32 (FP32 MFMA) and BF16 (bfloat16 products on BF16 MFMA, FP32 storage)."""
    p, lmax, A, B, d = big
    X0 = wl.random_block(p.n, p.block, 2001)
    o = rr.rayleigh_ritz(X0, filters.dense_op(p.A), filters.dense_op(p.B))
    lam = o["lam"]
    bounds = (lam[0] - 0.05 * (lam[-1] - lam[0]), lmax, lam[-1])
    prm = P.make_params(256, 320, 20, method=P.METHOD_RCHFSI, filter_prec=prec,
                        lambda_max=lmax)
    ctx = P.chfsi_create(P.dense_operator(A), P.dense_operator(B), d, prm, keep=(A, B, d))
    Y = P.colmajor_empty(p.n, p.block)
    P.chfsi_filter(ctx, P.to_colmajor(o["X"]), lam, P.to_colmajor(o["R"]), Y, *bounds)
    torch.cuda.synchronize()
    cols = np.array([0, 1, 37, 128, 255, 256, 300, 319])
    ref, RYp, _ = filters.residual_filter(filters.dense_op(p.A), filters.diag_op(p.dinv),
                                          o["X"][:, cols], lam[cols], o["R"][:, cols], 20, *bounds,
                                          return_parts=True)
    g = Y.cpu().numpy()[:, cols]
    assert_columns(g, ref, residual_part(RYp, p.dinv), prec_name(prec), 20, p.n,
                   "N=8192 filter samples")


@pytest.mark.parametrize("prec", [P.PREC_FP32, P.PREC_BF16])
def test_rchfsi_solve_full_size(big, prec):
    p, lmax, A, B, d = big
    gold = json.load(open(GOLD))
    wref = np.asarray(gold["eigenvalues"])
    prm = P.make_params(256, 320, 20, max_iter=60, tol=1e-8, method=P.METHOD_RCHFSI,
                        filter_prec=prec, lambda_max=lmax)
    ctx = P.chfsi_create(P.dense_operator(A), P.dense_operator(B), d, prm, keep=(A, B, d))
    Xd = P.to_colmajor(wl.random_block(p.n, p.block, 2001))
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    print(rep["iterations"], rep["max_residual"], rep["time_total_ms"])
    assert st == P.OK
    ev = np.asarray(ev)
    scale = 1e-3 * max(abs(wref[0]), lmax)
    rel = np.abs(ev[:256] - wref[:256]) / np.maximum(np.abs(wref[:256]), scale)
    assert rel.max() <= 1e-10
    assert np.count_nonzero(ev < 0) == 256 == gold["negative_count_A"]
    X = Xd.cpu().numpy()
    res = np.linalg.norm(p.A @ X[:, :256] - (p.B @ X[:, :256]) * ev[None, :256], axis=0)
    assert res.max() <= 1e-8 * 1.01
    G = X[:, :64].T @ (p.B @ X[:, :64])
    np.testing.assert_allclose(G, np.eye(64), atol=1e-9)


@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_FP32, P.PREC_BF16])
def test_complex_filter_column_samples(prec):
    """The complex Hermitian counterpart that bench.py's dense run times (N = 8192,
    320 complex vectors, 256 wanted, degree 20, device-built pencil with
    ||D^-1 eps S||_2 = 0.05), in every filter precision: sampled columns of one
    filter pass against the oracle on the host copies."""
    from workloads.gpu import hermitian_problem
    n, b, p = 8192, 320, 20
    A, B, dinv, _ = hermitian_problem(n, 256, seed=1003)
    lmax = 10.0 / (0.95 * float((1.0 / dinv).min())) + 0.1
    g = torch.Generator(device="cuda")
    g.manual_seed(2003)
    X = torch.complex(torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g),
                      torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g)).t()
    R = (1e-3 * torch.complex(torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g),
                              torch.randn((b, n), dtype=torch.float64, device="cuda",
                                          generator=g))).t()
    lam = np.sort(np.random.default_rng(2003).uniform(-1.0, 0.2, b))
    bounds = (lam[0] - 0.05 * (lam[-1] - lam[0]), lmax, lam[-1])
    prm = P.make_params(256, b, p, method=P.METHOD_RCHFSI, filter_prec=prec, lambda_max=lmax)
    ctx = P.chfsi_create(P.hermitian_operator(A), P.hermitian_operator(B), dinv, prm,
                         keep=(A, B, dinv))
    Y = P.colmajor_empty_complex(n, b)
    print("complex N=8192 b=320 filter, prec", prec, flush=True)
    P.chfsi_filter(ctx, X, lam, R, Y, *bounds)
    torch.cuda.synchronize()
    cols = np.array([0, 1, 37, 128, 255, 256, 300, 319])
    got = Y[:, cols].cpu().numpy()
    Xc, Rc = X[:, cols].cpu().numpy(), R[:, cols].cpu().numpy()
    Ah, dh = A.cpu().numpy(), dinv.cpu().numpy()
    ctx.close()
    del X, R, Y, A, B
    ref, RYp, _ = filters.residual_filter(filters.dense_op(Ah), filters.diag_op(dh), Xc,
                                          lam[cols], Rc, p, *bounds, return_parts=True)
    assert np.all(np.isfinite(got))
    scale = np.linalg.norm(ref, axis=0) if prec == P.PREC_FP64 else residual_part(RYp, dh)
    assert_columns(got, ref, scale, prec_name(prec), p, 2 * n, "complex N=8192 samples")
