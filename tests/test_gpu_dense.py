"""GPU parity of the dense path through the C ABI against the CPU oracle.

Sizes span several GEMM tiles with ragged tails (n not a multiple of the
tile, block not a multiple of 16, a padded leading dimension).  Filters are
compared column by column with the bounds of tests/parity.py: G u sqrt(K p)
of the column's norm (FP64, and the plain filter) or of its residual part
D^{-1} R_Y (FP32 / BF16 residual filter; Theorem 3.4: the error of the
residual form scales with ||R||).  Full solves must reach the same
eigenvalues to 1e-10 relative.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import filters, rr, solver
from parity import assert_columns, prec_name, residual_part

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402


def dev(a):
    return P.to_colmajor(a)


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def gen_problem():
    p = wl.dense_generalized(n=701, n_low=24, block=40, degree=8, seed=77)
    w = sla.eigvalsh(p.A, p.B)
    return p, w


def _ctx(p, params, dinv=True):
    A = dev(p.A)
    B = dev(p.B) if p.B is not None else None
    d = torch.from_numpy(p.dinv).cuda() if (dinv and p.dinv is not None) else None
    opA = P.dense_operator(A)
    opB = P.dense_operator(B) if B is not None else None
    ctx = P.chfsi_create(opA, opB, d, params, keep=(A, B, d))
    return ctx


def _ritz_start(p, seed=5):
    X0 = wl.random_block(p.n, p.block, seed)
    Bop = filters.dense_op(p.B) if p.B is not None else filters.identity_op()
    return rr.rayleigh_ritz(X0, filters.dense_op(p.A), Bop)


@pytest.mark.parametrize("n,block", [(768, 128), (1024, 128), (1280, 320)])
def test_rchfsi_bf16_filter_aligned_shapes(n, block):
    """Shapes the 32 x 32 x 16 BF16 product takes (n a multiple of 128, the
    block of 128 or 320): one split with the epilogue in the product (768),
    two splits with the reduction (1024, 1280); column-by-column bounds as for
    the other BF16 filters."""
    p = wl.dense_generalized(n=n, n_low=block // 2, block=block, degree=8, seed=n + block)
    w = sla.eigvalsh(p.A, p.B)
    bounds = (w[0] - 0.1, w[-1] + 0.5, 0.5 * (w[block - 1] + w[block]))
    params = P.make_params(block // 2, block, 8, method=P.METHOD_RCHFSI,
                           filter_prec=P.PREC_BF16, lambda_max=bounds[1])
    ctx = _ctx(p, params)
    st = _ritz_start(p)
    X, lam, R = st["X"], st["lam"], st["R"]
    Yd = P.colmajor_empty(p.n, p.block)
    P.chfsi_filter(ctx, dev(X), lam, dev(R), Yd, *bounds, degree=8)
    torch.cuda.synchronize()
    ref, RYp, _ = filters.residual_filter(filters.dense_op(p.A), filters.diag_op(p.dinv), X, lam,
                                          R, 8, *bounds, return_parts=True)
    assert_columns(host(Yd), ref, residual_part(RYp, p.dinv), "bf16", 8, p.n,
                   f"bf16 aligned n={n} b={block}")


@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_FP32])
def test_chfsi_filter_matches_oracle(gen_problem, prec):
    p, w = gen_problem
    bounds = (w[0] - 0.1, w[-1] + 0.5, 0.5 * (w[p.block - 1] + w[p.block]))
    params = P.make_params(p.n_wanted, p.block, p.degree, method=P.METHOD_CHFSI, filter_prec=prec,
                           lambda_max=bounds[1])
    ctx = _ctx(p, params)
    X = wl.random_block(p.n, p.block, 3)
    Xd = dev(X)
    Yd = P.colmajor_empty(p.n, p.block)
    P.chfsi_filter(ctx, Xd, None, None, Yd, *bounds, degree=p.degree)
    torch.cuda.synchronize()
    ref = filters.chebyshev_filter(lambda V: p.dinv[:, None] * (p.A @ V), X, p.degree, *bounds)
    assert_columns(host(Yd), ref, np.linalg.norm(ref, axis=0), prec_name(prec), p.degree, p.n,
                   "chfsi filter")


@pytest.mark.parametrize("prec,degree", [(P.PREC_FP64, 8), (P.PREC_FP64, 1), (P.PREC_FP64, 2),
                                         (P.PREC_FP32, 8), (P.PREC_FP32, 20),
                                         (P.PREC_BF16, 8), (P.PREC_BF16, 20)])
def test_rchfsi_filter_matches_oracle(gen_problem, prec, degree):
    p, w = gen_problem
    bounds = (w[0] - 0.1, w[-1] + 0.5, 0.5 * (w[p.block - 1] + w[p.block]))
    params = P.make_params(p.n_wanted, p.block, max(degree, 1), method=P.METHOD_RCHFSI,
                           filter_prec=prec, lambda_max=bounds[1])
    ctx = _ctx(p, params)
    st = _ritz_start(p)
    X, lam, R = st["X"], st["lam"], st["R"]
    Xd, Rd = dev(X), dev(R)
    Yd = P.colmajor_empty(p.n, p.block)
    P.chfsi_filter(ctx, Xd, lam, Rd, Yd, *bounds, degree=degree)
    torch.cuda.synchronize()
    ref, RYp, LYp = filters.residual_filter(filters.dense_op(p.A), filters.diag_op(p.dinv), X, lam,
                                            R, degree, *bounds, return_parts=True)
    g = host(Yd)
    if prec == P.PREC_FP64:
        assert_columns(g, ref, np.linalg.norm(ref, axis=0), "fp64", degree, p.n, "rchfsi")
    else:
        # FP32 blocks and products, or BF16 product inputs (A and D^{-1} R_Y
        # rounded to bfloat16, FP32 accumulation): the rounding touches only the
        # residual part D^{-1} R_Y of each column
        assert_columns(g, ref, residual_part(RYp, p.dinv), prec_name(prec), degree, p.n,
                       "rchfsi")


def test_rayleigh_ritz_matches_oracle(gen_problem):
    p, w = gen_problem
    params = P.make_params(p.n_wanted, p.block, 4, lambda_max=w[-1] + 1)
    ctx = _ctx(p, params)
    rng = np.random.default_rng(9)
    # a filtered-looking block: span near the low eigenvectors plus noise
    _, U = sla.eigh(p.A, p.B)
    Y = U[:, : p.block] @ rng.standard_normal((p.block, p.block)) + 1e-3 * rng.standard_normal(
        (p.n, p.block))
    Yd = dev(Y)
    Xd = P.colmajor_empty(p.n, p.block)
    Rd = P.colmajor_empty(p.n, p.block)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, Yd, Xd, Rd)
    o = rr.rayleigh_ritz(Y, filters.dense_op(p.A), filters.dense_op(p.B))
    scale = np.abs(o["lam"]).max()
    np.testing.assert_allclose(ritz, o["lam"], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(norms, o["resnorm"], rtol=1e-6, atol=1e-11 * scale)
    Xg = host(Xd)
    np.testing.assert_allclose(Xg.T @ p.B @ Xg, np.eye(p.block), atol=1e-10)
    # same Ritz vectors up to sign (distinct Ritz values)
    M = np.abs(Xg.T @ p.B @ o["X"])
    np.testing.assert_allclose(np.diag(M), 1.0, atol=1e-8)
    # residual block recomputed on the CPU from the returned pairs
    Rg = host(Rd)
    np.testing.assert_allclose(Rg, p.A @ Xg - (p.B @ Xg) * np.asarray(ritz)[None, :],
                               atol=1e-10 * scale)


def test_rayleigh_ritz_wide_block_matches_oracle():
    """b = 300 > 256: the symmetric Gram matrices are formed as lower block
    panels (several panel widths, a ragged last panel) and mirrored."""
    p = wl.dense_generalized(n=1100, n_low=40, block=300, degree=8, seed=78)
    params = P.make_params(p.n_wanted, p.block, 4, lambda_max=20.0)
    ctx = _ctx(p, params)
    rng = np.random.default_rng(10)
    _, U = sla.eigh(p.A, p.B)
    Y = U[:, : p.block] @ rng.standard_normal((p.block, p.block)) + 1e-3 * rng.standard_normal(
        (p.n, p.block))
    Xd, Rd = P.colmajor_empty(p.n, p.block), P.colmajor_empty(p.n, p.block)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, dev(Y), Xd, Rd)
    o = rr.rayleigh_ritz(Y, filters.dense_op(p.A), filters.dense_op(p.B))
    scale = np.abs(o["lam"]).max()
    np.testing.assert_allclose(ritz, o["lam"], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(norms, o["resnorm"], rtol=1e-6, atol=1e-11 * scale)
    Xg = host(Xd)
    np.testing.assert_allclose(Xg.T @ p.B @ Xg, np.eye(p.block), atol=1e-10)


def test_rayleigh_ritz_padded_leading_dimension(gen_problem):
    p, w = gen_problem
    params = P.make_params(p.n_wanted, p.block, 4, lambda_max=w[-1] + 1)
    ctx = _ctx(p, params)
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((p.n, p.block))
    big = torch.zeros((p.block, p.n + 13), dtype=torch.float64, device="cuda")
    big[:, : p.n] = torch.from_numpy(Y.T.copy()).cuda()
    Yd = big.t()[: p.n]
    assert P._ld(Yd) == p.n + 13
    Xd = P.colmajor_empty(p.n, p.block)
    Rd = P.colmajor_empty(p.n, p.block)
    ritz, _ = P.chfsi_rayleigh_ritz(ctx, Yd, Xd, Rd)
    o = rr.rayleigh_ritz(Y, filters.dense_op(p.A), filters.dense_op(p.B))
    np.testing.assert_allclose(ritz, o["lam"], atol=1e-10 * np.abs(o["lam"]).max())


def test_solve_dense_standard_full_size():
    """N = 1024 standard problem, FP64 plain filter, fixed bounds: the prescribed spectrum."""
    p = wl.dense_standard()
    lam = p.lam_A
    bounds = (lam[0] - 0.05, lam[-1] + 0.1, 0.5 * (lam[p.block - 1] + lam[p.block]))
    params = P.make_params(p.n_wanted, p.block, p.degree, max_iter=30, tol=p.tol,
                           method=P.METHOD_CHFSI, filter_prec=P.PREC_FP64, lambda_min=bounds[0],
                           lambda_max=bounds[1], lambda_T=bounds[2])
    ctx = _ctx(p, params)
    X0 = wl.random_block(p.n, p.block, 2000)
    Xd = dev(X0)
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    print(rep["iterations"], rep["history"][:12])
    assert st == P.OK and rep["converged"]
    ev = np.asarray(ev)
    relerr = np.abs(ev[:32] - lam[:32]) / np.maximum(np.abs(lam[:32]), 1e-3 * 10.1)
    assert relerr.max() <= 1e-10
    X = host(Xd)
    rcpu = np.linalg.norm(p.A @ X[:, :32] - X[:, :32] * ev[None, :32], axis=0)
    assert rcpu.max() <= 1e-10
    # oracle runs the same iteration: same number of passes
    o = solver.solve(filters.dense_op(p.A), filters.identity_op(), filters.identity_op(), X0, 32,
                     p.degree, p.tol, 30, bounds, method="chfsi")
    assert abs(o["iters"] - rep["iterations"]) <= 1
    np.testing.assert_allclose(ev[:32], o["lam"][:32], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("method,prec", [("rchfsi", P.PREC_FP64), ("rchfsi", P.PREC_FP32),
                                         ("rchfsi", P.PREC_BF16)])
def test_solve_generalized_reduced(method, prec):
    p = wl.dense_generalized(n=1536, n_low=48, block=64, degree=20, seed=1001)
    w = sla.eigvalsh(p.A, p.B)
    lmax = float(w[-1]) + 0.5
    params = P.make_params(48, 64, 20, max_iter=40, tol=1e-9, method=P.METHOD_RCHFSI,
                           filter_prec=prec, lambda_max=lmax)
    ctx = _ctx(p, params)
    X0 = wl.random_block(p.n, p.block, 2001)
    Xd = dev(X0)
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    print(prec, rep["iterations"], ["%.2e" % h for h in rep["history"]])
    assert st == P.OK
    ev = np.asarray(ev)
    scale = 1e-3 * max(abs(w[0]), abs(w[-1]))
    relerr = np.abs(ev[:48] - w[:48]) / np.maximum(np.abs(w[:48]), scale)
    assert relerr.max() <= 1e-10
    X = host(Xd)
    rcpu = np.linalg.norm(p.A @ X[:, :48] - (p.B @ X[:, :48]) * ev[None, :48], axis=0)
    assert rcpu.max() <= 1e-9 * 1.01
    np.testing.assert_allclose(X.T @ p.B @ X, np.eye(64), atol=1e-9)


def test_plain_filter_with_approximate_inverse_stagnates():
    """ChFSI with D^{-1} != B^{-1} stalls (Theorem 3.2); R-ChFSI above converges."""
    p = wl.dense_generalized(n=1536, n_low=48, block=64, degree=20, seed=1001)
    w = sla.eigvalsh(p.A, p.B)
    params = P.make_params(48, 64, 20, max_iter=12, tol=1e-9, method=P.METHOD_CHFSI,
                           filter_prec=P.PREC_FP64, lambda_max=float(w[-1]) + 0.5)
    ctx = _ctx(p, params)
    Xd = dev(wl.random_block(p.n, p.block, 2001))
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    assert st == P.ERR_NOCONV and rep["max_residual"] > 1e-6


def test_invalid_arguments_are_rejected(gen_problem):
    p, w = gen_problem
    A = dev(p.A)
    opA = P.dense_operator(A)
    with pytest.raises(P.ChfsiError) as e:
        P.chfsi_create(opA, None, None, P.make_params(50, 40, 8, lambda_max=10.0))
    assert e.value.status == P.ERR_ARG
    with pytest.raises(P.ChfsiError):
        P.chfsi_create(opA, None, None, P.make_params(10, 40, 0, lambda_max=10.0))
    with pytest.raises(P.ChfsiError):
        P.chfsi_create(opA, None, None, P.make_params(10, 40, 8, lambda_max=float("inf")))
    ctx = P.chfsi_create(opA, None, None, P.make_params(10, 40, 8, method=P.METHOD_CHFSI,
                                                        lambda_max=10.0), keep=(A,))
    Xd = dev(np.ones((p.n, 40)))
    Yd = P.colmajor_empty(p.n, 40)
    with pytest.raises(P.ChfsiError):
        P.chfsi_filter(ctx, Xd, None, None, Yd, 1.0, 10.0, 0.5)      # lmin > lT


def test_rayleigh_ritz_singular_gram_uses_svqb(gen_problem):
    """A block with a repeated column: the scaled Gram matrix is singular, the
    SVQB reading keeps the b-1 independent directions (here an invariant
    subspace, so their Ritz values are exact eigenvalues), refills one column
    and repeats Rayleigh-Ritz."""
    p, w = gen_problem
    params = P.make_params(p.n_wanted, p.block, 4, lambda_max=w[-1] + 1)
    ctx = _ctx(p, params)
    _, U = sla.eigh(p.A, p.B)
    Y = U[:, : p.block].copy()
    Y[:, -1] = Y[:, 0]
    Xd = P.colmajor_empty(p.n, p.block)
    Rd = P.colmajor_empty(p.n, p.block)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, dev(Y), Xd, Rd)
    ritz = np.asarray(ritz)
    exact = w[: p.block - 1]
    for lam in exact:
        assert np.min(np.abs(ritz - lam)) <= 1e-10 * max(1.0, abs(lam))
    Xg = host(Xd)
    np.testing.assert_allclose(Xg.T @ p.B @ Xg, np.eye(p.block), atol=1e-9)
    Rg = p.A @ Xg - (p.B @ Xg) * ritz[None, :]
    np.testing.assert_allclose(norms, np.linalg.norm(Rg, axis=0), rtol=1e-6, atol=1e-9)


def test_chfsi_exact_inverse_filter_and_solve():
    """Algorithm 2 with the exact inverse, H = B^{-1} A (binv_exact): the filter
    matches the oracle's Algorithm 2 with that operator, and the solve reaches
    LAPACK's eigenvalues of the generalized pencil."""
    p = wl.dense_generalized(n=1024, n_low=32, block=40, degree=16, seed=71)
    w = sla.eigh(p.A, p.B, eigvals_only=True)
    lmax = float(w[-1]) + 0.5
    params = P.make_params(32, 40, 16, max_iter=60, tol=1e-10, method=P.METHOD_CHFSI,
                           filter_prec=P.PREC_FP64, lambda_max=lmax, binv_exact=1)
    ctx = _ctx(p, params)
    X = wl.random_block(p.n, 40, 72)
    Y = P.colmajor_empty(p.n, 40)
    bounds = (float(w[0]) - 0.1, lmax, float(w[40]))
    P.chfsi_filter(ctx, dev(X), None, None, Y, *bounds, degree=16)
    torch.cuda.synchronize()
    apply_H = lambda U: np.linalg.solve(p.B, p.A @ U)
    ref = filters.chebyshev_filter(apply_H, X, 16, *bounds)
    # per column, relative to the column: the operator is formed through the
    # Cholesky factor of B, whose error (u kappa(B) n) sits far above the
    # product's rounding, so this bound is the formation's, not G u sqrt(K p)
    rel = np.linalg.norm(host(Y) - ref, axis=0) / np.linalg.norm(ref, axis=0)
    print("exact-inverse ChFSI filter max column rel err", rel.max())
    assert rel.max() <= 1e-10
    Xs = dev(wl.random_block(p.n, 40, 73))
    st, ev, rn, rep = P.chfsi_solve(ctx, Xs)
    print("exact-inverse ChFSI solve:", rep["iterations"], "iterations", rep["max_residual"])
    assert st == P.OK
    np.testing.assert_allclose(ev[:32], w[:32], rtol=0, atol=1e-10 * np.max(np.abs(w[:32])))


def test_stagnation_stops_early_and_returns_best_pairs():
    """ChFSI with D^{-1} != B^{-1} stalls (Theorem 3.2).  With stall_iters the
    solve stops once its lowest max residual has not halved for that many
    passes (report flags bit 2, CHFSI_ERR_NOCONV), and with keep_best the
    returned pairs are those of the lowest max residual: their residuals,
    recomputed on the CPU, are the reported ones."""
    p = wl.dense_generalized(n=1536, n_low=48, block=64, degree=20, seed=1001)
    w = sla.eigvalsh(p.A, p.B)
    params = P.make_params(48, 64, 20, max_iter=60, tol=1e-9, method=P.METHOD_CHFSI,
                           filter_prec=P.PREC_FP64, lambda_max=float(w[-1]) + 0.5,
                           stall_iters=4, keep_best=1)
    ctx = _ctx(p, params)
    Xd = dev(wl.random_block(p.n, p.block, 2001))
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    print(rep["iterations"], rep["best_iteration"], rep["best_residual"],
          ["%.2e" % h for h in rep["history"]])
    assert st == P.ERR_NOCONV
    assert rep["flags"] & 4
    assert rep["iterations"] < 60
    hist = rep["history"]
    # stopped because the lowest max residual did not halve over the last 4 passes
    assert min(hist) >= 0.5 * min(hist[: len(hist) - 4])
    assert rep["best_residual"] == min(hist)
    assert rep["max_residual"] == rep["best_residual"]
    X = host(Xd)
    ev = np.asarray(ev)
    rcpu = np.linalg.norm(p.A @ X[:, :48] - (p.B @ X[:, :48]) * ev[None, :48], axis=0)
    np.testing.assert_allclose(rcpu, np.asarray(rn[:48]), rtol=1e-6, atol=1e-12)
    assert abs(rcpu.max() - rep["best_residual"]) <= 1e-6 * rep["best_residual"]


@pytest.mark.parametrize("cap", ["1", "2"])
def test_jacobi_sweep_cap_is_reported(monkeypatch, cap):
    """An eigensolve stopped by its sweep cap (forced to 1 or 2 sweeps here;
    with 2, the second sweep's first launches are queued before the first
    sweep's flags are read) with rotations still pending raises report flags
    bit 1."""
    p = wl.dense_generalized(n=512, n_low=16, block=40, degree=8, seed=1001)
    w = sla.eigvalsh(p.A, p.B)
    params = P.make_params(16, 40, 8, max_iter=1, tol=1e-12, method=P.METHOD_RCHFSI,
                           filter_prec=P.PREC_FP64, lambda_max=float(w[-1]) + 0.5)
    ctx = _ctx(p, params)
    monkeypatch.setenv("CHFSI_JACOBI_MAX_SWEEPS", cap)
    st, ev, rn, rep = P.chfsi_solve(ctx, dev(wl.random_block(p.n, 40, 7)))
    assert rep["flags"] & 2
    monkeypatch.delenv("CHFSI_JACOBI_MAX_SWEEPS")
    st, ev, rn, rep = P.chfsi_solve(ctx, dev(wl.random_block(p.n, 40, 7)))
    assert not rep["flags"] & 2


@pytest.mark.parametrize("n,b", [(512, 40), (1024, 100), (2048, 320)])
def test_jacobi_pipelined_rounds_bitwise(monkeypatch, n, b):
    """The pipelined outer rounds (a round's pair solves launched with the
    previous round's rotations, the pair workgroups forming their rotated
    blocks themselves) give bit-identical Rayleigh-Ritz results to a pair-solve
    launch followed by a rotation launch per round (knob CHFSI_JACOBI_PIPE=0):
    padded blocks of 2, 4 and 10 pairs."""
    p = wl.dense_generalized(n=n, n_low=b // 2, block=b, degree=8, seed=1001)
    w = sla.eigvalsh(p.A, p.B)
    params = P.make_params(b // 2, b, 8, method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP64,
                           lambda_max=float(w[-1]) + 0.5)
    ctx = _ctx(p, params)
    Y = dev(wl.random_block(n, b, 13))
    out = {}
    for pipe in ("0", "1"):
        monkeypatch.setenv("CHFSI_JACOBI_PIPE", pipe)
        X, R = P.colmajor_empty(n, b), P.colmajor_empty(n, b)
        print("Rayleigh-Ritz n", n, "b", b, "pipelined", pipe, flush=True)
        ritz, norms = P.chfsi_rayleigh_ritz(ctx, Y, X, R)
        out[pipe] = (np.asarray(ritz), np.asarray(norms), host(X), host(R))
    for a, c in zip(out["0"], out["1"]):
        assert np.array_equal(a, c)
    lam = out["1"][0]
    scale = np.abs(w).max()
    o = rr.rayleigh_ritz(host(Y), filters.dense_op(p.A), filters.dense_op(p.B))
    np.testing.assert_allclose(lam, o["lam"], rtol=0, atol=1e-11 * scale)


def test_bf16_stagnation_escalates_to_fp32():
    """A reduced-precision filter has a largest usable degree (Section 3.1's
    condition): on the toy spectrum of Section 4.1 (m = 1000, 10 wanted, gap 1)
    the BF16-product residual filter stalls at degree 64.  With escalate the
    stalled solve continues in FP32 and converges to LAPACK's eigenvalues;
    without it the same solve stops on stagnation."""
    t = wl.toy_standard(1000, 10, seed=31)
    A = t["A"]
    w = np.linalg.eigvalsh(A)
    Ad = dev(A)
    anorm = float(np.abs(w).max())
    for escalate in (0, 1):
        # the bounds of the controlled experiments (Section 4.1), block = n
        params = P.make_params(10, 10, 64, max_iter=80, tol=1e-9 * anorm,
                               method=P.METHOD_RCHFSI, filter_prec=P.PREC_BF16,
                               lambda_min=float(w[0]) - 0.05, lambda_max=float(w[-1]) + 0.1,
                               lambda_T=0.5 * float(w[9] + w[10]), stall_iters=5,
                               escalate=escalate)
        ctx = P.chfsi_create(P.dense_operator(Ad), None, None, params, keep=(Ad,))
        Xd = dev(wl.random_block(1000, 10, 42))
        st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
        print("escalate", escalate, P.STATUS_NAMES[st], rep["iterations"],
              rep["escalation_iteration"], ["%.1e" % h for h in rep["history"]])
        if escalate:
            assert st == P.OK and rep["flags"] & 8 and rep["escalation_iteration"] > 0
            np.testing.assert_allclose(ev[:10], w[:10], rtol=1e-10, atol=1e-10 * anorm)
        else:
            assert st == P.ERR_NOCONV and rep["flags"] & 4


def test_amplification_guard_reports_and_caps():
    """Section 3.1's amplification T_p(|L(lambda_min)|) of a pass: one pass is
    reported as the oracle's closed form from the start block's Ritz values
    (bounds policy: lambda_min = eps_1 - 0.05 (eps_b - eps_1), lambda_T = eps_b);
    a degree-40 pass exceeds 1e12 (flags bit 4); with amp_cap every pass stays
    within the cap at a lower degree (flags bit 5) and the solve still reaches
    LAPACK's eigenvalues."""
    from oracle import chebyshev
    p = wl.dense_generalized(n=1024, n_low=32, block=40, degree=40, seed=91)
    w = sla.eigvalsh(p.A, p.B)
    lmax = float(w[-1]) + 0.5
    X0 = wl.random_block(p.n, p.block, 92)
    st0 = rr.rayleigh_ritz(X0, filters.dense_op(p.A), filters.dense_op(p.B))
    e1, eb = float(st0["lam"][0]), float(st0["lam"][-1])
    lmin, lT = e1 - 0.05 * (eb - e1), eb
    e, c, _ = chebyshev.affine(lmin, lmax, lT)
    ref = float(chebyshev.cheb_T(40, np.array([(lmin - c) / e]))[0])
    ref = abs(ref)
    params = P.make_params(32, 40, 40, max_iter=1, tol=1e-30, method=P.METHOD_RCHFSI,
                           filter_prec=P.PREC_FP32, lambda_max=lmax)
    ctx = _ctx(p, params)
    st, ev, rn, rep = P.chfsi_solve(ctx, dev(X0))
    print("one pass: amplification", rep["max_amplification"], "oracle", ref, "flags", rep["flags"])
    assert rep["min_degree_used"] == 40
    assert abs(rep["max_amplification"] - ref) <= 1e-6 * ref
    assert bool(rep["flags"] & 16) == (ref > 1e12) and not rep["flags"] & 32
    cap = 1e8
    params = P.make_params(32, 40, 40, max_iter=100, tol=1e-10, method=P.METHOD_RCHFSI,
                           filter_prec=P.PREC_FP32, lambda_max=lmax, amp_cap=cap)
    ctx = _ctx(p, params)
    st, ev, rn, rep = P.chfsi_solve(ctx, dev(X0))
    print("capped:", rep["iterations"], "passes, degree >=", rep["min_degree_used"],
          "amplification", rep["max_amplification"], "flags", rep["flags"])
    assert st == P.OK
    assert rep["flags"] & 32 and not rep["flags"] & 16
    assert 1 <= rep["min_degree_used"] < 40 and rep["max_amplification"] <= cap
    np.testing.assert_allclose(ev[:32], w[:32], rtol=0, atol=1e-10 * np.max(np.abs(w[:32])))
    with pytest.raises(P.ChfsiError):
        P.chfsi_create(P.dense_operator(dev(p.A)), None, None,
                       P.make_params(8, 16, 8, lambda_max=lmax, amp_cap=math.nan))
