"""GPU parity of the complex Hermitian residual filter (Section 4.3) through the
C ABI against the CPU oracle.

The pencil is the complex counterpart of the dense generalized workload
(complex reflectors, B = D + eps S with complex Hermitian S, the real
diagonal approximate inverse D^{-1}) at a ragged size (N = 701, block 40: no
tile divides either).  FP64 filters match the oracle to 1e-11 relative; FP32
and bfloat16 products have an error bounded by the residual part they carry
(Theorem 3.4), with the bounds of the real dense tests.  The GPU
Rayleigh-Ritz (on the real embedding of the projected Hermitian pencil)
matches the oracle's Ritz values to 1e-11; full solves, with the GPU filter
inside the oracle's Algorithm 1 and entirely on the GPU through chfsi_solve,
reach LAPACK's eigenvalues of the Hermitian pencil.
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



@pytest.fixture(scope="module")
def herm():
    p = wl.dense_hermitian(n=701, n_low=24, block=40, degree=8, seed=77)
    lmax = 10.0 / (0.95 * p.meta["dmin"]) + 0.1
    return p, lmax


def _ctx(p, prec, lmax, degree):
    A = P.to_colmajor_complex(p.A)
    B = P.to_colmajor_complex(p.B)
    d = torch.from_numpy(p.dinv).cuda()
    prm = P.make_params(p.n_wanted, p.block, degree, method=P.METHOD_RCHFSI, filter_prec=prec,
                        lambda_max=lmax)
    return P.chfsi_create(P.hermitian_operator(A), P.hermitian_operator(B), d, prm,
                          keep=(A, B, d))


@pytest.mark.parametrize("prec,degree", [(P.PREC_FP64, 8), (P.PREC_FP64, 1), (P.PREC_FP64, 2),
                                         (P.PREC_FP32, 8), (P.PREC_BF16, 8)])
def test_complex_residual_filter_matches_oracle(herm, prec, degree):
    p, lmax = herm
    ctx = _ctx(p, prec, lmax, 8)
    o = rr.rayleigh_ritz(wl.random_block_complex(p.n, p.block, 5), filters.dense_op(p.A),
                         filters.dense_op(p.B))
    lam = o["lam"]
    bounds = (lam[0] - 0.05 * (lam[-1] - lam[0]), lmax, lam[-1])
    Y = P.colmajor_empty_complex(p.n, p.block)
    print("complex filter prec", prec, "degree", degree, "n", p.n, "b", p.block, flush=True)
    P.chfsi_filter(ctx, P.to_colmajor_complex(o["X"]), lam, P.to_colmajor_complex(o["R"]), Y,
                   *bounds, degree=degree)
    torch.cuda.synchronize()
    got = Y.cpu().numpy()
    ref, RYp, _ = filters.residual_filter(filters.dense_op(p.A), filters.diag_op(p.dinv), o["X"],
                                          lam, o["R"], degree, *bounds, return_parts=True)
    assert got.dtype == np.complex128 and np.all(np.isfinite(got))
    # the complex product is one real product with K = 2n terms per element
    scale = np.linalg.norm(ref, axis=0) if prec == P.PREC_FP64 else residual_part(RYp, p.dinv)
    assert_columns(got, ref, scale, prec_name(prec), degree, 2 * p.n, "complex filter")


@pytest.mark.parametrize("prec", [P.PREC_FP32, P.PREC_BF16])
def test_complex_solve_with_gpu_filter(prec):
    """Algorithm 1 with the GPU residual filter and the oracle's Rayleigh-Ritz."""
    p = wl.dense_hermitian(n=1024, n_low=32, block=40, degree=16, seed=78)
    lmax = 10.0 / (0.95 * p.meta["dmin"]) + 0.1
    w = sla.eigh(p.A, p.B, eigvals_only=True, subset_by_index=(0, 31))
    ctx = _ctx(p, prec, lmax, 16)
    opA, opB = filters.dense_op(p.A), filters.dense_op(p.B)
    o = rr.rayleigh_ritz(wl.random_block_complex(p.n, p.block, 9), opA, opB)
    Y = P.colmajor_empty_complex(p.n, p.block)
    it = 0
    while np.max(o["resnorm"][:32]) >= 1e-10 and it < 40:
        lam = o["lam"]
        bounds = (lam[0] - 0.05 * (lam[-1] - lam[0]), lmax, lam[-1])
        P.chfsi_filter(ctx, P.to_colmajor_complex(o["X"]), lam, P.to_colmajor_complex(o["R"]), Y,
                       *bounds, degree=16)
        torch.cuda.synchronize()
        o = rr.rayleigh_ritz(Y.cpu().numpy(), opA, opB)
        it += 1
    print("complex solve prec", prec, "iterations", it, "max residual",
          float(np.max(o["resnorm"][:32])))
    assert np.max(o["resnorm"][:32]) < 1e-10
    assert np.max(np.abs(o["lam"][:32] - w)) <= 1e-10 * np.max(np.abs(w))


def test_complex_rayleigh_ritz_matches_oracle(herm):
    """Rayleigh-Ritz on the real embedding of the projected Hermitian pencil."""
    p, lmax = herm
    ctx = _ctx(p, P.PREC_FP32, lmax, 8)
    Yh = wl.random_block_complex(p.n, p.block, 6)
    X = P.colmajor_empty_complex(p.n, p.block)
    R = P.colmajor_empty_complex(p.n, p.block)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, P.to_colmajor_complex(Yh), X, R)
    o = rr.rayleigh_ritz(Yh, filters.dense_op(p.A), filters.dense_op(p.B))
    lam = np.array(ritz)
    scale = np.max(np.abs(o["lam"]))
    assert np.max(np.abs(lam - o["lam"])) <= 1e-11 * scale
    Xg, Rg = X.cpu().numpy(), R.cpu().numpy()
    assert np.linalg.norm(Xg.conj().T @ p.B @ Xg - np.eye(p.block)) <= 1e-10
    Rref = p.A @ Xg - p.B @ Xg * lam[None, :]
    assert np.linalg.norm(Rg - Rref) <= 1e-10 * np.linalg.norm(p.A, 2)
    assert np.allclose(norms, np.linalg.norm(Rref, axis=0), rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_FP32, P.PREC_BF16])
def test_complex_solve_on_gpu(prec):
    """Algorithm 1 entirely on the GPU (filter, Rayleigh-Ritz, residuals)."""
    p = wl.dense_hermitian(n=1024, n_low=32, block=40, degree=16, seed=78)
    lmax = 10.0 / (0.95 * p.meta["dmin"]) + 0.1
    w = sla.eigh(p.A, p.B, eigvals_only=True, subset_by_index=(0, 31))
    A = P.to_colmajor_complex(p.A)
    B = P.to_colmajor_complex(p.B)
    d = torch.from_numpy(p.dinv).cuda()
    prm = P.make_params(32, 40, 16, max_iter=40, tol=1e-10, method=P.METHOD_RCHFSI,
                        filter_prec=prec, lambda_max=lmax)
    ctx = P.chfsi_create(P.hermitian_operator(A), P.hermitian_operator(B), d, prm, keep=(A, B, d))
    X = P.to_colmajor_complex(wl.random_block_complex(p.n, p.block, 9))
    st, ev, rn, rep = P.chfsi_solve(ctx, X)
    print("complex GPU solve prec", prec, rep["iterations"], "iterations, max residual",
          rep["max_residual"])
    assert st == P.OK and rep["converged"]
    assert np.max(np.abs(np.array(ev[:32]) - w)) <= 1e-10 * np.max(np.abs(w))
    Xg = X.cpu().numpy()[:, :32]
    res = np.linalg.norm(p.A @ Xg - p.B @ Xg * np.array(ev[:32])[None, :], axis=0)
    assert np.max(res) < 1e-9


def test_complex_context_limits(herm):
    p, lmax = herm
    A = P.to_colmajor_complex(p.A)
    prm = P.make_params(p.n_wanted, p.block, 8, method=P.METHOD_CHFSI, filter_prec=P.PREC_FP64,
                        lambda_max=lmax)
    with pytest.raises(RuntimeError, match="residual filter"):
        P.chfsi_create(P.hermitian_operator(A), None, None, prm, keep=(A,))


def test_complex_standard_problem_padded_leading_dimensions():
    """B = I (D^{-1} = I), blocks with padded leading dimensions, block 37."""
    p = wl.dense_hermitian(n=517, n_low=30, block=37, degree=12, seed=81, generalized=False)
    w = np.linalg.eigvalsh(p.A)[:30]
    A = P.to_colmajor_complex(p.A)
    prm = P.make_params(30, 37, 12, max_iter=60, tol=1e-10, method=P.METHOD_RCHFSI,
                        filter_prec=P.PREC_FP32, lambda_max=10.1)
    ctx = P.chfsi_create(P.hermitian_operator(A), None, None, prm, keep=(A,))
    ld = 530
    buf = torch.zeros((37, ld), dtype=torch.complex128, device="cuda")
    X = buf.t()[:517]
    X.copy_(P.to_colmajor_complex(wl.random_block_complex(517, 37, 12)))
    assert X.stride(1) == ld
    st, ev, rn, rep = P.chfsi_solve(ctx, X)
    print("complex standard solve:", rep["iterations"], "iterations, max residual",
          rep["max_residual"])
    assert st == P.OK
    assert np.max(np.abs(np.array(ev[:30]) - w)) <= 1e-10 * np.max(np.abs(w))
    assert torch.all(buf.t()[517:] == 0)          # the padding rows are untouched
    # the filter on padded blocks matches the oracle (D^{-1} = I)
    o = rr.rayleigh_ritz(wl.random_block_complex(517, 37, 13), filters.dense_op(p.A),
                         filters.identity_op())
    lam = o["lam"]
    bounds = (lam[0] - 0.05 * (lam[-1] - lam[0]), 10.1, lam[-1])
    Xb = torch.zeros((37, ld), dtype=torch.complex128, device="cuda").t()[:517]
    Rb = torch.zeros((37, ld), dtype=torch.complex128, device="cuda").t()[:517]
    Yb = torch.zeros((37, ld), dtype=torch.complex128, device="cuda").t()[:517]
    Xb.copy_(P.to_colmajor_complex(o["X"]))
    Rb.copy_(P.to_colmajor_complex(o["R"]))
    P.chfsi_filter(ctx, Xb, lam, Rb, Yb, *bounds, degree=12)
    torch.cuda.synchronize()
    ref, RYp, _ = filters.residual_filter(filters.dense_op(p.A), filters.identity_op(), o["X"], lam,
                                          o["R"], 12, *bounds, return_parts=True)
    assert np.linalg.norm(Yb.cpu().numpy() - ref) <= 1e-4 * np.linalg.norm(RYp)


def test_complex_rayleigh_ritz_singular_gram_uses_svqb(herm):
    """A block with a repeated column: the embedded Gram matrix has a zero
    eigenvalue pair, the SVQB reading keeps the b - 1 independent complex
    directions (here an invariant subspace, so their Ritz values are exact
    eigenvalues), refills one column and repeats Rayleigh-Ritz."""
    p, lmax = herm
    ctx = _ctx(p, P.PREC_FP32, lmax, 8)
    w, U = sla.eigh(p.A, p.B)
    Y = U[:, : p.block].copy()
    Y[:, -1] = Y[:, 0]
    X = P.colmajor_empty_complex(p.n, p.block)
    R = P.colmajor_empty_complex(p.n, p.block)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, P.to_colmajor_complex(Y), X, R)
    ritz = np.asarray(ritz)
    for lam in w[: p.block - 1]:
        assert np.min(np.abs(ritz - lam)) <= 1e-10 * max(1.0, abs(lam))
    Xg = X.cpu().numpy()
    assert np.linalg.norm(Xg.conj().T @ p.B @ Xg - np.eye(p.block)) <= 1e-9
    Rg = p.A @ Xg - (p.B @ Xg) * ritz[None, :]
    np.testing.assert_allclose(norms, np.linalg.norm(Rg, axis=0), rtol=1e-6, atol=1e-9)
    assert np.linalg.norm(R.cpu().numpy() - Rg) <= 1e-9 * np.linalg.norm(p.A, 2)


def test_complex_rayleigh_ritz_equal_ritz_values():
    """Equal Ritz values: a block spanning an invariant subspace with a 6-fold
    and a double eigenvalue.  The embedded problem's eigenspaces of equal
    values are 12- and 4-dimensional, and the complex Ritz vectors must still
    be an orthonormal basis of them."""
    n, b = 300, 12
    lam = np.concatenate([[-1.0], np.full(6, -0.5), [0.0, 0.0, 0.25], np.linspace(1.0, 10.0, n - 10)])
    rng = np.random.default_rng(61)
    A = wl.hermitian_from_spectrum(lam, wl.complex_householder_vectors(rng, n, 8))
    A = 0.5 * (A + A.conj().T)
    w, U = np.linalg.eigh(A)
    # a basis of the lowest 12 eigenvectors, mixed within the span (not orthonormal)
    M = rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b))
    Y = U[:, :b] @ M
    Ad = P.to_colmajor_complex(A)
    prm = P.make_params(b, b, 4, method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP64, lambda_max=10.5)
    ctx = P.chfsi_create(P.hermitian_operator(Ad), None, None, prm, keep=(Ad,))
    X, R = P.colmajor_empty_complex(n, b), P.colmajor_empty_complex(n, b)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, P.to_colmajor_complex(Y), X, R)
    np.testing.assert_allclose(ritz, w[:b], rtol=0, atol=1e-11)
    Xg = X.cpu().numpy()
    assert np.linalg.norm(Xg.conj().T @ Xg - np.eye(b)) <= 1e-10
    assert np.max(np.linalg.norm(A @ Xg - Xg * np.array(ritz)[None, :], axis=0)) <= 1e-10
    assert np.max(norms) <= 1e-10
