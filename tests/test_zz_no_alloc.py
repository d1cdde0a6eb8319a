"""The filter entry point that allocates nothing (chfsi_filter_static) against
the context-based FP64 residual filter (chfsi_filter), through the C ABI.

Two calls in a row on the static scratch array, the second with a smaller
input (fewer rows and columns, lower degree), for a dense pencil and for a
27-point grid pencil: every column agrees with chfsi_filter's within the FP64
per-column bound of tests/parity.py (both run the same kernels; only the
split-K factor of the dense product may differ).  Inputs beyond the static
array's size are refused with CHFSI_ERR_ARG before any work is queued.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import filters, rr, stencil
from parity import GRID_TERMS, assert_columns

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402


def _inputs(apply_A, apply_B, n, b, seed):
    o = rr.rayleigh_ritz(wl.random_block(n, b, seed), apply_A, apply_B)
    return o["X"], o["lam"], o["R"]


def _pair(opA, dinv_d, keep, X, lam, R, bounds, degree, terms, label):
    n, b = X.shape
    prm = P.make_params(min(b, 4), b, degree, method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP64,
                        lambda_max=bounds[1])
    ctx = P.chfsi_create(opA, None, dinv_d, prm, keep=keep)
    Xd, Rd = P.to_colmajor(X), P.to_colmajor(R)
    Y_ctx = P.colmajor_empty(n, b)
    P.chfsi_filter(ctx, Xd, lam, Rd, Y_ctx, *bounds, degree=degree)
    Y_static = P.colmajor_empty(n, b)
    ritz_d = torch.tensor(np.asarray(lam, dtype=np.float64), device="cuda")
    P.chfsi_filter_static(opA, dinv_d, Xd, ritz_d, Rd, Y_static, *bounds, degree=degree)
    torch.cuda.synchronize()
    got, ref = Y_static.cpu().numpy(), Y_ctx.cpu().numpy()
    print(f"{label}: n={n} b={b} p={degree} bitwise equal: {np.array_equal(got, ref)}", flush=True)
    assert_columns(got, ref, np.linalg.norm(ref, axis=0), "fp64", degree, terms, label)
    ctx.close()


def test_static_filter_dense_two_calls():
    for i, (n, b, p, seed) in enumerate(((640, 48, 14, 11), (300, 20, 9, 12))):
        rng = np.random.default_rng(seed)
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam = np.concatenate([np.linspace(-1.0, -0.2, b // 2), rng.uniform(0.0, 10.0, n - b // 2)])
        A = (Q * lam) @ Q.T
        A = 0.5 * (A + A.T)
        d = rng.uniform(0.5, 2.0, n)
        B = np.diag(d)
        Ad = P.to_colmajor(A)
        dd = torch.from_numpy(1.0 / d).cuda()
        opA = P.dense_operator(Ad)
        if i == 0:
            # b = 0: binds the static array on this device and queues nothing
            P.chfsi_filter_static(opA, dd, None, None, None, None, -1.0, 1.0, 0.0, 1)
        w = sla.eigvalsh(A, B)
        X, lam_r, R = _inputs(filters.dense_op(A), filters.dense_op(B), n, b, seed + 100)
        bounds = (float(w[0]) - 0.1, float(w[-1]) + 0.5, float(lam_r[-1]))
        _pair(opA, dd, (Ad, dd), X, lam_r, R, bounds, p, n, f"dense call n={n}")


def test_static_filter_grid_two_calls():
    for shape, b, p, seed in (((9, 10, 12), 12, 10, 8), ((6, 9, 10), 5, 6, 9)):
        rng = np.random.default_rng(seed)
        V, _ = wl.gaussian_wells(shape, 3, rng)
        cA = 0.5 * wl.tensor_stencil_27("stiffness")
        cB = wl.tensor_stencil_27("mass")
        apply_A, apply_B = stencil.make_ops(cA, cB, V, shape, 2)
        n = int(np.prod(shape))
        Vd = torch.from_numpy(np.ascontiguousarray(V).reshape(-1)).cuda()
        opA = P.stencil_operator(shape, cA, coef_mass=cB, field=Vd, field_mode=2)
        X, lam_r, R = _inputs(apply_A, apply_B, n, b, seed + 100)
        bounds = (float(lam_r[0]) - 6.0, 18.5, float(lam_r[-1]))
        _pair(opA, None, (Vd,), X, lam_r, R, bounds, p, GRID_TERMS, f"grid call {shape}")


def test_static_filter_refuses_oversized_input():
    shape = (160, 160, 160)
    opA = P.stencil_operator(shape, 0.5 * wl.tensor_stencil_27("stiffness"))
    need = P.chfsi_filter_static_bytes(opA.n, 2400, 40)
    assert need > P.STATIC_SCRATCH_BYTES
    # the size check comes before any use of the (here never dereferenced) blocks
    fake = torch.empty(1, dtype=torch.float64, device="cuda")
    lib = P.lib()
    p = fake.data_ptr()
    st = lib.chfsi_filter_static(P.C.byref(opA), None, 2400, p, opA.n, p, p, opA.n, p, opA.n,
                                 -1.0, 18.5, 0.0, 40, None)
    assert st == P.ERR_ARG
    assert "static scratch" in P.chfsi_last_error()
