"""GPU parity of the Lanczos bound estimate (chfsi_estimate_bounds) against
oracle.bounds, and solves with lambda_max = NaN (estimated inside the library).

The filter's bounds are estimates (Section 2.1).  Both sides run k Lanczos
steps on B^{-1} A in the B-inner product from the same seeded start vector;
the library solves with B by preconditioned CG to relative residual 1e-10,
the oracle exactly, so the Ritz values theta_1, theta_k and the safeguarded
estimates agree to ~1e-10.  Pencils: the dense generalized recipe (dense B,
D^{-1} preconditioner), the grid pencil with wells (mass matrix B, no
preconditioner), a complex Hermitian dense pencil and a Bloch grid pencil.
Solves with lambda_max = NaN reach LAPACK's eigenvalues like the solves with
a given bound (dense N = 1536 and the 8^3 grid).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import bounds, stencil

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402

STEPS = 12


def _dense_ops(A, B):
    cf = sla.cho_factor(B)
    return (lambda x: A @ x), (lambda x: B @ x), (lambda y: sla.cho_solve(cf, y))


def _compare(ctx, v0_dev, ref, w, label):
    lo, hi, tmin, tmax = P.chfsi_estimate_bounds(ctx, v0_dev, STEPS)
    scale = np.abs(w).max()
    print(f"{label}: GPU theta [{tmin:.12g}, {tmax:.12g}] bounds [{lo:.12g}, {hi:.12g}]; "
          f"oracle theta [{ref['theta'][0]:.12g}, {ref['theta'][-1]:.12g}] bounds "
          f"[{ref['lower']:.12g}, {ref['upper']:.12g}]; spectrum [{w[0]:.12g}, {w[-1]:.12g}]",
          flush=True)
    for g, o in ((tmin, ref["theta"][0]), (tmax, ref["theta"][-1]), (lo, ref["lower"]),
                 (hi, ref["upper"])):
        assert abs(g - o) <= 1e-9 * scale, (label, g, o)
    assert hi >= w[-1] and lo <= w[0]


def test_bounds_dense_generalized():
    p = wl.dense_generalized(n=700, n_low=24, block=32, degree=12, seed=21)
    w = sla.eigvalsh(p.A, p.B)
    A, B = P.to_colmajor(p.A), P.to_colmajor(p.B)
    d = torch.from_numpy(p.dinv).cuda()
    prm = P.make_params(24, 32, 12, method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP32)
    ctx = P.chfsi_create(P.dense_operator(A), P.dense_operator(B), d, prm, keep=(A, B, d))
    v0 = wl.random_block(p.n, 1, 5)[:, 0]
    ref = bounds.lanczos_bounds(*_dense_ops(p.A, p.B), v0, STEPS)
    _compare(ctx, torch.from_numpy(v0).cuda(), ref, w, "dense generalized N=700")


def test_bounds_grid_with_wells():
    shape = (8, 10, 12)
    rng = np.random.default_rng(4)
    V, _ = wl.gaussian_wells(shape, 3, rng)
    cA = 0.5 * wl.tensor_stencil_27("stiffness")
    cB = wl.tensor_stencil_27("mass")
    apply_A, apply_B = stencil.make_ops(cA, cB, V, shape, 2)
    n = int(np.prod(shape))
    I = np.eye(n)
    Am, Bm = apply_A(I), apply_B(I)
    Am, Bm = 0.5 * (Am + Am.T), 0.5 * (Bm + Bm.T)
    w = sla.eigvalsh(Am, Bm)
    Vd = torch.from_numpy(np.ascontiguousarray(V).reshape(-1)).cuda()
    opA = P.stencil_operator(shape, cA, coef_mass=cB, field=Vd, field_mode=2)
    opB = P.stencil_operator(shape, cB)
    prm = P.make_params(6, 8, 8, method=P.METHOD_RCHFSI, filter_prec=P.PREC_BF16)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    v0 = wl.random_block(n, 1, 6)[:, 0]
    ref = bounds.lanczos_bounds(*_dense_ops(Am, Bm), v0, STEPS)
    _compare(ctx, torch.from_numpy(v0).cuda(), ref, w, "grid (8,10,12) with wells")


def test_bounds_complex_hermitian():
    rng = np.random.default_rng(8)
    n = 300
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Ah = 0.5 * (G + G.conj().T)
    H = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Bh = np.eye(n) + (0.05 / n) * (H @ H.conj().T)
    w = sla.eigvalsh(Ah, Bh)
    A, B = P.to_colmajor_complex(Ah), P.to_colmajor_complex(Bh)
    prm = P.make_params(8, 12, 8, method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP32)
    ctx = P.chfsi_create(P.hermitian_operator(A), P.hermitian_operator(B), None, prm, keep=(A, B))
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = bounds.lanczos_bounds(*_dense_ops(Ah, Bh), v0, STEPS)
    _compare(ctx, torch.from_numpy(v0).cuda(), ref, w, "complex Hermitian N=300")


def test_bounds_bloch_grid():
    shape, k = (6, 8, 10), (0.3, -0.7, 1.1)
    rng = np.random.default_rng(9)
    V, _ = wl.gaussian_wells(shape, 2, rng)
    cA = 0.5 * wl.tensor_stencil_27("stiffness")
    cB = wl.tensor_stencil_27("mass")
    apply_A, apply_B = stencil.make_ops_bloch(cA, cB, V, shape, 2, k)
    n = int(np.prod(shape))
    I = np.eye(n, dtype=np.complex128)
    Am, Bm = apply_A(I), apply_B(I)
    Am, Bm = 0.5 * (Am + Am.conj().T), 0.5 * (Bm + Bm.conj().T)
    w = sla.eigvalsh(Am, Bm)
    Vd = torch.from_numpy(np.ascontiguousarray(V).reshape(-1)).cuda()
    opA = P.stencil_operator(shape, cA, coef_mass=cB, field=Vd, field_mode=2, bloch=k)
    opB = P.stencil_operator(shape, cB, bloch=k)
    prm = P.make_params(6, 8, 8, method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP64)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = bounds.lanczos_bounds(*_dense_ops(Am, Bm), v0, STEPS)
    _compare(ctx, torch.from_numpy(v0).cuda(), ref, w, "Bloch grid (6,8,10)")


@pytest.mark.parametrize("prec", [P.PREC_FP32, P.PREC_BF16])
def test_solve_dense_with_estimated_lambda_max(prec):
    p = wl.dense_generalized(n=1536, n_low=48, block=64, degree=20, seed=1001)
    w = sla.eigvalsh(p.A, p.B)
    A, B = P.to_colmajor(p.A), P.to_colmajor(p.B)
    d = torch.from_numpy(p.dinv).cuda()
    prm = P.make_params(48, 64, 20, max_iter=40, tol=1e-9, method=P.METHOD_RCHFSI,
                        filter_prec=prec)          # lambda_max = NaN: estimated
    ctx = P.chfsi_create(P.dense_operator(A), P.dense_operator(B), d, prm, keep=(A, B, d))
    Xd = P.to_colmajor(wl.random_block(p.n, 64, 2001))
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    print(prec, rep["iterations"], "lambda_max used %.6g (true %.6g), estimate %.1f ms"
          % (rep["lambda_max_used"], w[-1], rep["time_bounds_ms"]))
    assert st == P.OK
    assert rep["lambda_max_used"] >= w[-1]
    scale = 1e-3 * max(abs(w[0]), abs(w[-1]))
    rel = np.abs(np.asarray(ev[:48]) - w[:48]) / np.maximum(np.abs(w[:48]), scale)
    assert rel.max() <= 1e-10


@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_BF16])
def test_solve_grid_with_estimated_lambda_max(prec):
    shape = (8, 8, 8)
    rng = np.random.default_rng(5)
    V, _ = wl.gaussian_wells(shape, 2, rng)
    cA = 0.5 * wl.tensor_stencil_27("stiffness")
    cB = wl.tensor_stencil_27("mass")
    apply_A, apply_B = stencil.make_ops(cA, cB, V, shape, 2)
    I = np.eye(512)
    w = sla.eigvalsh(apply_A(I), apply_B(I))
    Vd = torch.from_numpy(np.ascontiguousarray(V).reshape(-1)).cuda()
    opA = P.stencil_operator(shape, cA, coef_mass=cB, field=Vd, field_mode=2)
    opB = P.stencil_operator(shape, cB)
    prm = P.make_params(6, 8, 8, max_iter=200, tol=1e-9, method=P.METHOD_RCHFSI,
                        filter_prec=prec)          # lambda_max = NaN: estimated
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    Xd = P.to_colmajor(wl.random_block(512, 8, 31))
    st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
    print(prec, rep["iterations"], "lambda_max used %.6g (true %.6g)"
          % (rep["lambda_max_used"], w[-1]))
    assert st == P.OK
    assert rep["lambda_max_used"] >= w[-1]
    np.testing.assert_allclose(ev[:6], w[:6], rtol=1e-9, atol=1e-10)


def test_overlapped_estimate_matches_sequential(monkeypatch):
    """The estimate of lambda_max made on a second stream during the first
    Rayleigh-Ritz pass (dense real operators) is bit-identical to the one made
    before it on the context's stream (knob CHFSI_LANCZOS_OVERLAP=0), and so is
    the whole solve."""
    p = wl.dense_generalized(n=1536, n_low=48, block=64, degree=20, seed=1001)
    A, B = P.to_colmajor(p.A), P.to_colmajor(p.B)
    d = torch.from_numpy(p.dinv).cuda()
    out = {}
    for knob in ("0", "1"):
        monkeypatch.setenv("CHFSI_LANCZOS_OVERLAP", knob)
        prm = P.make_params(48, 64, 20, max_iter=40, tol=1e-9, method=P.METHOD_RCHFSI,
                            filter_prec=P.PREC_FP32)          # lambda_max = NaN: estimated
        ctx = P.chfsi_create(P.dense_operator(A), P.dense_operator(B), d, prm, keep=(A, B, d))
        Xd = P.to_colmajor(wl.random_block(p.n, 64, 2001))
        print("solve with the estimate overlapped:", knob, flush=True)
        st, ev, rn, rep = P.chfsi_solve(ctx, Xd)
        assert st == P.OK
        out[knob] = (rep["lambda_max_used"], rep["iterations"], np.asarray(ev), np.asarray(rn),
                     Xd.cpu().numpy())
        print(knob, rep["lambda_max_used"], rep["iterations"], rep["time_bounds_ms"],
              rep["time_total_ms"] if "time_total_ms" in rep else "")
    a, b = out["0"], out["1"]
    assert a[0] == b[0] and a[1] == b[1]
    for x, y in zip(a[2:], b[2:]):
        assert np.array_equal(x, y)
