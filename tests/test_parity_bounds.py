"""The per-column parity bounds of tests/parity.py, checked on the CPU.

1. FP32 and bfloat16 arithmetic of the residual filter (Algorithm 3), emulated
   with numpy float32 and round-to-nearest-even bfloat16, stays within the
   bounds on the dense and grid shapes the GPU tests use.
2. A mistake planted in the oracle -- one step's product term scaled by
   (1 + 1e-3), i.e. one coefficient a_k wrong by 1e-3 -- breaks the FP32 and
   FP64 bounds on every one of those shapes, so the GPU parity tests would
   catch it.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import filters, rr, stencil
from parity import GRID_TERMS, bound, column_errors, residual_part


def _bf16(x):
    x = np.ascontiguousarray(np.asarray(x, np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _emulated_filter(apply32, dinv, X, lam, Yres, p, lmin, lmax, lT, mode):
    """Algorithm 3 in reduced precision.  mode 'fp32': FP32 blocks and products;
    'bf16_products': the product's inputs rounded to bfloat16 (apply32 holds the
    rounded operator), FP32 blocks; 'bf16_storage': blocks stored in bfloat16,
    FP32 arithmetic.  Coefficients are FP64 rounded once to FP32."""
    f = np.float32
    store = _bf16 if mode == "bf16_storage" else (lambda v: np.asarray(v, f))
    e, c = (lmax - lT) / 2, (lmax + lT) / 2
    sigma = e / (lmin - c)
    s1, gamma = sigma, 2 / sigma
    Yc = store(Yres)
    RX = store(np.zeros_like(Yres))
    RY = store((s1 / e) * Yres)
    LX, LY = np.ones_like(lam), (s1 / e) * (lam - c)
    d32 = np.asarray(dinv, f)[:, None]
    for _k in range(2, p + 1):
        s2 = 1 / (gamma - sigma)
        a = 2 * s2 / e
        Z = (d32 * RY.astype(f)).astype(f)
        if mode == "bf16_products":
            Z = _bf16(Z)
        new = (f(a) * apply32(Z) + f(-a * c) * RY.astype(f) + f(-sigma * s2) * RX.astype(f)
               + f(a) * Yc.astype(f) * LY.astype(f)[None, :])
        RX = store(new)
        LX = a * LY * lam - a * c * LY - sigma * s2 * LX
        RX, RY, LX, LY = RY, RX, LY, LX
        sigma = s2
    return np.asarray(dinv)[:, None] * RY.astype(np.float64) + X * LY[None, :]


def _planted(apply_A, step):
    """apply_A whose `step`-th call (1-based) returns (1 + 1e-3) times the product."""
    calls = {"n": 0}

    def op(V):
        calls["n"] += 1
        out = apply_A(V)
        return out * (1 + 1e-3) if calls["n"] == step else out
    return op


@pytest.fixture(scope="module")
def dense_case():
    p = wl.dense_generalized(n=701, n_low=24, block=40, degree=8, seed=77)
    w = sla.eigvalsh(p.A, p.B)
    bounds = (w[0] - 0.1, w[-1] + 0.5, 0.5 * (w[39] + w[40]))
    o = rr.rayleigh_ritz(wl.random_block(701, 40, 5), filters.dense_op(p.A), filters.dense_op(p.B))
    return p, bounds, o


GRID_SHAPES = [(9, 10, 12), (5, 20, 64), (4, 30, 40)]


def _grid_case(shape):
    V, _ = wl.gaussian_wells(shape, 3, np.random.default_rng(8))
    cA, cB = 0.5 * wl.tensor_stencil_27("stiffness"), wl.tensor_stencil_27("mass")
    aA, aB = stencil.make_ops(cA, cB, V, shape, 2)
    n = int(np.prod(shape))
    o = rr.rayleigh_ritz(wl.random_block(n, 9, 4), aA, aB)
    return aA, o, (o["lam"][0] - 0.5, 18.5, o["lam"][-1])


@pytest.mark.parametrize("degree", [2, 8, 20])
def test_dense_emulated_arithmetic_within_bounds(dense_case, degree):
    p, bnd, o = dense_case
    ref, RYp, _ = filters.residual_filter(filters.dense_op(p.A), filters.diag_op(p.dinv), o["X"],
                                          o["lam"], o["R"], degree, *bnd, return_parts=True)
    part = residual_part(RYp, p.dinv)
    A32, A16 = p.A.astype(np.float32), _bf16(p.A)
    got = _emulated_filter(lambda V: A32 @ V, p.dinv, o["X"], o["lam"], o["R"], degree, *bnd,
                           "fp32")
    assert column_errors(got, ref, part).max() <= bound("fp32", degree, p.n)
    got = _emulated_filter(lambda V: A16 @ V, p.dinv, o["X"], o["lam"], o["R"], degree, *bnd,
                           "bf16_products")
    assert column_errors(got, ref, part).max() <= bound("bf16", degree, p.n)


@pytest.mark.parametrize("shape", GRID_SHAPES)
@pytest.mark.parametrize("degree", [4, 10, 30])
def test_grid_emulated_arithmetic_within_bounds(shape, degree):
    aA, o, bnd = _grid_case(shape)
    ones = np.ones(o["X"].shape[0])
    ref, RYp, _ = filters.residual_filter(aA, filters.identity_op(), o["X"], o["lam"], o["R"],
                                          degree, *bnd, return_parts=True)
    part = residual_part(RYp)
    a32 = lambda V: aA(V.astype(np.float64)).astype(np.float32)   # noqa: E731
    for mode, prec in (("fp32", "fp32"), ("bf16_storage", "bf16")):
        got = _emulated_filter(a32, ones, o["X"], o["lam"], o["R"], degree, *bnd, mode)
        assert column_errors(got, ref, part).max() <= bound(prec, degree, GRID_TERMS), mode


@pytest.mark.parametrize("degree", [8, 20])
def test_planted_coefficient_error_breaks_dense_bounds(dense_case, degree):
    p, bnd, o = dense_case
    ref, RYp, _ = filters.residual_filter(filters.dense_op(p.A), filters.diag_op(p.dinv), o["X"],
                                          o["lam"], o["R"], degree, *bnd, return_parts=True)
    bad = filters.residual_filter(_planted(filters.dense_op(p.A), degree // 2),
                                  filters.diag_op(p.dinv), o["X"], o["lam"], o["R"], degree, *bnd)
    r = column_errors(bad, ref, residual_part(RYp, p.dinv))
    assert r.max() > 10 * bound("fp32", degree, p.n)
    # the largest dense FP32 parity case (n = 8192) still resolves it
    assert r.max() > 3 * bound("fp32", degree, 8192)
    assert column_errors(bad, ref, np.linalg.norm(ref, axis=0)).max() > 1e3 * bound(
        "fp64", degree, p.n)


@pytest.mark.parametrize("shape", GRID_SHAPES)
@pytest.mark.parametrize("degree", [4, 10, 30])
def test_planted_coefficient_error_breaks_grid_bounds(shape, degree):
    aA, o, bnd = _grid_case(shape)
    ref, RYp, _ = filters.residual_filter(aA, filters.identity_op(), o["X"], o["lam"], o["R"],
                                          degree, *bnd, return_parts=True)
    bad = filters.residual_filter(_planted(aA, degree // 2), filters.identity_op(), o["X"],
                                  o["lam"], o["R"], degree, *bnd)
    r = column_errors(bad, ref, residual_part(RYp))
    assert r.max() > 10 * bound("fp32", degree, GRID_TERMS)
