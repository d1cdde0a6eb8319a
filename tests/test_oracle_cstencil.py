"""Pins for the oracle's C grid kernels (oracle/stencil27.c via oracle.cstencil):
the pencil application and Algorithm 3 agree with the NumPy oracle
(``stencil.make_ops``, ``filters.residual_filter``) to FP64 rounding on ragged
grids, for every field_mode, with D^{-1} = I and with a diagonal D^{-1}."""
import numpy as np
import pytest

import workloads as wl
from oracle import cstencil, filters, stencil


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_c_pencil_apply_matches_numpy(mode):
    shape = (5, 7, 9)
    rng = np.random.default_rng(mode)
    V, _ = wl.gaussian_wells(shape, 2, rng)
    cA = 0.5 * wl.tensor_stencil_27("stiffness")
    cB = wl.tensor_stencil_27("mass")
    apply_A, _ = stencil.make_ops(cA, cB, V, shape, mode)
    x = rng.standard_normal(int(np.prod(shape)))
    ref = apply_A(x)
    got = cstencil.pencil_apply(cA, cB, V, mode, shape, x)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("use_dinv", [False, True])
def test_c_residual_filter_matches_numpy(use_dinv):
    shape = (6, 8, 10)
    rng = np.random.default_rng(11)
    V, _ = wl.gaussian_wells(shape, 3, rng)
    cA = 0.5 * wl.tensor_stencil_27("stiffness")
    cB = wl.tensor_stencil_27("mass")
    apply_A, _ = stencil.make_ops(cA, cB, V, shape, 2)
    n, b, p = int(np.prod(shape)), 5, 12
    X = rng.standard_normal((n, b))
    R = 1e-2 * rng.standard_normal((n, b))
    lam = np.sort(rng.uniform(-4.0, 0.5, b))
    dinv = rng.uniform(0.8, 1.2, n) if use_dinv else None
    bounds = (-4.5, 18.5, 0.6)
    Dop = filters.diag_op(dinv) if use_dinv else filters.identity_op()
    ref = filters.residual_filter(apply_A, Dop, X, lam, R, p, *bounds)
    got = cstencil.rchfsi_filter(cA, cB, V, 2, shape, dinv, X, lam, R, p, *bounds)
    err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= 1e-12, err
