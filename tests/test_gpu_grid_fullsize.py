"""Parity of the grid pencil's BF16 residual filter at full size (128^3
periodic grid, 64 Gaussian wells, mass-weighted potential, block 1200), in the
launch configuration that bench.py's grid workload times.

The filter is column-independent (Lambda is diagonal), so the oracle filters a
sample of columns exactly and the GPU block must agree on those columns, with
an error bounded by the residual part it carries (Theorem 3.4).  The sample
takes every position of one column group and the last column.  Degree 4 runs
three recurrence steps -- the same kernel launch as each step of the degree-30
filter -- and keeps the oracle within seconds.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import filters, stencil
from parity import GRID_TERMS, assert_columns, residual_part

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402


def test_bf16_grid_filter_fullsize_sampled_columns():
    prob = wl.stencil_problem()
    shape, b = prob.shape, prob.block
    n = int(np.prod(shape))
    apply_A, _ = stencil.make_ops(prob.coef_A, prob.coef_B, prob.V, shape, prob.field_mode)
    Vd = torch.from_numpy(np.ascontiguousarray(prob.V).reshape(-1)).cuda()
    opA = P.stencil_operator(shape, prob.coef_A, coef_mass=prob.coef_B, field=Vd,
                             field_mode=prob.field_mode)
    opB = P.stencil_operator(shape, prob.coef_B)
    prm = P.make_params(prob.n_wanted, b, prob.degree, method=P.METHOD_RCHFSI,
                        filter_prec=P.PREC_BF16, lambda_max=18.5, memory_mode=1)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    g = torch.Generator(device="cuda")
    g.manual_seed(2002)
    X = torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g).t()
    R = torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g).t().mul_(1e-3)
    lam = np.sort(np.random.default_rng(2002).uniform(-4.0, 1.0, b))
    bounds = (lam[0] - 0.5, 18.5, lam[-1])
    Y = P.colmajor_empty(n, b)
    print("grid 128^3 b=1200 BF16 filter, degree 4", flush=True)
    P.chfsi_filter(ctx, X, lam, R, Y, *bounds, degree=4)
    torch.cuda.synchronize()
    cols = [0, 1, 2, 3, 1199]
    Xc = X[:, cols].cpu().numpy()
    Rc = R[:, cols].cpu().numpy()
    got = Y[:, cols].cpu().numpy()
    del X, R, Y
    ref, RYp, _ = filters.residual_filter(apply_A, filters.identity_op(), Xc, lam[cols], Rc, 4,
                                          *bounds, return_parts=True)
    assert np.all(np.isfinite(got))
    assert_columns(got, ref, residual_part(RYp), "bf16", 4, GRID_TERMS, "grid full size")


def test_bf16_bloch_grid_filter_fullsize_sampled_columns():
    """The same pencil at wave vector k = (0.013, -0.021, 0.034) (complex, Section
    4.3) with 600 complex vectors -- the 1200 planar columns of the real case --
    as bench.py's grid workload with --bloch times it."""
    k = (0.013, -0.021, 0.034)
    torch.cuda.empty_cache()          # the complex context needs about 175 GiB
    prob = wl.stencil_problem()
    shape, b = prob.shape, prob.block // 2
    n = int(np.prod(shape))
    apply_A, _ = stencil.make_ops_bloch(prob.coef_A, prob.coef_B, prob.V, shape, prob.field_mode,
                                        k)
    Vd = torch.from_numpy(np.ascontiguousarray(prob.V).reshape(-1)).cuda()
    opA = P.stencil_operator(shape, prob.coef_A, coef_mass=prob.coef_B, field=Vd,
                             field_mode=prob.field_mode, bloch=k)
    opB = P.stencil_operator(shape, prob.coef_B, bloch=k)
    prm = P.make_params(prob.n_wanted // 2, b, prob.degree, method=P.METHOD_RCHFSI,
                        filter_prec=P.PREC_BF16, lambda_max=18.5)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    g = torch.Generator(device="cuda")
    g.manual_seed(2003)
    X = torch.randn((b, n), dtype=torch.complex128, device="cuda", generator=g).t()
    R = torch.randn((b, n), dtype=torch.complex128, device="cuda", generator=g).t().mul_(1e-3)
    lam = np.sort(np.random.default_rng(2003).uniform(-4.0, 1.0, b))
    bounds = (lam[0] - 0.5, 18.5, lam[-1])
    Y = P.colmajor_empty_complex(n, b)
    print("Bloch grid 128^3 b=600 complex BF16 filter, degree 4", flush=True)
    P.chfsi_filter(ctx, X, lam, R, Y, *bounds, degree=4)
    torch.cuda.synchronize()
    cols = [0, 1, 2, 3, b - 1]
    Xc = X[:, cols].cpu().numpy()
    Rc = R[:, cols].cpu().numpy()
    got = Y[:, cols].cpu().numpy()
    del X, R, Y
    ctx.close()
    ref, RYp, _ = filters.residual_filter(apply_A, filters.identity_op(), Xc, lam[cols], Rc, 4,
                                          *bounds, return_parts=True)
    assert np.all(np.isfinite(got))
    assert_columns(got, ref, residual_part(RYp), "bf16", 4, GRID_TERMS, "grid full size")


def test_bf16_grid160_filter_fullsize_sampled_columns():
    """The 160^3 pencil with 200 Gaussian wells (N = 4.1M), BF16 residual filter.
    The 2400-column block of the large grid workload leaves no room for FP64
    copies of X, R and Y beside it (79 GB each), so this runs 240 columns: the
    column groups are independent, and each is launched with the same tile
    shape (rows of 160 points, the same slab height) as in the full block."""
    torch.cuda.empty_cache()
    prob = wl.stencil_problem(grid=160, n_wells=200, n_wanted=2000, block=2400, degree=40,
                              seed=1004)
    shape, b = prob.shape, 240
    n = int(np.prod(shape))
    apply_A, _ = stencil.make_ops(prob.coef_A, prob.coef_B, prob.V, shape, prob.field_mode)
    Vd = torch.from_numpy(np.ascontiguousarray(prob.V).reshape(-1)).cuda()
    opA = P.stencil_operator(shape, prob.coef_A, coef_mass=prob.coef_B, field=Vd,
                             field_mode=prob.field_mode)
    opB = P.stencil_operator(shape, prob.coef_B)
    prm = P.make_params(200, b, prob.degree, method=P.METHOD_RCHFSI, filter_prec=P.PREC_BF16,
                        lambda_max=18.5, memory_mode=1)
    ctx = P.chfsi_create(opA, opB, None, prm, keep=(Vd,))
    g = torch.Generator(device="cuda")
    g.manual_seed(2004)
    X = torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g).t()
    R = torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g).t().mul_(1e-3)
    lam = np.sort(np.random.default_rng(2004).uniform(-4.0, 1.0, b))
    bounds = (lam[0] - 0.5, 18.5, lam[-1])
    Y = P.colmajor_empty(n, b)
    print("grid 160^3 b=240 BF16 filter, degree 4", flush=True)
    P.chfsi_filter(ctx, X, lam, R, Y, *bounds, degree=4)
    torch.cuda.synchronize()
    cols = [0, 1, 2, 3, 121, b - 1]
    Xc = X[:, cols].cpu().numpy()
    Rc = R[:, cols].cpu().numpy()
    got = Y[:, cols].cpu().numpy()
    del X, R, Y
    ctx.close()
    ref, RYp, _ = filters.residual_filter(apply_A, filters.identity_op(), Xc, lam[cols], Rc, 4,
                                          *bounds, return_parts=True)
    assert np.all(np.isfinite(got))
    assert_columns(got, ref, residual_part(RYp), "bf16", 4, GRID_TERMS, "grid full size")
