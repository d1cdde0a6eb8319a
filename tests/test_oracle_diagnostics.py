"""Pins for oracle.diagnostics (the convergence condition of Section 3.1, as
verified in the controlled experiment of Section 4.1.3).

* The B^{1/2} norm helper equals the norm formed with an explicit B^{1/2}.
* With D^{-1} = B^{-1} the filtering error is zero to rounding for both
  methods (Algorithm 3 is an identity rewrite of Algorithm 2).
* Theorem 3.1: at every iteration whose premise holds, the angle of the
  filtered span is within the bound computed from the measured error, angle
  and the two Chebyshev values (any slip in C_p's scaling, the B-norm or the
  angle breaks it where the bound is tight, near convergence of ChFSI).
* Generalized toy problem, zeta = 1e-3 (the setting of Section 4.1.3):
  - ChFSI: the error saturates at O(zeta) and the condition is violated once
    the subspace is close (the two sides cross); the residual stalls.
  - R-ChFSI: the error tracks the residual norm (Theorem 3.4: ||Delta|| is
    bounded by a constant times ||R||) and the condition holds at every
    iteration between the random start and the machine-precision floor.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import diagnostics as dg

GOLD = os.path.join(os.path.dirname(__file__), "golden", "toy_problem.json")


def _toy(zeta):
    g = json.load(open(GOLD))
    m, n, p = g["m"], g["n"], g["p"]
    t = wl.toy_generalized(m, n, zeta=zeta, seed=21, pert_seed=22)
    lam = np.sort(t["lam_gen"])
    # Section 4.1.1 bounds: lambda_1 - 0.05, (lambda_n + lambda_{n+1}) / 2, lambda_m + 0.1
    bounds = (lam[0] - 0.05, lam[-1] + g["lambda_max_offset"], 0.5 * (lam[n - 1] + lam[n]))
    w, U = sla.eigh(t["A"], t["B"])
    return t, n, p, bounds, w, U[:, :n]


def test_b_norm_matches_explicit_square_root(rng):
    G = rng.standard_normal((40, 40))
    B = G @ G.T / 40 + np.eye(40)
    D = rng.standard_normal((40, 6))
    Bh = np.real(sla.sqrtm(B))
    np.testing.assert_allclose(dg.b_norm2(D, B), np.linalg.norm(Bh @ D, 2), rtol=1e-10)
    np.testing.assert_allclose(dg.b_norm2(D, None), np.linalg.norm(D, 2), rtol=1e-12)


@pytest.mark.parametrize("method", ["chfsi", "rchfsi"])
def test_exact_inverse_has_no_filtering_error(method):
    t, n, p, bounds, w, U = _toy(0.0)
    h = dg.run(method, t["A"], t["B"], t["Binv"], t["Dinv"], wl.random_block(t["A"].shape[0], n, 23),
               n, p, bounds, 12, w, U)
    assert max(x["filter_error"] for x in h) <= 1e-13


@pytest.fixture(scope="module")
def toy_runs():
    t, n, p, bounds, w, U = _toy(1e-3)
    X0 = wl.random_block(t["A"].shape[0], n, 23)
    return {m: dg.run(m, t["A"], t["B"], t["Binv"], t["Dinv"], X0, n, p, bounds, 36, w, U)
            for m in ("chfsi", "rchfsi")}


def test_chfsi_error_saturates_and_condition_fails(toy_runs):
    h = toy_runs["chfsi"]
    late = np.array([x["filter_error"] for x in h[12:]])
    assert np.all(np.abs(late / late[-1] - 1.0) < 0.05)          # saturated
    assert 1e-3 * 1e-3 < late[-1] < 10 * 1e-3                     # O(zeta)
    assert not h[-1]["holds"] and h[-1]["rhs"] > h[-1]["lhs"]     # curves crossed
    assert h[-1]["max_res"] > 1e-4                                # residual stalls


def test_rchfsi_error_tracks_residual_and_condition_holds(toy_runs):
    h = toy_runs["rchfsi"]
    mid = [x for x in h if 1e-11 < x["max_res"] < 1.0]
    assert len(mid) >= 15
    # above the rounding floor of the error (~1e-14) it is proportional to ||R||
    ratio = np.array([x["filter_error"] / x["res_norm"] for x in mid if x["filter_error"] > 1e-12])
    assert len(ratio) >= 10 and ratio.max() / ratio.min() < 3.0
    assert all(x["holds"] for x in mid)
    assert h[-1]["max_res"] < 1e-12
    # the filtering error falls by many decades, unlike ChFSI's
    assert h[-1]["filter_error"] < 1e-8 * h[1]["filter_error"]


@pytest.mark.parametrize("method", ["chfsi", "rchfsi"])
def test_theorem31_bound_holds(toy_runs, method):
    h = toy_runs[method]
    checked = 0
    tight = 0.0
    for x in h:
        if x["angle"] < 1e-10 or not np.isfinite(x["tan_bound"]):
            continue
        checked += 1
        t_next = np.tan(x["angle_next"])
        assert t_next <= x["tan_bound"] * (1 + 1e-8) + 1e-14
        tight = max(tight, t_next / x["tan_bound"])
    assert checked >= 10
    print(method, "largest tan ratio to the bound:", tight)
