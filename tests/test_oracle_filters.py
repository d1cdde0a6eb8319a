"""Pins for oracle.filters (Algorithms 2 and 3) and oracle.angles.

* Algorithm 2 on a matrix with known eigenvectors equals Q C_p(Lambda) Q^T X,
  with C_p evaluated by numpy's Chebyshev series (not the oracle's).
* Algorithm 3 with the exact inverse equals Algorithm 2 with H = B^{-1} A for
  any block X and any diagonal Lambda (Proposition 3.3 is an identity).
* Theorems 3.2 / 3.4: with an approximate inverse the residual filter's error
  shrinks with ||R|| while the plain filter's error does not.
* Definition 2.1 written out equals the sine-based angle.
* Theorem 2.1: one exact filter step contracts tan(angle) by
  max_{j>n}|C_p(l_j)| / min_{j<=n}|C_p(l_j)| (the bound its proof establishes).
"""
import numpy as np
import pytest
import scipy.linalg as sla
from numpy.polynomial import chebyshev as npcheb

import workloads as wl
from oracle import angles, filters, rr


def _Cp_numpy(x, p, lmin, lmax, lT):
    e, c = (lmax - lT) / 2, (lmax + lT) / 2
    coeff = np.zeros(p + 1)
    coeff[p] = 1.0
    return npcheb.chebval((np.asarray(x) - c) / e, coeff) / npcheb.chebval((lmin - c) / e, coeff)


def _sym_from_spectrum(rng, lam):
    Q, _ = np.linalg.qr(rng.standard_normal((len(lam), len(lam))))
    return Q, (Q * lam) @ Q.T


@pytest.mark.parametrize("p", [1, 2, 8, 16])
def test_chebyshev_filter_on_known_spectrum(rng, p):
    n = 120
    lam = np.sort(np.concatenate([np.linspace(-1, -0.2, 10), rng.uniform(0, 10, n - 10)]))
    Q, A = _sym_from_spectrum(rng, lam)
    X = rng.standard_normal((n, 12))
    bounds = (lam[0] - 0.05, lam[-1] + 0.1, 0.5 * (lam[11] + lam[12]))
    Y = filters.chebyshev_filter(filters.dense_op(A), X, p, *bounds)
    ref = Q @ (_Cp_numpy(lam, p, *bounds)[:, None] * (Q.T @ X))
    assert np.linalg.norm(Y - ref) <= 1e-12 * np.linalg.norm(ref)


def _generalized(rng, n=150):
    lam = np.sort(np.concatenate([np.linspace(-1, -0.1, 12), rng.uniform(0, 10, n - 12)]))
    _, A = _sym_from_spectrum(rng, lam)
    Gm = rng.standard_normal((n, n))
    B = Gm @ Gm.T / n + np.eye(n)
    return A, B


def test_residual_filter_equals_chebyshev_filter_with_exact_inverse(rng):
    A, B = _generalized(rng)
    Binv = np.linalg.inv(B)
    X = rng.standard_normal((A.shape[0], 14))
    lam = rng.uniform(-1.5, 3.0, 14)           # any diagonal works: the identity is algebraic
    Yres = A @ X - (B @ X) * lam[None, :]
    bounds = (-1.6, 120.0, 0.5)
    for p in (2, 5, 10):
        y3 = filters.residual_filter(filters.dense_op(A), filters.dense_op(Binv), X, lam, Yres, p,
                                     *bounds)
        y2 = filters.chebyshev_filter(filters.dense_op(Binv @ A), X, p, *bounds)
        assert np.linalg.norm(y3 - y2) <= 1e-11 * np.linalg.norm(y2)


def test_residual_filter_eigenvalue_recurrence_is_closed_form(rng):
    n = 60
    lam_all = np.sort(rng.uniform(-2, 8, n))
    Q, A = _sym_from_spectrum(rng, lam_all)
    X = Q[:, :7]
    lam = lam_all[:7]
    Yres = A @ X - X * lam[None, :]
    bounds = (lam_all[0] - 0.1, lam_all[-1] + 0.1, 0.5 * (lam_all[7] + lam_all[8]))
    _, _, LY = filters.residual_filter(filters.dense_op(A), filters.identity_op(), X, lam, Yres,
                                       9, *bounds, return_parts=True)
    np.testing.assert_allclose(LY, _Cp_numpy(lam, 9, *bounds), rtol=1e-11)


def test_residual_filter_error_scales_with_residual(rng):
    """Theorem 3.4 vs 3.2: with D^{-1} != B^{-1} only the residual form's error follows ||R||."""
    n, b, p = 160, 10, 8
    A, B = _generalized(rng, n)
    Binv = np.linalg.inv(B)
    E = wl.unit_sym_perturbation(rng, n)
    Dinv = Binv + 1e-3 * E
    w, U = sla.eigh(A, B)
    bounds = (w[0] - 0.05, w[-1] + 0.1, 0.5 * (w[b - 1] + w[b]))
    ratios, plain = [], []
    for delta in (1e-2, 1e-4, 1e-6):
        Xp = U[:, :b] + delta * rng.standard_normal((n, b))
        out = rr.rayleigh_ritz(Xp, filters.dense_op(A), filters.dense_op(B))
        X, lam, R = out["X"], out["lam"], out["R"]
        exact = filters.chebyshev_filter(filters.dense_op(Binv @ A), X, p, *bounds)
        y3 = filters.residual_filter(filters.dense_op(A), filters.dense_op(Dinv), X, lam, R, p,
                                     *bounds)
        y2 = filters.chebyshev_filter(filters.dense_op(Dinv @ A), X, p, *bounds)
        nr = np.linalg.norm(R, 2)
        ratios.append(np.linalg.norm(y3 - exact, 2) / nr)
        plain.append(np.linalg.norm(y2 - exact, 2))
    # residual form: error / ||R|| stays within a constant band over 4 decades of ||R||
    assert max(ratios) / min(ratios) < 10.0
    # plain form: error does not follow ||R|| down (stagnates at O(zeta))
    assert plain[-1] > 1e-3 * plain[0]
    assert ratios[-1] * 1e-4 < plain[-1]


def test_angle_definition_matches_sine_route(rng):
    n, q = 80, 6
    Xo, _ = np.linalg.qr(rng.standard_normal((n, n)))
    S, Sperp = Xo[:, :q], Xo[:, q:]
    Y = S + 0.03 * rng.standard_normal((n, q))
    Yo, _ = np.linalg.qr(Y)
    t = angles.tan_angle_def21(S, Sperp, Yo)
    th = angles.max_principal_angle(S, Y)
    assert abs(np.arctan(t) - th) < 1e-10


def test_theorem_2_1_contraction(rng):
    n, b, p = 200, 8, 6
    lam = np.sort(np.concatenate([np.linspace(1, 4, b), 5 + 0.2 * np.arange(n - b)]))
    Q, A = _sym_from_spectrum(rng, lam)
    bounds = (lam[0] - 0.05, lam[-1] + 0.1, 0.5 * (lam[b - 1] + lam[b]))
    # The proof of Theorem 2.1 bounds the step by max_{j>n}|C_p(l_j)| / min_{j<=n}|C_p(l_j)|;
    # its final equality with |C_p(l_{n+1})/C_p(l_n)| only holds when l_T = l_{n+1}.
    cp = np.abs(_Cp_numpy(lam, p, *bounds))
    rate = cp[b:].max() / cp[:b].min()
    X = rng.standard_normal((n, b))
    for _ in range(4):
        X, _ = np.linalg.qr(X)
        t0 = np.tan(angles.max_principal_angle(Q[:, :b], X))
        Y = filters.chebyshev_filter(filters.dense_op(A), X, p, *bounds)
        t1 = np.tan(angles.max_principal_angle(Q[:, :b], Y))
        assert t1 <= rate * t0 * (1 + 1e-8) + 1e-13
        X = Y
