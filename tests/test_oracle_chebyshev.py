"""Pins for oracle.chebyshev (scaled Chebyshev polynomials, Section 2.1).

Each check compares the oracle against something it does not share code with:
numpy's Chebyshev series, the defining three-term recurrence of T_k, the
trigonometric identity T_m(cos t) = cos(m t), and the closed form of C_k.
"""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import chebyshev as ch


@pytest.mark.parametrize("k", [0, 1, 2, 3, 7, 16, 20, 30, 40])
def test_cheb_T_matches_numpy_series(k):
    x = np.concatenate([np.linspace(-1, 1, 41), np.linspace(-3.5, -1.001, 15),
                        np.linspace(1.001, 2.5, 15)])
    coeff = np.zeros(k + 1)
    coeff[k] = 1.0
    ref = npcheb.chebval(x, coeff)
    got = ch.cheb_T(k, x)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12)


def test_cheb_T_three_term_and_trig_identity():
    theta = np.linspace(0, np.pi, 37)
    x = np.cos(theta)
    T = [np.ones_like(x), x.copy()]
    for k in range(1, 25):
        T.append(2 * x * T[k] - T[k - 1])
    for m in range(25):
        np.testing.assert_allclose(ch.cheb_T(m, x), T[m], atol=1e-11)
        np.testing.assert_allclose(ch.cheb_T(m, x), np.cos(m * theta), atol=1e-11)


@pytest.mark.parametrize("bounds", [(0.95, 202.9, 4.5), (-1.05, 10.1, 0.085), (-2.5, 25.0, -0.05),
                                    (-4.3, 18.0, -1.2)])
def test_sigma_ratio_of_T(bounds):
    lmin, lmax, lT = bounds
    e, c, s1 = ch.affine(lmin, lmax, lT)
    L0 = (lmin - c) / e
    assert abs(L0 - 1.0 / s1) < 1e-14 * abs(L0)
    s = ch.sigmas(s1, 30)
    for k in range(1, 31):
        ref = npcheb.chebval(L0, [0] * (k - 1) + [1]) / npcheb.chebval(L0, [0] * k + [1])
        assert abs(s[k - 1] - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("bounds,p", [((0.95, 202.9, 4.5), 8), ((-1.05, 10.1, 0.085), 16),
                                      ((-2.5, 25.0, -0.05), 20), ((-4.3, 18.0, -1.2), 40)])
def test_scalar_recurrence_equals_closed_form(bounds, p):
    lmin, lmax, lT = bounds
    x = np.concatenate([np.linspace(lmin, lT, 25), np.linspace(lT, lmax, 25)])
    rec = ch.scalar_recurrence(x, lmin, lmax, lT, p)
    e, c, _ = ch.affine(lmin, lmax, lT)
    for k in range(p + 1):
        coeff = np.zeros(k + 1)
        coeff[k] = 1.0
        ref = npcheb.chebval((x - c) / e, coeff) / npcheb.chebval((lmin - c) / e, coeff)
        np.testing.assert_allclose(rec[k], ref, rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(ch.scaled_cheb(x, k, lmin, lmax, lT), ref, rtol=1e-10,
                                   atol=1e-13)


def test_scaled_cheb_normalisation_and_damping():
    lmin, lmax, lT = -1.05, 10.1, 0.085
    for k in range(0, 30):
        assert abs(ch.scaled_cheb(np.array([lmin]), k, lmin, lmax, lT)[0] - 1.0) < 1e-12
        vals = ch.scaled_cheb(np.linspace(lT, lmax, 200), k, lmin, lmax, lT)
        assert np.all(np.abs(vals) <= 1.0 + 1e-12)


def test_recurrence_coefficient_sign_mistake_is_caught(monkeypatch):
    """A planted sign error in b_k must break the closed-form pin."""
    good = ch.recurrence_coeffs

    def bad(lmin, lmax, lT, p):
        r = good(lmin, lmax, lT, p).copy()
        r[:, 1] *= -1.0
        return r

    monkeypatch.setattr(ch, "recurrence_coeffs", bad)
    lmin, lmax, lT = -1.05, 10.1, 0.085
    x = np.linspace(lmin, lmax, 30)
    rec = ch.scalar_recurrence(x, lmin, lmax, lT, 6)
    e, c, _ = ch.affine(lmin, lmax, lT)
    ref = npcheb.chebval((x - c) / e, [0] * 6 + [1]) / npcheb.chebval((lmin - c) / e, [0] * 6 + [1])
    assert not np.allclose(rec[6], ref, rtol=1e-6)
