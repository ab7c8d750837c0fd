"""Pins of the ensemble-statistics oracle (oracle/stats.py) against closed
forms and an independent library routine (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats as sps

from oracle import stats


def test_moments_match_scipy_central_moments():
    rng = np.random.default_rng(7)
    beta = rng.normal(0.3, 0.05, size=(37, 11)) + rng.exponential(0.02, size=(37, 11))
    mu = stats.ensemble_moments(beta, 5)
    np.testing.assert_allclose(mu[:, 0], beta.mean(axis=0), rtol=1e-14)
    for p in range(2, 6):
        ref = sps.moment(beta, moment=p, axis=0)  # population central moment
        np.testing.assert_allclose(mu[:, p - 1], ref, rtol=1e-10, atol=1e-18)


def test_moments_closed_forms():
    # constant members: mean c, central moments 0
    mu = stats.ensemble_moments(np.full((8, 3), 0.25), 4)
    assert np.all(mu[:, 0] == 0.25) and np.all(mu[:, 1:] == 0.0)
    # symmetric two-point distribution +-a: mu_2 = a^2, mu_3 = 0, mu_4 = a^4
    a = 0.125
    beta = np.array([[a], [-a]] * 5)
    mu = stats.ensemble_moments(beta, 4)
    assert mu[0, 0] == 0.0 and mu[0, 1] == a * a and mu[0, 2] == 0.0 and mu[0, 3] == a ** 4
    # a shift moves mu_1 only
    rng = np.random.default_rng(1)
    b = rng.uniform(size=(20, 4))
    m0, m1 = stats.ensemble_moments(b, 3), stats.ensemble_moments(b + 2.0, 3)
    np.testing.assert_allclose(m1[:, 0], m0[:, 0] + 2.0, rtol=1e-15)
    np.testing.assert_allclose(m1[:, 1:], m0[:, 1:], rtol=1e-12, atol=1e-15)


def test_window_exact_for_linear_data():
    t = np.arange(0, 41) * 0.5
    mu1 = 0.3 + 0.01 * t          # trapezoid rule is exact for a linear mu_1
    mu2 = 0.004 * t                # exactly k t
    beta0, k = stats.ensemble_window(t, mu1, mu2, 5.0, 15.0)
    assert math.isclose(beta0, 0.3 + 0.01 * 10.0, rel_tol=1e-14)
    assert math.isclose(k, 0.004, rel_tol=1e-14)
    # window edges are inclusive; fewer than two samples: no average
    b, kk = stats.ensemble_window(t, mu1, mu2, 5.0, 5.2)
    assert math.isnan(b) and math.isclose(kk, 0.004, rel_tol=1e-14)
    b, kk = stats.ensemble_window(t, mu1, mu2, 5.1, 5.2)
    assert math.isnan(b) and math.isnan(kk)


def test_window_average_of_a_quadratic():
    # trapezoid error of t^2 on a uniform grid h over [a, b]: (b - a) h^2 / 6
    h = 0.25
    t = np.arange(0, 81) * h
    mu1 = t ** 2
    beta0, _ = stats.ensemble_window(t, mu1, np.zeros_like(t), 2.0, 10.0)
    exact = (10.0 ** 3 - 2.0 ** 3) / 3.0 / 8.0
    assert math.isclose(beta0, exact + h * h / 6.0, rel_tol=1e-13)


def test_histogram_counts():
    t = np.array([0.0, 1.0, 2.0])
    beta = np.array([[0.05, 0.15, 0.25], [-1.0, 0.35, 1.0], [np.nan, 0.0, 0.999999]])
    c = stats.beta_histogram(beta, t, 0.0, 2.0, 0.0, 1.0, 10)
    # below: -1.0; above: 1.0; NaN dropped; bins of width 0.1
    assert c[0] == 1 and c[-1] == 1 and c.sum() == 8
    assert c[1] == 2 and c[2] == 1 and c[3] == 1 and c[4] == 1 and c[10] == 1
    # interior values off the edges agree with numpy.histogram
    rng = np.random.default_rng(3)
    b = rng.uniform(-0.2, 1.2, size=(50, 6))
    tt = np.arange(6.0)
    c = stats.beta_histogram(b, tt, 1.0, 4.0, 0.0, 1.0, 7)
    w = b[:, 1:5].ravel()
    ref, _ = np.histogram(w[(w >= 0) & (w < 1)], bins=7, range=(0.0, 1.0))
    np.testing.assert_array_equal(c[1:-1], ref)
    assert c[0] == np.count_nonzero(w < 0) and c[-1] == np.count_nonzero(w >= 1)
