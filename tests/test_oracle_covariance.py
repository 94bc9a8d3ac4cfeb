"""Pins of oracle.covariance against closed forms (Section 2.1)."""

import numpy as np

from oracle import covariance as cv


def test_matern_half_is_exponential_of_euclidean_distance():
    # nu = 1/2: 2^{1/2}/Gamma(1/2) x^{1/2} K_{1/2}(x) = e^{-x}  (K_{1/2}(x) = sqrt(pi/(2x)) e^{-x})
    rng = np.random.default_rng(1)
    t1, t2 = rng.uniform(-1, 1, (2, 200))
    lam, s2 = 0.3, 1.7
    x = np.sqrt(t1 ** 2 + t2 ** 2) / lam
    np.testing.assert_allclose(cv.matern(t1, t2, 0.5, lam, s2), s2 * np.exp(-x), rtol=1e-13)


def test_matern_three_halves_closed_form():
    rng = np.random.default_rng(2)
    t1, t2 = rng.uniform(-1, 1, (2, 200))
    lam, s2 = 0.1, 2.0
    x = np.sqrt(3.0) * np.sqrt(t1 ** 2 + t2 ** 2) / lam
    np.testing.assert_allclose(cv.matern(t1, t2, 1.5, lam, s2), s2 * (1 + x) * np.exp(-x), rtol=1e-12)


def test_matern_value_and_continuity_at_zero():
    for nu in (0.5, 1.0, 1.5, 2.7):
        assert cv.matern(0.0, 0.0, nu, 0.2, 1.3) == 1.3
        near = cv.matern(1e-9, 0.0, nu, 0.2, 1.3)
        assert abs(near - 1.3) < 1e-4


def test_matern_nu_one_monotone_and_positive():
    r = np.linspace(0.0, 2.0, 401)
    c = cv.matern(r, 0 * r, 1.0, 0.1, 1.0)
    assert np.all(np.diff(c) < 0) and np.all(c > 0)


def test_separable_exponential_definition_and_difference_from_matern_half():
    t1 = np.array([0.3, 0.0, 0.2])
    t2 = np.array([0.0, 0.4, 0.2])
    se = cv.sepexp(t1, t2, 0.3, 1.0)
    np.testing.assert_allclose(se, np.exp(-(np.abs(t1) + np.abs(t2)) / 0.3), rtol=1e-15)
    ma = cv.matern(t1, t2, 0.5, 0.3, 1.0)
    # equal on the axes, different off the axes (1-norm vs 2-norm)
    np.testing.assert_allclose(se[:2], ma[:2], rtol=1e-13)
    assert abs(se[2] - ma[2]) > 1e-3
