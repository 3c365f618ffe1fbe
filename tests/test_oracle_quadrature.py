"""Pins of oracle.quadrature: Gauss-Legendre rule on [0,1] and Lagrange bases."""

import math

import numpy as np
import pytest

from oracle.quadrature import gauss_legendre_01, lagrange


def test_degree2_closed_form():
    # 3-point Gauss-Legendre: nodes (1 -+ sqrt(3/5))/2 and 1/2, weights 5/18, 8/18, 5/18
    x, w = gauss_legendre_01(2)
    s = math.sqrt(3.0 / 5.0)
    np.testing.assert_allclose(x, [(1 - s) / 2, 0.5, (1 + s) / 2], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [5 / 18, 8 / 18, 5 / 18], rtol=0, atol=1e-15)


@pytest.mark.parametrize("degree", range(0, 7))
def test_exact_to_degree_2l_plus_1(degree):
    x, w = gauss_legendre_01(degree)
    assert np.all(np.diff(x) > 0) and x[0] > 0 and x[-1] < 1
    for p in range(2 * degree + 2):
        assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 1e-14
    p = 2 * degree + 2       # first degree the rule misses
    assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) > 1e-12


@pytest.mark.parametrize("degree", range(0, 6))
def test_lagrange_is_exact_kronecker_at_nodes(degree):
    x, _ = gauss_legendre_01(degree)
    L = lagrange(x, x)
    assert np.array_equal(L, np.eye(degree + 1))


@pytest.mark.parametrize("degree", range(1, 6))
def test_lagrange_matches_numpy_polynomial(degree):
    x, _ = gauss_legendre_01(degree)
    t = np.linspace(-0.3, 1.4, 37)
    L = lagrange(x, t)
    for l in range(degree + 1):
        others = np.delete(x, l)
        p = np.polynomial.Polynomial.fromroots(others)
        ref = p(t) / p(x[l])
        np.testing.assert_allclose(L[l], ref, rtol=1e-12, atol=1e-12)
