"""Pins of oracle.spline: the periodic spline system, the closed-form inverse,
the B-spline formula of the paper evaluated directly, and invariants."""

import math

import numpy as np
import pytest

from oracle import spline
from vp_inputs import random_field, random_shifts


def _paper_matrix(n):
    # (1/6) [4 1 0 ... 0 1; 1 4 1 ...; ...; 1 0 ... 0 1 4], periodic, n >= 3
    M = 4.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    M[0, -1] = M[-1, 0] = 1.0
    return M / 6.0


def _S(x):
    # the cubic B-spline of Sec. 3 with unit spacing, written from its formula
    a = abs(x)
    if a <= 1.0:
        return (4.0 - 6.0 * a * a + 3.0 * a ** 3) / 6.0
    if a <= 2.0:
        return (2.0 - a) ** 3 / 6.0
    return 0.0


@pytest.mark.parametrize("n", [3, 4, 7, 24, 96])
def test_coefficients_solve_the_printed_system(n):
    u = random_field((5, n), seed=n)
    om = spline.coefficients(u)
    ref = np.linalg.solve(_paper_matrix(n), u.T).T
    np.testing.assert_allclose(om, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [5, 24, 96, 288])
def test_closed_form_circulant_inverse(n):
    # inverse column c_j = sqrt(3) (r^j + r^(n-j)) / (1 - r^n), r = sqrt(3) - 2
    r = math.sqrt(3.0) - 2.0
    j = np.arange(n)
    c = math.sqrt(3.0) * (r ** j + r ** (n - j)) / (1.0 - r ** n)
    e0 = np.zeros((1, n))
    e0[0, 0] = 1.0
    col = spline.coefficients(e0)[0]
    np.testing.assert_allclose(col, c, rtol=0, atol=1e-15)


def test_weights_partition_and_interpolation():
    np.testing.assert_allclose(spline.weights(0.0), [0, 1 / 6, 4 / 6, 1 / 6],
                               rtol=0, atol=1e-16)
    for a in np.linspace(0, 1, 13):
        b = spline.weights(a)
        assert abs(b.sum() - 1.0) < 1e-15
        # the cubic B-spline reproduces linear data and has variance 1/3:
        # sum_k k S(y-k) = y and sum_k k^2 S(y-k) = y^2 + 1/3, y = t
        t = 1.0 - a
        q = np.array([-1.0, 0.0, 1.0, 2.0])
        assert abs(np.dot(b, q) - t) < 1e-15
        assert abs(np.dot(b, q * q) - (t * t + 1.0 / 3.0)) < 1e-15


@pytest.mark.parametrize("n", [8, 24])
def test_shift_of_a_spline_is_the_spline_evaluated(n):
    # u = C omega for a random omega: the sweep must return the spline
    # sum_k omega_k S(i - sigma - k) summed over periodic images, computed
    # directly from the B-spline formula
    om = random_field((n,), seed=5)
    u = (np.roll(om, 1) + 4 * om + np.roll(om, -1)) / 6.0
    for sigma in random_shifts(10, seed=6, n_cells=n):
        out = spline.sweep(u[None, :], 1, np.array([[sigma]]))[0]
        ref = np.zeros(n)
        for i in range(n):
            y = i - sigma
            for k in range(n):
                d = (y - k) % n             # distance modulo the period
                for img in (d - 2 * n, d - n, d, d + n):
                    ref[i] += om[k] * _S(img)
        np.testing.assert_allclose(out, ref, rtol=0, atol=5e-15)


@pytest.mark.parametrize("n", [6, 24])
def test_mass_and_integer_roll(n):
    f = random_field((3, n, 2), seed=9)
    for s in random_shifts(15, seed=10, n_cells=n):
        g = spline.sweep(f, 1, np.full((3, 1, 2), s))
        np.testing.assert_allclose(g.sum(axis=1), f.sum(axis=1), rtol=0, atol=1e-13)
    for s in (-3, 0, 2, n + 1):
        g = spline.sweep(f, 1, np.full((3, 1, 2), float(s)))
        np.testing.assert_allclose(g, np.roll(f, s, axis=1), rtol=0, atol=1e-14)


def test_cubic_reproduced_away_from_seam():
    n = 120
    x = np.arange(n, dtype=np.float64)
    p = np.polynomial.Polynomial([0.2, -0.01, 3e-4, -2e-6])
    u = p(x)[None, :]
    for sigma in (0.3, -0.45, 1.7):
        out = spline.sweep(u, 1, np.array([[sigma]]))[0]
        sl = slice(30, n - 30)
        np.testing.assert_allclose(out[sl], p(x - sigma)[sl], rtol=0, atol=1e-12)
