"""Pins of oracle.adjoint: transposes by the dot-product identity, shift
derivatives and gradients by finite differences, derivative matrices by exact
symbolic differentiation."""

import math

import numpy as np
import pytest
import sympy as sp

from oracle import adjoint, field, sldg, spline, strang
from oracle.quadrature import gauss_legendre_01
from vp_inputs import random_field, random_shifts


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_lagrange_derivative(degree):
    xi, _ = gauss_legendre_01(degree)
    t = np.linspace(-0.2, 1.3, 17)
    d = adjoint.lagrange_deriv(xi, t)
    for l in range(degree + 1):
        p = np.polynomial.Polynomial.fromroots(np.delete(xi, l))
        np.testing.assert_allclose(d[l], p.deriv()(t) / p(xi[l]), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
@pytest.mark.parametrize("alpha", [0.05, 0.4, 0.77])
def test_projection_derivatives_match_differences(degree, alpha):
    dA, dB = adjoint.projection_derivatives(degree, alpha)
    h = 1e-6
    Ap, Bp = sldg.projection_matrices(degree, alpha + h)
    Am, Bm = sldg.projection_matrices(degree, alpha - h)
    np.testing.assert_allclose(dA, (Ap - Am) / (2 * h), rtol=0, atol=2e-8)
    np.testing.assert_allclose(dB, (Bp - Bm) / (2 * h), rtol=0, atol=2e-8)


def test_projection_derivatives_exact_degree2():
    a, t = sp.symbols("a t")
    s = sp.sqrt(sp.Rational(3, 5))
    xi = [(1 - s) / 2, sp.Rational(1, 2), (1 + s) / 2]
    w = [sp.Rational(5, 18), sp.Rational(8, 18), sp.Rational(5, 18)]

    def L(l, z):
        e = sp.Integer(1)
        for k in range(3):
            if k != l:
                e *= (z - xi[k]) / (xi[l] - xi[k])
        return e

    alpha = sp.Rational(1, 3)
    dA, dB = adjoint.projection_derivatives(2, 1.0 / 3.0)
    for j in range(3):
        for l in range(3):
            Aj = sp.integrate(sp.expand(L(l, t + 1 - a) * L(j, t)), (t, 0, a)) / w[j]
            Bj = sp.integrate(sp.expand(L(l, t - a) * L(j, t)), (t, a, 1)) / w[j]
            assert abs(float(sp.diff(Aj, a).subs(a, alpha)) - dA[j, l]) < 1e-13
            assert abs(float(sp.diff(Bj, a).subs(a, alpha)) - dB[j, l]) < 1e-13


@pytest.mark.parametrize("degree", [0, 1, 2])
def test_sldg_adjoint_dot_product(degree):
    m = degree + 1
    dims = (3 * m, 4 * m, 2 * m, 5 * m)
    u = random_field(dims, seed=1)
    lam = random_field(dims, seed=2)
    for axis in range(4):
        shape = list(dims)
        shape[axis] = 1
        sig = random_shifts(int(np.prod(shape)), seed=axis, n_cells=dims[axis] // m).reshape(shape)
        lhs = np.sum(sldg.sweep(u, axis, sig, degree) * lam)
        rhs = np.sum(u * adjoint.sldg_sweep_adjoint(lam, axis, sig, degree))
        assert _rel(lhs, rhs) < 1e-13


def test_spline_adjoint_dot_product():
    dims = (6, 7, 5, 9)
    u = random_field(dims, seed=3)
    lam = random_field(dims, seed=4)
    for axis in range(4):
        shape = list(dims)
        shape[axis] = 1
        sig = random_shifts(int(np.prod(shape)), seed=axis, n_cells=dims[axis]).reshape(shape)
        lhs = np.sum(spline.sweep(u, axis, sig) * lam)
        rhs = np.sum(u * adjoint.spline_sweep_adjoint(lam, axis, sig))
        assert _rel(lhs, rhs) < 1e-13


@pytest.mark.parametrize("method", ["sldg", "spline"])
def test_shift_derivative_matches_differences(method):
    degree = 2
    m = degree + 1 if method == "sldg" else 1
    dims = (2 * m, 3 * m, 4 * m, 2 * m)
    u = random_field(dims, seed=5)
    lam = random_field(dims, seed=6)
    rng = np.random.default_rng(7)
    for axis in range(4):
        shape = list(dims)
        shape[axis] = 1
        sig = rng.uniform(-2.0, 2.0, size=shape)
        if method == "sldg":
            g = adjoint.sldg_sweep_dshift(u, lam, axis, sig, degree)
            fwd = lambda s: np.sum(sldg.sweep(u, axis, s, degree) * lam)  # noqa: E731
        else:
            g = adjoint.spline_sweep_dshift(u, lam, axis, sig)
            fwd = lambda s: np.sum(spline.sweep(u, axis, s) * lam)  # noqa: E731
        h = 1e-6
        for idx in [tuple(int(rng.integers(0, d)) for d in shape) for _ in range(4)]:
            sp_, sm_ = sig.copy(), sig.copy()
            sp_[idx] += h
            sm_[idx] -= h
            fd = (fwd(sp_) - fwd(sm_)) / (2 * h)
            gi = g[tuple(i for d, i in enumerate(idx) if d != axis)]
            assert abs(gi - fd) < 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("degree", [None, 1, 2])
def test_density_and_poisson_adjoint_dot_products(degree):
    m = 1 if degree is None else degree + 1
    dims = (4 * m, 6 * m, 3 * m, 2 * m)
    f = random_field(dims, seed=8)
    g = random_field(dims[:2], seed=9)
    lhs = np.sum(field.density(f, degree, 12.0, 18.0) * g)
    rhs = np.sum(f * adjoint.density_adjoint(g, dims, degree, 12.0, 18.0))
    assert _rel(lhs, rhs) < 1e-13
    rho = random_field(dims[:2], seed=10)
    g1 = random_field(dims[:2], seed=11)
    g2 = random_field(dims[:2], seed=12)
    e1, e2, _ = field.poisson(rho, degree, 4 * math.pi, 3.0)
    lhs = np.sum(e1 * g1) + np.sum(e2 * g2)
    rhs = np.sum(rho * adjoint.poisson_adjoint(g1, g2, degree, 4 * math.pi, 3.0))
    assert _rel(lhs, rhs) < 1e-12


def _small_grid(method):
    degree = 1 if method == "sldg" else None
    m = 2 if method == "sldg" else 1
    dims = (4 * m, 4 * m, 6 * m, 6 * m) if method == "sldg" else (8, 8, 12, 12)
    return strang.Grid(dims, (0.0, 0.0, -6.0, -6.0), (4 * math.pi, 4 * math.pi, 12.0, 12.0),
                       degree)


@pytest.mark.parametrize("method", ["sldg", "spline"])
def test_final_energy_gradient_matches_central_differences(method):
    # dJ/d eps at eps = 0.5 and a random directional derivative, against
    # central differences with h = 1e-4 (FP64): agreement to 1e-6 relative
    grid = _small_grid(method)
    tau, nsteps = 0.1, 3

    def f0(eps):
        return field.initial_condition("landau", grid.dims, grid.lo, grid.length,
                                       grid.degree, eps, 0.5)

    def J(f):
        return strang.run(f, grid, tau, nsteps)[1][-1]

    J0, grad = adjoint.final_energy_gradient(f0(0.5), grid, tau, nsteps)
    assert abs(J0 - J(f0(0.5))) < 1e-14 * J0
    df0 = f0(1.0) - f0(0.0)             # f0 is affine in eps
    g_eps = np.sum(grad * df0)
    h = 1e-4
    fd = (J(f0(0.5 + h)) - J(f0(0.5 - h))) / (2 * h)
    assert _rel(g_eps, fd) < 1e-6, (g_eps, fd)
    d = random_field(grid.dims, seed=13) * f0(0.5)
    g_d = np.sum(grad * d)
    fd = (J(f0(0.5) + h * d) - J(f0(0.5) - h * d)) / (2 * h)
    assert _rel(g_d, fd) < 1e-6, (g_d, fd)


@pytest.mark.parametrize("method,degree", [("sldg", 1), ("sldg", 2), ("sldg", 3), ("spline", None)])
def test_shift_derivative_just_below_zero_is_the_left_one(method, degree):
    # For sigma in (-1, 0) the floor is -1 and the line map is a polynomial
    # in sigma (degree 2l+1 in alpha for SLDG, 3 for the spline), so the
    # derivative at sigma = -1e-17 is fixed by samples inside (-1, 0): an
    # exact fit differentiated at -1e-17, and a one-sided difference below
    # zero.
    m = 1 if method == "spline" else degree + 1
    n_pts = 7 * m
    rng = np.random.default_rng(21)
    u = rng.uniform(-1.0, 1.0, size=(3, n_pts))
    lam = rng.uniform(-1.0, 1.0, size=(3, n_pts))
    if method == "sldg":
        fwd = lambda s: np.sum(sldg.sweep(u, 1, np.full((3, 1), s), degree) * lam, axis=1)  # noqa: E731
        dshift = lambda s: adjoint.sldg_sweep_dshift(u, lam, 1, np.full((3, 1), s), degree)  # noqa: E731
        pdeg = 2 * degree + 1
    else:
        fwd = lambda s: np.sum(spline.sweep(u, 1, np.full((3, 1), s)) * lam, axis=1)  # noqa: E731
        dshift = lambda s: adjoint.spline_sweep_dshift(u, lam, 1, np.full((3, 1), s))  # noqa: E731
        pdeg = 3
    s0 = -1e-17
    n, alpha = sldg.split_shift(s0)
    assert n == -1 and alpha == 1.0
    got = dshift(s0)
    # exact: polynomial through pdeg+3 points of (-1, 0), differentiated at s0
    xs = -np.linspace(0.05, 0.95, pdeg + 3)
    ys = np.array([fwd(x) for x in xs])
    for r in range(3):
        p = np.polynomial.Polynomial.fit(xs, ys[:, r], pdeg)
        assert abs(p.deriv()(s0) - got[r]) < 1e-9 * max(1.0, abs(got[r]))
    # one-sided difference below zero (second order: from -h and -2h)
    h = 1e-5
    fd = (3 * fwd(s0) - 4 * fwd(s0 - h) + fwd(s0 - 2 * h)) / (2 * h)
    np.testing.assert_allclose(got, fd, rtol=1e-7, atol=1e-7)
    # SLDG: the right derivative at zero is another number (the projected
    # map has a kink at whole cells); spline: the cubic B-spline has a
    # continuous first derivative, so both sides agree
    right = dshift(0.0)
    if method == "sldg":
        assert np.max(np.abs(right - got)) > 1e-3 * np.max(np.abs(got))
    else:
        np.testing.assert_allclose(right, got, rtol=1e-13, atol=1e-13)
    # the forward map is continuous across zero: bitwise the same lines
    assert np.array_equal(fwd(s0), fwd(0.0))
