"""Pins of oracle.sldg against closed forms, exact arithmetic, brute-force
integration and invariants of the translate-and-project step."""

import numpy as np
import pytest
import sympy as sp
from scipy.integrate import quad

from oracle import sldg
from oracle.quadrature import gauss_legendre_01
from vp_inputs import random_field, random_shifts


def _np_lagrange(x, l):
    others = np.delete(x, l)
    p = np.polynomial.Polynomial.fromroots(others)
    return lambda t: p(t) / p(x[l])


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.77])
def test_degree0_is_donor_cell(alpha):
    # piecewise constants: the projection is the textbook upwind average
    A, B = sldg.projection_matrices(0, alpha)
    assert abs(A[0, 0] - alpha) < 1e-15 and abs(B[0, 0] - (1 - alpha)) < 1e-15


@pytest.mark.parametrize("degree", range(0, 6))
def test_alpha_zero_and_one_bitwise(degree):
    m = degree + 1
    A, B = sldg.projection_matrices(degree, 0.0)
    assert np.array_equal(A, np.zeros((m, m))) and np.array_equal(B, np.eye(m))
    A, B = sldg.projection_matrices(degree, 1.0)
    assert np.array_equal(A, np.eye(m)) and np.array_equal(B, np.zeros((m, m)))


@pytest.mark.parametrize("degree", [1, 2, 3])
@pytest.mark.parametrize("alpha", [0.125, 0.5, 0.8])
def test_against_adaptive_quadrature(degree, alpha):
    # the defining integrals, integrated by scipy.quad with numpy polynomials
    x, w = gauss_legendre_01(degree)
    A, B = sldg.projection_matrices(degree, alpha)
    L = [_np_lagrange(x, l) for l in range(degree + 1)]
    for j in range(degree + 1):
        for l in range(degree + 1):
            a = quad(lambda t: L[l](t + 1 - alpha) * L[j](t), 0, alpha,
                     epsabs=1e-15, epsrel=1e-14)[0] / w[j]
            b = quad(lambda t: L[l](t - alpha) * L[j](t), alpha, 1,
                     epsabs=1e-15, epsrel=1e-14)[0] / w[j]
            assert abs(A[j, l] - a) < 2e-13
            assert abs(B[j, l] - b) < 2e-13


def _exact_AB(degree, alpha):
    t = sp.symbols("t")
    if degree == 1:
        s = sp.sqrt(sp.Rational(1, 3))
        xi = [(1 - s) / 2, (1 + s) / 2]
        w = [sp.Rational(1, 2)] * 2
    else:
        s = sp.sqrt(sp.Rational(3, 5))
        xi = [(1 - s) / 2, sp.Rational(1, 2), (1 + s) / 2]
        w = [sp.Rational(5, 18), sp.Rational(8, 18), sp.Rational(5, 18)]
    m = len(xi)

    def L(l, z):
        e = sp.Integer(1)
        for k in range(m):
            if k != l:
                e *= (z - xi[k]) / (xi[l] - xi[k])
        return e

    A = np.zeros((m, m))
    B = np.zeros((m, m))
    for j in range(m):
        for l in range(m):
            A[j, l] = float(sp.integrate(sp.expand(L(l, t + 1 - alpha) * L(j, t)),
                                         (t, 0, alpha)) / w[j])
            B[j, l] = float(sp.integrate(sp.expand(L(l, t - alpha) * L(j, t)),
                                         (t, alpha, 1)) / w[j])
    return A, B


@pytest.mark.parametrize("degree", [1, 2])
@pytest.mark.parametrize("alpha", [sp.Rational(1, 4), sp.Rational(1, 2)])
def test_against_exact_symbolic_integration(degree, alpha):
    Ae, Be = _exact_AB(degree, alpha)
    A, B = sldg.projection_matrices(degree, float(alpha))
    np.testing.assert_allclose(A, Ae, rtol=0, atol=2e-15)
    np.testing.assert_allclose(B, Be, rtol=0, atol=2e-15)


def test_degree2_half_shift_rational_entries():
    # exact values: A(1/2) has -1/12 at both diagonal ends and -1/48 in the middle
    A, B = sldg.projection_matrices(2, 0.5)
    assert abs(A[0, 0] + 1 / 12) < 1e-15 and abs(A[2, 2] + 1 / 12) < 1e-15
    assert abs(A[1, 1] + 1 / 48) < 1e-15


@pytest.mark.parametrize("degree", range(0, 6))
@pytest.mark.parametrize("alpha", [0.1, 0.37, 0.5, 0.93])
def test_reflection_and_mass(degree, alpha):
    m = degree + 1
    J = np.eye(m)[::-1]
    A, B = sldg.projection_matrices(degree, alpha)
    A2, _ = sldg.projection_matrices(degree, 1 - alpha)
    np.testing.assert_allclose(B, J @ A2 @ J, rtol=0, atol=5e-15)
    _, w = gauss_legendre_01(degree)
    np.testing.assert_allclose(w @ (A + B), w, rtol=0, atol=1e-15)


# ------------------------------------------------------------------ sweeps ---

@pytest.mark.parametrize("degree", [0, 2, 3])
def test_integer_shift_is_exact_roll(degree):
    m = degree + 1
    f = random_field((4, 5 * m, 3, 2), seed=1)
    for s in (-7, -1, 0, 1, 3, 5, 11):
        out = sldg.sweep(f, 1, np.full((4, 1, 3, 2), float(s)), degree)
        ref = np.roll(f.reshape(4, 5, m, 3, 2), s, axis=1).reshape(f.shape)
        assert np.array_equal(out, ref)


@pytest.mark.parametrize("degree", [1, 2])
def test_period_shift_invariance_and_mass(degree):
    m = degree + 1
    nc = 6
    f = random_field((3, 2, nc * m, 4), seed=2)
    _, w = gauss_legendre_01(degree)
    wv = np.tile(w, nc)
    for s in random_shifts(12, seed=3, n_cells=nc):
        sig = np.full((3, 2, 1, 4), s)
        a = sldg.sweep(f, 2, sig, degree)
        b = sldg.sweep(f, 2, sig + nc, degree)
        assert np.array_equal(a, b)
        mass0 = np.einsum("abce,c->abe", f, wv)
        mass1 = np.einsum("abce,c->abe", a, wv)
        np.testing.assert_allclose(mass1, mass0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_polynomial_reproduced_away_from_seam(degree):
    # data equal to one polynomial of degree <= l on a run of cells is
    # translated exactly: the projection has nothing to do there
    m = degree + 1
    nc = 10
    xi, _ = gauss_legendre_01(degree)
    x = (np.repeat(np.arange(nc), m) + np.tile(xi, nc))   # unit cell width
    coeffs = np.linspace(0.3, -0.2, degree + 1)
    poly = np.polynomial.Polynomial(coeffs)
    f = np.broadcast_to(poly(x)[None, :], (2, nc * m)).copy()
    for sigma in (0.3, 1.75, -0.6):
        out = sldg.sweep(f, 1, np.full((2, 1), sigma), degree)
        ref = poly(x - sigma)
        # interior cells whose feet stay inside [0, nc)
        lo = int(np.ceil(max(sigma, 0))) + 1
        hi = nc - int(np.ceil(max(-sigma, 0))) - 1
        sl = slice(lo * m, hi * m)
        scale = np.max(np.abs(f))
        np.testing.assert_allclose(out[0, sl], ref[sl], rtol=0, atol=1e-14 * scale)


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_matches_brute_force_projection(degree):
    # project the translated piecewise polynomial by high-order quadrature on
    # each piece, with bases built from numpy polynomials
    m = degree + 1
    nc = 5
    xi, w = gauss_legendre_01(degree)
    u = random_field((nc, m), seed=7)
    L = [_np_lagrange(xi, l) for l in range(m)]
    gx, gw = np.polynomial.legendre.leggauss(12)

    def uval(y):
        c = int(np.floor(y)) % nc
        s = y - np.floor(y)
        return sum(u[c, l] * L[l](s) for l in range(m))

    for sigma in (0.41, -1.3, 2.9):
        out = sldg.sweep(u.reshape(1, -1), 1, np.array([[sigma]]), degree).reshape(nc, m)
        frac = sigma - np.floor(sigma)
        for i in range(nc):
            for j in range(m):
                tot = 0.0
                for a, b in ((0.0, frac), (frac, 1.0)):
                    if b <= a:
                        continue
                    tq = a + (b - a) * 0.5 * (gx + 1)
                    vals = np.array([uval(i + t - sigma) for t in tq])
                    tot += 0.5 * (b - a) * np.sum(gw * vals * L[j](tq))
                assert abs(out[i, j] - tot / w[j]) < 1e-13


@pytest.mark.parametrize("degree", [1, 2])
def test_l2_never_increases(degree):
    m = degree + 1
    nc = 8
    _, w = gauss_legendre_01(degree)
    wv = np.tile(w, nc)
    f = random_field((3, nc * m), seed=11)
    n0 = np.einsum("ab,b->a", f * f, wv)
    for s in random_shifts(20, seed=12, n_cells=nc):
        g = sldg.sweep(f, 1, np.full((3, 1), s), degree)
        n1 = np.einsum("ab,b->a", g * g, wv)
        assert np.all(n1 <= n0 * (1 + 1e-14))


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_convergence_order(degree):
    # smooth periodic data: one shift, error at the nodes falls like h^(l+1)
    m = degree + 1
    xi, _ = gauss_legendre_01(degree)
    errs = []
    for nc in (16, 32, 64):
        h = 1.0 / nc
        x = (np.repeat(np.arange(nc), m) + np.tile(xi, nc)) * h
        f = np.sin(2 * np.pi * x)[None, :]
        a = (nc // 4 + 0.37) * h      # same fractional part at every h
        out = sldg.sweep(f, 1, np.array([[a / h]]), degree)
        errs.append(np.max(np.abs(out[0] - np.sin(2 * np.pi * (x - a)))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > degree + 1 - 0.3), rates
