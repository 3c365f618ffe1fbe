"""Pins of oracle.field: density, Poisson, transfer matrices, diagnostics."""

import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import field
from oracle.quadrature import gauss_legendre_01


@pytest.mark.parametrize("degree", [None, 0, 2, 3])
def test_density_of_constant(degree):
    m = 1 if degree is None else degree + 1
    dims = (2, 3, 4 * m, 5 * m)
    f = np.full(dims, 0.7)
    rho = field.density(f, degree, 12.0, 18.0)
    np.testing.assert_allclose(rho, 0.7 * 12.0 * 18.0, rtol=1e-14)


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_density_exact_for_cellwise_polynomials(degree):
    # a polynomial of degree <= 2l+1 in v is integrated exactly by the GL nodes
    m = degree + 1
    nc = 4
    L = 3.0
    v = field.nodes_1d(-1.5, L, nc * m, degree)
    p = np.polynomial.Polynomial(np.linspace(1.0, -0.5, 2 * degree + 2))
    f = (p(v)[:, None] * np.ones(nc * m)[None, :])[None, None]
    exact = (p.integ()(1.5) - p.integ()(-1.5)) * L
    assert abs(field.density(f, degree, L, L)[0, 0] - exact) < 1e-12 * abs(exact)


@pytest.mark.parametrize("n", [16, 24, 30])
def test_poisson_pure_mode_spline_grid(n):
    # rho - 1 = eps cos(k x1) on a uniform grid: E1 = (eps/k) sin(k x1), E2 = 0
    Lx = 4 * math.pi
    k = 2 * math.pi / Lx * 2
    eps = 0.3
    x = field.nodes_1d(0.0, Lx, n, None)
    rho = 1.0 + eps * np.cos(k * x)[:, None] * np.ones(n + 2)[None, :]
    rho = rho[:, :n]
    e1, e2, W = field.poisson(rho, None, Lx, Lx)
    np.testing.assert_allclose(e1, (eps / k) * np.sin(k * x)[:, None] * np.ones((1, n)),
                               rtol=0, atol=1e-14)
    np.testing.assert_allclose(e2, 0.0, atol=1e-15)
    # W = 1/2 int E^2 = 1/2 (eps/k)^2 * Lx^2 / 2
    assert abs(W - 0.25 * (eps / k) ** 2 * Lx * Lx) < 1e-12
    # the other direction, with a non-square box
    rho2 = 1.0 + eps * np.cos(k * x)[None, :] * np.ones((n, 1))
    e1b, e2b, _ = field.poisson(rho2, None, Lx, Lx)
    np.testing.assert_allclose(e2b, (eps / k) * np.sin(k * x)[None, :] * np.ones((n, 1)),
                               rtol=0, atol=1e-14)
    np.testing.assert_allclose(e1b, 0.0, atol=1e-15)


def test_poisson_uniform_density_gives_zero_field():
    for degree in (None, 2):
        n = 12
        e1, e2, W = field.poisson(np.full((n, n), 1.37), degree, 5.0, 7.0)
        assert np.max(np.abs(e1)) < 1e-14 and np.max(np.abs(e2)) < 1e-14 and W < 1e-26


def test_poisson_gauss_law_spectrally():
    # for a band-limited density the divergence of E, taken spectrally,
    # returns rho minus its mean
    n1, n2 = 16, 20
    L1, L2 = 3.0, 5.0
    x1 = field.nodes_1d(0.0, L1, n1, None)
    x2 = field.nodes_1d(0.0, L2, n2, None)
    rho = (1.0 + 0.2 * np.sin(2 * np.pi * 3 * x1 / L1)[:, None] * np.cos(2 * np.pi * 2 * x2 / L2)[None, :]
           + 0.1 * np.cos(2 * np.pi * x1 / L1)[:, None])
    e1, e2, _ = field.poisson(rho, None, L1, L2)
    k1 = 2 * np.pi / L1 * np.fft.fftfreq(n1) * n1
    k2 = 2 * np.pi / L2 * np.fft.fftfreq(n2) * n2
    div = np.real(np.fft.ifft2(1j * k1[:, None] * np.fft.fft2(e1) + 1j * k2[None, :] * np.fft.fft2(e2)))
    np.testing.assert_allclose(div, rho - rho.mean(), rtol=0, atol=1e-13)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_transfer_matrix(degree):
    Q = field.transfer_matrix(degree)
    m = degree + 1
    # rows sum to one (constants are preserved) and a degree-l polynomial
    # sampled at the GL nodes is mapped to its values at the sub-cell midpoints
    np.testing.assert_allclose(Q.sum(axis=1), 1.0, atol=1e-14)
    xi, _ = gauss_legendre_01(degree)
    e = (np.arange(m) + 0.5) / m
    p = np.polynomial.Polynomial(np.linspace(0.5, -1.0, m))
    np.testing.assert_allclose(Q @ p(xi), p(e), atol=1e-14)


@pytest.mark.parametrize("degree", [1, 2])
def test_poisson_sldg_converges(degree):
    # E of a smooth density converges at order >= l+1 at the nodes
    Lx = 4 * math.pi
    k = 0.5
    eps = 0.4
    errs = []
    for nc in (8, 16, 32):
        n = nc * (degree + 1)
        x = field.nodes_1d(0.0, Lx, n, degree)
        rho = 1.0 + eps * np.cos(k * x)[:, None] * np.ones((1, n))
        e1, _, _ = field.poisson(rho, degree, Lx, Lx)
        errs.append(np.max(np.abs(e1 - (eps / k) * np.sin(k * x)[:, None])))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > degree + 1 - 0.3), rates


def test_landau_initial_energy_spline_grid():
    # rho = M^2 (1 + eps (cos k x1 + cos k x2)), M the midpoint-rule mass of
    # the Maxwellian on [-6, 6]; W(0) = 1/2 M^4 (eps/k)^2 L1 L2 = 8 pi^2 M^4
    n = 32
    dims = (n, n, n, n)
    lo = (0.0, 0.0, -6.0, -6.0)
    ln = (4 * math.pi, 4 * math.pi, 12.0, 12.0)
    f = field.initial_condition("landau", dims, lo, ln, None, 0.5, 0.5)
    rho = field.density(f, None, 12.0, 12.0)
    _, _, W = field.poisson(rho, None, ln[0], ln[1])
    M = erf(6.0 / math.sqrt(2.0))        # midpoint rule is spectrally accurate here
    assert abs(W - 8 * math.pi ** 2 * M ** 4) < 1e-8 * W


def test_moments_of_landau_state():
    n = 24
    dims = (n, n, n, n)
    lo = (0.0, 0.0, -6.0, -6.0)
    ln = (4 * math.pi, 4 * math.pi, 12.0, 12.0)
    f = field.initial_condition("landau", dims, lo, ln, None, 0.5, 0.5)
    mass, l1, l2, kin = field.moments(f, None, lo, ln)
    M = erf(6.0 / math.sqrt(2.0))
    area = ln[0] * ln[1]
    assert abs(mass - area * M * M) < 1e-8 * mass
    assert abs(l1 - mass) < 1e-14 * mass           # f > 0
    # <v^2> of the unit Maxwellian truncated to [-6,6]: 1 - 12 phi(6)/M per direction
    phi6 = math.exp(-18.0) / math.sqrt(2 * math.pi)
    v2 = 1.0 - 2 * 6 * phi6 / M
    assert abs(kin - area * M * M * v2) < 1e-7 * kin
    # int f^2 = area (1 + eps^2) * (int g^2 dv)^2, int g^2 = 1/(2 sqrt(pi)) erf(6)
    g2 = erf(6.0) / (2 * math.sqrt(math.pi))
    assert abs(l2 ** 2 - area * (1 + 0.25) * g2 ** 2) < 1e-8 * l2 ** 2
