"""Grids, initial conditions, density, Poisson solve and diagnostics (oracle).

Model (Sec. 1, Eq. (1)): d_t f + v . grad_x f + E . grad_v f = 0 with
div E = rho - 1, curl E = 0 and rho = int f dv, on a box periodic in all four
directions.  E = -grad phi with -Lap phi = rho - 1, solved spectrally.

Methods: ``degree >= 0`` selects the SLDG space (nodes at Gauss-Legendre
points of every cell); ``degree = None`` selects the equidistant spline grid
with points at cell centres (i + 1/2) h.
"""

import numpy as np

from .quadrature import gauss_legendre_01, lagrange


# ----------------------------------------------------------------- grids ---

def nodes_1d(lo, length, n_dofs, degree):
    """Coordinates of the n_dofs points of one axis."""
    if degree is None:
        h = length / n_dofs
        return lo + (np.arange(n_dofs) + 0.5) * h
    m = degree + 1
    nc = n_dofs // m
    h = length / nc
    xi, _ = gauss_legendre_01(degree)
    return lo + (np.repeat(np.arange(nc), m) + np.tile(xi, nc)) * h


def weights_1d(length, n_dofs, degree):
    """Quadrature weights of one axis (integral = sum weights * values)."""
    if degree is None:
        return np.full(n_dofs, length / n_dofs)
    m = degree + 1
    nc = n_dofs // m
    _, w = gauss_legendre_01(degree)
    return np.tile(w, nc) * (length / nc)


def cell_width(length, n_dofs, degree):
    """Shift unit: the cell width (SLDG) or the grid spacing (spline)."""
    if degree is None:
        return length / n_dofs
    return length / (n_dofs // (degree + 1))


# ---------------------------------------------------- initial conditions ---

def initial_condition_at(kind, x1, x2, v1, v2, eps, k, v0=0.0, form="sum"):
    """f0 at coordinate arrays that broadcast against each other.

    landau:     (2 pi)^-1 exp(-(v1^2+v2^2)/2) (1 + eps (cos k x1 + cos k x2))
                (Sec. 4, Eq. (6)).
    two_stream: (8 pi)^-1 [g(v1-v0)+g(v1+v0)][g(v2-v0)+g(v2+v0)] p(x),
                g(s) = exp(-s^2/2) (Sec. 5, Eq. (7)); p = 1 + eps cos k x1
                cos k x2 for form="product", 1 + eps (cos k x1 + cos k x2)
                for form="sum".
    """
    if kind == "landau":
        px = 1.0 + eps * (np.cos(k * x1) + np.cos(k * x2))
        fv = np.exp(-0.5 * v1 ** 2) * np.exp(-0.5 * v2 ** 2) / (2.0 * np.pi)
    elif kind == "two_stream":
        if form == "product":
            px = 1.0 + eps * np.cos(k * x1) * np.cos(k * x2)
        else:
            px = 1.0 + eps * (np.cos(k * x1) + np.cos(k * x2))
        g1 = np.exp(-0.5 * (v1 - v0) ** 2) + np.exp(-0.5 * (v1 + v0) ** 2)
        g2 = np.exp(-0.5 * (v2 - v0) ** 2) + np.exp(-0.5 * (v2 + v0) ** 2)
        fv = g1 * g2 / (8.0 * np.pi)
    else:
        raise ValueError(kind)
    return px * fv


def initial_condition(kind, dims, lo, length, degree, eps, k, v0=0.0,
                      form="sum"):
    """Sample f0 at the nodes (the dofs are point values, Sec. 3)."""
    x1, x2, v1, v2 = (nodes_1d(lo[d], length[d], dims[d], degree)
                      for d in range(4))
    return initial_condition_at(kind, x1[:, None, None, None], x2[None, :, None, None],
                                v1[None, None, :, None], v2[None, None, None, :],
                                eps, k, v0, form)


# ---------------------------------------------------------------- density ---

def density(f, degree, length_v1, length_v2):
    """rho(x1, x2) = int f dv with the quadrature of the velocity grid."""
    f = np.asarray(f, dtype=np.float64)
    w1 = weights_1d(length_v1, f.shape[2], degree)
    w2 = weights_1d(length_v2, f.shape[3], degree)
    return np.einsum("abce,c,e->ab", f, w1, w2)


# ---------------------------------------------------------------- Poisson ---

def transfer_matrix(degree):
    """Q[p, m] = L_m(e_p), e_p = (p + 1/2)/(l+1): values of the cell
    polynomial at l+1 equidistant sub-cell midpoints."""
    xi, _ = gauss_legendre_01(degree)
    e = (np.arange(degree + 1) + 0.5) / (degree + 1)
    return lagrange(xi, e).T


def _block(Q, nc):
    return np.kron(np.eye(nc), Q)


def poisson(rho, degree, length_x1, length_x2):
    """E1, E2 on the x-nodes and W = 1/2 int |E|^2 dx.

    SLDG: the nodal density is moved to the uniform grid of sub-cell
    midpoints by Q, E is computed there spectrally and moved back by Q^-1.
    Modes: k = 2 pi m / L with m in FFT order; E_hat = -i k rho_hat / |k|^2,
    set to zero for m = 0 and wherever m1 or m2 is the Nyquist index n/2.
    """
    rho = np.asarray(rho, dtype=np.float64)
    n1, n2 = rho.shape
    if degree is not None:
        Q = transfer_matrix(degree)
        m = degree + 1
        Q1, Q2 = _block(Q, n1 // m), _block(Q, n2 // m)
        r = Q1 @ rho @ Q2.T
    else:
        r = rho
    rh = np.fft.fft2(r)
    m1 = np.fft.fftfreq(n1) * n1
    m2 = np.fft.fftfreq(n2) * n2
    k1 = (2.0 * np.pi / length_x1) * m1[:, None]
    k2 = (2.0 * np.pi / length_x2) * m2[None, :]
    kk = k1 ** 2 + k2 ** 2
    zero = (kk == 0.0)
    if n1 % 2 == 0:
        zero = zero | (np.abs(m1) == n1 // 2)[:, None]
    if n2 % 2 == 0:
        zero = zero | (np.abs(m2) == n2 // 2)[None, :]
    kk_safe = np.where(zero, 1.0, kk)
    e1h = np.where(zero, 0.0, -1j * k1 * rh / kk_safe)
    e2h = np.where(zero, 0.0, -1j * k2 * rh / kk_safe)
    e1 = np.real(np.fft.ifft2(e1h))
    e2 = np.real(np.fft.ifft2(e2h))
    if degree is not None:
        e1 = np.linalg.solve(Q1, np.linalg.solve(Q2, e1.T).T)
        e2 = np.linalg.solve(Q1, np.linalg.solve(Q2, e2.T).T)
    wx1 = weights_1d(length_x1, n1, degree)
    wx2 = weights_1d(length_x2, n2, degree)
    W = 0.5 * np.einsum("ab,a,b->", e1 ** 2 + e2 ** 2, wx1, wx2)
    return e1, e2, float(W)


# ------------------------------------------------------------ diagnostics ---

def moments(f, degree, lo, length):
    """mass, L1, L2 = sqrt(int f^2), kinetic energy 1/2 int |v|^2 f, using
    the nodal quadrature of the grid (Sec. 4 diagnostics)."""
    f = np.asarray(f, dtype=np.float64)
    w = [weights_1d(length[d], f.shape[d], degree) for d in range(4)]
    v1 = nodes_1d(lo[2], length[2], f.shape[2], degree)
    v2 = nodes_1d(lo[3], length[3], f.shape[3], degree)

    def q(g):
        return float(np.einsum("abce,a,b,c,e->", g, *w))

    vv = (v1 ** 2)[:, None] + (v2 ** 2)[None, :]
    return (q(f), q(np.abs(f)), float(np.sqrt(q(f * f))),
            0.5 * q(f * vv[None, None, :, :]))
