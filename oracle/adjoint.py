"""Adjoint (transposed) operators and gradients of the split step (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Transposes are with respect to the plain Euclidean inner product of the
arrays of degrees of freedom, <a, b> = sum a*b, which is what reverse-mode
differentiation of the discrete map needs.

* SLDG sweep, fixed shift (Sec. 3, Eq. (5)): out_i = A u_{i-s-1} + B u_{i-s}
  gives u_bar_c = A^T lam_{c+s+1} + B^T lam_{c+s} (indices mod n_c).
* Its derivative with respect to a line's shift: d out_i / d sigma =
  A'(alpha) u_{i-s-1} + B'(alpha) u_{i-s}, with, by Leibniz' rule on the
  integrals that define A and B,
    A'_jl = (1/w_j) [ L_l(1) L_j(alpha) - int_0^alpha L_l'(t+1-alpha) L_j(t) dt ]
    B'_jl = (1/w_j) [ -L_l(0) L_j(alpha) - int_alpha^1 L_l'(t-alpha) L_j(t) dt ]
  (integrands of degree 2l-1: exact with the (l+1)-point Gauss rule).
* Spline sweep: out = E(alpha) C^{-1} u with E the four-tap evaluation; C is
  symmetric, so u_bar = C^{-1} E^T lam; d out/d sigma uses d beta/d alpha.
* Density rho = D f: D^T g broadcasts g over v with the quadrature weights.
* Poisson E_d = P_d rho: on the uniform grid P_d is a real Fourier multiplier
  m_d(k) = -i k_d/|k|^2 whose conjugate is -m_d(k), so its transpose is -P_d;
  the SLDG maps Q, Q^{-1} act per cell and are transposed as matrices.
* Objective: the final electric energy J = W(f^N) = 1/2 sum w_a w_b |E|^2.
"""

import numpy as np

from . import field, sldg, spline, strang
from .quadrature import gauss_legendre_01, lagrange


# --------------------------------------------------------------- helpers ---

def lagrange_deriv(nodes, t):
    """L_l'(t) for the Lagrange basis on ``nodes``: shape (len(nodes),)+shape(t)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    m = len(nodes)
    out = np.zeros((m,) + t.shape)
    for l in range(m):
        denom = np.prod([nodes[l] - nodes[k] for k in range(m) if k != l])
        for q in range(m):
            if q == l:
                continue
            term = np.ones_like(t)
            for k in range(m):
                if k != l and k != q:
                    term = term * (t - nodes[k])
            out[l] = out[l] + term
        out[l] = out[l] / denom
    return out


def _lines(f, axis, sigma):
    f = np.asarray(f, dtype=np.float64)
    g = np.moveaxis(f, axis, -1)
    sig = np.asarray(sigma, dtype=np.float64)
    if sig.ndim == f.ndim:
        sig = np.moveaxis(sig, axis, -1)[..., 0]
    sig = np.broadcast_to(sig, g.shape[:-1]).reshape(-1)
    return g, g.reshape(-1, g.shape[-1]), sig


# ----------------------------------------------------------------- SLDG ---

def projection_derivatives(degree, alpha):
    """dA/dalpha and dB/dalpha (Leibniz' rule on the defining integrals)."""
    alpha = float(alpha)
    xi, w = gauss_legendre_01(degree)
    m = degree + 1
    L_at_1 = lagrange(xi, np.array(1.0))       # L_l(1)
    L_at_0 = lagrange(xi, np.array(0.0))       # L_l(0)
    L_at_a = lagrange(xi, np.array(alpha))     # L_j(alpha)
    dA = np.outer(L_at_a, L_at_1)              # [j, l] = L_j(alpha) L_l(1)
    dB = -np.outer(L_at_a, L_at_0)
    ta = alpha * xi
    dA -= (lagrange(xi, ta) * (alpha * w)) @ lagrange_deriv(xi, ta + (1.0 - alpha)).T
    tb = alpha + (1.0 - alpha) * xi
    dB -= (lagrange(xi, tb) * ((1.0 - alpha) * w)) @ lagrange_deriv(xi, tb - alpha).T
    return dA / w[:, None], dB / w[:, None]


def sldg_sweep_adjoint(lam, axis, sigma, degree):
    """Transpose of sldg.sweep for fixed shifts, applied to ``lam``."""
    m = degree + 1
    g, lines, sig = _lines(lam, axis, sigma)
    nl, N = lines.shape
    nc = N // m
    out = np.empty_like(lines)
    values, inverse = np.unique(sig, return_inverse=True)
    c = np.arange(nc)
    for k, s in enumerate(values):
        sel = np.nonzero(inverse == k)[0]
        n, alpha = sldg.split_shift(s)
        A, B = sldg.projection_matrices(degree, alpha)
        la = lines[sel].reshape(-1, nc, m)
        out[sel] = (la[:, (c + n + 1) % nc, :] @ A + la[:, (c + n) % nc, :] @ B).reshape(-1, N)
    return np.moveaxis(out.reshape(g.shape), -1, axis)


def sldg_sweep_dshift(f, lam, axis, sigma, degree):
    """d <lam, sweep(f, sigma)> / d sigma for every line (array of the line
    index shape, i.e. f.shape without ``axis``)."""
    m = degree + 1
    g, fl, sig = _lines(f, axis, sigma)
    _, ll, _ = _lines(lam, axis, sigma)
    nl, N = fl.shape
    nc = N // m
    out = np.empty(nl)
    values, inverse = np.unique(sig, return_inverse=True)
    i = np.arange(nc)
    for k, s in enumerate(values):
        sel = np.nonzero(inverse == k)[0]
        n, alpha = sldg.split_shift(s)
        dA, dB = projection_derivatives(degree, alpha)
        u = fl[sel].reshape(-1, nc, m)
        d = u[:, (i - n - 1) % nc, :] @ dA.T + u[:, (i - n) % nc, :] @ dB.T
        out[sel] = np.sum(d.reshape(len(sel), -1) * ll[sel], axis=1)
    return out.reshape(g.shape[:-1])


# --------------------------------------------------------------- spline ---

def spline_weight_derivatives(alpha):
    """d beta_q / d alpha (beta as in spline.weights, t = 1 - alpha)."""
    t = 1.0 - float(alpha)
    dbdt = np.array([-3.0 * (1.0 - t) ** 2 / 6.0,
                     (9.0 * t ** 2 - 12.0 * t) / 6.0,
                     (-9.0 * t ** 2 + 6.0 * t + 3.0) / 6.0,
                     3.0 * t ** 2 / 6.0])
    return -dbdt


def spline_sweep_adjoint(lam, axis, sigma):
    """Transpose of spline.sweep for fixed shifts: C^{-1} E^T lam."""
    g, lines, sig = _lines(lam, axis, sigma)
    nl, n_pts = lines.shape
    mu = np.zeros_like(lines)
    values, inverse = np.unique(sig, return_inverse=True)
    i = np.arange(n_pts)
    for k, s in enumerate(values):
        sel = np.nonzero(inverse == k)[0]
        n, alpha = sldg.split_shift(s)
        beta = spline.weights(alpha)
        lsel = lines[sel]
        acc = np.zeros_like(lsel)
        m0 = i - n - 1
        for q in range(4):
            # out_i += beta_q omega_{m0_i - 1 + q}: scatter lam_i to that index
            np.add.at(acc, (slice(None), (m0 - 1 + q) % n_pts), beta[q] * lsel)
        mu[sel] = acc
    out = spline.coefficients(mu)       # C^{-1} is symmetric
    return np.moveaxis(out.reshape(g.shape), -1, axis)


def spline_sweep_dshift(f, lam, axis, sigma):
    g, fl, sig = _lines(f, axis, sigma)
    _, ll, _ = _lines(lam, axis, sigma)
    nl, n_pts = fl.shape
    out = np.empty(nl)
    values, inverse = np.unique(sig, return_inverse=True)
    i = np.arange(n_pts)
    for k, s in enumerate(values):
        sel = np.nonzero(inverse == k)[0]
        n, alpha = sldg.split_shift(s)
        db = spline_weight_derivatives(alpha)
        omega = spline.coefficients(fl[sel])
        m0 = i - n - 1
        d = np.zeros_like(omega)
        for q in range(4):
            d += db[q] * omega[:, (m0 - 1 + q) % n_pts]
        out[sel] = np.sum(d * ll[sel], axis=1)
    return out.reshape(g.shape[:-1])


# ------------------------------------------------------ density, Poisson ---

def density_adjoint(g_rho, shape, degree, length_v1, length_v2):
    """D^T: the weighted broadcast of g_rho over the velocity axes."""
    w1 = field.weights_1d(length_v1, shape[2], degree)
    w2 = field.weights_1d(length_v2, shape[3], degree)
    return g_rho[:, :, None, None] * w1[None, None, :, None] * w2[None, None, None, :]


def _spectral(Y, length_x1, length_x2, comp):
    n1, n2 = Y.shape
    m1 = np.fft.fftfreq(n1) * n1
    m2 = np.fft.fftfreq(n2) * n2
    k1 = (2.0 * np.pi / length_x1) * m1[:, None]
    k2 = (2.0 * np.pi / length_x2) * m2[None, :]
    kk = k1 ** 2 + k2 ** 2
    zero = kk == 0.0
    if n1 % 2 == 0:
        zero = zero | (np.abs(m1) == n1 // 2)[:, None]
    if n2 % 2 == 0:
        zero = zero | (np.abs(m2) == n2 // 2)[None, :]
    kd = k1 if comp == 0 else k2
    mult = np.where(zero, 0.0, -1j * kd / np.where(zero, 1.0, kk))
    return np.real(np.fft.ifft2(mult * np.fft.fft2(Y)))


def poisson_adjoint(g1, g2, degree, length_x1, length_x2):
    """rho_bar = P_1^T g1 + P_2^T g2 for (E1, E2) = poisson(rho)."""
    g1 = np.asarray(g1, dtype=np.float64)
    g2 = np.asarray(g2, dtype=np.float64)
    n1, n2 = g1.shape
    if degree is not None:
        Q = field.transfer_matrix(degree)
        m = degree + 1
        Q1 = np.kron(np.eye(n1 // m), Q)
        Q2 = np.kron(np.eye(n2 // m), Q)
        Q1i, Q2i = np.linalg.inv(Q1), np.linalg.inv(Q2)
        # E_d = Q1^-1 S_d(Q1 rho Q2^T) Q2^-T ; transpose: Q1^T S_d^T(Q1^-T G Q2^-1) Q2
        y1 = Q1i.T @ g1 @ Q2i
        y2 = Q1i.T @ g2 @ Q2i
        r = -_spectral(y1, length_x1, length_x2, 0) - _spectral(y2, length_x1, length_x2, 1)
        return Q1.T @ r @ Q2
    return -_spectral(g1, length_x1, length_x2, 0) - _spectral(g2, length_x1, length_x2, 1)


# ------------------------------------------------------------- the step ---

def _advect(f, axis, sigma, grid):
    return strang.advect(f, axis, sigma, grid)


def _advect_adjoint(lam, axis, sigma, grid):
    if grid.degree is None:
        return spline_sweep_adjoint(lam, axis, sigma)
    return sldg_sweep_adjoint(lam, axis, sigma, grid.degree)


def _advect_dshift(f, lam, axis, sigma, grid):
    if grid.degree is None:
        return spline_sweep_dshift(f, lam, axis, sigma)
    return sldg_sweep_dshift(f, lam, axis, sigma, grid.degree)


def step_adjoint(f, lam, grid, tau):
    """Given f^m and lam = dJ/df^{m+1}, return dJ/df^m (one Strang step)."""
    sx1 = strang.x_shift(grid, 0, 0.5 * tau)
    sx2 = strang.x_shift(grid, 1, 0.5 * tau)
    f1 = _advect(f, 0, sx1, grid)
    f2 = _advect(f1, 1, sx2, grid)
    e1, e2, _ = strang.electric_field(f2, grid)
    s1 = (tau * e1 / grid.h(2))[:, :, None, None]
    s2 = (tau * e2 / grid.h(3))[:, :, None, None]
    f3 = _advect(f2, 2, s1, grid)
    # backward
    l5 = _advect_adjoint(lam, 1, sx2, grid)
    l4 = _advect_adjoint(l5, 0, sx1, grid)
    l3 = _advect_adjoint(l4, 3, s2, grid)
    g2 = _advect_dshift(f3, l4, 3, s2, grid).sum(axis=2)        # sum over v1
    l2 = _advect_adjoint(l3, 2, s1, grid)
    g1 = _advect_dshift(f2, l3, 2, s1, grid).sum(axis=2)        # sum over v2
    rho_bar = poisson_adjoint(tau / grid.h(2) * g1, tau / grid.h(3) * g2, grid.degree,
                              grid.length[0], grid.length[1])
    l2 = l2 + density_adjoint(rho_bar, f.shape, grid.degree, grid.length[2], grid.length[3])
    l1 = _advect_adjoint(l2, 1, sx2, grid)
    return _advect_adjoint(l1, 0, sx1, grid)


def energy_gradient(f, grid):
    """J = W(f) = 1/2 sum w_a w_b (E1^2 + E2^2) and dJ/df."""
    e1, e2, W = strang.electric_field(f, grid)
    wx1 = field.weights_1d(grid.length[0], f.shape[0], grid.degree)
    wx2 = field.weights_1d(grid.length[1], f.shape[1], grid.degree)
    wx = wx1[:, None] * wx2[None, :]
    rho_bar = poisson_adjoint(wx * e1, wx * e2, grid.degree, grid.length[0], grid.length[1])
    return W, density_adjoint(rho_bar, f.shape, grid.degree, grid.length[2], grid.length[3])


def final_energy_gradient(f0, grid, tau, nsteps):
    """J = W(f^N) after ``nsteps`` Strang steps from f0, and dJ/df0.

    Every intermediate state is stored (the oracle has no memory pressure)."""
    states = [np.asarray(f0, dtype=np.float64)]
    for _ in range(nsteps):
        states.append(strang.step(states[-1], grid, tau))
    J, lam = energy_gradient(states[-1], grid)
    for m in range(nsteps - 1, -1, -1):
        lam = step_adjoint(states[m], lam, grid, tau)
    return J, lam
