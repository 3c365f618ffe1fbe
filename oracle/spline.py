"""Periodic cubic-spline semi-Lagrangian sweep (oracle).

What is computed (Sec. 3): on an equidistant periodic grid of n points the
values u_i are interpolated by sum_k omega_k S(x - x_k), S the cubic B-spline
with 6 S(x) = 4 - 6 (x/h)^2 + 3 |x/h|^3 for |x| <= h, (2 - |x/h|)^3 for
h <= |x| <= 2h and 0 beyond.  Interpolation at the grid points gives the
periodic tridiagonal (circulant) system (1/6) circ(4, 1, 0, ..., 0, 1) omega
= u printed in Sec. 3; the new values are the spline evaluated at the feet of
the characteristics, u'_i = s(x_i - a).

With the shift in grid points sigma = a/h, n = floor(sigma), alpha = sigma-n,
t = 1 - alpha and m = i - n - 1, the point x_i - a sits at x_m + t h, so only
omega_{m-1..m+2} contribute, with weights 6 S at distances 1+t, t, 1-t, 2-t:

    beta_0 = (1-t)^3/6, beta_1 = (3t^3 - 6t^2 + 4)/6,
    beta_2 = (-3t^3 + 3t^2 + 3t + 1)/6, beta_3 = t^3/6.
"""

import numpy as np
from scipy.linalg import solve_circulant

from .sldg import split_shift


def circulant_column(n):
    """First column of (1/6)(u_{i-1} + 4 u_i + u_{i+1}) with periodic indices."""
    c = np.zeros(n)
    np.add.at(c, [0, 1 % n, (n - 1) % n], [4.0, 1.0, 1.0])
    return c / 6.0


def coefficients(lines):
    """Spline coefficients omega for every row of ``lines`` (shape (L, n))."""
    lines = np.asarray(lines, dtype=np.float64)
    n = lines.shape[-1]
    return solve_circulant(circulant_column(n), lines.T).T


def weights(alpha):
    """beta_0..beta_3 for the fractional shift alpha in [0, 1]."""
    t = 1.0 - float(alpha)
    return np.array([(1.0 - t) ** 3 / 6.0,
                     (3.0 * t ** 3 - 6.0 * t ** 2 + 4.0) / 6.0,
                     (-3.0 * t ** 3 + 3.0 * t ** 2 + 3.0 * t + 1.0) / 6.0,
                     t ** 3 / 6.0])


def shift_lines(lines, sigma):
    """Shift every row of ``lines`` by ``sigma`` grid points (periodic)."""
    omega = coefficients(lines)
    n_pts = lines.shape[-1]
    n, alpha = split_shift(sigma)
    beta = weights(alpha)
    m = np.arange(n_pts) - n - 1
    out = np.zeros_like(omega)
    for q in range(4):
        out += beta[q] * omega[:, (m - 1 + q) % n_pts]
    return out


def sweep(f, axis, sigma):
    """Cubic-spline sweep of ``f`` along ``axis``; ``sigma`` as in sldg.sweep."""
    f = np.asarray(f, dtype=np.float64)
    g = np.moveaxis(f, axis, -1)
    sig = np.asarray(sigma, dtype=np.float64)
    if sig.ndim == f.ndim:
        sig = np.moveaxis(sig, axis, -1)[..., 0]
    sig = np.broadcast_to(sig, g.shape[:-1]).reshape(-1)
    lines = g.reshape(-1, g.shape[-1])
    out = np.empty_like(lines)
    values, inverse = np.unique(sig, return_inverse=True)
    for k, s in enumerate(values):
        sel = np.nonzero(inverse == k)[0]
        out[sel] = shift_lines(lines[sel], s)
    return np.moveaxis(out.reshape(g.shape), -1, axis)
