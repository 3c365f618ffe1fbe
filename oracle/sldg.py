"""Semi-Lagrangian discontinuous Galerkin translate-and-project (oracle).

What is computed (Sec. 2, last part; Sec. 3, Eq. (5)): a function that is a
polynomial of degree l on every cell is translated, u'(x) = u(x - a), and the
result is L2-projected back onto cell-wise polynomials of degree l.  The
degrees of freedom are values at the Gauss-Legendre nodes of every cell.  Each
output cell needs two adjacent input cells, and the update is linear:

    u'_{i,j} = sum_l A_{jl} u_{i*,l} + sum_l B_{jl} u_{i*+1,l}

(the second sum of Eq. (5) runs over l; the printed index j is a typo).

The paper defers the entries of A and B to another article.  They follow from
the definition: write the shift in cells as sigma = a/h, n = floor(sigma) and
alpha = sigma - n in [0, 1).  On the normalised output cell t in [0, 1) the
translated point lies in input cell i-n-1 (local coordinate t+1-alpha) for
t < alpha and in input cell i-n (local coordinate t-alpha) for t >= alpha, so
i* = i-n-1.  The Gauss-Legendre mass matrix is diagonal with entries w_j, so

    A_jl(alpha) = (1/w_j) int_0^alpha  L_l(t+1-alpha) L_j(t) dt
    B_jl(alpha) = (1/w_j) int_alpha^1  L_l(t-alpha)   L_j(t) dt.

Both integrands are polynomials of degree 2l, so the (l+1)-point
Gauss-Legendre rule mapped onto [0, alpha] and [alpha, 1] evaluates them
exactly; this is how the paper says the coefficients are obtained (Sec. 2).
"""

import numpy as np

from .quadrature import gauss_legendre_01, lagrange


def projection_matrices(degree, alpha):
    """A(alpha), B(alpha), each (l+1)x(l+1), for 0 <= alpha <= 1."""
    alpha = float(alpha)
    xi, w = gauss_legendre_01(degree)
    # integral over [0, alpha]: points alpha*xi_q, weights alpha*w_q
    ta = alpha * xi
    La_out = lagrange(xi, ta)                   # L_j(t_q)        [j, q]
    La_in = lagrange(xi, ta + (1.0 - alpha))    # L_l(t_q+1-alpha) [l, q]
    A = (La_out * (alpha * w)) @ La_in.T / w[:, None]
    # integral over [alpha, 1]: points alpha+(1-alpha)*xi_q, weights (1-alpha)*w_q
    tb = alpha + (1.0 - alpha) * xi
    Lb_out = lagrange(xi, tb)
    Lb_in = lagrange(xi, tb - alpha)
    B = (Lb_out * ((1.0 - alpha) * w)) @ Lb_in.T / w[:, None]
    return A, B


def split_shift(sigma):
    """n = floor(sigma) (a Python int) and alpha = sigma - n, both from FP64.

    This is the exact floor branch: the translated point lies in the cell
    that sigma itself falls in.  For sigma in [-2^-54, 0) the difference
    sigma - floor(sigma) = 1 + sigma rounds to 1.0, so alpha may equal one.
    The forward map is unaffected (A(1) = I, B(1) = 0 shifted by one cell is
    A(0) = 0, B(0) = I), but a shift derivative taken here is the derivative
    at sigma, i.e. the one from the left of the whole cell, not from the
    right.  Only an exactly integer sigma gives alpha = 0 and the one-sided
    derivative from the right.
    """
    sigma = float(sigma)
    n = np.floor(sigma)
    alpha = sigma - n
    return int(n), alpha


def shift_lines(lines, sigma, degree):
    """Apply the SLDG shift by ``sigma`` cells to every row of ``lines``.

    ``lines`` has shape (n_lines, n_cells*(degree+1)); all rows share sigma.
    Periodic in the cell index.
    """
    m = degree + 1
    nl, N = lines.shape
    nc = N // m
    u = lines.reshape(nl, nc, m)
    n, alpha = split_shift(sigma)
    A, B = projection_matrices(degree, alpha)
    i = np.arange(nc)
    left = (i - n - 1) % nc
    right = (i - n) % nc
    out = u[:, left, :] @ A.T + u[:, right, :] @ B.T
    return out.reshape(nl, N)


def sweep(f, axis, sigma, degree):
    """SLDG sweep of the 4D (any-D) array ``f`` along ``axis``.

    ``sigma`` holds the shift in cells for every line along ``axis``: an
    array broadcastable to ``f`` once the ``axis`` dimension is dropped (pass
    it with that dimension of length 1, or with it removed).  Computation is
    in float64 whatever the dtype of ``f``.
    """
    f = np.asarray(f, dtype=np.float64)
    m = degree + 1
    if f.shape[axis] % m:
        raise ValueError("axis length must be a multiple of degree+1")
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
        out[sel] = shift_lines(lines[sel], s, degree)
    return np.moveaxis(out.reshape(g.shape), -1, axis)
