"""Gauss-Legendre nodes and Lagrange bases on the unit cell.

The SLDG degrees of freedom are point values at the l+1 Gauss-Legendre nodes
of each cell (Sec. 2, end; Sec. 3 around Eq. (5)).  Nodes xi_j are returned on
[0, 1] in ascending order with weights w_j summing to one, so that the
integral over a cell of width h is h * sum_j w_j g(xi_j).
"""

import numpy as np


def gauss_legendre_01(degree):
    """Nodes and weights of the (degree+1)-point Gauss-Legendre rule on [0,1]."""
    if degree < 0:
        raise ValueError("degree must be >= 0")
    x, w = np.polynomial.legendre.leggauss(degree + 1)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange(nodes, t):
    """Values L_l(t) of the Lagrange basis on ``nodes``.

    Returns an array of shape (len(nodes),) + shape(t).  Each L_l is the
    product over k != l of (t - x_k) / (x_l - x_k), so L_l(x_q) is exactly
    delta_lq in floating point.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    out = np.ones((len(nodes),) + t.shape)
    for l, xl in enumerate(nodes):
        for k, xk in enumerate(nodes):
            if k != l:
                out[l] = out[l] * ((t - xk) / (xl - xk))
    return out
