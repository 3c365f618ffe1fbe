"""Strang splitting step (oracle), Sec. 2.

f^{m+1} = exp(tau/2 A) exp(tau B) exp(tau/2 A) f^m, with A the free streaming
(exact flow g(x - tau v, v)) and B the acceleration (exact flow
g(x, v - tau E(x))).  A and B are applied direction by direction, which adds
no error because the directional parts commute.  E is computed once per step
from the density after the first half step; the acceleration leaves the
density unchanged, so E stays fixed during B.

Shifts, in cells (SLDG) or grid points (spline):
  x_d sweep:  sigma = (tau/2) v_d / h_{x_d}, one value per v_d node;
  v_d sweep:  sigma = tau E_d(x1, x2) / h_{v_d}, one value per (x1, x2).
Sweep order: x1, x2, (rho -> E), v1, v2, x1, x2.

``run_merged`` takes the same steps but joins the closing x half-steps of one
step and the opening x half-steps of the next into x sweeps of the whole step
tau (the exact free-streaming flows compose: exp(tau/2 A) exp(tau/2 A) =
exp(tau A)); the state f^m itself is only formed, and its diagnostics taken,
every ``every`` steps.  With every = 1 it is ``run``.
"""

from dataclasses import dataclass

import numpy as np

from . import field, sldg, spline


@dataclass
class Grid:
    dims: tuple
    lo: tuple
    length: tuple
    degree: object      # int >= 0 for SLDG, None for the spline grid

    def h(self, d):
        return field.cell_width(self.length[d], self.dims[d], self.degree)

    def nodes(self, d):
        return field.nodes_1d(self.lo[d], self.length[d], self.dims[d],
                              self.degree)


def advect(f, axis, sigma, grid):
    if grid.degree is None:
        return spline.sweep(f, axis, sigma)
    return sldg.sweep(f, axis, sigma, grid.degree)


def x_shift(grid, d, tau_part):
    """Shift of the x_d sweep as an array broadcastable to f (axis d kept)."""
    v = grid.nodes(d + 2)
    s = tau_part * v / grid.h(d)
    shape = [1, 1, 1, 1]
    shape[d + 2] = len(v)
    return s.reshape(shape)


def electric_field(f, grid):
    rho = field.density(f, grid.degree, grid.length[2], grid.length[3])
    return field.poisson(rho, grid.degree, grid.length[0], grid.length[1])


def step(f, grid, tau):
    """One Strang step; returns f^{m+1}."""
    f = advect(f, 0, x_shift(grid, 0, 0.5 * tau), grid)
    f = advect(f, 1, x_shift(grid, 1, 0.5 * tau), grid)
    e1, e2, _ = electric_field(f, grid)
    s1 = (tau * e1 / grid.h(2))[:, :, None, None]
    s2 = (tau * e2 / grid.h(3))[:, :, None, None]
    f = advect(f, 2, s1, grid)
    f = advect(f, 3, s2, grid)
    f = advect(f, 0, x_shift(grid, 0, 0.5 * tau), grid)
    f = advect(f, 1, x_shift(grid, 1, 0.5 * tau), grid)
    return f


def run(f0, grid, tau, nsteps, with_moments=False):
    """Integrate ``nsteps`` Strang steps.

    Returns (f, W) with W[m] the electric energy of f^m, m = 0..nsteps, and,
    when ``with_moments``, also the (nsteps+1, 4) array of mass, L1, L2 and
    kinetic energy of every f^m.
    """
    f = np.asarray(f0, dtype=np.float64)
    W = [electric_field(f, grid)[2]]
    mom = [field.moments(f, grid.degree, grid.lo, grid.length)]
    for _ in range(nsteps):
        f = step(f, grid, tau)
        W.append(electric_field(f, grid)[2])
        if with_moments:
            mom.append(field.moments(f, grid.degree, grid.lo, grid.length))
    if with_moments:
        return f, np.array(W), np.array(mom)
    return f, np.array(W)


def run_merged(f0, grid, tau, nsteps, every, with_moments=False):
    """``nsteps`` Strang steps in segments of ``every`` steps, each segment
    x(tau/2) [field, v1, v2, x(tau)] ... [field, v1, v2, x(tau/2)].

    Returns (f, W) with W[j] the electric energy of f^{j*every}, and, when
    ``with_moments``, the moments of the same states.
    """
    if every < 1 or nsteps % every:
        raise ValueError("nsteps must be a multiple of every >= 1")
    f = np.asarray(f0, dtype=np.float64)
    W = [electric_field(f, grid)[2]]
    mom = [field.moments(f, grid.degree, grid.lo, grid.length)]
    for _ in range(nsteps // every):
        f = advect(f, 0, x_shift(grid, 0, 0.5 * tau), grid)
        f = advect(f, 1, x_shift(grid, 1, 0.5 * tau), grid)
        for j in range(every):
            e1, e2, _ = electric_field(f, grid)
            f = advect(f, 2, (tau * e1 / grid.h(2))[:, :, None, None], grid)
            f = advect(f, 3, (tau * e2 / grid.h(3))[:, :, None, None], grid)
            part = tau if j < every - 1 else 0.5 * tau
            f = advect(f, 0, x_shift(grid, 0, part), grid)
            f = advect(f, 1, x_shift(grid, 1, part), grid)
        W.append(electric_field(f, grid)[2])
        if with_moments:
            mom.append(field.moments(f, grid.degree, grid.lo, grid.length))
    if with_moments:
        return f, np.array(W), np.array(mom)
    return f, np.array(W)
