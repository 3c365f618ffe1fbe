"""Seeded random arrays for parity tests.

Every generator takes an explicit seed and returns float64 NumPy arrays; the
caller casts to the storage precision it tests.
"""

import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def random_field(shape, seed, positive=False):
    """Uniform values in [-1, 1) (or [0, 1) when ``positive``), float64."""
    g = rng(seed)
    a = g.random(size=tuple(shape))
    return a if positive else 2.0 * a - 1.0


def edge_shifts(n_cells):
    """Shifts (in cells or grid points) that probe the floor/modulo logic.

    Integers of both signs, values a rounding step either side of an integer,
    shifts beyond one period and zero.
    """
    n = float(n_cells)
    base = [0.0, 1.0, -1.0, 2.0, -3.0, n, -n, n + 1.0, 2.5 * n + 0.25,
            -2.5 * n - 0.75, 0.5, -0.5, 1e-17, -1e-17]
    out = list(base)
    for v in (1.0, -1.0, 3.0, -2.0, 0.0):
        out.append(float(np.nextafter(v, np.inf)))
        out.append(float(np.nextafter(v, -np.inf)))
    return np.array(out, dtype=np.float64)


def random_shifts(count, seed, scale=3.0, n_cells=None):
    """``count`` shifts uniform in [-scale, scale), with the edge cases of
    :func:`edge_shifts` (when ``n_cells`` is given) written over the front."""
    g = rng(seed)
    s = scale * (2.0 * g.random(size=int(count)) - 1.0)
    if n_cells is not None:
        e = edge_shifts(n_cells)
        m = min(len(e), len(s))
        s[:m] = e[:m]
    return s
