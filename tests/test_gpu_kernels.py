"""Kernel parity: every C-ABI entry point against the FP64 oracle, element by
element, on seeded inputs (grids that span several tiles and ragged tails,
non-cubic so that axis mix-ups fail)."""

import math

import numpy as np
import pytest

from gpu_common import (announce, assert_close, rel_l2, rel_max, require_gpu, to_dev,
                        to_host, torch)
from oracle import field, sldg, spline
from vp_inputs import random_field, random_shifts

pytestmark = pytest.mark.gpu


def _line_shifts(dims, axis, seed, n_cells, scale=3.0):
    shape = list(dims)
    shape[axis] = 1
    count = int(np.prod(shape))
    return random_shifts(count, seed, scale=scale, n_cells=n_cells).reshape(shape)


SLDG_CASES = [
    # (cells per axis, degree)
    ((3, 4, 5, 6), 2),
    ((5, 3, 4, 7), 1),
    ((2, 3, 3, 2), 3),
    ((4, 2, 3, 5), 0),
    ((2, 2, 2, 3), 5),
    ((1, 3, 2, 4), 2),        # a single cell along x1
    ((11, 3, 2, 37), 2),      # strided lines longer than a wavefront, long rows
    # whole workgroups of columns along x1 and x2 (row-segment blocks in
    # memory order), lines that end in a partial segment of cells
    ((3, 5, 4, 16), 3),
    ((11, 9, 4, 16), 1),
]


@pytest.mark.parametrize("cells,degree", SLDG_CASES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_sldg_advect_parity(cells, degree, dt):
    vp = require_gpu()
    m = degree + 1
    dims = tuple(c * m for c in cells)
    f = random_field(dims, seed=sum(cells) + degree)
    fin = to_dev(f, dt)
    f_ref_in = to_host(fin)               # the values the kernel sees
    for axis in range(4):
        announce(f"sldg_advect cells={cells} degree={degree} {dt} axis={axis}")
        sig = _line_shifts(dims, axis, seed=10 * axis + degree, n_cells=cells[axis])
        out = torch.empty_like(fin)
        vp.sldg_advect(axis, degree, fin, out, to_dev(sig))
        ref = sldg.sweep(f_ref_in, axis, sig, degree)
        assert_close(to_host(out), ref, dt, f"axis {axis}")


@pytest.mark.parametrize("cells,degree", [((2, 4, 8, 32), 2), ((4, 2, 8, 32), 1)])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_sldg_advect_parity_shift_shared_along_v2(cells, degree, dt):
    # shifts that do not depend on v2 (as in the x1 sweep of a step): a
    # thread takes 2 or 4 adjacent v2 columns with vector loads and stores
    vp = require_gpu()
    m = degree + 1
    dims = tuple(c * m for c in cells)
    f = random_field(dims, seed=7 + degree)
    fin = to_dev(f, dt)
    fr = to_host(fin)
    rng = np.random.default_rng(8)
    for axis in range(3):
        shape = list(dims)
        shape[axis] = 1
        shape[3] = 1
        sig = rng.uniform(-2.5, 2.5, size=shape)
        sig.flat[0] = -1e-17
        announce(f"sldg_advect shared-v2 shift {cells} degree={degree} {dt} axis={axis}")
        out = torch.empty_like(fin)
        vp.sldg_advect(axis, degree, fin, out, to_dev(sig))
        assert_close(to_host(out), sldg.sweep(fr, axis, sig, degree), dt, f"axis {axis}")
        lam = torch.empty_like(fin)
        vp.sldg_advect_adjoint(axis, degree, fin, lam, to_dev(sig))
        from oracle import adjoint as oadj
        assert_close(to_host(lam), oadj.sldg_sweep_adjoint(fr, axis, sig, degree), dt,
                     f"adjoint axis {axis}")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_sldg_integer_shift_is_exact_permutation(dt):
    vp = require_gpu()
    cells, degree = (4, 5, 3, 6), 2
    m = degree + 1
    dims = tuple(c * m for c in cells)
    f = random_field(dims, seed=3)
    fin = to_dev(f, dt)
    for axis in range(4):
        announce(f"sldg integer shift {dt} axis={axis}")
        shape = list(dims)
        shape[axis] = 1
        k = np.random.default_rng(axis).integers(-9, 9, size=shape).astype(np.float64)
        out = torch.empty_like(fin)
        vp.sldg_advect(axis, degree, fin, out, to_dev(k))
        got = out.cpu().numpy()
        src = fin.cpu().numpy()
        g = np.moveaxis(src, axis, -1)
        kk = np.moveaxis(k, axis, -1)[..., 0]
        exp = np.empty_like(g)
        nc = cells[axis]
        for idx in np.ndindex(g.shape[:-1]):
            exp[idx] = np.roll(g[idx].reshape(nc, m), int(kk[idx]), axis=0).ravel()
        assert np.array_equal(got, np.moveaxis(exp, -1, axis))


def test_sldg_mass_conserved_to_roundoff():
    vp = require_gpu()
    cells, degree = (6, 5, 7, 4), 2
    m = degree + 1
    dims = tuple(c * m for c in cells)
    f = random_field(dims, seed=4, positive=True)
    fin = to_dev(f)
    _, w = np.polynomial.legendre.leggauss(m)
    for axis in range(4):
        announce(f"sldg mass axis={axis}")
        sig = _line_shifts(dims, axis, seed=axis, n_cells=cells[axis])
        out = torch.empty_like(fin)
        vp.sldg_advect(axis, degree, fin, out, to_dev(sig))
        wl = np.tile(w, cells[axis])
        shape = [1, 1, 1, 1]
        shape[axis] = dims[axis]
        m0 = (f * wl.reshape(shape)).sum(axis=axis)
        m1 = (to_host(out) * wl.reshape(shape)).sum(axis=axis)
        assert np.max(np.abs(m1 - m0)) <= 1e-13 * np.max(np.abs(m0))


# (contiguous rows of 1, 3, 16, 67, 96 and 130 points: the padded row
# windows with wrapped copies shorter and longer than the row; strided lines
# of 80 points: FP64 column segments over 16 points; of 130 and 200 points:
# 32-line column tiles in FP64 and FP32, 16-line ones in FP64)
SPLINE_DIMS = [(12, 10, 9, 16), (7, 24, 5, 3), (3, 5, 40, 6), (4, 3, 6, 67), (2, 2, 2, 1),
               (3, 2, 5, 96), (2, 3, 4, 130), (3, 80, 5, 4), (3, 130, 4, 5), (2, 200, 3, 4)]


@pytest.mark.parametrize("dims", SPLINE_DIMS)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_spline_advect_parity(dims, dt):
    vp = require_gpu()
    f = random_field(dims, seed=sum(dims))
    fin = to_dev(f, dt)
    f_ref_in = to_host(fin)
    for axis in range(4):
        announce(f"spline_advect dims={dims} {dt} axis={axis}")
        sig = _line_shifts(dims, axis, seed=20 + axis, n_cells=dims[axis])
        out = torch.empty_like(fin)
        vp.spline_advect(axis, fin, out, to_dev(sig))
        ref = spline.sweep(f_ref_in, axis, sig)
        assert_close(to_host(out), ref, dt, f"axis {axis}")


def test_broadcast_shift_patterns_of_the_step():
    # x-sweeps: one shift per velocity node; v-sweeps: one per (x1, x2)
    vp = require_gpu()
    cells, degree = (5, 4, 6, 3), 2
    m = degree + 1
    dims = tuple(c * m for c in cells)
    f = random_field(dims, seed=8)
    fin = to_dev(f)
    rng = np.random.default_rng(9)
    cases = [(0, rng.uniform(-2, 2, size=(1, 1, dims[2], 1))),
             (1, rng.uniform(-2, 2, size=(1, 1, 1, dims[3]))),
             (2, rng.uniform(-2, 2, size=(dims[0], dims[1], 1, 1))),
             (3, rng.uniform(-2, 2, size=(dims[0], dims[1], 1, 1)))]
    for axis, sig in cases:
        announce(f"step shift pattern axis={axis}")
        st = [0, 0, 0, 0]
        if axis == 0:
            st[2] = 1
        elif axis == 1:
            st[3] = 1
        else:
            st[0], st[1] = dims[1], 1
        out = torch.empty_like(fin)
        vp.sldg_advect(axis, degree, fin, out, to_dev(sig.ravel()), shift_stride=st)
        assert_close(to_host(out), sldg.sweep(f, axis, sig, degree), "f64", f"axis {axis}")
        out2 = torch.empty_like(fin)
        vp.spline_advect(axis, fin, out2, to_dev(sig.ravel()), shift_stride=st)
        assert_close(to_host(out2), spline.sweep(f, axis, sig), "f64", f"spline axis {axis}")


def test_nonfinite_shift_gives_nan_line_only():
    vp = require_gpu()
    dims = (6, 6, 6, 6)
    f = random_field(dims, seed=1)
    fin = to_dev(f)
    sig = np.zeros((6, 6, 1, 6))
    sig[1, 2, 0, 3] = np.nan
    sig[4, 0, 0, 5] = np.inf
    announce("non-finite shifts")
    out = torch.empty_like(fin)
    vp.sldg_advect(2, 2, fin, out, to_dev(sig))
    got = to_host(out)
    assert np.all(np.isnan(got[1, 2, :, 3])) and np.all(np.isnan(got[4, 0, :, 5]))
    mask = np.ones(dims, bool)
    mask[1, 2, :, 3] = False
    mask[4, 0, :, 5] = False
    assert np.array_equal(got[mask], f[mask])


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("axis", [0, 2, 3])
def test_spline_nonfinite_shift_gives_nan_line_only(dt, axis):
    # strided (column tile) and contiguous (row tile) lines: a NaN or an
    # infinite shift poisons its own line and leaves the others of the tile
    vp = require_gpu()
    dims = (8, 6, 10, 12)
    f = random_field(dims, seed=2)
    fin = to_dev(f, dt)
    fr = to_host(fin)
    shape = list(dims)
    shape[axis] = 1
    sig = np.random.default_rng(3).uniform(-2.0, 2.0, size=shape)
    bad = [(1, 2, 0, 3), (4, 0, 5, 7)]
    for b, v in zip(bad, (np.nan, -np.inf)):
        idx = list(b)
        idx[axis] = 0
        sig[tuple(idx)] = v
    announce(f"spline non-finite shifts {dt} axis={axis}")
    out = torch.empty_like(fin)
    vp.spline_advect(axis, fin, out, to_dev(sig))
    got = to_host(out)
    mask = np.ones(dims, bool)
    for b in bad:
        sl = list(b)
        sl[axis] = slice(None)
        assert np.all(np.isnan(got[tuple(sl)])), b
        mask[tuple(sl)] = False
    assert np.all(np.isfinite(got[mask]))
    ref = spline.sweep(fr, axis, np.where(np.isfinite(sig), sig, 0.0))
    tol = 1e-12 if dt == "f64" else 2e-6
    assert rel_max(got[mask], ref[mask]) < tol


# --------------------------------------------------------- field kernels ---

@pytest.mark.parametrize("degree", [2, 1, 3, 5, -1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n4_cells", [5, 8])
def test_density_and_moments_parity(degree, dt, n4_cells):
    # 5 cells along v2: weights from tables; 8 cells: the weight pattern
    # repeats within a few rounds of 64 values (register weights)
    vp = require_gpu()
    m = 1 if degree < 0 else degree + 1
    dims = (3 * m, 2 * m, 7 * m, n4_cells * m)
    lo = (0.0, 0.0, -6.0, -9.0)
    ln = (4 * math.pi, 10 * math.pi, 12.0, 18.0)
    f = random_field(dims, seed=5, positive=False)
    fin = to_dev(f, dt)
    fr = to_host(fin)
    od = None if degree < 0 else degree
    announce(f"vp_density degree={degree} {dt}")
    rho = torch.empty(dims[0], dims[1], dtype=torch.float64, device="cuda")
    vp.vp_density(degree, fin, ln[2], ln[3], rho)
    ref = field.density(fr, od, ln[2], ln[3])
    assert rel_l2(to_host(rho), ref) < 1e-13
    announce(f"vp_moments degree={degree} {dt}")
    out4 = torch.empty(4, dtype=torch.float64, device="cuda")
    vp.vp_moments(degree, fin, lo, ln, out4)
    got = to_host(out4)
    exp = np.array(field.moments(fr, od, lo, ln))
    np.testing.assert_allclose(got, exp, rtol=1e-12, atol=0)


@pytest.mark.parametrize("degree,n1,n2", [(2, 24, 18), (1, 10, 16), (-1, 32, 20), (-1, 9, 7),
                                          (3, 8, 12), (5, 18, 12), (0, 7, 5), (3, 128, 128),
                                          (2, 96, 96)])
def test_poisson_parity(degree, n1, n2):
    vp = require_gpu()
    L1, L2 = 4 * math.pi, 3.0
    rho = 1.0 + 0.3 * random_field((n1, n2), seed=n1 + n2)
    announce(f"vp_poisson degree={degree} {n1}x{n2}")
    e1 = torch.empty(n1, n2, dtype=torch.float64, device="cuda")
    e2 = torch.empty_like(e1)
    W = torch.empty(1, dtype=torch.float64, device="cuda")
    vp.vp_poisson(degree, L1, L2, to_dev(rho), e1, e2, W)
    r1, r2, rW = field.poisson(rho, None if degree < 0 else degree, L1, L2)
    scale = max(np.max(np.abs(r1)), np.max(np.abs(r2)))
    assert np.max(np.abs(to_host(e1) - r1)) <= 1e-12 * scale
    assert np.max(np.abs(to_host(e2) - r2)) <= 1e-12 * scale
    assert abs(to_host(W)[0] - rW) <= 1e-12 * rW


@pytest.mark.parametrize("kind,form", [(0, None), (1, "sum"), (2, "product")])
@pytest.mark.parametrize("degree", [2, -1])
def test_init_parity(kind, form, degree):
    vp = require_gpu()
    m = 1 if degree < 0 else degree + 1
    dims = (4 * m, 3 * m, 5 * m, 6 * m)
    if kind == 0:
        lo, ln, eps, k, v0 = (0, 0, -6, -6), (4 * math.pi, 4 * math.pi, 12, 12), 0.5, 0.5, 0.0
    else:
        lo, ln, eps, k, v0 = (0, 0, -9, -9), (10 * math.pi, 10 * math.pi, 18, 18), 1e-3, 0.2, 2.4
    announce(f"vp_init kind={kind} degree={degree}")
    f = torch.empty(dims, dtype=torch.float64, device="cuda")
    vp.vp_init(kind, eps, k, v0, degree, f, lo, ln)
    ref = field.initial_condition("landau" if kind == 0 else "two_stream", dims, lo, ln,
                                  None if degree < 0 else degree, eps, k, v0,
                                  form=form or "sum")
    assert rel_l2(to_host(f), ref) < 1e-14


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("dims", [(7, 5, 9, 13), (4, 6, 96, 256), (3, 130, 2, 128)])
def test_copy_patterns_are_exact_copies(dt, dims):
    # the bandwidth references of the bench copy every element (ragged
    # tiles, segments and flat tails included)
    vp = require_gpu()
    f = to_dev(random_field(dims, seed=3), dt)
    for pid in (vp.PATTERN_CONTIGUOUS, vp.PATTERN_TILES, vp.PATTERN_SEGMENTS, vp.PATTERN_LINES):
        for axis in ((0,) if pid == vp.PATTERN_CONTIGUOUS else (0, 1, 2)):
            announce(f"vp_copy_pattern {pid} axis {axis} {dt} {dims}")
            g = torch.full_like(f, float("nan"))
            vp.vp_copy_pattern(pid, f, g, axis)
            torch.cuda.synchronize()
            assert torch.equal(f, g), (pid, axis)
