"""Pins of oracle.strang: the whole split step against physics that fixes
signs and normalisations (linear Landau damping), and conservation laws."""

import math

import numpy as np
import pytest
from scipy.special import erf, wofz

from oracle import field, strang
from vp_inputs import workload


def _landau_root(k):
    # plasma dispersion relation of the Maxwellian: 1 + (1 + z Z(z))/k^2 = 0,
    # z = omega/(sqrt(2) k), Z(z) = i sqrt(pi) w(z) (Faddeeva), Newton from 1.4-0.15i
    def D(w):
        z = w / (math.sqrt(2.0) * k)
        return 1.0 + (1.0 + z * 1j * math.sqrt(math.pi) * wofz(z)) / k ** 2
    w = 1.4 - 0.15j
    for _ in range(60):
        h = 1e-7
        w = w - D(w) / ((D(w + h) - D(w - h)) / (2 * h))
    return w


def test_dispersion_root_value():
    w = _landau_root(0.5)
    assert abs(w.real - 1.4156618886) < 1e-8 and abs(w.imag + 0.1533594669) < 1e-8


@pytest.mark.slow
def test_linear_landau_damping_rate():
    # 1D-1V Landau damping embedded in the 4D code: perturbation in x1 only,
    # one cell in x2 and v2, Maxwellian in v1 renormalised to discrete mass 1.
    # The electric energy decays like exp(2 gamma t) with gamma the imaginary
    # part of the dispersion root; a wrong sign of E or of a shift fails this.
    k = 0.5
    deg = 2
    dims = (24, 3, 96, 3)
    lo = (0.0, 0.0, -6.0, -6.0)
    ln = (4 * math.pi, 4 * math.pi, 12.0, 12.0)
    g = strang.Grid(dims, lo, ln, deg)
    x1 = g.nodes(0)
    v1 = g.nodes(2)
    fv = np.exp(-0.5 * v1 ** 2)
    fv /= np.sum(fv * field.weights_1d(ln[2], dims[2], deg))
    f = ((1 + 0.01 * np.cos(k * x1))[:, None, None, None] * fv[None, None, :, None]
         * np.ones((1, dims[1], 1, dims[3])) / ln[3])
    nsteps = 180
    _, W = strang.run(f, g, 0.1, nsteps)
    t = 0.1 * np.arange(nsteps + 1)
    pk = [i for i in range(1, nsteps) if W[i] > W[i - 1] and W[i] >= W[i + 1] and t[i] > 1.5]
    assert len(pk) >= 6
    slope = np.polyfit(t[pk], np.log(W[pk]), 1)[0]
    gamma = _landau_root(k).imag
    assert abs(slope - 2 * gamma) < 0.03 * abs(2 * gamma), (slope, 2 * gamma)


@pytest.mark.parametrize("method", ["sldg", "spline"])
def test_mass_and_energy_over_landau_steps(method):
    w = workload("landau_8")
    degree = w.degree if method == "sldg" else None
    dims = w.dofs
    g = strang.Grid(dims, w.lo, w.length, degree)
    f0 = field.initial_condition("landau", dims, w.lo, w.length, degree, w.eps, w.k)
    f, W, mom = strang.run(f0, g, w.dt, 6, with_moments=True)
    mass = mom[:, 0]
    np.testing.assert_allclose(mass, mass[0], rtol=2e-14)
    # total energy = kinetic + electric is conserved up to the splitting error
    # (the paper reports errors of order 1e-3 for these runs, Sec. 4)
    etot = mom[:, 3] + W
    assert np.max(np.abs(etot - etot[0])) < 2e-3 * etot[0]
    # the strongly perturbed field first loses energy (nonlinear Landau damping)
    assert np.all(np.diff(W) < 0) and W[-1] < 0.7 * W[0]


def test_step_is_deterministic_and_restartable():
    w = workload("landau_8")
    g = strang.Grid(w.dofs, w.lo, w.length, w.degree)
    f0 = field.initial_condition("landau", w.dofs, w.lo, w.length, w.degree, w.eps, w.k)
    a, _ = strang.run(f0, g, w.dt, 2)
    b, _ = strang.run(strang.run(f0, g, w.dt, 1)[0], g, w.dt, 1)
    assert np.array_equal(a, b)


def test_merged_run_with_every_one_is_the_plain_run():
    w = workload("landau_8")
    g = strang.Grid(w.dofs, w.lo, w.length, w.degree)
    f0 = field.initial_condition("landau", w.dofs, w.lo, w.length, w.degree, w.eps, w.k)
    a, Wa = strang.run(f0, g, w.dt, 3)
    b, Wb = strang.run_merged(f0, g, w.dt, 3, 1)
    assert np.array_equal(a, b) and np.array_equal(Wa, Wb)


@pytest.mark.parametrize("degree", [0, None])
def test_merged_run_equals_plain_run_for_whole_cell_x_shifts(degree):
    # tau = 4 h_x and velocity nodes at half-integers: every x half-step
    # shifts by an odd whole number of cells, so x(tau/2) x(tau/2) = x(tau)
    # exactly (permutations) and merging changes nothing but round-off;
    # a wrong merged shift, a missing closing half-step or a field taken at
    # the wrong state would not
    dims = (8, 8, 12, 12)
    lo = (0.0, 0.0, -6.0, -6.0)
    ln = (8.0, 8.0, 12.0, 12.0)
    g = strang.Grid(dims, lo, ln, degree)
    tau = 4.0 * g.h(0)
    assert np.allclose(strang.x_shift(g, 0, 0.5 * tau) % 1.0, 0.0)
    f0 = field.initial_condition("landau", dims, lo, ln, degree, 0.3, 2 * math.pi / 8.0)
    a, Wa = strang.run(f0, g, tau, 4)
    b, Wb = strang.run_merged(f0, g, tau, 4, 4)
    tol = 0.0 if degree == 0 else 1e-13
    assert np.max(np.abs(a - b)) <= tol * np.max(np.abs(a))
    assert abs(Wa[-1] - Wb[-1]) <= max(tol, 1e-15) * Wa[-1] * 10
    assert len(Wb) == 2 and Wb[0] == Wa[0]


def test_merged_run_converges_to_the_plain_run():
    # the two schemes differ only by how often the x flows are projected
    # (x(tau/2) twice against x(tau) once): with the perturbation along x1
    # only, the difference after a fixed time shrinks as x1 and v1 are refined
    diffs = []
    for nc in (8, 16):
        dims = (3 * nc, 3, 3 * nc, 3)
        lo = (0.0, 0.0, -6.0, -6.0)
        ln = (4 * math.pi, 4 * math.pi, 12.0, 12.0)
        g = strang.Grid(dims, lo, ln, 2)
        x1, v1, v2 = g.nodes(0), g.nodes(2), g.nodes(3)
        f0 = ((1 + 0.2 * np.cos(0.5 * x1))[:, None, None, None]
              * np.exp(-0.5 * v1 ** 2)[None, None, :, None]
              * np.exp(-0.5 * v2 ** 2)[None, None, None, :]
              * np.ones((1, dims[1], 1, 1)) / (2 * math.pi))
        a, _ = strang.run(f0, g, 0.2, 4)
        b, _ = strang.run_merged(f0, g, 0.2, 4, 4)
        diffs.append(np.max(np.abs(a - b)) / np.max(np.abs(a)))
    assert 0 < diffs[1] < diffs[0] / 2.5 and diffs[0] < 1e-3, diffs


def _golden():
    import json
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")
    with open(p) as fh:
        return json.load(fh)


def test_landau_workload_matches_paper():
    g = _golden()["landau_4d"]
    w = workload("landau_8")
    assert (w.eps, w.k, w.dt) == (g["eps"], g["k"], g["tau"])
    assert w.lo == (0.0, 0.0, g["v_domain"][0], g["v_domain"][0])
    np.testing.assert_allclose(w.length, (4 * math.pi, 4 * math.pi,
                                          g["v_domain"][1] - g["v_domain"][0],
                                          g["v_domain"][1] - g["v_domain"][0]))


def test_two_stream_product_form_matches_paper():
    g = _golden()["two_stream_4d"]
    w = workload("two_stream_64")
    assert (w.eps, w.k, w.v0) == (g["eps"], g["k"], g["v0"])
    # product perturbation of Eq. (7) at a point where cos k x1 cos k x2 = 1/2
    dims = (2, 2, 2, 2)
    lo = (0.0, 0.0, -6.0, -6.0)
    ln = (10 * math.pi, 10 * math.pi, 12.0, 12.0)
    f = field.initial_condition("two_stream", dims, lo, ln, None, g["eps"], g["k"],
                                g["v0"], form="product")
    x = 10 * math.pi / 4          # first node of each x axis
    v = -6.0 + 12.0 / 4
    gv = math.exp(-0.5 * (v - 2.4) ** 2) + math.exp(-0.5 * (v + 2.4) ** 2)
    ref = (1 + 1e-3 * math.cos(0.2 * x) ** 2) * gv * gv / (8 * math.pi)
    assert abs(f[0, 0, 0, 0] - ref) < 1e-16


def test_two_stream_sum_form_point_value_and_mass():
    # The two-stream workloads use the sum perturbation 1 + eps (cos k x1 +
    # cos k x2) on v in [-9, 9) (Sec. 5, Eq. (7) with the sum in place of the
    # product).  Point value: x nodes at (i + 1/2) L / 3, where k x = pi/3
    # for i = 0 (cos = 1/2, so the sum form gives 1 + eps and the product
    # form 1 + eps/4).
    w = workload("two_stream_64")
    assert w.form == "sum" and w.lo[2] == -9.0 and w.length[2] == 18.0
    dims = (3, 3, 2, 2)
    f = field.initial_condition("two_stream", dims, w.lo, w.length, None, w.eps, w.k, w.v0)
    v = -9.0 + 18.0 / 4
    gv = math.exp(-0.5 * (v - 2.4) ** 2) + math.exp(-0.5 * (v + 2.4) ** 2)
    ref = (1.0 + 1e-3 * (0.5 + 0.5)) * gv * gv / (8.0 * math.pi)
    assert abs(f[0, 0, 0, 0] - ref) < 1e-16
    # i = 1: k x = pi, cos = -1 for both axes
    ref11 = (1.0 - 2e-3) * gv * gv / (8.0 * math.pi)
    assert abs(f[1, 1, 1, 1] - ref11) < 1e-16
    # Mass: the x integral of the perturbation vanishes over whole periods
    # (k L = 2 pi), each velocity factor integrates to
    # sqrt(pi/2) [erf((9 - v0)/sqrt 2) + erf((9 + v0)/sqrt 2)] per bump, so
    # mass = L1 L2 / (8 pi) G^2 with G = 2 sqrt(pi/2)[...].  The midpoint
    # rule of the spline grid is spectrally accurate for the bumps.
    n = 48
    f = field.initial_condition("two_stream", (8, 8, n, n), w.lo, w.length, None,
                                w.eps, w.k, w.v0)
    mass, l1, _, _ = field.moments(f, None, w.lo, w.length)
    s2 = math.sqrt(2.0)
    G = 2.0 * math.sqrt(math.pi / 2.0) * (erf((9.0 - 2.4) / s2) + erf((9.0 + 2.4) / s2))
    exact = w.length[0] * w.length[1] / (8.0 * math.pi) * G * G
    assert abs(mass - exact) < 1e-10 * exact
    assert abs(l1 - mass) < 1e-14 * mass
