"""Adjoint parity: the transposed kernels, shift derivatives, field
transposes, the Strang-step adjoint and whole-run gradients against the FP64
oracle and against central finite differences of the device forward map."""

import math

import numpy as np
import pytest

from gpu_common import announce, assert_close, rel_l2, require_gpu, to_dev, to_host, torch
from oracle import adjoint, field, strang
from vp_inputs import random_field, random_shifts, workload

pytestmark = pytest.mark.gpu


def _line_shifts(dims, axis, seed, n_cells, scale=2.5):
    shape = list(dims)
    shape[axis] = 1
    return random_shifts(int(np.prod(shape)), seed, scale=scale, n_cells=n_cells).reshape(shape)


@pytest.mark.parametrize("method", ["sldg", "spline"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_adjoint_sweeps_and_shift_derivatives(method, dt):
    vp = require_gpu()
    degree = 2
    m = degree + 1 if method == "sldg" else 1
    dims = (3 * m, 4 * m, 5 * m, 6 * m) if method == "sldg" else (9, 12, 10, 21)
    u = random_field(dims, seed=1)
    lam = random_field(dims, seed=2)
    ud, ld = to_dev(u, dt), to_dev(lam, dt)
    ur, lr = to_host(ud), to_host(ld)
    for axis in range(4):
        announce(f"{method} adjoint/dshift {dt} axis={axis}")
        sig = _line_shifts(dims, axis, seed=axis + 3, n_cells=dims[axis] // m)
        out = torch.empty_like(ld)
        g = torch.empty(int(np.prod(dims)) // dims[axis], dtype=torch.float64, device="cuda")
        if method == "sldg":
            vp.sldg_advect_adjoint(axis, degree, ld, out, to_dev(sig))
            vp.sldg_advect_dshift(axis, degree, ud, ld, to_dev(sig), g)
            ref = adjoint.sldg_sweep_adjoint(lr, axis, sig, degree)
            gref = adjoint.sldg_sweep_dshift(ur, lr, axis, sig, degree)
        else:
            vp.spline_advect_adjoint(axis, ld, out, to_dev(sig))
            vp.spline_advect_dshift(axis, ud, ld, to_dev(sig), g)
            ref = adjoint.spline_sweep_adjoint(lr, axis, sig)
            gref = adjoint.spline_sweep_dshift(ur, lr, axis, sig)
        assert_close(to_host(out), ref, dt, f"adjoint axis {axis}")
        assert_close(to_host(g), gref.reshape(-1), dt, f"dshift axis {axis}")


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n", [100, 150, 192, 257])
def test_spline_shift_derivative_long_contiguous_rows(dt, n):
    # rows of the contiguous axis longer than one and two wavefronts, a
    # ragged last tile; the shift derivative by rows (100, 192 and 257
    # points) and by segments (150)
    vp = require_gpu()
    dims = (3, 4, 5, n)
    u = random_field(dims, seed=11)
    lam = random_field(dims, seed=12)
    ud, ld = to_dev(u, dt), to_dev(lam, dt)
    sig = _line_shifts(dims, 3, seed=13, n_cells=n, scale=4.0)
    g = torch.empty(int(np.prod(dims[:3])), dtype=torch.float64, device="cuda")
    announce(f"spline dshift {dt} n={n}")
    vp.spline_advect_dshift(3, ud, ld, to_dev(sig), g)
    gref = adjoint.spline_sweep_dshift(to_host(ud), to_host(ld), 3, sig)
    assert_close(to_host(g), gref.reshape(-1), dt, "dshift along the contiguous axis")


@pytest.mark.parametrize("degree", [2, -1])
def test_density_and_poisson_adjoint(degree):
    vp = require_gpu()
    m = 1 if degree < 0 else degree + 1
    dims = (4 * m, 3 * m, 5 * m, 6 * m)
    od = None if degree < 0 else degree
    announce(f"density/poisson adjoint degree={degree}")
    rb = random_field(dims[:2], seed=4)
    lam0 = random_field(dims, seed=5)
    lam = to_dev(lam0)
    vp.vp_density_adjoint(degree, to_dev(rb), 12.0, 18.0, lam, accumulate=True)
    ref = lam0 + adjoint.density_adjoint(rb, dims, od, 12.0, 18.0)
    assert_close(to_host(lam), ref, "f64", "density adjoint")
    g1 = random_field(dims[:2], seed=6)
    g2 = random_field(dims[:2], seed=7)
    out = torch.empty(dims[:2], dtype=torch.float64, device="cuda")
    vp.vp_poisson_adjoint(degree, 4 * math.pi, 3.0, to_dev(g1), to_dev(g2), out)
    assert_close(to_host(out), adjoint.poisson_adjoint(g1, g2, od, 4 * math.pi, 3.0),
                 "f64", "poisson adjoint")


def _small(method):
    # 16 x 16 velocity nodes: the x2 sweep before the field solve also forms
    # the density (256 columns per SLDG workgroup, 64-line spline tiles)
    degree = 1 if method == "sldg" else None
    dims = (8, 8, 16, 16)
    return strang.Grid(dims, (0.0, 0.0, -6.0, -6.0), (4 * math.pi, 4 * math.pi, 12.0, 12.0),
                       degree)


@pytest.mark.parametrize("method", ["sldg", "spline"])
def test_energy_gradient_and_step_adjoint(method):
    vp = require_gpu()
    g = _small(method)
    deg = -1 if g.degree is None else g.degree
    f = field.initial_condition("landau", g.dims, g.lo, g.length, g.degree, 0.5, 0.5)
    lam0 = random_field(g.dims, seed=8)
    st = vp.VPState(vp.METHOD_SLDG if method == "sldg" else vp.METHOD_SPLINE, max(deg, 0),
                    torch.float64, g.dims, g.lo, g.length)
    announce(f"energy gradient {method}")
    lam = torch.empty(g.dims, dtype=torch.float64, device="cuda")
    W = torch.empty(1, dtype=torch.float64, device="cuda")
    st.energy_gradient(to_dev(f), lam, W)
    Wr, gref = adjoint.energy_gradient(f, g)
    assert abs(to_host(W)[0] - Wr) <= 1e-12 * Wr
    assert_close(to_host(lam), gref, "f64", "energy gradient")
    announce(f"step adjoint {method}")
    lam = to_dev(lam0)
    work = st.adjoint_workspace()
    st.adjoint_step(to_dev(f), lam, 0.1, work)
    assert_close(to_host(lam), adjoint.step_adjoint(f, lam0, g, 0.1), "f64", "step adjoint")
    st.close()


@pytest.mark.parametrize("method", ["sldg", "spline"])
def test_whole_run_gradient_vs_oracle_and_differences(method):
    vp = require_gpu()
    from paper_1803_02143_amd.autograd import final_electric_energy
    g = _small(method)
    deg = -1 if g.degree is None else g.degree
    tau, nsteps = 0.1, 5
    st = vp.VPState(vp.METHOD_SLDG if method == "sldg" else vp.METHOD_SPLINE, max(deg, 0),
                    torch.float64, g.dims, g.lo, g.length)

    def f0_dev(eps):
        f = torch.empty(g.dims, dtype=torch.float64, device="cuda")
        vp.vp_init(vp.IC_LANDAU, eps, 0.5, 0.0, deg, f, g.lo, g.length)
        return f

    announce(f"whole-run gradient {method}")
    f0 = f0_dev(0.5).requires_grad_(True)
    J = final_electric_energy(f0, st, nsteps, tau, every=2)
    J.backward()
    grad = f0.grad.detach()
    # the lean schedule (states recomputed from the checkpoint) gives the
    # same gradient bit for bit
    f0b = f0_dev(0.5).requires_grad_(True)
    final_electric_energy(f0b, st, nsteps, tau, every=3, store_segment=False).backward()
    assert torch.equal(f0b.grad, grad)
    # against the oracle gradient from its own initial condition
    fo = field.initial_condition("landau", g.dims, g.lo, g.length, g.degree, 0.5, 0.5)
    Jr, gr = adjoint.final_energy_gradient(fo, g, tau, nsteps)
    assert abs(J.item() - Jr) <= 1e-11 * Jr
    assert rel_l2(to_host(grad), gr) < 1e-10
    # d J / d eps against central differences of the device forward map
    df0 = f0_dev(1.0) - f0_dev(0.0)
    g_eps = float((grad * df0).sum())
    h = 1e-4

    def J_of(eps):
        f = f0_dev(eps)
        tmp = torch.empty_like(f)
        W = torch.empty(nsteps + 1, dtype=torch.float64, device="cuda")
        st.step(f, tmp, nsteps, tau, W)
        return float(W[-1])

    fd = (J_of(0.5 + h) - J_of(0.5 - h)) / (2 * h)
    assert abs(g_eps - fd) <= 1e-6 * abs(fd), (g_eps, fd)
    st.close()


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        return json.load(fh)


def test_differentiated_landau_full_size():
    # 32^4 cells, degree 2, 40 steps, checkpoints every 10.  FP64: J = W(f^40)
    # and dJ/d eps against the stored oracle values (the oracle's reverse
    # sweep over the same steps, tests/golden/make_landau96_golden.py), the
    # gradient's entries at fixed dofs and its sums over all axes but one,
    # and dJ/d eps against FP64 central differences (h = 1e-4) of the device
    # run.  FP32 forward and adjoint: the same quantities, with the error of
    # the gradient bounded by a small multiple of what FP32 storage does to
    # J itself.
    vp = require_gpu()
    from paper_1803_02143_amd.autograd import final_electric_energy
    w = workload("landau_32_adjoint")
    gold = _golden("landau96_adjoint_gradient.json")
    assert tuple(gold["dims"]) == w.dofs and gold["steps"] == w.steps and gold["tau"] == w.dt
    res = {}
    for dt, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        announce(f"differentiated Landau 96^4 {dt}: forward + adjoint")
        st = vp.VPState(vp.METHOD_SLDG, w.degree, tdt, w.dofs, w.lo, w.length)

        def f0_dev(eps):
            f = torch.empty(w.dofs, dtype=tdt, device="cuda")
            vp.vp_init(vp.IC_LANDAU, eps, w.k, 0.0, w.degree, f, w.lo, w.length)
            return f

        f0 = f0_dev(w.eps).requires_grad_(True)
        J = final_electric_energy(f0, st, w.steps, w.dt, every=10)
        J.backward()
        grad = f0.grad.double()
        df0 = (f0_dev(1.0).double() - f0_dev(0.0).double())
        res[dt] = {
            "J": J.item(), "dJ_deps": float((grad * df0).sum()),
            "probes": [float(grad[tuple(p)]) for p, _ in gold["grad_probes"]],
            "marginals": [grad.sum(dim=tuple(a for a in range(4) if a != d)).cpu().numpy()
                          for d in range(4)],
            "l2": float(grad.norm()),
        }
        del grad, df0
        if dt == "f64":
            h = 1e-4

            def J_of(eps):
                f = f0_dev(eps)
                tmp = torch.empty_like(f)
                W = torch.empty(w.steps + 1, dtype=torch.float64, device="cuda")
                st.step(f, tmp, w.steps, w.dt, W)
                return float(W[-1])

            announce("differentiated Landau 96^4 f64: central differences")
            fd = (J_of(w.eps + h) - J_of(w.eps - h)) / (2 * h)
            res["fd"] = fd
            assert abs(res["f64"]["dJ_deps"] - fd) <= 1e-6 * abs(fd), (res["f64"]["dJ_deps"], fd)
        st.close()
        del f0
        torch.cuda.empty_cache()
    # FP64 against the oracle
    r = res["f64"]
    assert abs(r["J"] - gold["J"]) <= 1e-11 * gold["J"], (r["J"], gold["J"])
    assert abs(r["dJ_deps"] - gold["dJ_deps"]) <= 1e-10 * abs(gold["dJ_deps"]), \
        (r["dJ_deps"], gold["dJ_deps"])
    assert abs(r["l2"] - gold["grad_l2"]) <= 1e-10 * gold["grad_l2"]
    scale = max(abs(v) for _, v in gold["grad_probes"])
    for got, (p, ref) in zip(r["probes"], gold["grad_probes"]):
        assert abs(got - ref) <= 1e-10 * scale, (p, got, ref)
    for d in range(4):
        ref = np.array(gold["grad_marginals"][d])
        assert rel_l2(r["marginals"][d], ref) <= 1e-10, d
    # FP32: errors against the oracle, recorded in the output
    q = res["f32"]
    err_J = abs(q["J"] - gold["J"]) / gold["J"]
    err_g = abs(q["dJ_deps"] - gold["dJ_deps"]) / abs(gold["dJ_deps"])
    err_fd = abs(q["dJ_deps"] - res["fd"]) / abs(res["fd"])
    err_m = max(rel_l2(q["marginals"][d], np.array(gold["grad_marginals"][d])) for d in range(4))
    announce(f"FP32 differentiated Landau: rel err J {err_J:.3e}, dJ/deps {err_g:.3e} "
             f"(vs FP64 central differences {err_fd:.3e}), gradient marginals {err_m:.3e}")
    # (measured on MI355X: 1.3e-6 for J, 1.2e-6 for dJ/d eps against the
    # oracle and against FP64 central differences, 1.3e-6 for the marginals)
    assert err_J <= 1e-5, err_J
    assert err_g <= max(3.0 * err_J, 3e-6), (err_g, err_J)
    assert err_fd <= max(3.0 * err_J, 3e-6), (err_fd, err_J)
    assert err_m <= 1e-5, err_m


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n", [80, 96, 150])
@pytest.mark.parametrize("axis", [1, 3])
def test_spline_adjoint_segment_lengths(dt, n, axis):
    # lines whose per-thread segments span the three register bounds of the
    # transposed sweep and the shift derivative (16, 24 and 48 points),
    # along a strided axis and the contiguous one, ragged last tiles
    vp = require_gpu()
    dims = (3, n, 5, 7) if axis == 1 else (3, 4, 5, n)
    u = random_field(dims, seed=21)
    lam = random_field(dims, seed=22)
    ud, ld = to_dev(u, dt), to_dev(lam, dt)
    ur, lr = to_host(ud), to_host(ld)
    sig = _line_shifts(dims, axis, seed=23, n_cells=n, scale=4.0)
    out = torch.empty_like(ld)
    g = torch.empty(int(np.prod(dims)) // n, dtype=torch.float64, device="cuda")
    announce(f"spline adjoint/dshift {dt} axis={axis} n={n}")
    vp.spline_advect_adjoint(axis, ld, out, to_dev(sig))
    vp.spline_advect_dshift(axis, ud, ld, to_dev(sig), g)
    assert_close(to_host(out), adjoint.spline_sweep_adjoint(lr, axis, sig), dt, "adjoint")
    assert_close(to_host(g), adjoint.spline_sweep_dshift(ur, lr, axis, sig).reshape(-1), dt, "dshift")
