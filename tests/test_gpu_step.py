"""Strang step parity: vp_strang_step against the oracle step by step and over
whole runs, plus full-size checks at the 96^4 workload that the bench times."""

import math

import numpy as np
import pytest

from gpu_common import (announce, assert_close, rel_l2, require_gpu, to_dev,
                        to_host, torch)
from oracle import field, sldg, spline, strang
from vp_inputs import random_field, workload

pytestmark = pytest.mark.gpu


def _grid(w, method):
    degree = w.degree if method == "sldg" else None
    return strang.Grid(w.dofs, w.lo, w.length, degree)


@pytest.mark.parametrize("method", ["sldg", "spline"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_step_by_step_parity(method, dt):
    vp = require_gpu()
    w = workload("landau_8")
    g = _grid(w, method)
    f = field.initial_condition("landau", w.dofs, w.lo, w.length, g.degree, w.eps, w.k)
    st = vp.VPState(vp.METHOD_SLDG if method == "sldg" else vp.METHOD_SPLINE,
                    w.degree, torch.float64 if dt == "f64" else torch.float32,
                    w.dofs, w.lo, w.length)
    for m in range(3):
        announce(f"strang step {method} {dt} step {m}")
        fd = to_dev(f, dt)
        tmp = torch.empty_like(fd)
        st.step(fd, tmp, 1, w.dt)
        f_in = to_host(to_dev(f, dt))          # what the device started from
        ref = strang.step(f_in, g, w.dt)
        assert_close(to_host(fd), ref, dt, f"step {m}")
        f = ref
    st.close()


@pytest.mark.parametrize("method", ["sldg", "spline"])
def test_whole_run_energy_and_moments(method):
    vp = require_gpu()
    w = workload("landau_8")
    g = _grid(w, method)
    deg = w.degree if method == "sldg" else -1
    f0 = field.initial_condition("landau", w.dofs, w.lo, w.length, g.degree, w.eps, w.k)
    _, W_ref, mom_ref = strang.run(f0, g, w.dt, w.steps, with_moments=True)
    announce(f"whole run {method} {w.steps} steps")
    st = vp.VPState(vp.METHOD_SLDG if method == "sldg" else vp.METHOD_SPLINE,
                    w.degree, torch.float64, w.dofs, w.lo, w.length)
    fd = torch.empty(w.dofs, dtype=torch.float64, device="cuda")
    vp.vp_init(vp.IC_LANDAU, w.eps, w.k, 0.0, deg, fd, w.lo, w.length)
    tmp = torch.empty_like(fd)
    W = torch.empty(w.steps + 1, dtype=torch.float64, device="cuda")
    mom = torch.empty(4 * (w.steps + 1), dtype=torch.float64, device="cuda")
    st.step(fd, tmp, w.steps, w.dt, W, mom)
    Wg = to_host(W)
    mg = to_host(mom).reshape(-1, 4)
    np.testing.assert_allclose(Wg, W_ref, rtol=1e-10, atol=0)
    np.testing.assert_allclose(mg, mom_ref, rtol=1e-10, atol=0)
    # mass to round-off along the whole run
    assert np.max(np.abs(mg[:, 0] - mg[0, 0])) <= 1e-13 * mg[0, 0]
    st.close()


def test_chunked_run_equals_single_run_bitwise():
    vp = require_gpu()
    w = workload("landau_8")
    announce("chunked vs single run")
    st = vp.VPState(vp.METHOD_SLDG, w.degree, torch.float64, w.dofs, w.lo, w.length)
    a = torch.empty(w.dofs, dtype=torch.float64, device="cuda")
    vp.vp_init(vp.IC_LANDAU, w.eps, w.k, 0.0, w.degree, a, w.lo, w.length)
    b = a.clone()
    tmp = torch.empty_like(a)
    st.step(a, tmp, 4, w.dt)
    st.step(b, tmp, 2, w.dt)
    st.step(b, tmp, 2, w.dt)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    st.close()


# ----------------------------------------------- full size (96^4, bench) ---

def _sample_lines(axis, dims, count, seed):
    rng = np.random.default_rng(seed)
    idx = []
    for _ in range(count):
        i = [int(rng.integers(0, d)) for d in dims]
        i[axis] = slice(None)
        idx.append(tuple(i))
    return idx


@pytest.mark.parametrize("method", ["sldg", "spline"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_full_size_sweeps_sampled(method, dt):
    # the 96^4 workload, shifts with the step's broadcast patterns; sampled
    # lines are recomputed by the oracle one by one
    vp = require_gpu()
    w = workload("landau_32")
    dims = w.dofs
    announce(f"full size {method} {dt} {dims}: host input")
    f = random_field(dims, seed=32, positive=True)
    fin = to_dev(f, dt)
    fr = f.astype(np.float32).astype(np.float64) if dt == "f32" else f
    rng = np.random.default_rng(33)
    out = torch.empty_like(fin)
    for axis in range(4):
        if axis < 2:
            sig = rng.uniform(-1.6, 1.6, size=dims[axis + 2])
            st = [0, 0, 0, 0]
            st[axis + 2] = 1
        else:
            sig = rng.uniform(-0.9, 0.9, size=dims[0] * dims[1])
            st = [dims[1], 1, 0, 0]
        announce(f"full size {method} {dt} axis={axis}")
        if method == "sldg":
            vp.sldg_advect(axis, w.degree, fin, out, to_dev(sig), shift_stride=st)
        else:
            vp.spline_advect(axis, fin, out, to_dev(sig), shift_stride=st)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        lines = _sample_lines(axis, dims, 64, seed=axis)
        for ix in lines:
            off = sum(ix[d] * st[d] for d in range(4) if d != axis)
            u = fr[ix][None, :]
            if method == "sldg":
                ref = sldg.shift_lines(u, sig[off], w.degree)[0]
            else:
                ref = spline.shift_lines(u, sig[off])[0]
            assert_close(got[ix], ref, dt, f"axis {axis} line {ix}")
        # mass per swept line is conserved everywhere (a property at any size)
        if method == "sldg":
            _, wq = np.polynomial.legendre.leggauss(w.degree + 1)
            wl = np.tile(wq, dims[axis] // (w.degree + 1))
        else:
            wl = np.ones(dims[axis])
        shape = [1, 1, 1, 1]
        shape[axis] = dims[axis]
        m0 = np.tensordot(fr, wl, axes=([axis], [0]))
        m1 = np.tensordot(got, wl, axes=([axis], [0]))
        tol = 1e-12 if dt == "f64" else 1e-5
        assert np.max(np.abs(m1 - m0)) <= tol * np.max(np.abs(m0))


_FULL_SIZE_REF = {}


def _full_size_reference(method):
    """f0 and the oracle's FP64 Strang step of the 96^4 Landau workload."""
    if method not in _FULL_SIZE_REF:
        w = workload("landau_32")
        g = _grid(w, method)
        announce(f"full size step {method}: oracle step")
        f0 = field.initial_condition("landau", w.dofs, w.lo, w.length, g.degree, w.eps, w.k)
        _FULL_SIZE_REF.clear()           # one method's arrays at a time
        _FULL_SIZE_REF[method] = (f0, strang.step(f0, g, w.dt))
    return _FULL_SIZE_REF[method]


@pytest.mark.parametrize("method,dt", [("sldg", "f64"), ("sldg", "f32"),
                                       ("spline", "f64"), ("spline", "f32")])
def test_full_size_step_parity(method, dt):
    # one whole Strang step of the 96^4 workload (32^4 cells of degree 2, or
    # the spline on 96^4 points) against the oracle, every dof compared
    vp = require_gpu()
    w = workload("landau_32")
    f0, ref = _full_size_reference(method)
    tdt = torch.float64 if dt == "f64" else torch.float32
    st = vp.VPState(vp.METHOD_SLDG if method == "sldg" else vp.METHOD_SPLINE, w.degree,
                    tdt, w.dofs, w.lo, w.length)
    fd = to_dev(f0, dt)
    tmp = torch.empty_like(fd)
    W = torch.empty(2, dtype=torch.float64, device="cuda")
    mom = torch.empty(8, dtype=torch.float64, device="cuda")
    announce(f"full size step {method} {dt}: device step")
    st.step(fd, tmp, 1, w.dt, W, mom)
    got = to_host(fd)
    del fd, tmp
    st.close()
    # W and the moments of f^1 from the fused x2 sweep's partial sums (the
    # spline's 13824 workgroup sums take the two-stage moment reduction)
    g = _grid(w, method)
    W_ref = strang.electric_field(ref, g)[2]
    m_ref = np.array(field.moments(ref, g.degree, g.lo, g.length))
    tol = 1e-12 if dt == "f64" else 1e-5
    assert abs(to_host(W)[1] - W_ref) <= tol * W_ref
    np.testing.assert_allclose(to_host(mom)[4:], m_ref, rtol=tol)
    if dt == "f32":
        # the oracle stepped the FP64 state; the FP32 input differs from it
        # by its rounding, which the (linear, L2-bounded) step carries over
        # unamplified: it must leave room for the 1e-5 bound
        r_in = rel_l2(f0.astype(np.float32).astype(np.float64), f0)
        assert r_in < 1e-7
    assert_close(got, ref, dt, f"96^4 {method} {dt} step")


@pytest.mark.parametrize("cells,degree", [((8, 6, 8, 10), 1), ((4, 3, 4, 5), 3),
                                          ((3, 2, 3, 4), 5)])
def test_step_parity_other_degrees(cells, degree):
    # two FP64 Strang steps of degree 1, 3 (the dG4 of Table 1) and 5 on
    # non-cubic grids, against the oracle
    vp = require_gpu()
    w = workload("landau_8")
    dims = tuple(c * (degree + 1) for c in cells)
    g = strang.Grid(dims, w.lo, w.length, degree)
    f = field.initial_condition("landau", dims, w.lo, w.length, degree, w.eps, w.k)
    st = vp.VPState(vp.METHOD_SLDG, degree, torch.float64, dims, w.lo, w.length)
    fd = to_dev(f)
    tmp = torch.empty_like(fd)
    W = torch.empty(3, dtype=torch.float64, device="cuda")
    announce(f"strang steps degree {degree} {dims}")
    st.step(fd, tmp, 2, w.dt, W)
    ref, Wr = strang.run(f, g, w.dt, 2)
    assert_close(to_host(fd), ref, "f64", f"degree {degree}")
    assert np.max(np.abs(to_host(W) - Wr) / Wr) <= 1e-12
    st.close()


@pytest.mark.parametrize("name", ["landau_table1_64", "landau_table1_128"])
def test_table1_workloads(name):
    # dG4 at 64 and 128 dofs per direction: one full FP64 step against the
    # oracle at 64^4; sampled lines of every sweep at 128^4
    vp = require_gpu()
    w = workload(name)
    g = _grid(w, "sldg")
    dims = w.dofs
    st = vp.VPState(vp.METHOD_SLDG, w.degree, torch.float64, dims, w.lo, w.length)
    if dims[0] == 64:
        announce(f"{name}: oracle step")
        f0 = field.initial_condition("landau", dims, w.lo, w.length, w.degree, w.eps, w.k)
        ref = strang.step(f0, g, w.dt)
        fd = to_dev(f0)
        tmp = torch.empty_like(fd)
        announce(f"{name}: device step")
        st.step(fd, tmp, 1, w.dt)
        assert_close(to_host(fd), ref, "f64", "64^4 dG4 step")
    else:
        announce(f"{name}: host input")
        f = random_field(dims, seed=64, positive=True)
        fin = to_dev(f)
        out = torch.empty_like(fin)
        rng = np.random.default_rng(65)
        for axis in range(4):
            if axis < 2:
                sig = rng.uniform(-1.6, 1.6, size=dims[axis + 2])
                sst = [0, 0, 0, 0]
                sst[axis + 2] = 1
            else:
                sig = rng.uniform(-0.9, 0.9, size=dims[0] * dims[1])
                sst = [dims[1], 1, 0, 0]
            announce(f"{name}: sldg axis={axis}")
            vp.sldg_advect(axis, w.degree, fin, out, to_dev(sig), shift_stride=sst)
            got = to_host(out)
            for ix in _sample_lines(axis, dims, 32, seed=axis + 10):
                off = sum(ix[d] * sst[d] for d in range(4) if d != axis)
                ref = sldg.shift_lines(f[ix][None, :], sig[off], w.degree)[0]
                assert_close(got[ix], ref, "f64", f"axis {axis} line {ix}")
            # spline on the same grid
            announce(f"{name}: spline axis={axis}")
            vp.spline_advect(axis, fin, out, to_dev(sig), shift_stride=sst)
            got = to_host(out)
            for ix in _sample_lines(axis, dims, 32, seed=axis + 20):
                off = sum(ix[d] * sst[d] for d in range(4) if d != axis)
                ref = spline.shift_lines(f[ix][None, :], sig[off])[0]
                assert_close(got[ix], ref, "f64", f"spline axis {axis} line {ix}")
        del fin, out
    st.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("method", ["sldg", "spline"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_merged_run_parity(method, dt):
    # 10 steps with the x half-steps merged inside segments of 5 steps: the
    # two formed states, their W and moments against the oracle's merged run
    vp = require_gpu()
    w = workload("landau_8")
    g = _grid(w, method)
    f0 = field.initial_condition("landau", w.dofs, w.lo, w.length, g.degree, w.eps, w.k)
    st = vp.VPState(vp.METHOD_SLDG if method == "sldg" else vp.METHOD_SPLINE,
                    w.degree, torch.float64 if dt == "f64" else torch.float32,
                    w.dofs, w.lo, w.length)
    fd = to_dev(f0, dt)
    f_in = to_host(fd)
    tmp = torch.empty_like(fd)
    W = torch.empty(3, dtype=torch.float64, device="cuda")
    mom = torch.empty(12, dtype=torch.float64, device="cuda")
    announce(f"merged run {method} {dt}")
    st.run(fd, tmp, 10, w.dt, 5, W, mom)
    ref, Wr, mr = strang.run_merged(f_in, g, w.dt, 10, 5, with_moments=True)
    assert_close(to_host(fd), ref, dt, "merged run state")
    tol = 1e-12 if dt == "f64" else 1e-5
    assert np.max(np.abs(to_host(W) - Wr) / Wr) <= tol
    np.testing.assert_allclose(to_host(mom).reshape(3, 4), mr, rtol=tol)
    st.close()


def test_diagnostics_are_ordered_on_the_callers_stream():
    # the diagnostics of the fused states run on the state's second stream;
    # on return, work queued on the caller's stream must see all of them:
    # copies queued right after the call, on a stream of the caller's own,
    # equal the results of the same run on the default stream
    vp = require_gpu()
    w = workload("landau_8")
    dims = (12, 12, 16, 16)   # fused x2 sweeps for both methods (SLDG degree 1)
    for method in (vp.METHOD_SLDG, vp.METHOD_SPLINE):
        st = vp.VPState(method, 1, torch.float64, dims, w.lo, w.length)
        f0 = torch.empty(dims, dtype=torch.float64, device="cuda")
        vp.vp_init(vp.IC_LANDAU, w.eps, w.k, 0.0, 1 if method == vp.METHOD_SLDG else -1, f0,
                   w.lo, w.length)
        torch.cuda.synchronize()
        nsteps = 6
        # reference: default stream, synchronised
        a = f0.clone()
        tmp = torch.empty_like(a)
        Wa = torch.empty(nsteps + 1, dtype=torch.float64, device="cuda")
        ma = torch.empty(4 * (nsteps + 1), dtype=torch.float64, device="cuda")
        announce(f"diagnostics stream order, method {method}")
        st.timing_enable(True)
        st.step(a, tmp, nsteps, w.dt, Wa, ma)
        torch.cuda.synchronize()
        timers = st.timing_read()
        st.timing_enable(False)
        assert timers["sweep_x2_rho"][1] == 2 * nsteps, timers
        # the caller's own stream; the copies are queued behind the call
        s1 = torch.cuda.Stream()
        b = f0.clone()
        Wb = torch.full((nsteps + 1,), float("nan"), dtype=torch.float64, device="cuda")
        mb = torch.full((4 * (nsteps + 1),), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            st.step(b, tmp, nsteps, w.dt, Wb, mb, stream=s1)
            Wc = Wb.clone()
            mc = mb.clone()
        s1.synchronize()
        assert torch.equal(a, b)
        assert torch.equal(Wa, Wc), (Wa, Wc)
        assert torch.equal(ma, mc), (ma, mc)
        st.close()


def test_run_with_every_step_formed_is_the_plain_step():
    vp = require_gpu()
    w = workload("landau_8")
    st = vp.VPState(vp.METHOD_SLDG, w.degree, torch.float64, w.dofs, w.lo, w.length)
    a = torch.empty(w.dofs, dtype=torch.float64, device="cuda")
    vp.vp_init(vp.IC_LANDAU, w.eps, w.k, 0.0, w.degree, a, w.lo, w.length)
    b = a.clone()
    tmp = torch.empty_like(a)
    Wa = torch.empty(5, dtype=torch.float64, device="cuda")
    Wb = torch.empty(5, dtype=torch.float64, device="cuda")
    announce("run every=1 against step")
    st.step(a, tmp, 4, w.dt, Wa)
    st.run(b, tmp, 4, w.dt, 1, Wb)
    assert torch.equal(a, b) and torch.equal(Wa, Wb)
    with pytest.raises(vp.VPError):
        st.run(b, tmp, 5, w.dt, 2)
    st.close()


@pytest.mark.parametrize("method,dt,dims", [
    ("sldg", "f64", (12, 10, 16, 16)), ("sldg", "f32", (12, 10, 16, 16)),
    # (N2 a multiple of 256/L, 4 for 64-line tiles)
    ("spline", "f64", (10, 16, 16, 16)), ("spline", "f32", (12, 12, 16, 16)),
    # 64-line FP64 tiles (one segment a wavefront) up to 128 points a line
    # (64 KiB tiles), and 32-line tiles (two segments per wavefront)
    ("spline", "f64", (6, 104, 16, 16)), ("spline", "f64", (2, 136, 8, 16)),
    ("spline", "f32", (2, 264, 8, 16)),
    ("spline", "f64", (6, 16, 16, 16)), ("spline", "f64", (4, 96, 8, 16)),
    ("spline", "f64", (4, 48, 8, 16)), ("spline", "f64", (4, 112, 8, 16)),
    ("spline", "f64", (2, 128, 8, 16)), ("spline", "f64", (2, 192, 8, 16)),
    # FP32 64-line tiles up to the longest line the tile holds
    ("spline", "f32", (6, 48, 8, 16)), ("spline", "f32", (4, 192, 8, 16)),
    ("spline", "f32", (4, 40, 8, 16)), ("spline", "f32", (4, 200, 8, 16)),
])
def test_step_parity_with_density_from_the_x2_sweep(method, dt, dims):
    # the x2 sweep before each field solve also forms the density of its
    # output (groups of 256 velocity columns for SLDG, of 64 or 32 for the
    # spline) and, before the diagnostics, the moments; two steps against
    # the oracle, W and the moments included
    vp = require_gpu()
    degree = 1 if method == "sldg" else None
    w = workload("landau_8")
    g = strang.Grid(dims, w.lo, w.length, degree)
    f = field.initial_condition("landau", dims, w.lo, w.length, degree, w.eps, w.k)
    st = vp.VPState(vp.METHOD_SLDG if method == "sldg" else vp.METHOD_SPLINE, 1,
                    torch.float64 if dt == "f64" else torch.float32, dims, w.lo, w.length)
    fd = to_dev(f, dt)
    f_in = to_host(fd)
    tmp = torch.empty_like(fd)
    W = torch.empty(3, dtype=torch.float64, device="cuda")
    mom = torch.empty(12, dtype=torch.float64, device="cuda")
    announce(f"fused x2 density {method} {dt}")
    st.timing_enable(True)
    st.step(fd, tmp, 2, w.dt, W, mom)
    timers = st.timing_read()
    st.timing_enable(False)
    # every x2 sweep of the two steps formed a density: none went separately
    assert timers["sweep_x2_rho"][1] == 4, timers
    assert timers["sweep_x2"][1] == 0, timers
    ref, Wr, mr = strang.run(f_in, g, w.dt, 2, with_moments=True)
    assert_close(to_host(fd), ref, dt, "two steps")
    tol = 1e-12 if dt == "f64" else 1e-5
    assert np.max(np.abs(to_host(W) - Wr) / Wr) <= tol
    np.testing.assert_allclose(to_host(mom).reshape(3, 4), mr, rtol=tol)
    # the same steps with W only (density without the moment sums), timing
    # only the x1 sweeps: the other categories record nothing
    fd2 = to_dev(f_in, dt)
    W2 = torch.empty(3, dtype=torch.float64, device="cuda")
    st.timing_select(["sweep_x1"])
    st.step(fd2, tmp, 2, w.dt, W2)
    timers = st.timing_read()
    st.timing_enable(False)
    assert timers["sweep_x1"][1] == 4, timers
    assert all(c == 0 for k, (_, c) in timers.items() if k != "sweep_x1"), timers
    assert torch.equal(fd2, fd)
    assert np.max(np.abs(to_host(W2) - Wr) / Wr) <= tol
    with pytest.raises(ValueError):
        st.timing_select(["sweep_x3"])
    from paper_1803_02143_amd import _lib as L
    assert vp.lib().vp_timing_select(st._h, 1 << L.VP_TIMER_COUNT) == L.VP_ERR_ARG
    st.close()


def test_merged_run_parity_table1_64():
    # dG4 at 64^4 (the x2 sweeps form the density and moments of their
    # output): two steps merged into one segment against the oracle
    vp = require_gpu()
    w = workload("landau_table1_64")
    g = _grid(w, "sldg")
    announce("merged run dG4 64^4: oracle")
    f0 = field.initial_condition("landau", w.dofs, w.lo, w.length, w.degree, w.eps, w.k)
    ref, Wr, mr = strang.run_merged(f0, g, w.dt, 2, 2, with_moments=True)
    st = vp.VPState(vp.METHOD_SLDG, w.degree, torch.float64, w.dofs, w.lo, w.length)
    fd = to_dev(f0)
    tmp = torch.empty_like(fd)
    W = torch.empty(2, dtype=torch.float64, device="cuda")
    mom = torch.empty(8, dtype=torch.float64, device="cuda")
    announce("merged run dG4 64^4: device")
    st.run(fd, tmp, 2, w.dt, 2, W, mom)
    assert_close(to_host(fd), ref, "f64", "merged 64^4")
    assert np.max(np.abs(to_host(W) - Wr) / Wr) <= 1e-12
    np.testing.assert_allclose(to_host(mom).reshape(2, 4), mr, rtol=1e-12)
    st.close()


@pytest.mark.parametrize("method", ["sldg", "spline"])
def test_landau96_whole_run_against_stored_oracle_trace(method):
    # the 96^4 Landau run of Sec. 4 (tau = 0.05, 200 Strang steps, FP64):
    # W(t_m) of every state and its mass, L1, L2 and kinetic energy against
    # the oracle's run (tests/golden/make_landau96_golden.py), whole run at
    # 1e-10 relative
    import json
    import os
    vp = require_gpu()
    w = workload("landau_32")
    path = os.path.join(os.path.dirname(__file__), "golden", f"landau96_trace_{method}.json")
    if not os.path.exists(path):
        pytest.skip(f"the oracle's {method} trace has not been written to {path}")
    with open(path) as fh:
        gold = json.load(fh)
    assert tuple(gold["dims"]) == w.dofs and gold["steps"] == w.steps and gold["tau"] == w.dt
    st = vp.VPState(vp.METHOD_SLDG if method == "sldg" else vp.METHOD_SPLINE, w.degree,
                    torch.float64, w.dofs, w.lo, w.length)
    f = torch.empty(w.dofs, dtype=torch.float64, device="cuda")
    vp.vp_init(vp.IC_LANDAU, w.eps, w.k, 0.0, w.degree if method == "sldg" else -1, f,
               w.lo, w.length)
    tmp = torch.empty_like(f)
    W = torch.empty(w.steps + 1, dtype=torch.float64, device="cuda")
    mom = torch.empty(4 * (w.steps + 1), dtype=torch.float64, device="cuda")
    announce(f"96^4 Landau {method}: {w.steps} steps against the oracle trace")
    st.step(f, tmp, w.steps, w.dt, W, mom)
    Wd = to_host(W)
    md = to_host(mom).reshape(-1, 4)
    st.close()
    Wr = np.array(gold["W"])
    mr = np.array(gold["moments"])
    err_W = np.abs(Wd - Wr) / np.abs(Wr)
    announce(f"max rel diff of W over the run {err_W.max():.3e} (step {int(err_W.argmax())})")
    assert err_W.max() <= 1e-10, (err_W.max(), int(err_W.argmax()))
    err_m = np.abs(md - mr) / np.abs(mr)
    assert err_m.max() <= 1e-10, err_m.max(axis=0)
    # mass conservation to round-off over the whole run
    assert np.max(np.abs(md[:, 0] - md[0, 0])) <= 1e-12 * md[0, 0]
