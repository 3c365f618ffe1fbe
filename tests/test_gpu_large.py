"""Full-size checks at the two-stream workloads: 192^4 (FP32 and FP64) and
288^4 (FP32, 27.5 GB per copy of f).  The device state comes from vp_init;
the oracle evaluates the same initial condition itself at the nodes of each
sampled line and recomputes that line's sweep."""

import numpy as np
import pytest

from gpu_common import announce, assert_close, require_gpu, torch
from oracle import field, sldg, spline
from vp_inputs import workload

pytestmark = pytest.mark.gpu


def _nodes(w, degree):
    return [field.nodes_1d(w.lo[d], w.length[d], w.dofs[d], degree) for d in range(4)]


def _line_input(w, nodes, ix, axis, dt):
    coords = [nodes[d][ix[d]] if d != axis else nodes[d] for d in range(4)]
    u = field.initial_condition_at("two_stream", *coords, w.eps, w.k, w.v0, w.form)
    u = np.broadcast_to(u, (len(nodes[axis]),)).astype(np.float64)
    if dt == "f32":
        u = u.astype(np.float32).astype(np.float64)
    return u


@pytest.mark.parametrize("name,dt", [("two_stream_64", "f32"), ("two_stream_64", "f64"),
                                     ("two_stream_96", "f32")])
def test_large_sweeps_sampled(name, dt):
    vp = require_gpu()
    w = workload(name)
    dims = w.dofs
    tdt = torch.float32 if dt == "f32" else torch.float64
    rng = np.random.default_rng(7)
    announce(f"{name} {dt}: allocating 2 x {np.prod(dims) * (4 if dt == 'f32' else 8) / 1e9:.1f} GB")
    f = torch.empty(dims, dtype=tdt, device="cuda")
    out = torch.empty_like(f)
    for method in ("sldg", "spline"):
        degree = w.degree if method == "sldg" else None
        announce(f"{name} {dt} {method}: vp_init")
        vp.vp_init(vp.IC_TWO_STREAM_SUM, w.eps, w.k, w.v0, -1 if degree is None else degree,
                   f, w.lo, w.length)
        nodes = _nodes(w, degree)
        for axis in range(4):
            if axis < 2:
                h = field.cell_width(w.length[axis], dims[axis], degree)
                sig = 0.5 * w.dt * nodes[axis + 2] / h
                st = [0, 0, 0, 0]
                st[axis + 2] = 1
            else:
                sig = rng.uniform(-0.9, 0.9, size=dims[0] * dims[1])
                st = [dims[1], 1, 0, 0]
            announce(f"{name} {dt} {method} axis={axis}")
            shift = torch.from_numpy(np.ascontiguousarray(sig)).cuda()
            if method == "sldg":
                vp.sldg_advect(axis, w.degree, f, out, shift, shift_stride=st)
            else:
                vp.spline_advect(axis, f, out, shift, shift_stride=st)
            torch.cuda.synchronize()
            for q in range(24):
                ix = [int(rng.integers(0, d)) for d in dims]
                sel = list(ix)
                sel[axis] = slice(None)
                got = out[tuple(sel)].double().cpu().numpy()
                off = sum(ix[d] * st[d] for d in range(4) if d != axis)
                u = _line_input(w, nodes, ix, axis, dt)
                if method == "sldg":
                    ref = sldg.shift_lines(u[None, :], sig[off], w.degree)[0]
                else:
                    ref = spline.shift_lines(u[None, :], sig[off])[0]
                assert_close(got, ref, dt, f"{method} axis {axis} line {ix}")
    del f, out
    torch.cuda.empty_cache()


def test_capacity_run_288_f32_conserves_mass():
    # two Strang steps of the 288^4 FP32 workload with diagnostics
    vp = require_gpu()
    w = workload("two_stream_96")
    announce("two_stream_96 f32: two Strang steps")
    f = torch.empty(w.dofs, dtype=torch.float32, device="cuda")
    tmp = torch.empty_like(f)
    vp.vp_init(vp.IC_TWO_STREAM_SUM, w.eps, w.k, w.v0, w.degree, f, w.lo, w.length)
    st = vp.VPState(vp.METHOD_SLDG, w.degree, torch.float32, w.dofs, w.lo, w.length)
    W = torch.empty(3, dtype=torch.float64, device="cuda")
    mom = torch.empty(12, dtype=torch.float64, device="cuda")
    st.step(f, tmp, 2, w.dt, W, mom)
    torch.cuda.synchronize()
    m = mom.cpu().numpy().reshape(3, 4)
    Wh = W.cpu().numpy()
    assert np.all(np.isfinite(m)) and np.all(np.isfinite(Wh))
    assert np.max(np.abs(m[:, 0] - m[0, 0])) <= 1e-6 * m[0, 0]
    # the exact initial mass: area times the two-stream normalisation
    # (each velocity factor integrates to 2 sqrt(2 pi) over the real line)
    assert abs(m[0, 0] - w.length[0] * w.length[1]) < 1e-6 * m[0, 0]
    st.close()
    del f, tmp
    torch.cuda.empty_cache()


def test_capacity_run_288_f32_with_adjoint_tail():
    # 100 FP32 Strang steps of the 288^4 workload, then dW(f^100)/df^80
    # through the last 20 steps with checkpoints every 4 steps and every
    # state recomputed from its checkpoint (at most 9 copies of f, 248 GB).
    # The directional derivative along the perturbation mode is checked
    # against FP64 central differences of the 20 steps from the same f^80.
    vp = require_gpu()
    import time
    from paper_1803_02143_amd.autograd import final_electric_energy
    w = workload("two_stream_96")
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    nb = int(np.prod(w.dofs)) * 4
    announce(f"two_stream_96 f32: 80 Strang steps ({nb / 1e9:.1f} GB per copy)")
    st = vp.VPState(vp.METHOD_SLDG, w.degree, torch.float32, w.dofs, w.lo, w.length)
    f = torch.empty(w.dofs, dtype=torch.float32, device="cuda")
    tmp = torch.empty_like(f)
    vp.vp_init(vp.IC_TWO_STREAM_SUM, w.eps, w.k, w.v0, w.degree, f, w.lo, w.length)
    mom = torch.empty(4 * 81, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    st.step(f, tmp, 80, w.dt, None, mom)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    del tmp
    m = mom.cpu().numpy().reshape(81, 4)
    assert np.max(np.abs(m[:, 0] - m[0, 0])) <= 1e-5 * m[0, 0]

    announce("two_stream_96 f32: last 20 steps with checkpoints, adjoint")
    f80 = f.requires_grad_(True)
    t0 = time.perf_counter()
    J = final_electric_energy(f80, st, 20, w.dt, every=4, store_segment=False)
    J.backward()
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    peak = torch.cuda.max_memory_allocated()
    announce(f"80 steps {t_fwd:.2f} s; 20 steps + adjoint {t_adj:.2f} s; "
             f"peak {peak / 1e9:.1f} GB ({peak / nb:.2f} copies of f)")
    assert peak <= 9.2 * nb
    grad = f80.grad.detach()
    f80 = f80.detach()
    del f
    # perturbation direction d f0 / d eps, and the directional derivative
    delta = torch.empty_like(f80)
    vp.vp_init(vp.IC_TWO_STREAM_SUM, 1.0, w.k, w.v0, w.degree, delta, w.lo, w.length)
    base = torch.empty_like(f80)
    vp.vp_init(vp.IC_TWO_STREAM_SUM, 0.0, w.k, w.v0, w.degree, base, w.lo, w.length)
    delta.sub_(base)
    del base
    g_dir = float(sum((grad[i].double() * delta[i].double()).sum() for i in range(w.dofs[0])))
    del grad
    torch.cuda.empty_cache()

    announce("two_stream_96 f64: central differences over the last 20 steps")
    st64 = vp.VPState(vp.METHOD_SLDG, w.degree, torch.float64, w.dofs, w.lo, w.length)
    h = 1e-5
    Js = []
    for sgn in (1.0, -1.0):
        g64 = f80.double()
        g64.add_(delta.double(), alpha=sgn * h)
        t64 = torch.empty_like(g64)
        W = torch.empty(21, dtype=torch.float64, device="cuda")
        st64.step(g64, t64, 20, w.dt, W)
        Js.append(float(W[-1]))
        del g64, t64
        torch.cuda.empty_cache()
    fd = (Js[0] - Js[1]) / (2 * h)
    announce(f"adjoint {g_dir:.10e} vs central difference {fd:.10e}: "
             f"rel {abs(g_dir - fd) / abs(fd):.2e}; W(f^100) = {J.item():.6e}")
    assert abs(g_dir - fd) <= 1e-6 * abs(fd)
    st.close()
    st64.close()
    del f80, delta
    torch.cuda.empty_cache()
