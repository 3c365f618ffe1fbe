"""Throughput of the split-step semi-Lagrangian Vlasov-Poisson hot path.

One step = one Strang step of the SLDG solver (degree 2) plus one Strang step
of the cubic-spline solver on the same grid, each with its density, Poisson
solve and per-step diagnostics (electric energy, mass, L1, L2, kinetic
energy).  Every step performs 12 one-dimensional advection sweeps over the
whole 4D array.  The workload is nonlinear Landau damping on 32^4 cells of
degree 2 (96^4 dofs), FP64, dt = 0.05, synthetic initial data generated on
the device.

Prints one JSON line: value = dof-updates per second over the whole timed
region (12 * 96^4 per step / time per step), the roofline of the dominant
sweep kernel (timed with HIP events on the launch stream) and the CPU
oracle's rate on a bounded sample.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SWEEPS_PER_STEP = 6
# Strang steps of the pass before the timed region that times every kernel
TABLE_STEPS = 20


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="landau_32")
    ap.add_argument("--dtype", default=None, help="f64 or f32 (default: the config's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-precision", action="store_true",
                    help="skip the second timed run in the other storage precision")
    ap.add_argument("--methods", default="sldg,spline")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the timing of the adjoint step and its kernels")
    ap.add_argument("--adjoint-steps", type=int, default=20)
    ap.add_argument("--no-microbench", action="store_true",
                    help="skip the isolated per-axis sweep timings")
    ap.add_argument("--no-merged", action="store_true",
                    help="skip the timing of runs with merged x half-steps")
    ap.add_argument("--diag-every", type=int, default=10)
    ap.add_argument("--no-two-stream", action="store_true",
                    help="skip the two-stream legs (192^4 FP64 and FP32, 288^4 FP32)")
    ap.add_argument("--two-stream-steps", type=int, default=10,
                    help="timed Strang steps of each two-stream leg at 192^4 (half at 288^4)")
    ap.add_argument("--copy-ref", type=int, default=0,
                    help="plain device copies of one f buffer before the run (a "
                         "reference kernel of known size for hardware counters)")
    return ap.parse_args()


def counter_traffic(kernel_key, workload_name, dtype):
    """HBM bytes per launch of one sweep kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary, or None when no summary covers it or the
    kernel sources changed since the counters were taken."""
    import glob
    import hashlib
    import re

    csrc = os.path.join(ROOT, "paper_1803_02143_amd", "csrc")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_counters.md"))):
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
        if not m:
            continue
        data = json.loads(m.group(1))
        if data.get("workload") != workload_name or data.get("dtype") != dtype:
            continue
        entry = data["per_launch"].get(kernel_key)
        if entry is None:
            return None
        src = "sldg.hip" if kernel_key.startswith("sldg") else "spline.hip"
        for f in (src, "vp4d_internal.hpp"):
            h = hashlib.sha256(open(os.path.join(csrc, f), "rb").read()).hexdigest()[:16]
            if data["sources"].get(f) != h:
                return None
        return entry["read_bytes"] + entry["written_bytes"]
    return None


def host_info():
    """CPU model and the number of host cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu_model": model, "nproc": usable, "os_cpu_count": os.cpu_count()}


def cpu_baseline(w, dtype):
    """The oracle's sweep rate on a bounded sample: one SLDG and one spline
    sweep along every axis of the full grid, shifts of the step's shape."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import sldg, spline
    from vp_inputs import random_field

    dims = w.dofs
    rng = np.random.default_rng(0)
    f = random_field(dims, seed=1, positive=True)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    updates = 0
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        for axis in range(4):
            shape = [1, 1, 1, 1]
            if axis < 2:
                shape[axis + 2] = dims[axis + 2]
            else:
                shape[0], shape[1] = dims[0], dims[1]
            sig = rng.uniform(-1.2, 1.2, size=shape)
            sldg.sweep(f, axis, sig, w.degree)
            spline.sweep(f, axis, sig)
            updates += 2 * int(np.prod(dims))
    dt = time.perf_counter() - t0
    return {"value": updates / dt, "unit": "dof-updates/s", "cores": 1,
            "kind": "oracle", "host": host_info(),
            "sample": f"one SLDG (degree {w.degree}) and one cubic-spline sweep along "
                      f"each of the 4 axes of the full {'x'.join(map(str, dims))} grid, "
                      f"float64, 1 thread, {dt:.1f} s"}


def run_precision(vp, torch, w, dt, methods, steps, warmup, stream, copy_ref=0):
    """Init, warm up and time `steps` Strang steps of every method in one
    precision; returns the timed seconds and the per-method runs."""
    tdt = torch.float64 if dt == "f64" else torch.float32
    dims = w.dofs
    runs = []
    for m in methods:
        method = vp.METHOD_SLDG if m == "sldg" else vp.METHOD_SPLINE
        deg = w.degree if m == "sldg" else -1
        st = vp.VPState(method, w.degree, tdt, dims, w.lo, w.length)
        f = torch.empty(dims, dtype=tdt, device="cuda")
        tmp = torch.empty_like(f)
        vp.vp_init(vp.IC_LANDAU if w.ic == "landau" else vp.IC_TWO_STREAM_SUM,
                   w.eps, w.k, w.v0, deg, f, w.lo, w.length)
        runs.append({"name": m, "st": st, "f": f, "tmp": tmp})

    for _ in range(copy_ref):
        runs[0]["tmp"].copy_(runs[0]["f"])
    torch.cuda.synchronize()

    # untimed warm-up, then a pass with every timer on: the per-kernel table,
    # and the sweep with the largest total time (the roofline kernel), whose
    # launches alone carry HIP events in the timed region (each timed launch
    # costs two event records on the stream)
    for r in runs:
        if warmup:
            r["st"].step(r["f"], r["tmp"], warmup, w.dt, None, None, stream)
    tsteps = min(steps, TABLE_STEPS)
    for r in runs:
        Wt = torch.empty(tsteps + 1, dtype=torch.float64, device="cuda")
        mt = torch.empty(4 * (tsteps + 1), dtype=torch.float64, device="cuda")
        r["st"].timing_enable(True)
        r["st"].step(r["f"], r["tmp"], tsteps, w.dt, Wt, mt, stream)
    torch.cuda.synchronize()
    best = None
    for r in runs:
        r["timers"] = r["st"].timing_read()
        r["table_steps"] = tsteps
        for name, (ms, cnt) in r["timers"].items():
            if name.startswith("sweep") and cnt and (best is None or ms > best[2]):
                best = (r["name"], name, ms)
    for r in runs:
        if r["name"] == best[0]:
            r["st"].timing_select([best[1]])
        else:
            r["st"].timing_enable(False)
        r["W"] = torch.empty(steps + 1, dtype=torch.float64, device="cuda")
        r["mom"] = torch.empty(4 * (steps + 1), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    # the timed region: each solver advances `steps` Strang steps in one call,
    # recording W and the moments of every state
    t0 = time.perf_counter()
    for r in runs:
        r["ev"] = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        r["ev"][0].record(stream)
        r["st"].step(r["f"], r["tmp"], steps, w.dt, r["W"], r["mom"], stream)
        r["ev"][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for r in runs:
        r["ms_per_step"] = r["ev"][0].elapsed_time(r["ev"][1]) / steps
        r["timed"] = r["st"].timing_read()
        r["st"].timing_enable(False)
        r["st"].close()
        del r["tmp"]
    return elapsed, runs


def two_stream_legs(vp, torch, methods, steps, stream):
    """The two-stream workloads at one GPU: 192^4 dofs (64^4 cells, degree 2)
    in FP64 and FP32, with the difference of the FP32 run from the FP64 one
    after the timed steps, and 288^4 dofs (96^4 cells) in FP32.  Per leg:
    ms per Strang step and dof-updates/s per method, and every sweep kernel's
    average launch time and algorithmic rate from the library's HIP events."""
    import numpy as np

    from vp_inputs import workload

    out = {}
    w = workload("two_stream_64")
    n4 = int(np.prod(w.dofs))
    leg = {"dofs": list(w.dofs), "steps": steps, "warmup": 2, "dt": w.dt}
    keep = {}
    for dt in ("f64", "f32"):
        esize = 8 if dt == "f64" else 4
        elapsed, runs = run_precision(vp, torch, w, dt, methods, steps, 2, stream)
        detail, dominant = kernel_table(runs, n4, esize)
        leg[dt] = {
            "ms_per_step": elapsed / steps * 1e3,
            "dof_updates_per_s": SWEEPS_PER_STEP * len(runs) * n4 * steps / elapsed,
            "ms_per_step_by_method": {r["name"]: r["ms_per_step"] for r in runs},
            "kernels": detail, "dominant": dominant,
            "dominant_frac_of_peak": detail[dominant]["alg_GBs"] / HBM_PEAK_GBS,
        }
        keep[dt] = runs
    diffs = {}
    for r, q in zip(keep["f64"], keep["f32"]):
        fa = r["f"]
        num = 0.0
        den = 0.0
        for a0 in range(0, fa.shape[0], 16):        # in slabs: no full FP64 temporaries
            x = fa[a0:a0 + 16]
            y = q["f"][a0:a0 + 16].double()
            num += float(((y - x) ** 2).sum())
            den += float((x ** 2).sum())
        diffs[r["name"]] = {
            "rel_l2_f": math.sqrt(num / den),
            "rel_max_W": float(((q["W"] - r["W"]).abs() / r["W"].abs()).max()),
            "W_el_last_f64": float(r["W"][-1].item()),
        }
    leg["f32_vs_f64_after_run"] = diffs
    leg["f32_speedup_vs_f64"] = leg["f64"]["ms_per_step"] / leg["f32"]["ms_per_step"]
    del keep, runs, r, q
    torch.cuda.empty_cache()
    out[w.name] = leg

    w = workload("two_stream_96")
    n4 = int(np.prod(w.dofs))
    st = max(1, steps // 2)
    elapsed, runs = run_precision(vp, torch, w, "f32", methods, st, 1, stream)
    detail, dominant = kernel_table(runs, n4, 4)
    out[w.name] = {
        "dofs": list(w.dofs), "dtype": "f32", "steps": st, "warmup": 1, "dt": w.dt,
        "ms_per_step": elapsed / st * 1e3,
        "dof_updates_per_s": SWEEPS_PER_STEP * len(runs) * n4 * st / elapsed,
        "ms_per_step_by_method": {r["name"]: r["ms_per_step"] for r in runs},
        "kernels": detail, "dominant": dominant,
        "dominant_frac_of_peak": detail[dominant]["alg_GBs"] / HBM_PEAK_GBS,
        "rel_mass_drift": {r["name"]: float(((r["mom"][0::4] - r["mom"][0]).abs().max()
                                             / r["mom"][0]).item()) for r in runs},
    }
    del runs
    torch.cuda.empty_cache()
    return out


def _event_ms(torch, stream, fn, reps):
    """Average milliseconds of `fn()` over `reps` calls, HIP events recorded
    on the stream the library launches on."""
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    fn()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def sweep_microbench(vp, torch, w, methods, stream, reps=20, warmup=3):
    """Every sweep on its own: per method, storage precision and axis, the
    median of `reps` launches (after `warmup`) with the shifts of the first
    step, a 512 MB read between launches so that no launch finds its data
    (or dirty lines of the previous launch) in the caches; and the rate of a
    plain device copy of one f buffer measured the same way (the practical
    streaming ceiling)."""
    import numpy as np

    dims = w.dofs
    n4 = int(np.prod(dims))
    flush = torch.ones(512 * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
    out = {}

    def timed(fn):
        ts = []
        for r in range(warmup + reps):
            flush.sum()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            if r >= warmup:
                ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    for dt, tdt, es in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        f = torch.empty(dims, dtype=tdt, device="cuda")
        g = torch.empty_like(f)
        f.uniform_()
        ms = timed(lambda: g.copy_(f))
        res = {"copy": {"ms": ms, "GBs": 2 * n4 * es / (ms * 1e-3) / 1e9}}
        copy_gbs = res["copy"]["GBs"]
        # copies with each sweep family's access pattern (the library's
        # vp_copy_pattern): the bandwidth that pattern reaches here
        ceilings = {}
        for pname, pid in (("contiguous", vp.PATTERN_CONTIGUOUS), ("tiles", vp.PATTERN_TILES),
                           ("segments", vp.PATTERN_SEGMENTS), ("lines", vp.PATTERN_LINES)):
            for axis in ((0,) if pname == "contiguous" else (0, 1, 2)):
                pms = timed(lambda: vp.vp_copy_pattern(pid, f, g, axis, stream=stream))
                torch.cuda.synchronize()
                assert torch.equal(f, g), f"vp_copy_pattern {pname} axis {axis} is no copy"
                key = pname if pname == "contiguous" else f"{pname}_{('x1', 'x2', 'v1')[axis]}"
                ceilings[key] = 2 * n4 * es / (pms * 1e-3) / 1e9
        res["pattern_copy_GBs"] = ceilings
        for m in methods:
            deg = w.degree if m == "sldg" else -1
            shifts = step_shifts(w, deg)
            per = {}
            for axis in range(4):
                sig = torch.from_numpy(shifts[axis]).cuda()
                if m == "sldg":
                    fn = lambda: vp.sldg_advect(axis, w.degree, f, g, sig, stream=stream)
                else:
                    fn = lambda: vp.spline_advect(axis, f, g, sig, stream=stream)
                ms = timed(fn)
                gbs = 2 * n4 * es / (ms * 1e-3) / 1e9
                pkey = sweep_pattern(m, axis)
                per[("x1", "x2", "v1", "v2")[axis]] = {
                    "us": ms * 1e3, "dof_updates_per_s": n4 / (ms * 1e-3), "alg_GBs": gbs,
                    "frac_of_peak": gbs / HBM_PEAK_GBS, "frac_of_copy": gbs / copy_gbs,
                    "pattern": pkey, "frac_of_pattern_copy": gbs / ceilings[pkey]}
            per["mean_frac_of_peak"] = float(np.mean([v["frac_of_peak"] for v in per.values()]))
            res[m] = per
        out[dt] = res
        del f, g
    del flush
    torch.cuda.empty_cache()
    return out


def run_merged(vp, torch, w, dt, methods, steps, every, stream):
    """The same steps with the x half-steps merged between states formed
    every `every` steps (4 + 2/every sweeps per step instead of 6)."""
    tdt = torch.float64 if dt == "f64" else torch.float32
    steps = max(every, steps // every * every)
    out = {"diag_every": every, "steps": steps, "sweeps_per_step": 4 + 2.0 / every}
    for m in methods:
        method = vp.METHOD_SLDG if m == "sldg" else vp.METHOD_SPLINE
        deg = w.degree if m == "sldg" else -1
        st = vp.VPState(method, w.degree, tdt, w.dofs, w.lo, w.length)
        f = torch.empty(w.dofs, dtype=tdt, device="cuda")
        tmp = torch.empty_like(f)
        vp.vp_init(vp.IC_LANDAU if w.ic == "landau" else vp.IC_TWO_STREAM_SUM,
                   w.eps, w.k, w.v0, deg, f, w.lo, w.length)
        W = torch.empty(steps // every + 1, dtype=torch.float64, device="cuda")
        mom = torch.empty(4 * (steps // every + 1), dtype=torch.float64, device="cuda")
        st.run(f, tmp, every, w.dt, every, None, None, stream)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        st.run(f, tmp, steps, w.dt, every, W, mom, stream)
        b.record(stream)
        b.synchronize()
        out[m] = {"ms_per_step": a.elapsed_time(b) / steps,
                  "W_el_last": float(W[-1].item())}
        st.close()
        del f, tmp
    return out


def sweep_pattern(method, axis, fused=False):
    """The vp_copy_pattern access pattern of a sweep kernel: row sweeps
    stream contiguous tiles, spline columns load 64-line tiles, plain SLDG
    columns run by row segments, and the fused SLDG x2 sweep walks whole
    lines."""
    if axis == 3:
        return "contiguous"
    name = ("x1", "x2", "v1")[axis]
    if method == "spline":
        return f"tiles_{name}"
    return f"lines_{name}" if fused else f"segments_{name}"


def step_shifts(w, degree):
    """The shifts (in cells or grid points) of the first Strang step of the
    Landau run: x sweeps (tau/2) v / h_x at the velocity nodes, v sweeps
    tau E / h_v with the field of the initial perturbation,
    E_d = (eps / k) sin(k x_d)."""
    import numpy as np

    m = 1 if degree < 0 else degree + 1
    if degree < 0:
        xi = np.array([0.5])
    else:
        xi = (np.polynomial.legendre.leggauss(m)[0] + 1.0) / 2.0
    nodes, h = [], []
    for d in range(4):
        nc = w.dofs[d] // m
        hd = w.length[d] / nc
        nodes.append(w.lo[d] + (np.arange(nc)[:, None] + xi[None, :]).ravel() * hd)
        h.append(hd)
    out = []
    for axis in range(4):
        shape = [1, 1, 1, 1]
        if axis < 2:
            shape[axis + 2] = w.dofs[axis + 2]
            sig = 0.5 * w.dt * nodes[axis + 2] / h[axis]
        else:
            shape[0], shape[1] = w.dofs[0], w.dofs[1]
            x = nodes[axis - 2]
            e = (w.eps / w.k) * np.sin(w.k * x)
            sig = w.dt * e / h[axis]
            sig = sig[:, None] if axis == 2 else sig[None, :]
            sig = np.broadcast_to(sig, (w.dofs[0], w.dofs[1]))
        out.append(np.ascontiguousarray(np.asarray(sig, dtype=np.float64).reshape(shape)))
    return out


def run_adjoint(vp, torch, w, dt, methods, steps, stream):
    """Reverse-mode cost on the same grid: whole adjoint Strang steps
    (recompute of the forward half step, six transposed sweeps, two shift
    derivatives, the field transposes), and each transposed sweep and shift
    derivative on its own with the shifts of the step."""
    import numpy as np

    tdt = torch.float64 if dt == "f64" else torch.float32
    esize = 8 if dt == "f64" else 4
    dims = w.dofs
    n4 = int(np.prod(dims))
    out = {}
    for m in methods:
        method = vp.METHOD_SLDG if m == "sldg" else vp.METHOD_SPLINE
        deg = w.degree if m == "sldg" else -1
        st = vp.VPState(method, w.degree, tdt, dims, w.lo, w.length)
        f = torch.empty(dims, dtype=tdt, device="cuda")
        vp.vp_init(vp.IC_LANDAU if w.ic == "landau" else vp.IC_TWO_STREAM_SUM,
                   w.eps, w.k, w.v0, deg, f, w.lo, w.length)
        lam = torch.empty_like(f)
        st.energy_gradient(f, lam, None, stream)
        work = st.adjoint_workspace()
        ms_step = _event_ms(torch, stream, lambda: st.adjoint_step(f, lam, w.dt, work, stream),
                            steps)
        res = {"ms_per_adjoint_step": ms_step, "kernels": {}}
        # per-axis kernels with the shifts of the first step
        buf = torch.empty_like(f)
        shifts = step_shifts(w, deg)
        for axis in range(4):
            sig = torch.from_numpy(shifts[axis]).cuda()
            g = torch.empty(n4 // dims[axis], dtype=torch.float64, device="cuda")
            if m == "sldg":
                adj = lambda: vp.sldg_advect_adjoint(axis, w.degree, buf, lam, sig, stream=stream)
                dsh = lambda: vp.sldg_advect_dshift(axis, w.degree, f, lam, sig, g, stream=stream)
            else:
                adj = lambda: vp.spline_advect_adjoint(axis, buf, lam, sig, stream=stream)
                dsh = lambda: vp.spline_advect_dshift(axis, f, lam, sig, g, stream=stream)
            name = ("x1", "x2", "v1", "v2")[axis]
            for kind, fn in (("adjoint_sweep", adj), ("dshift", dsh)):
                ms = _event_ms(torch, stream, fn, 10)
                # adjoint sweep: read lam, write lam'; shift derivative: read f
                # and lam, write one value per line
                nbytes = 2 * n4 * esize + (8 * (n4 // dims[axis]) if kind == "dshift" else 0)
                res["kernels"][f"{m}_{kind}_{name}"] = {
                    "avg_ms": ms, "alg_GBs": nbytes / (ms * 1e-3) / 1e9}
        st.close()
        out[m] = res
        del f, lam, work, buf
        torch.cuda.empty_cache()
    return out


def timed_kernel(runs, n4, esize):
    """The roofline kernel's average launch in the timed region (the only
    category whose launches carry HIP events there) and its rates."""
    for r in runs:
        for name, (ms, cnt) in r["timed"].items():
            if cnt:
                avg = ms / cnt
                return f"{r['name']}_{name}", {
                    "avg_ms": avg, "launches": cnt, "total_ms": ms,
                    "dof_updates_per_s": n4 / (avg * 1e-3),
                    "alg_GBs": 2.0 * n4 * esize / (avg * 1e-3) / 1e9}
    raise RuntimeError("no timed launches in the timed region")


def kernel_table(runs, n4, esize):
    """Per-kernel averages from the library's HIP events over the pass before
    the timed region (every category timed), and the sweep with the largest
    total time."""
    detail = {}
    dominant = None
    for r in runs:
        for name, (ms, cnt) in r["timers"].items():
            if cnt == 0:
                continue
            key = f"{r['name']}_{name}"
            avg = ms / cnt
            d = {"avg_ms": avg, "launches": cnt, "total_ms": ms}
            if name.startswith("sweep"):
                d["dof_updates_per_s"] = n4 / (avg * 1e-3)
                d["alg_GBs"] = 2.0 * n4 * esize / (avg * 1e-3) / 1e9
            detail[key] = d
            if name.startswith("sweep") and (dominant is None or ms > detail[dominant]["total_ms"]):
                dominant = key
    return detail, dominant


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); the "
              "multi-GPU sharding is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1803_02143_amd as vp
    from vp_inputs import workload

    w = workload(a.config)
    dt = a.dtype or w.dtype
    esize = 8 if dt == "f64" else 4
    dims = w.dofs
    n4 = int(np.prod(dims))
    methods = [m for m in a.methods.split(",") if m]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    elapsed, runs = run_precision(vp, torch, w, dt, methods, a.steps, a.warmup, stream,
                                  a.copy_ref)
    sweeps = SWEEPS_PER_STEP * len(runs)
    value = sweeps * n4 * a.steps / elapsed
    detail, _ = kernel_table(runs, n4, esize)
    dominant, dom = timed_kernel(runs, n4, esize)
    roofline = {"kernel": dominant, "bound": "hbm", "achieved": dom["alg_GBs"],
                "launches": dom["launches"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["alg_GBs"] / HBM_PEAK_GBS,
                "traffic": counter_traffic(dominant, w.name, dt),
                "alg_bytes_per_launch": 2 * n4 * esize}
    W_last = {r["name"]: float(r["W"][-1].item()) for r in runs}
    mass_drift = {r["name"]: float(((r["mom"][0::4] - r["mom"][0]).abs().max() / r["mom"][0]).item())
                  for r in runs}

    out = {
        "metric": "4D dof-updates/s per advection sweep (whole Strang steps, SLDG + spline)",
        "value": value,
        "unit": "dof-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic (Landau initial condition sampled on the device)",
        "config": {"workload": f"{w.name}: nonlinear Landau 2D-2V, {w.cells[0]}^4 cells, "
                               f"SLDG degree {w.degree} ({dims[0]}^4 dofs) + cubic spline "
                               f"on {dims[0]}^4 points, dt={w.dt}",
                   "dofs": list(dims), "methods": methods, "sweeps_per_step": sweeps},
        "roofline": roofline,
        "ms_per_step_by_method": {r["name"]: r["ms_per_step"] for r in runs},
        "kernels": detail,
        "W_el_last": W_last,
        "rel_mass_drift": mass_drift,
    }

    if not a.no_microbench:
        out["sweep_microbench"] = sweep_microbench(vp, torch, w, methods, stream)
        # the dominant kernel against a copy with its own access pattern
        meth, _, kind = dominant.partition("_sweep_")
        axis = {"x1": 0, "x2": 1, "v1": 2, "v2": 3, "x2_rho": 1}[kind]
        pkey = sweep_pattern(meth, axis, fused=kind == "x2_rho")
        ceil_gbs = out["sweep_microbench"][dt]["pattern_copy_GBs"][pkey]
        roofline["pattern_copy"] = {"pattern": pkey, "GBs": ceil_gbs,
                                    "frac": roofline["achieved"] / ceil_gbs}

    if not a.no_merged:
        mr = run_merged(vp, torch, w, dt, methods, a.steps, a.diag_every, stream)
        for r in runs:
            mr[r["name"]]["speedup_vs_every_step"] = r["ms_per_step"] / mr[r["name"]]["ms_per_step"]
        out["merged_run"] = mr

    if w.name.startswith("landau_table1_"):
        # the paper's Table 1 (whole Strang steps, FP64 assumed, 16 threads
        # on two Xeon E5-2630 v3 / one VSC3 node of two E5-2650 v2): context
        paper = {64: {"sldg_dG4": (0.105, 0.151), "selalib_spline": (0.194, 0.219)},
                 128: {"sldg_dG4": (1.62, 2.31), "selalib_spline": (3.25, 4.02)}}[dims[0]]
        out["paper_table1"] = {
            "dofs_per_direction": dims[0],
            "this_run_s_per_step": {r["name"]: r["ms_per_step"] * 1e-3 for r in runs},
            "paper_s_per_step": {k: {"workstation_2x_E5-2630v3": v[0],
                                     "vsc3_node_2x_E5-2650v2": v[1]}
                                 for k, v in paper.items()},
        }

    if not a.no_adjoint:
        adj = run_adjoint(vp, torch, w, dt, methods, a.adjoint_steps, stream)
        for m, r in adj.items():
            # forward step time of the method: its library timers per step
            fwd = sum(v["total_ms"] for k, v in detail.items()
                      if k.startswith(m + "_")) / runs[0]["table_steps"]
            r["adjoint_over_forward_kernel_time"] = r["ms_per_adjoint_step"] / fwd
        out["adjoint"] = adj

    if not a.no_other_precision:
        # the same steps in the other storage precision: its rates, and its
        # difference from this run (which matches the FP64 oracle to 1e-12)
        odt = "f32" if dt == "f64" else "f64"
        oes = 8 if odt == "f64" else 4
        oel, oruns = run_precision(vp, torch, w, odt, methods, a.steps, a.warmup, stream)
        odetail, _ = kernel_table(oruns, n4, oes)
        diffs = {}
        for r, q in zip(runs, oruns):
            fa = r["f"].double()
            fb = q["f"].double()
            diffs[r["name"]] = {
                "rel_l2_f": float((fb - fa).norm() / fa.norm()),
                "rel_max_W": float(((q["W"] - r["W"]).abs() / r["W"].abs()).max()),
            }
        out["other_precision"] = {
            "dtype": odt, "ms_per_step": oel / a.steps * 1e3,
            "value": sweeps * n4 * a.steps / oel,
            "speedup_vs_main": elapsed / oel,
            "difference_vs_main_after_run": diffs,
            "kernels": {k: {kk: v[kk] for kk in ("avg_ms", "dof_updates_per_s", "alg_GBs") if kk in v}
                        for k, v in odetail.items()},
        }
    if not a.no_two_stream:
        out["two_stream"] = two_stream_legs(vp, torch, methods, a.two_stream_steps, stream)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, dt)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
