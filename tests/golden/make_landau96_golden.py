"""Writes the stored expected values of the 96^4 Landau workloads.

Every number written here comes from the FP64 oracle (``oracle/``) and
nothing else; the GPU tests compare the device runs against these files.

    python tests/golden/make_landau96_golden.py trace sldg
    python tests/golden/make_landau96_golden.py trace spline
    python tests/golden/make_landau96_golden.py gradient

trace:    the Landau run on 32^4 cells, degree 2 (96^4 dofs; the spline on
          the same 96^4 point grid), tau = 0.05, 200 Strang steps: the
          electric energy W(t_m) = 1/2 int |E|^2 of every f^m (Sec. 4) and
          the mass, L1 norm, L2 norm and kinetic energy of every f^m.
          -> landau96_trace_<method>.json
gradient: the differentiated Landau run (same grid, SLDG degree 2, tau =
          0.05, 40 steps): J = W(f^40) and dJ/d eps at eps = 1/2, with
          f0 affine in eps, dJ/d eps = <dJ/df0, f0(1) - f0(0)>; the
          gradient is the oracle's reverse sweep with every state stored
          (about 28 GB of host memory).  Also a few components of dJ/df0
          at fixed indices and its sums over all axes but one.
          -> landau96_adjoint_gradient.json

A run takes one to three hours on one host core per job.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import adjoint, field, strang  # noqa: E402
from vp_inputs import workload  # noqa: E402

# fixed dof indices (x1, x2, v1, v2) whose gradient entries are stored
GRADIENT_PROBES = [(0, 0, 48, 48), (17, 5, 40, 61), (95, 95, 0, 0), (48, 12, 30, 66),
                   (3, 90, 55, 47), (60, 60, 47, 48)]


def _grid(w, method):
    degree = w.degree if method == "sldg" else None
    return strang.Grid(w.dofs, w.lo, w.length, degree)


def trace(method):
    w = workload("landau_32")
    g = _grid(w, method)
    f0 = field.initial_condition("landau", g.dims, g.lo, g.length, g.degree, w.eps, w.k)
    t0 = time.time()
    f = np.asarray(f0, dtype=np.float64)
    W = [strang.electric_field(f, g)[2]]
    mom = [field.moments(f, g.degree, g.lo, g.length)]
    for m in range(w.steps):
        f = strang.step(f, g, w.dt)
        W.append(strang.electric_field(f, g)[2])
        mom.append(field.moments(f, g.degree, g.lo, g.length))
        print(f"step {m + 1}/{w.steps} W={W[-1]:.17g} ({time.time() - t0:.0f} s)", flush=True)
    out = {
        "about": "FP64 oracle: Landau 32^4 cells, 96^4 dofs, tau = 0.05, 200 Strang steps; "
                 "W[m] = electric energy of f^m, moments[m] = (mass, L1, L2, kinetic) of f^m",
        "written_by": "tests/golden/make_landau96_golden.py trace " + method,
        "workload": w.name, "method": method, "degree": g.degree, "dims": list(g.dims),
        "tau": w.dt, "steps": w.steps,
        "W": [float(x) for x in W],
        "moments": [[float(x) for x in row] for row in mom],
    }
    path = os.path.join(HERE, f"landau96_trace_{method}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", path)


def gradient():
    w = workload("landau_32_adjoint")
    g = _grid(w, "sldg")

    def f0(eps):
        return field.initial_condition("landau", g.dims, g.lo, g.length, g.degree, eps, w.k)

    t0 = time.time()
    J, grad = adjoint.final_energy_gradient(f0(w.eps), g, w.dt, w.steps)
    print(f"J={J:.17g} ({time.time() - t0:.0f} s)", flush=True)
    d_eps = f0(1.0) - f0(0.0)
    dJ = float(np.sum(grad * d_eps))
    out = {
        "about": "FP64 oracle: Landau 32^4 cells, SLDG degree 2 (96^4 dofs), tau = 0.05, "
                 "40 Strang steps from f0(eps = 0.5); J = W(f^40); dJ_deps = <dJ/df0, "
                 "f0(1) - f0(0)>; grad_probes = dJ/df0 at the listed dof indices; "
                 "grad_marginals[d] = dJ/df0 summed over every axis but d",
        "written_by": "tests/golden/make_landau96_golden.py gradient",
        "workload": w.name, "degree": g.degree, "dims": list(g.dims), "tau": w.dt,
        "steps": w.steps, "eps": w.eps,
        "J": float(J), "dJ_deps": dJ,
        "grad_l2": float(np.sqrt(np.sum(grad * grad))),
        "grad_marginals": [[float(x) for x in np.sum(grad, axis=tuple(a for a in range(4) if a != d))]
                           for d in range(4)],
        "grad_probes": [[list(p), float(grad[p])] for p in GRADIENT_PROBES],
    }
    path = os.path.join(HERE, "landau96_adjoint_gradient.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2])
    elif sys.argv[1] == "gradient":
        gradient()
    else:
        raise SystemExit(__doc__)
