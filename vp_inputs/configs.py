"""Named workloads of the 2D-2V Vlasov-Poisson runs.

Each workload is plain data: the initial condition and its parameters, the
phase-space box, the number of cells per axis, the polynomial degree of the
semi-Lagrangian discontinuous Galerkin (SLDG) space, the storage precision,
the time step and the number of Strang steps.

* Landau damping follows Sec. 4 (Eq. (6)): f0 = (2 pi)^-1 exp(-|v|^2/2)
  (1 + eps (cos k x1 + cos k x2)), eps = 1/2, k = 1/2, x in [0, 4 pi)^2,
  v in [-6, 6)^2.  The Table 1 workloads use it with degree 3 (dG4) at 64
  and 128 dofs per direction.
* Two-stream follows Sec. 5 (Eq. (7)) with the perturbation written as a sum
  (1 + eps (cos k x1 + cos k x2)) and the velocity box widened to [-9, 9)^2;
  the product form cos k x1 cos k x2 of Eq. (7) is available as ``form``.
"""

from dataclasses import dataclass, field, replace
import math


@dataclass(frozen=True)
class Workload:
    name: str
    ic: str                      # "landau" | "two_stream"
    cells: tuple                 # cells per axis (x1, x2, v1, v2)
    degree: int                  # SLDG polynomial degree l (dofs per cell = l+1)
    dtype: str                   # "f64" | "f32" storage of f
    dt: float
    steps: int
    lo: tuple
    length: tuple
    eps: float
    k: float
    v0: float = 0.0
    form: str = "sum"            # two-stream perturbation: "sum" | "product"
    notes: str = ""

    @property
    def dofs(self):
        return tuple(c * (self.degree + 1) for c in self.cells)

    def with_(self, **kw):
        return replace(self, **kw)


_FOUR_PI = 4.0 * math.pi
_TEN_PI = 10.0 * math.pi

_LANDAU = dict(ic="landau", lo=(0.0, 0.0, -6.0, -6.0),
               length=(_FOUR_PI, _FOUR_PI, 12.0, 12.0), eps=0.5, k=0.5)
_TWO_STREAM = dict(ic="two_stream", lo=(0.0, 0.0, -9.0, -9.0),
                   length=(_TEN_PI, _TEN_PI, 18.0, 18.0), eps=1e-3, k=0.2,
                   v0=2.4)

CONFIGS = {
    "landau_8": Workload(name="landau_8", cells=(8, 8, 8, 8), degree=2,
                         dtype="f64", dt=0.1, steps=20, **_LANDAU,
                         notes="24^4 dofs; small case"),
    "landau_32": Workload(name="landau_32", cells=(32, 32, 32, 32), degree=2,
                          dtype="f64", dt=0.05, steps=200, **_LANDAU,
                          notes="96^4 dofs; spline on the same 96^4 grid"),
    "two_stream_64": Workload(name="two_stream_64", cells=(64, 64, 64, 64),
                              degree=2, dtype="f32", dt=0.1, steps=500,
                              **_TWO_STREAM, notes="192^4 dofs"),
    "landau_32_adjoint": Workload(name="landau_32_adjoint",
                                 cells=(32, 32, 32, 32), degree=2, dtype="f32",
                                 dt=0.05, steps=40, **_LANDAU,
                                 notes="differentiated run"),
    # the comparison workload of Table 1: dG4 (degree 3), 64 and 128 dofs per
    # direction, the spline on the same grid, tau = 0.1 as in Sec. 4
    "landau_table1_64": Workload(name="landau_table1_64", cells=(16, 16, 16, 16),
                                 degree=3, dtype="f64", dt=0.1, steps=20, **_LANDAU,
                                 notes="64^4 dofs, degree 3"),
    "landau_table1_128": Workload(name="landau_table1_128", cells=(32, 32, 32, 32),
                                  degree=3, dtype="f64", dt=0.1, steps=20, **_LANDAU,
                                  notes="128^4 dofs, degree 3"),
    "two_stream_96": Workload(name="two_stream_96", cells=(96, 96, 96, 96),
                              degree=2, dtype="f32", dt=0.1, steps=100,
                              **_TWO_STREAM, notes="288^4 dofs"),
}


def workload(name, **overrides):
    w = CONFIGS[name]
    return w.with_(**overrides) if overrides else w
