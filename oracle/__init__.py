"""FP64 CPU oracle for the split-step semi-Lagrangian Vlasov-Poisson solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, NumPy/SciPy
implementation of what the HIP library computes, written from the paper
(Einkemmer, "A comparison of semi-Lagrangian discontinuous Galerkin and
spline based Vlasov solvers in four dimensions", arXiv:1803.02143).  Only the
tests, the smoke check and the bench's CPU-baseline leg may import it.  It
shares no code with the HIP library and imports nothing from it.

Modules
  quadrature  Gauss-Legendre nodes/weights on [0,1] and Lagrange bases
  sldg        translate-and-project operator and 1D sweep (Sec. 2, Sec. 3 Eq. (5))
  spline      periodic cubic-spline interpolation sweep (Sec. 3)
  field       grids, initial conditions, density, Poisson, diagnostics
  strang      Strang step composition (Sec. 2)

Parity status: every function here is pinned by a test under ``tests/``
(see ``tests/test_oracle_*.py``) against closed forms, exact invariants,
brute-force integration or independent library routines.
"""

from . import quadrature, sldg, spline, field, strang  # noqa: F401
