"""FP64 CPU oracle for the coarse-grid-projection (CGP) QG time step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference against which the HIP path is checked.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path never does.  It shares no code with the HIP path:
the only common module is ``cgp_inputs`` (seeded inputs, no method
arithmetic).

Paper: O. San and A. E. Staples, "An Efficient Coarse Grid Projection Method
for Quasigeostrophic Models of Large-Scale Ocean Circulation" (arXiv 1308.3290).

Modules
  grid        node grid and coordinates (Sec. 4.4 index ranges)
  operators   Arakawa Jacobian J1/J2/J3 (Sec. 4.1), 5-point Laplacian, beta term,
              and exact transposes of every 9-point operator (scatter form)
  transfer    full-weighting restriction and bilinear prolongation (Sec. 3.1)
  elliptic    sine-transform Poisson / two-layer solves (Sec. 4.3), three routes
  multigrid   V-cycle multigrid for the coarse Poisson problem (CGP's black box)
  model       right-hand sides, the CGP elliptic map, CGPRK3 step (Sec. 3.2, 4.2)
  cfl         adaptive CFL step size (Sec. 4.2) and the adaptive trajectory
  statistics  time means over a window of a long run (Sec. 5.1)
  diagnostics basin energy (eq. 26) and enstrophy
  adjoint     tangent-linear and adjoint of the one-layer CGP step; loss gradient
  params      nondimensional parameters from Tables 1 and 2

Every array is y-major with x contiguous, shape (ny+1, nx+1), boundary ring 0.

Parity status: every function here is pinned by a test in tests/test_oracle_*.py
against closed forms, invariants, special cases or printed values, except the
absolute long-run trajectories, which the paper prints nowhere (parity
unpinned beyond the operator pins that compose them).
"""
from . import grid, operators, transfer, elliptic, multigrid, model, cfl, statistics, diagnostics, adjoint, params  # noqa: F401
