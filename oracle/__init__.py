"""FP64 CPU oracle of the IBDL hot path, restated from the thesis.

TEST INFRASTRUCTURE ONLY.  This package is the checker, not the product: only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code with the HIP library; the two meet only in the
seeded input generators.

Modules: delta (regularized delta kernels), ib (grid, S, S*), grid
(finite-difference / spectral operators and inverses), ibdl (boundary
operators A, right-hand sides, grid recovery, dense assembly), gmres
(textbook GMRES), norms (error norms), adjoint (exact gradients of a loss of the
grid solution with respect to the markers and the boundary data, by forward-mode
differentiation of the forward map with dense solves), nearbdry (the indicator function of the
discretized curve and the near-boundary interpolation, 2-D), drag (net force, torque, flux and the
dimensionless drag of a Stokes solution, 2-D), ibsl (the single layer method's Schur complements,
Chapter 2), minres (textbook MINRES) and ns (one step of the Navier-Stokes IMEX scheme).

Parity status: every function is pinned by tests/test_oracle_*.py against
closed forms, kernel identities, adjointness, real-space stencils, PDE
residuals and the iteration counts the thesis prints; the gradients by central
differences of the pinned forward map (tests/test_oracle_adjoint.py); the near-boundary tools by
linear exactness, brute force and the closed-form indicator of a circle
(tests/test_oracle_nearbdry.py); the drag by the thesis's printed drag table (asymptotic forms,
first-order convergence to the reference values), the solvability condition and symmetry
(tests/test_oracle_drag.py); MINRES against GMRES and dense solves, IBSL by symmetry, the
thesis's MINRES iteration table and closed-form solutions (tests/test_oracle_ibsl.py); the
Navier-Stokes step by the Taylor-Green nonlinear term, consistency on linear data and the exact
decaying shear wave (tests/test_oracle_ns.py).  The 3-D operator has
no printed thesis value; it is pinned by closed-form convergence only.
"""
from . import adjoint, delta, drag, gmres, grid, ib, ibdl, ibsl, minres, nearbdry, norms, ns  # noqa: F401
from .ibdl import Setup  # noqa: F401
