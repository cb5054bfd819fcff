"""One step of the Navier-Stokes IMEX scheme with the completed IBDL method (2-D).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 6.5 (Navier-Stokes: numerical implementation).  The nonlinear term is explicit (extrapolated
from the two previous steps), viscosity and the boundary layers implicit (BDF2):
  rho ((3 u^{n+1} - 4 u^n + u^{n-1}) / (2 dt) + 2 (u.grad u)^n - (u.grad u)^{n-1})
      = -grad p^{n+1} + mu Delta u^{n+1} + eta S Q^{n+1} + mu div(S A^{n+1}),
so u^{n+1} solves the completed Brinkman problem with k^2 = 3 rho / (2 dt) and the forcing
  g~ = rho ((-4 u^n + u^{n-1}) / (2 dt) + 2 N^n - N^{n-1}),   N = (u . grad) u,
with S* u^{n+1} + Q/2 = U_b^{n+1}.  The derivatives of the nonlinear term are taken after the
near-boundary interpolation of the recovered field (the thesis's choice), with the handle's
derivative symbols.  The flow is driven by resetting u = (u_inf, 0) on a strip of grid columns
along the left side of the box after every step.
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from . import nearbdry as NB
from .gmres import gmres


def advection(grid, u, disc):
    """(u . grad) u of the 2-D field u [2][ny][nx]: component c is u d_x u_c + v d_y u_c."""
    out = np.empty_like(u)
    for c in range(2):
        out[c] = u[0] * G.deriv(grid, u[c], 0, disc) + u[1] * G.deriv(grid, u[c], 1, disc)
    return out


def forcing(un, unm1, Nn, Nnm1, rho, dt):
    return rho * ((-4.0 * un + unm1) / (2.0 * dt) + 2.0 * Nn - Nnm1)


def strip_reset(u, width, u_inf):
    """u = u_inf, v = 0 on the first `width` grid columns (x index < width)."""
    u = u.copy()
    u[0][:, :width] = u_inf
    u[1][:, :width] = 0.0
    return u


def step(setup, Ub, un, unm1, Nn, Nnm1, rho, dt, omega=None, m1=0.0, m2=0.0, strip=0, u_inf=0.0,
         tol=1e-12, maxit=200):
    """Returns (q, u^{n+1}, N^{n+1}, GMRES iterations).  setup: a completed 2-D Stokes Setup with
    kappa^2 = 3 rho / (2 dt); Ub: [n_ib][2] boundary velocity at t^{n+1}; omega: fluid mask for the
    near-boundary interpolation (skipped when m1 = 0)."""
    g = forcing(un, unm1, Nn, Nnm1, rho, dt)
    Ub = np.asarray(Ub, dtype=np.float64)
    q, it, _ = gmres(setup.apply, setup.rhs(Ub, g), tol, maxit)
    u = setup.recover(q, Ub, g)
    if m1 > 0:
        u = np.stack([NB.near_boundary(setup.grid, setup.X, Ub[:, c], omega, u[c], m1, m2) for c in range(2)])
    if strip > 0:
        u = strip_reset(u, strip, u_inf)
    return q, u, advection(setup.grid, u, setup.disc), it
