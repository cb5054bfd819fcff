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

Pressure (from the completed Brinkman system, (mu Delta - k^2) u - grad p + eta S Q + mu div(S A)
= g~ and div u + S(Q.n) = 0): its divergence gives
  p = Delta_0^-1 [ div(eta S Q + mu div(S A) - g~) - (mu Delta - k^2) S(Q.n) ].
Force on the body by a control volume (Sec. 6.5): with R a grid-aligned box around the body and
R' its part in the fluid,
  B = -int_{R'} rho u_t dx + oint_{dR} (sigma - rho u u^T) . n_R dl,
  sigma = -p I + mu (grad u + grad u^T),
both integrals by the trapezoidal rule on the grid nodes of R and of its sides.
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from . import nearbdry as NB
from .gmres import gmres
from .ib import spread


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


def pressure(setup, q, g=None):
    """Mean-zero pressure of the completed (or plain) Brinkman / Stokes solution with density q and
    forcing g (Setup of a 2-D Stokes problem)."""
    o = setup
    Q, _ = o.split(q)
    D = o.dim
    grid = o.grid
    f = np.zeros((D,) + grid.shape)
    if o.eta != 0.0:
        f = f + o.eta * o.S(Q)
    A = o.tensor_A(Q)
    SA = o.S(A.reshape(o.n_ib, D * D)).reshape((D, D) + grid.shape)
    f = f + o.mu * np.stack([sum(G.deriv(grid, SA[i, j], j, o.disc) for j in range(D)) for i in range(D)])
    if g is not None:
        f = f - g
    s = o.S(np.sum(Q * o.nrm, axis=1))
    lap_s = np.real(np.fft.ifftn(G.laplacian_symbol(grid, o.disc) * np.fft.fftn(s)))
    rhs = G.div(grid, f, o.disc) - (o.mu * lap_s - o.kappa ** 2 * s)
    return G.solve(grid, rhs, o.disc, 0.0)


def _trap(n):
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    return w


def cv_force(grid, u, ut, p, omega, rho, mu, box, disc):
    """B of the control-volume formula over the box of grid indices box = (i0, i1, j0, j1) (x from
    i0 to i1, y from j0 to j1, inclusive); u, ut: [2][ny][nx]; p, omega: [ny][nx]."""
    i0, i1, j0, j1 = box
    h = grid.h
    du = [[G.deriv(grid, u[c], d, disc) for d in range(2)] for c in range(2)]   # du[c][d] = d_d u_c

    def flux(c, d, jj, ii):
        """(sigma - rho u u^T)_{c d} at the nodes (jj, ii)."""
        sig = mu * (du[c][d][jj, ii] + du[d][c][jj, ii]) - (p[jj, ii] if c == d else 0.0)
        return sig - rho * u[c][jj, ii] * u[d][jj, ii]

    B = np.zeros(2)
    wy = _trap(j1 - j0 + 1) * h
    wx = _trap(i1 - i0 + 1) * h
    jj = np.arange(j0, j1 + 1)
    ii = np.arange(i0, i1 + 1)
    for c in range(2):
        B[c] += np.sum(wy * flux(c, 0, jj, np.full_like(jj, i1)))      # right side, n = +x
        B[c] -= np.sum(wy * flux(c, 0, jj, np.full_like(jj, i0)))      # left side, n = -x
        B[c] += np.sum(wx * flux(c, 1, np.full_like(ii, j1), ii))      # top, n = +y
        B[c] -= np.sum(wx * flux(c, 1, np.full_like(ii, j0), ii))      # bottom, n = -y
        vol = (omega[j0:j1 + 1, i0:i1 + 1] * ut[c][j0:j1 + 1, i0:i1 + 1])
        B[c] -= rho * np.sum(wy[:, None] * wx[None, :] * vol)
    return B
