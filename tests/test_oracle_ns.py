"""Pins of the oracle's Navier-Stokes IMEX step (Sec. 6.5).

* the nonlinear term on the Taylor-Green field u = (sin kx cos ky, -cos kx sin ky), whose
  (u . grad) u = (k/2) (sin 2kx, sin 2ky) exactly (spectral derivatives are exact for these modes);
* the time discretisation by consistency: for u and N linear in t, the BDF2 difference and the
  extrapolation 2 N^n - N^{n-1} are exact, so 3 rho u^{n+1} / (2 dt) + g~ must equal
  rho (u_t + N) at t^{n+1};
* a whole run: the decaying shear wave u = (e^{-nu k^2 t} sin ky, 0) solves the Navier-Stokes
  equations (its nonlinear term vanishes); with a body whose boundary data follow the wave,
  20 steps on 128^2 stay within 1e-3 of it on the nodes 0.15 or more from the body, near-boundary
  interpolation included.
"""
import math

import numpy as np

import oracle
from oracle import ns
from oracle.ib import Grid
from workloads import geometry as geo


def test_advection_taylor_green():
    g = Grid(2, (64, 64), (2.0, 2.0), (-1.0, -1.0))
    xs, ys = g.nodes()
    k = math.pi
    u = np.stack([np.sin(k * xs) * np.cos(k * ys), -np.cos(k * xs) * np.sin(k * ys)])
    want = 0.5 * k * np.stack([np.sin(2 * k * xs), np.sin(2 * k * ys)])
    assert np.max(np.abs(ns.advection(g, u, "spectral") - want)) < 1e-12
    # the finite-difference symbols are second order: the error drops fourfold per refinement
    e = []
    for n in (32, 64):
        gg = Grid(2, (n, n), (2.0, 2.0), (-1.0, -1.0))
        x, y = gg.nodes()
        uu = np.stack([np.sin(k * x) * np.cos(k * y), -np.cos(k * x) * np.sin(k * y)])
        ww = 0.5 * k * np.stack([np.sin(2 * k * x), np.sin(2 * k * y)])
        e.append(np.max(np.abs(ns.advection(gg, uu, "fd2") - ww)))
    assert 3.5 < e[0] / e[1] < 4.5


def test_forcing_is_consistent_for_linear_data():
    rng = np.random.default_rng(0)
    U, M, u0, N0 = rng.standard_normal((4, 2, 8, 8))
    rho, dt, t = 1.3, 0.02, 0.7
    u = lambda s: u0 + s * U
    N = lambda s: N0 + s * M
    g = ns.forcing(u(t), u(t - dt), N(t), N(t - dt), rho, dt)
    lhs = 3 * rho * u(t + dt) / (2 * dt) + g
    assert np.allclose(lhs, rho * (U + N(t + dt)), rtol=0, atol=1e-11)


def test_shear_wave_run():
    N, dt, nsteps = 128, 0.01, 20
    rho, mu, eta, k = 1.0, 0.05, 10.0, 2 * math.pi
    curve = geo.PolarCurve((0.5, 0.5), 0.15)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), 1.0 / N, 1.0)).flipped()
    o = oracle.Setup(2, (N, N), (1.0, 1.0), (0.0, 0.0), mk.X, mk.nrm, mk.ds, "stokes",
                     math.sqrt(3 * rho / (2 * dt)), mu, "dirichlet", eta, "peskin4", "spectral")
    xs, ys = o.grid.nodes()
    nu = mu / rho

    def exact(t, x, y):
        return np.stack([np.exp(-nu * k * k * t) * np.sin(k * y), 0 * x])

    r = np.hypot(xs - 0.5, ys - 0.5)
    omega = (r >= 0.15).astype(float)
    un, unm1 = exact(0.0, xs, ys), exact(-dt, xs, ys)
    Nn, Nnm1 = ns.advection(o.grid, un, "spectral"), ns.advection(o.grid, unm1, "spectral")
    for s in range(nsteps):
        Ub = exact((s + 1) * dt, mk.X[:, 0], mk.X[:, 1]).T
        _, u, Nu, it = ns.step(o, Ub, un, unm1, Nn, Nnm1, rho, dt, omega, 3, 4)
        unm1, un, Nnm1, Nn = un, u, Nn, Nu
    err = np.max(np.abs(un - exact(nsteps * dt, xs, ys))[:, r > 0.3])
    assert err < 1e-3, err
    assert np.max(np.abs(un - exact(nsteps * dt, xs, ys))[:, omega > 0]) < 1e-2


def test_strip_reset():
    u = np.random.default_rng(1).standard_normal((2, 16, 16))
    v = ns.strip_reset(u, 4, 1.5)
    assert np.all(v[0][:, :4] == 1.5) and np.all(v[1][:, :4] == 0.0)
    assert np.array_equal(v[:, :, 4:], u[:, :, 4:])
