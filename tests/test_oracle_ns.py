"""Pins of the oracle's Navier-Stokes IMEX step (Sec. 6.5).

* the nonlinear term on the Taylor-Green field u = (sin kx cos ky, -cos kx sin ky), whose
  (u . grad) u = (k/2) (sin 2kx, sin 2ky) exactly (spectral derivatives are exact for these modes);
* the time discretisation by consistency: for u and N linear in t, the BDF2 difference and the
  extrapolation 2 N^n - N^{n-1} are exact, so 3 rho u^{n+1} / (2 dt) + g~ must equal
  rho (u_t + N) at t^{n+1};
* the control-volume force by the divergence theorem: a constant state exerts none; a linear
  pressure -G x alone gives G |R| along x; the shear u = (sin ky, 0) gives
  mu k (cos k y1 - cos k y0)(x1 - x0); a uniform u_t gives -rho u_t |R|;
* the pressure of a solved completed Brinkman problem satisfies its momentum equation
  (mu Delta - k^2) u - grad p + eta S Q + mu div(S A) = g~ on every node, to rounding;
* a whole run: the decaying shear wave u = (e^{-nu k^2 t} sin ky, 0) solves the Navier-Stokes
  equations (its nonlinear term vanishes); with a body whose boundary data follow the wave,
  20 steps on 128^2 stay within 1e-3 of it on the nodes 0.15 or more from the body, near-boundary
  interpolation included.
"""
import math

import numpy as np

import oracle
from oracle import ns
from oracle.gmres import gmres
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


def test_cv_force_divergence_theorem():
    g = Grid(2, (64, 64), (1.0, 1.0), (0.0, 0.0))
    xs, ys = g.nodes()
    box = (8, 40, 12, 50)
    x0, x1, y0, y1 = g.h * 8, g.h * 40, g.h * 12, g.h * 50
    area = (x1 - x0) * (y1 - y0)
    one = np.ones(g.shape)
    zero2 = np.zeros((2,) + g.shape)
    U = np.stack([0.7 * one, -0.2 * one])
    assert np.allclose(ns.cv_force(g, U, zero2, 3.0 * one, one, 1.3, 0.1, box, "spectral"), 0, atol=1e-12)
    Gp = 2.5
    B = ns.cv_force(g, zero2, zero2, -Gp * xs, one, 1.0, 0.1, box, "spectral")
    assert np.allclose(B, [Gp * area, 0.0], atol=1e-12)
    k, mu = 2 * np.pi, 0.3
    us = np.stack([np.sin(k * ys), 0 * xs])
    B = ns.cv_force(g, us, zero2, 0 * xs, one, 0.0, mu, box, "spectral")
    assert np.allclose(B, [mu * k * (np.cos(k * y1) - np.cos(k * y0)) * (x1 - x0), 0.0], atol=1e-12)
    B = ns.cv_force(g, zero2, np.stack([0.4 * one, -1.1 * one]), 0 * xs, one, 2.0, mu, box, "spectral")
    assert np.allclose(B, [-2.0 * 0.4 * area, 2.0 * 1.1 * area], atol=1e-12)


def test_pressure_satisfies_momentum():
    N, rho, mu, dt = 64, 1.0, 0.05, 0.01
    curve = geo.PolarCurve((0.5, 0.5), 0.15)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), 1.0 / N, 1.0)).flipped()
    kap = math.sqrt(3 * rho / (2 * dt))
    o = oracle.Setup(2, (N, N), (1.0, 1.0), (0.0, 0.0), mk.X, mk.nrm, mk.ds, "stokes", kap, mu, "dirichlet", 10.0,
                     "peskin4", "spectral")
    xs, ys = o.grid.nodes()
    gf = np.stack([np.sin(2 * np.pi * ys) + 0.3, np.cos(2 * np.pi * xs) * np.sin(4 * np.pi * ys)])
    Ub = np.stack([np.cos(mk.X[:, 1]), np.sin(mk.X[:, 0])], 1)
    q, _, _ = gmres(o.apply, o.rhs(Ub, gf), 1e-12, 300)
    u = o.recover(q, Ub, gf)
    p = ns.pressure(o, q, gf)
    from oracle import grid as G
    lap = G.laplacian_symbol(o.grid, "spectral")
    Lu = np.stack([np.real(np.fft.ifft2(mu * lap * np.fft.fft2(u[c]))) - kap ** 2 * u[c] for c in range(2)])
    Q, _ = o.split(q)
    SA = o.S(o.tensor_A(Q).reshape(o.n_ib, 4)).reshape((2, 2) + o.grid.shape)
    f = o.eta * o.S(Q) + mu * np.stack([sum(G.deriv(o.grid, SA[i, j], j, "spectral") for j in range(2))
                                        for i in range(2)])
    res = Lu - G.grad(o.grid, p, "spectral") + f - gf
    assert np.max(np.abs(res)) < 1e-9 * np.max(np.abs(gf))
