"""GPU parity of the Navier-Stokes pieces (ibdl_advection, ibdl_ns_step, the vector near-boundary
interpolation) against the oracle (oracle/ns.py), and the exact decaying shear wave.

Tolerances: the nonlinear term 1e-12 (FP64) / 2e-5 (mixed) relative to its max-norm; a run of
steps at GMRES tol 1e-12 (FP64) 1e-9 relative in u and N against the oracle's run; the shear wave
within 1e-3 of the exact solution away from the body (as the oracle's pin)."""
import math

import numpy as np
import pytest
import torch

import paper_2210_07403_amd as ibdl
import oracle
from oracle import nearbdry as NB
from oracle import ns
from workloads import geometry as geo

from _helpers import to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]


def _setup(N, rho, mu, dt, eta=10.0, center=(0.5, 0.5), r=0.15, disc="spectral", precision="fp64"):
    curve = geo.PolarCurve(center, r)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), 1.0 / N, 1.0)).flipped()
    kap = math.sqrt(3 * rho / (2 * dt))
    o = oracle.Setup(2, (N, N), (1.0, 1.0), (0.0, 0.0), mk.X, mk.nrm, mk.ds, "stokes", kap, mu, "dirichlet", eta,
                     "peskin4", disc)
    pr = ibdl.Problem(2, (N, N), (1.0, 1.0), (0.0, 0.0), mk.X, mk.nrm, mk.ds, pde="stokes", kappa=kap, mu=mu, eta=eta,
                      kernel="peskin4", disc=disc, precision=precision)
    return mk, o, pr


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("disc", ["spectral", "fd2"])
def test_advection_matches_oracle(disc, precision):
    mk, o, pr = _setup(64, 1.0, 0.05, 0.01, disc=disc, precision=precision)
    xs, ys = o.grid.nodes()
    rng = np.random.default_rng(4)
    u = np.stack([np.sin(2 * np.pi * ys) + 0.3 * np.cos(4 * np.pi * xs), np.cos(2 * np.pi * xs) * np.sin(2 * np.pi * ys)])
    u = u + 0.05 * rng.standard_normal(u.shape)
    dt_ = np.float64 if precision == "fp64" else np.float32
    u = u.astype(dt_).astype(np.float64)
    got = to_np(pr.advection(u))
    want = ns.advection(o.grid, u, disc)
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert np.max(np.abs(got - want)) < tol * np.max(np.abs(want))
    pr.close()


def test_vector_near_boundary_matches_oracle():
    mk, o, pr = _setup(128, 1.0, 0.05, 0.01)
    xs, ys = o.grid.nodes()
    omega = (np.hypot(xs - 0.5, ys - 0.5) >= 0.15).astype(np.float64)
    u = np.stack([np.sin(3 * xs + 1) * np.cos(2 * ys), np.cos(xs) + ys])
    Ub = np.random.default_rng(2).standard_normal((mk.X.shape[0], 2))
    got = to_np(pr.near_boundary(Ub, omega, u, 3, 4))
    for c in range(2):
        want = NB.near_boundary(o.grid, mk.X, Ub[:, c], omega, u[c], 3, 4)
        assert np.max(np.abs(got[c] - want)) < 1e-12 * np.max(np.abs(want))
    pr.close()


def _run_pair(N, nsteps, rho, mu, dt, u_inf, strip, m1, m2):
    mk, o, pr = _setup(N, rho, mu, dt, center=(0.4, 0.5), r=0.1)
    xs, ys = o.grid.nodes()
    omega = (np.hypot(xs - 0.4, ys - 0.5) >= 0.1).astype(np.float64)
    u0 = np.stack([u_inf + 0.1 * np.sin(2 * np.pi * ys), 0.05 * np.sin(2 * np.pi * xs)])
    Ub = np.zeros((mk.X.shape[0], 2))
    # oracle run
    un, unm1 = u0.copy(), u0.copy()
    Nn = ns.advection(o.grid, un, "spectral")
    Nnm1 = Nn.copy()
    its = []
    for _ in range(nsteps):
        q, u, Nu, it = ns.step(o, Ub, un, unm1, Nn, Nnm1, rho, dt, omega, m1, m2, strip, u_inf, tol=1e-12)
        unm1, un, Nnm1, Nn = un, u, Nn, Nu
        its.append(it)
    # GPU run
    dev = pr.device
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    state = [t(u0), t(u0), t(ns.advection(o.grid, u0, "spectral")), t(ns.advection(o.grid, u0, "spectral"))]
    gits = []
    for _ in range(nsteps):
        qg, info = pr.ns_step(state, Ub, rho, dt, omega, m1, m2, strip, u_inf, tol=1e-12, maxit=200)
        assert info.status == 0
        gits.append(info.iters)
    pr.close()
    return (un, Nn, unm1, q, its), ([to_np(s) for s in state], to_np(qg), gits)


def test_ns_steps_match_oracle():
    (un, Nn, unm1, q, its), (st, qg, gits) = _run_pair(64, 4, 1.0, 0.02, 0.01, 1.0, 4, 3, 4)
    u_prev, u, n_prev, n = st
    assert all(abs(a - b) <= 1 for a, b in zip(its, gits)), (its, gits)
    for got, want in ((u, un), (u_prev, unm1), (n, Nn)):
        assert np.max(np.abs(got - want)) < 1e-9 * np.max(np.abs(want))
    assert np.max(np.abs(qg - q)) < 1e-8 * np.max(np.abs(q))
    assert np.all(u[0][:, :4] == 1.0) and np.all(u[1][:, :4] == 0.0)


def test_shear_wave_on_the_gpu():
    N, dt, nsteps, rho, mu, k = 128, 0.01, 20, 1.0, 0.05, 2 * math.pi
    mk, o, pr = _setup(N, rho, mu, dt)
    xs, ys = o.grid.nodes()
    nu = mu / rho

    def exact(t, x, y):
        return np.stack([np.exp(-nu * k * k * t) * np.sin(k * y), 0 * x])

    r = np.hypot(xs - 0.5, ys - 0.5)
    omega = (r >= 0.15).astype(np.float64)
    dev = pr.device
    tt = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    u0, um = exact(0.0, xs, ys), exact(-dt, xs, ys)
    state = [tt(um), tt(u0), pr.advection(um), pr.advection(u0)]
    for s in range(nsteps):
        Ub = exact((s + 1) * dt, mk.X[:, 0], mk.X[:, 1]).T
        _, info = pr.ns_step(state, Ub, rho, dt, omega, 3, 4, tol=1e-10, maxit=200)
        assert info.status == 0
    u = to_np(state[1])
    assert np.max(np.abs(u - exact(nsteps * dt, xs, ys))[:, r > 0.3]) < 1e-3
    pr.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pressure_matches_oracle(precision):
    rho, mu, dt = 1.0, 0.05, 0.01
    mk, o, pr = _setup(64, rho, mu, dt, precision=precision)
    xs, ys = o.grid.nodes()
    gf = np.stack([np.sin(2 * np.pi * ys) + 0.3, np.cos(2 * np.pi * xs) * np.sin(4 * np.pi * ys)])
    Ub = np.stack([np.cos(mk.X[:, 1]), np.sin(mk.X[:, 0])], 1)
    q, _, info = pr.solve(Ub, gf, tol=1e-12 if precision == "fp64" else 1e-6, maxit=200)
    qn = to_np(q)
    gd = gf.astype(np.float64 if precision == "fp64" else np.float32).astype(np.float64)
    got = to_np(pr.pressure(q, gf))
    want = ns.pressure(o, qn, gd)
    tol = 1e-10 if precision == "fp64" else 2e-5
    assert np.max(np.abs(got - want)) < tol * np.max(np.abs(want))
    pr.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cv_force_matches_oracle(precision):
    mk, o, pr = _setup(64, 1.0, 0.05, 0.01, precision=precision)
    xs, ys = o.grid.nodes()
    dt_ = np.float64 if precision == "fp64" else np.float32
    rnd = lambda a: a.astype(dt_).astype(np.float64)
    u = rnd(np.stack([1 + 0.3 * np.sin(2 * np.pi * ys) * np.cos(2 * np.pi * xs), 0.2 * np.sin(4 * np.pi * xs)]))
    up = rnd(u - 0.01 * np.stack([np.cos(2 * np.pi * xs), np.sin(2 * np.pi * ys)]))
    ut = (u - up) / 0.01
    p = rnd(np.sin(2 * np.pi * (xs + ys)))
    omega = (np.hypot(xs - 0.5, ys - 0.5) >= 0.15).astype(np.float64)
    box = (8, 55, 6, 50)
    got = to_np(pr.cv_force(u, up, 0.01, p, omega, 1.3, box))
    want = ns.cv_force(o.grid, u, ut, p, omega, 1.3, 0.05, box, "spectral")
    tol = 1e-11 if precision == "fp64" else 2e-5
    assert np.max(np.abs(got - want)) < tol * (1 + np.max(np.abs(want)))
    steady = to_np(pr.cv_force(u, None, 0.0, p, omega, 1.3, box))
    want0 = ns.cv_force(o.grid, u, 0 * ut, p, omega, 1.3, 0.05, box, "spectral")
    assert np.max(np.abs(steady - want0)) < tol * (1 + np.max(np.abs(want0)))
    pr.close()


def test_rejects():
    mk, o, pr = _setup(64, 1.0, 0.05, 0.01)
    z = [torch.zeros((2, 64, 64), dtype=torch.float64, device=pr.device) for _ in range(4)]
    with pytest.raises(ibdl.IBDLError):   # kappa^2 != 3 rho / (2 dt)
        pr.ns_step(z, np.zeros((mk.X.shape[0], 2)), 1.0, 0.02)
    with pytest.raises(ibdl.IBDLError):   # aliased state
        pr.ns_step([z[0], z[0], z[2], z[3]], np.zeros((mk.X.shape[0], 2)), 1.0, 0.01)
    pr.close()
    spec_pr = ibdl.Problem(2, (64, 64), (1.0, 1.0), (0.0, 0.0), mk.X, mk.nrm, mk.ds, pde="screened", kappa=1.0)
    with pytest.raises(ibdl.IBDLError):
        spec_pr.advection(np.zeros((2, 64, 64)))
    spec_pr.close()


def test_step_from_rest_stays_at_rest():
    """u = 0 with U_b = 0 and no strip: the forcing, the solve and the nonlinear term are all zero."""
    mk, o, pr = _setup(64, 1.0, 0.05, 0.01)
    z = [torch.zeros((2, 64, 64), dtype=torch.float64, device=pr.device) for _ in range(4)]
    g = torch.ones_like(z[0])
    q, info = pr.ns_step(z, np.zeros((mk.X.shape[0], 2)), 1.0, 0.01, None, 0, 0, 0, 0.0, g_out=g)
    assert info.status == 0 and info.iters == 0
    assert all(bool(torch.all(t == 0)) for t in z) and bool(torch.all(g == 0))
    assert bool(torch.all(q == 0))
    pr.close()
