"""Pins of the oracle's gradients (CPU): kernel derivatives, derivatives of S and S* with respect
to the markers, and dL/dX, dL/ddata of the whole forward map, against central differences.

Markers are moved off the lattice by a small seeded jitter first: the 4-point kernel's second
derivative jumps at |r| = 1 and |r| = 2, and a marker placed exactly on a grid line (theta = 0
on a centred circle) would put that jump at the centre of the difference stencil.
"""
import numpy as np
import pytest

from oracle import Setup, delta
from oracle import adjoint as ADJ
from oracle.ib import Grid, interp, interp_dX, spread, spread_dX
from workloads import problems as P


@pytest.mark.parametrize("name", ["peskin4", "cos4", "bspline6"])
def test_dphi_central_difference(name):
    phi, S = delta.kernel(name)
    dphi = delta.dkernel(name)
    r = np.random.default_rng(0).uniform(-S, S, 2000)
    e = 1e-6
    fd = (phi(r + e) - phi(r - e)) / (2 * e)
    assert np.abs(fd - dphi(r)).max() < 1e-8


@pytest.mark.parametrize("name", ["peskin4", "cos4", "bspline6"])
def test_dphi_moment_identities(name):
    """d/dr of sum_j phi(r - j) = 1 gives sum_j phi'(r - j) = 0; where the first moment
    sum_j (r - j) phi(r - j) vanishes identically, sum_j (r - j) phi'(r - j) = -1."""
    _, S = delta.kernel(name)
    dphi = delta.dkernel(name)
    x = np.random.default_rng(1).uniform(0, 1, 200)
    rr = x[:, None] - np.arange(-S, S + 1)[None, :]
    assert np.abs(dphi(rr).sum(axis=1)).max() < 1e-13
    first = (rr * dphi(rr)).sum(axis=1) + 1.0
    if name == "cos4":
        assert np.abs(first).max() > 1e-2        # not first-moment exact
    else:
        assert np.abs(first).max() < 1e-13


@pytest.mark.parametrize("dim,kern", [(2, "peskin4"), (2, "bspline6"), (3, "cos4")])
def test_spread_interp_directional_derivatives(dim, kern):
    n = (16,) * dim
    grid = Grid(dim, n, (1.0,) * dim, (0.0,) * dim)
    rng = np.random.default_rng(2)
    X = rng.uniform(0, 1, (9, dim))
    ds = rng.uniform(0.5, 1.5, 9) / 16
    F = rng.standard_normal((9, 2))
    u = rng.standard_normal((2,) + grid.shape)
    dX = rng.standard_normal(X.shape)
    e = 1e-6
    fd_s = (spread(grid, X + e * dX, ds, F, kern) - spread(grid, X - e * dX, ds, F, kern)) / (2 * e)
    an_s = spread_dX(grid, X, ds, F, kern, dX)
    assert np.abs(fd_s - an_s).max() < 1e-7 * np.abs(an_s).max()
    fd_i = (interp(grid, X + e * dX, u, kern) - interp(grid, X - e * dX, u, kern)) / (2 * e)
    an_i = interp_dX(grid, X, u, kern, dX)
    assert np.abs(fd_i - an_i).max() < 1e-7 * np.abs(an_i).max()


def _jittered(spec, seed=7):
    m = spec.markers
    rng = np.random.default_rng(seed)
    h = spec.L[0] / spec.n[0]
    X = m.X + rng.uniform(-1e-3, 1e-3, m.X.shape) * h
    return Setup(spec.dim, spec.n, spec.L, spec.origin, X, m.nrm, m.ds, spec.pde, spec.kappa, spec.mu,
                 spec.bc, spec.eta, spec.kernel, spec.disc)


def _with_X(o, X):
    return Setup(o.dim, o.grid.n, o.grid.L, o.grid.origin, X, o.nrm, o.ds, o.pde, o.kappa, o.mu, o.bc,
                 o.eta, o.kernel, o.disc)


GRAD_CASES = {
    "helmholtz_fd": lambda: P.helmholtz_circle(32, 1.5),
    "helmholtz_spectral": lambda: P.helmholtz_circle(32, 1.5, disc="spectral"),
    "cos4_circle": lambda: P.ProblemSpec(**{**P.helmholtz_circle(32, 1.5).__dict__, "kernel": "cos4"}),
    "completed_poisson": lambda: P.completed_poisson_exterior(32, 2.0, 10.0, "trig"),
    "neumann": lambda: P.neumann_circle(32),
    "brinkman": lambda: P.brinkman_circle(16, 1.5),
    "stokes_exterior": lambda: P.stokes_exterior_circle(16, 10.0),
    "sphere_3d": lambda: P.cfg3_sphere(16, 2),
}


@pytest.mark.parametrize("name", sorted(GRAD_CASES))
def test_gradients_central_difference(name):
    spec = GRAD_CASES[name]()
    o = _jittered(spec)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((o.nq,) + o.grid.shape if o.nq > 1 else o.grid.shape)
    gX, gd = ADJ.gradients(o, spec.data, spec.g, psi)
    eps = 1e-6

    def LX(X):
        return ADJ.loss_value(_with_X(o, X), spec.data, spec.g, psi)

    dirs = [rng.standard_normal(o.X.shape)]
    for k in rng.choice(o.X.size, 4, replace=False):   # individual components
        v = np.zeros(o.X.size)
        v[k] = 1.0
        dirs.append(v.reshape(o.X.shape))
    scale = np.abs(gX).max()
    for v in dirs:
        fd = (LX(o.X + eps * v) - LX(o.X - eps * v)) / (2 * eps)
        assert abs(np.sum(gX * v) - fd) < 1e-6 * max(abs(fd), scale), (np.sum(gX * v), fd)
    data = np.asarray(spec.data, dtype=np.float64)
    w = rng.standard_normal(data.shape)
    fd = (ADJ.loss_value(o, data + eps * w, spec.g, psi) - ADJ.loss_value(o, data - eps * w, spec.g, psi)) / (2 * eps)
    assert abs(np.sum(gd * w.reshape(-1)) - fd) < 1e-7 * abs(fd)
