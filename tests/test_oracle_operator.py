"""Pins of the oracle's IBDL operators against what the thesis prints and what the
mathematics fixes.

* GMRES iteration counts of the thesis tables (stored under tests/golden/ with their
  section and table), +-1 where the marker phase and boundary data details are unprinted;
* closed-form solutions: first-order decrease of the error under refinement at a fixed
  physical distance from Gamma (Sec. 5.4.1, 5.7, 6.4.2, the 3-D sphere);
* the plain method's failure and the completed method's recovery on the large exterior
  domain (Sec. 5.4.3);
* the Stokes density-induced field satisfies the discrete IBDL PDE system of
  Sec. 6.1.3 (momentum with the pressure of Sec. 6.3.2, and the source continuity equation);
* GMRES agrees with a dense LU solve of the explicitly assembled operator;
* the assembled operator is well conditioned and its conditioning does not grow with N
  (second-kind equation, Sec. 3 and 5.1.1).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import grid as G
from oracle.gmres import gmres
from workloads import problems as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table(name):
    rows = {}
    for line in open(os.path.join(GOLD, name)):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        rows[int(parts[0].split("^-")[1])] = [int(v) for v in parts[1:]]
    return rows


def _solve(spec, tol=None, maxit=200):
    o = oracle.Setup.from_spec(spec)
    b = o.rhs(spec.data, spec.g)
    x, k, hist = gmres(o.apply, b, tol or spec.tol, maxit)
    return o, x, k


@pytest.mark.parametrize("N", [64, 128])
def test_helmholtz_circle_iterations(N):
    want = _table("ibdl_iterations_helmholtz_circle.txt")[int(np.log2(N))]
    got = [_solve(P.helmholtz_circle(N, a))[2] for a in (2, 1.5, 1, 0.75)]
    assert all(abs(g - w) <= 1 for g, w in zip(got, want)), (got, want)


def test_helmholtz_circle_tol_1e10():
    """Sec. 5.4.1: five GMRES iterations reach 1e-10."""
    assert _solve(P.helmholtz_circle(128, 0.75), tol=1e-10)[2] in (4, 5, 6)


def _band_error(spec, o, x, rmax):
    xs, ys = spec.nodes()
    u = o.recover(x, spec.data, spec.g)
    r = np.hypot(xs - (0.5 if spec.origin[0] == 0 else 0.0), ys - (0.5 if spec.origin[0] == 0 else 0.0))
    return np.abs(u - spec.exact(xs, ys))[..., r < rmax].max()


@pytest.mark.parametrize("data", ["sin2theta", "linear"])
def test_helmholtz_circle_first_order(data):
    errs = []
    for N in (64, 128, 256):
        s = P.helmholtz_circle(N, 0.75, data=data)
        o, x, _ = _solve(s, tol=1e-10)
        errs.append(_band_error(s, o, x, 0.22))
    assert errs[0] / errs[1] > 1.6 and errs[1] / errs[2] > 1.6, errs


@pytest.mark.parametrize("N", [64, 128])
def test_starfish_iterations(N):
    want = _table("ibdl_iterations_starfish.txt")[int(np.log2(N / 4.0))]   # dx = 4 / N
    got = [_solve(P.starfish_poisson(N, a))[2] for a in (2, 0.75)]
    assert all(abs(g - w) <= 1 for g, w in zip(got, want)), (got, want)


def test_neumann_iterations_and_convergence():
    its, eu, eb = [], [], []
    for N in (64, 128, 256):
        s = P.neumann_circle(N)
        o, x, k = _solve(s)
        its.append(k)
        xs, ys = s.nodes()
        u = o.recover(x, s.data, s.g)
        r = np.hypot(xs, ys)
        eu.append(np.abs(u - s.exact(xs, ys))[r < 0.2].max())
        eb.append(np.abs(x - s.exact(s.markers.X[:, 0], s.markers.X[:, 1])).max())
    assert all(4 <= k <= 6 for k in its), its           # Sec. 5.7: 4-6 iterations
    assert eu[0] / eu[1] > 1.6 and eu[1] / eu[2] > 1.6, eu
    assert eb[0] / eb[1] > 1.6 and eb[1] / eb[2] > 1.6, eb


@pytest.mark.parametrize("N", [64, 128])
def test_brinkman_iterations(N):
    want = _table("ibdl_iterations_brinkman.txt")[int(np.log2(N / 2.0))]
    got = [_solve(P.brinkman_circle(N, a))[2] for a in (2, 1.5, 1, 0.75)]
    assert all(abs(g - w) <= 1 for g, w in zip(got, want)), (got, want)


def test_stokes_exterior_completed():
    """Sec. 6.4.2: completed IBDL for exterior Stokes.  First order in u, iteration counts
    independent of N, more iterations at eta = 100 than at eta = 10.  (The thesis quotes
    about 8 and 13 iterations; with the printed border rows the oracle needs 15-16 and
    25-27.  The next test shows where the difference comes from.)"""
    errs, its10, its100 = [], [], []
    for N in (32, 64, 128):
        s = P.stokes_exterior_circle(N, 10.0)
        o, x, k = _solve(s)
        its10.append(k)
        xs, ys = s.nodes()
        u = o.recover(x, s.data, s.g)
        r = np.hypot(xs, ys)
        errs.append(np.abs(u - s.exact(xs, ys))[:, r > 0.85].max())
        its100.append(_solve(P.stokes_exterior_circle(N, 100.0))[2])
    assert errs[0] / errs[1] > 1.6 and errs[1] / errs[2] > 1.6, errs
    assert max(its10) - min(its10) <= 1 and max(its10) <= 20, its10
    assert min(its100) > max(its10), (its10, its100)


def test_stokes_exterior_count_without_bordered_rows():
    """Sec. 6.4.2 prints about 8 GMRES iterations at eta = 10 for the completed exterior
    problem.  The same completed operator with an invertible grid operator (Brinkman
    k = 0.01: no u-bar unknowns, no border rows) takes 8 +- 1 on this data.  At k = 0 the
    border rows eta sum_i ds_i Q_i and the u-bar columns add a pair of eigenvalues per
    component, (l0 +- sqrt(l0^2 + 4 eta sum ds)) / 2 with l0 the Rayleigh quotient of a
    constant density (here about 7.26 and -6.50, far from the cluster near 1/2), and these
    cost GMRES the extra iterations (15-16 in all)."""
    its = _solve(P.stokes_exterior_circle(64, 10.0, k=0.01))[2]
    assert abs(its - 8) <= 1, its
    s = P.stokes_exterior_circle(32, 10.0)
    o = oracle.Setup.from_spec(s)
    A = o.assemble()
    ev = np.linalg.eigvals(A)
    n = o.n_ib
    for d in range(2):
        e = np.zeros(o.n_aug)
        e[d:2 * n:2] = 1.0
        l0 = e @ A @ e / (e @ e)
        c = 10.0 * o.ds.sum()
        for lam in ((l0 + np.sqrt(l0 * l0 + 4 * c)) / 2, (l0 - np.sqrt(l0 * l0 + 4 * c)) / 2):
            assert np.min(np.abs(ev - lam)) < 0.01 * abs(lam), (lam, np.sort(ev.real)[[0, 1, -2, -1]])
    k0 = _solve(P.stokes_exterior_circle(64, 10.0))[2]
    assert k0 - its >= 4, (k0, its)


def test_completed_poisson_large_exterior():
    """Sec. 5.4.3: plain IBDL fails on [-4, 4]^2 for u = exp(sin(2 pi x / L)); eta = 10 converges."""
    plain, done = [], []
    for N in (128, 256):
        for eta, out in ((0.0, plain), (10.0, done)):
            s = P.completed_poisson_exterior(N, 8.0, eta, "exp")
            o, x, _ = _solve(s)
            xs, ys = s.nodes()
            u = o.recover(x, s.data, s.g)
            m = np.hypot(xs, ys) > 0.5
            out.append(np.abs(u - s.exact(xs, ys))[m].max())
    assert min(plain) > 0.5
    assert done[0] < 0.01 and done[0] / done[1] > 1.6, done


def test_sphere_3d_first_order():
    errs = []
    for N, freq in ((32, 11), (64, 22)):
        s = P.cfg3_sphere(N, freq)
        o, x, k = _solve(s)
        assert k <= 10
        xs, ys, zs = s.nodes()
        u = o.recover(x, s.data, s.g)
        r = np.sqrt((xs - .5) ** 2 + (ys - .5) ** 2 + (zs - .5) ** 2)
        errs.append(np.abs(u - s.exact(xs, ys, zs))[r < 0.2].max())
    assert errs[0] / errs[1] > 1.6, errs


@pytest.mark.parametrize("k,eta", [(1.0, 0.0), (0.0, 10.0)])
def test_stokes_field_solves_ibdl_pde(k, eta):
    """u[Q] with p = -Delta_0^-1 L S(Q.n) + Delta_0^-1 div(eta S Q + mu div S A) satisfies
    mu Delta u - k^2 u - grad p + eta S Q + mu div(S A) = 0 and div u + S(Q.n) = 0
    (off the Nyquist lines and the mean mode, whose balance is the solvability constraint that
    the border rows carry)."""
    s = P.stokes_exterior_circle(32, eta, k=k)
    o = oracle.Setup.from_spec(s)
    g = o.grid
    Q = np.random.default_rng(8).standard_normal((o.n_ib, 2))
    u = o.u_of_q(Q)
    sQn = o.S(np.sum(Q * o.nrm, axis=1))
    SA = o.S(o.tensor_A(Q).reshape(o.n_ib, 4)).reshape((2, 2) + g.shape)
    divSA = np.stack([G.deriv(g, SA[i, 0], 0, "spectral") + G.deriv(g, SA[i, 1], 1, "spectral")
                      for i in range(2)])
    src = eta * o.S(Q) + o.mu * divSA
    Ls = o.mu * G.laplacian(g, sQn, "spectral") - k ** 2 * sQn
    p = -G.solve(g, Ls, "spectral", 0.0) + G.solve(g, G.div(g, src, "spectral"), "spectral", 0.0)
    mom = np.stack([o.mu * G.laplacian(g, u[i], "spectral") - k ** 2 * u[i] for i in range(2)]) \
        - G.grad(g, p, "spectral") + src
    cont = G.div(g, u, "spectral") + sQn

    def off_nyquist(f):
        fh = np.fft.fft2(f)
        fh[..., 16, :] = 0.0
        fh[..., :, 16] = 0.0
        fh[..., 0, 0] = 0.0
        return np.abs(fh).max()
    scale = np.abs(np.fft.fft2(src)).max()
    assert off_nyquist(mom) < 1e-10 * scale
    assert off_nyquist(cont) < 1e-10 * np.abs(np.fft.fft2(sQn)).max()


@pytest.mark.parametrize("builder", [
    lambda: P.helmholtz_circle(32, 1.0),
    lambda: P.neumann_circle(32),
    lambda: P.completed_poisson_exterior(32, 2.0, 10.0, "trig"),
    lambda: P.stokes_exterior_circle(16, 10.0),
    lambda: P.brinkman_circle(16, 1.0),
])
def test_gmres_matches_dense(builder):
    s = builder()
    o = oracle.Setup.from_spec(s)
    A = o.assemble()
    b = o.rhs(s.data, s.g)
    xd = np.linalg.solve(A, b)
    xg, k, _ = gmres(o.apply, b, 1e-13, 400)
    np.testing.assert_allclose(xg, xd, rtol=0, atol=1e-10 * np.abs(xd).max())
    # the assembled matrix is the operator: A q == apply(q) for a random q
    q = np.random.default_rng(1).standard_normal(o.n_aug)
    np.testing.assert_allclose(A @ q, o.apply(q), atol=1e-12 * np.abs(A @ q).max())


def test_second_kind_conditioning():
    conds = []
    for N in (32, 64):
        o = oracle.Setup.from_spec(P.helmholtz_circle(N, 1.0))
        conds.append(np.linalg.cond(o.assemble()))
    assert max(conds) < 20 and conds[1] < 1.5 * conds[0], conds
