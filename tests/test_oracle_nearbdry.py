"""Pins of the oracle's indicator function and near-boundary interpolation (2-D).

* the nearest markers against a k-d tree query (a library routine);
* x_A is the closest point of the segment [x1, x2] to p (checked against a dense sample of it);
* the bilinear sample reproduces bilinear functions exactly;
* every step of the interpolation is exact for linear functions, so a field that is linear
  except on the near-boundary points is restored to the linear function there;
* the width rules give the values the thesis states: 6 and 8 with finite differences, and with
  spectral symbols m1 from 4 to 20 over N = 64 ... 16384, growing by 2 per doubling, m2 = m1 + 2;
* the indicator of a circle equals the closed-form inside test at distance of more than 2h from
  the circle, and the regularized field is close to 1/2 on the markers;
* on the thesis's linear-solution Helmholtz problem (Sec. 5.5: Delta u - u = -(x+y) in the disk,
  u = x + y on the circle), the interpolation lowers the maximum error over Omega to the interior
  error level.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from oracle import nearbdry as NB
from oracle.gmres import gmres
from oracle.ib import Grid
from workloads import problems as P


def test_width_rules():
    assert NB.widths("fd2", 1024) == (6.0, 8.0)
    assert NB.widths("spectral", 64) == (4.0, 6.0)
    assert NB.widths("spectral", 16384) == (20.0, 22.0)
    for k in range(6, 14):
        a, b = NB.widths("spectral", 2 ** k), NB.widths("spectral", 2 ** (k + 1))
        assert b[0] - a[0] == 2.0 and b[1] == b[0] + 2.0


def test_nearest_markers_match_kdtree():
    rng = np.random.default_rng(0)
    X = rng.uniform(0, 1, (500, 2))
    tree = cKDTree(X)
    for _ in range(50):
        p = rng.uniform(0, 1, 2)
        idx, d2 = NB.nearest_markers(X, p, 3)
        dd, ii = tree.query(p, k=3)
        assert list(idx) == list(ii)
        assert np.allclose(np.sqrt(d2), dd, rtol=0, atol=1e-15)


def test_segment_point_is_closest():
    rng = np.random.default_rng(1)
    s = np.linspace(0.0, 1.0, 20001)
    for _ in range(40):
        x1, x2, p = rng.normal(size=(3, 2))
        xa, t = NB.segment_point(p, x1, x2)
        seg = x2[None, :] + s[:, None] * (x1 - x2)[None, :]
        dmin = np.min(np.linalg.norm(seg - p[None, :], axis=1))
        assert np.linalg.norm(xa - p) <= dmin + 1e-12
        # x_A on the segment, and t the unclamped line parameter
        assert np.isclose(np.linalg.norm(xa - x1) + np.linalg.norm(xa - x2), np.linalg.norm(x1 - x2))
        line = x2 + t * (x1 - x2)
        assert abs(np.dot(p - line, x1 - x2)) < 1e-12 * (1 + np.linalg.norm(p))


def test_bilinear_reproduces_bilinear_functions():
    g = Grid(2, (32, 32), (1.0, 1.0), (0.0, 0.0))
    xs, ys = g.nodes()
    rng = np.random.default_rng(2)
    a, b, c, d = rng.normal(size=4)
    u = a + b * xs + c * ys + d * xs * ys
    for _ in range(30):
        p = rng.uniform(0.1, 0.85, 2)
        want = a + b * p[0] + c * p[1] + d * p[0] * p[1]
        assert abs(NB.bilinear(g, u, p) - want) < 1e-13


@pytest.mark.parametrize("N", [64, 128])
def test_interpolation_exact_for_linear_fields(N):
    s = P.helmholtz_circle(N, 0.75, data="linear")
    g = Grid(s.dim, s.n, s.L, s.origin)
    xs, ys = g.nodes()
    X = s.markers.X
    chi = (np.hypot(xs, ys) < 0.25).astype(np.float64)
    a, b, c = 0.3, -1.2, 0.7
    lin = a + b * xs + c * ys
    pts = NB.near_points(g, X, chi, 6)
    assert len(pts) > 100
    u = lin.copy()
    rng = np.random.default_rng(3)
    for j, i in pts:
        u[j, i] += rng.normal()
    Ub = a + b * X[:, 0] + c * X[:, 1]
    out = NB.near_boundary(g, X, Ub, chi, u, 6, 8)
    jj, ii = np.array(pts).T
    assert np.max(np.abs(out[jj, ii] - lin[jj, ii])) < 1e-12
    # points that are not near the boundary keep their values
    mask = np.ones(u.shape, dtype=bool)
    mask[jj, ii] = False
    assert np.array_equal(out[mask], u[mask])


def test_near_points_are_within_m1_of_the_markers():
    s = P.helmholtz_circle(64, 0.75)
    g = Grid(s.dim, s.n, s.L, s.origin)
    xs, ys = g.nodes()
    chi = (np.hypot(xs, ys) < 0.25).astype(np.float64)
    pts = set(NB.near_points(g, s.markers.X, chi, 6))
    # the markers lie on the circle r = 1/4 within a fraction of h, so inside points with
    # 1/4 - r < 5.5h are near and those with 1/4 - r > 6.5h are not
    h = g.h
    r = np.hypot(xs, ys)
    for j in range(g.n[1]):
        for i in range(g.n[0]):
            if r[j, i] < 0.25 and 0.25 - r[j, i] < 5.5 * h:
                assert (j, i) in pts
            if r[j, i] < 0.25 - 6.5 * h:
                assert (j, i) not in pts


@pytest.mark.parametrize("disc", ["fd2", "spectral"])
def test_indicator_of_a_circle(disc):
    s = P.helmholtz_circle(64, 0.75, disc=disc)
    g = Grid(s.dim, s.n, s.L, s.origin)
    m = s.markers
    chi = NB.indicator(g, m.X, m.nrm, m.ds, s.kernel, disc)
    xs, ys = g.nodes()
    r = np.hypot(xs, ys)
    far = np.abs(r - 0.25) > 2 * g.h
    assert np.array_equal(chi[far], (r[far] < 0.25).astype(np.float64))
    reg = NB.indicator(g, m.X, m.nrm, m.ds, s.kernel, disc, regularized=True)
    # regularized field: ~1 deep inside, ~0 outside, ~1/2 on the markers
    assert abs(np.median(reg[r < 0.15]) - 1.0) < 0.02
    assert abs(np.median(reg[r > 0.35]) - 0.0) < 0.02
    on = oracle.ib.interp(g, m.X, reg, s.kernel)
    assert abs(np.median(on) - 0.5) < 0.05


def test_interpolation_reduces_max_error_of_linear_problem():
    """Sec. 5.5, eq. (pde again 2) with FD symbols, m1 = 6, m2 = 8: the near-boundary errors,
    which the discontinuity across Gamma keeps at O(1) h^0 scale without the interpolation,
    drop to the size of the interior error."""
    s = P.helmholtz_circle(128, 0.75, data="linear")
    o = oracle.Setup.from_spec(s)
    q, _, _ = gmres(o.apply, o.rhs(s.data, s.g), 1e-12, 200)
    u = o.recover(q, s.data, s.g)
    g = o.grid
    xs, ys = g.nodes()
    r = np.hypot(xs, ys)
    omega = r < 0.25
    exact = s.exact(xs, ys)
    chi = NB.indicator(g, s.markers.X, s.markers.nrm, s.markers.ds, s.kernel, s.disc)
    assert np.array_equal(chi[np.abs(r - 0.25) > 2 * g.h], omega[np.abs(r - 0.25) > 2 * g.h])
    before = np.max(np.abs(u - exact)[omega & (chi == 1)])
    fixed = NB.near_boundary(g, s.markers.X, s.data, chi, u, 6, 8)
    after = np.max(np.abs(fixed - exact)[omega & (chi == 1)])
    interior = np.max(np.abs(u - exact)[r < 0.25 - 8 * g.h])
    assert after < 0.5 * before, (before, after)
    assert after < 3 * interior, (after, interior)
