"""Indicator function of the discretized boundary and the near-boundary interpolation (2-D).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Indicator (Sec. 5.3.4, flagging interior points): the indicator chi of the interior of Gamma
satisfies Delta chi + div(delta n) = 0; regularized, Delta chi + S~ 1 = 0 with S~ the IBDL dipole
spread of the constant density 1.  On the periodic box the mean-zero solution is taken, shifted
so that the value at the box corner (the node at the origin) is 0, which leaves about 1/2 on
Gamma; values of at least 1/2 are flagged 1 (interior), the others 0.

Near-boundary interpolation (Sec. 5.3.3, interpolation for near-boundary points), for a grid
point p of Omega (chi = 1) within m1 meshwidths of Gamma (distance to the nearest marker):
  1. x1, x2 = the two nearest markers; x_A = the point of the segment [x1, x2] closest to p;
     when the projection falls outside the segment, the third nearest marker is added and the two
     of the three farthest apart are used instead (and the projection is clamped to the segment);
  2. u(x_A) = U_b(x1) |x_A - x2| / |x2 - x1| + U_b(x2) |x_A - x1| / |x2 - x1|;
  3. x_B = x_A + m2 h (p - x_A) / |p - x_A|, and u(x_B) by bilinear interpolation of the grid
     values at the four nodes around x_B;
  4. u(p) = u(x_A) |x_B - p| / |x_B - x_A| + u(x_B) |x_A - p| / |x_B - x_A|
     (u(x_A) itself when p lies on the segment).
The bilinear samples read the uncorrected field.  Ties between equally distant markers go to the
lower marker index.

Widths (Sec. 5.5, interpolation widths): m1 = 6, m2 = 8 with finite differences; with Fourier
spectral symbols m1 grows by 2 per doubling of N, m1 = 2 (log2 N - 4), and m2 = m1 + 2.

Parity: pinned by tests/test_oracle_nearbdry.py (exactness on linear fields, geometric properties
of x_A and x_B, nearest markers against brute force, the indicator of a circle against its closed
form away from the boundary).
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from .ib import Grid, spread


def widths(disc: str, N: int):
    """(m1, m2) of the thesis's rules for a grid of N points per side; at least m1 = 2 on coarse
    spectral grids (N < 32), where the logarithmic rule would give no width at all."""
    if disc == "fd2":
        return 6.0, 8.0
    m1 = max(2.0 * (np.log2(N) - 4.0), 2.0)
    return m1, m1 + 2.0


def indicator(grid: Grid, X, nrm, ds, kernel: str, disc: str, regularized: bool = False):
    """chi on the grid ([y][x]); with regularized=True the shifted field before thresholding."""
    X = np.asarray(X, dtype=np.float64)
    if grid.dim != 2:
        raise ValueError("the near-boundary tools are two-dimensional")
    ones = np.ones(X.shape[0])
    stilde = G.div(grid, spread(grid, X, ds, ones[:, None] * nrm, kernel), disc)
    chi = -G.solve(grid, stilde, disc, 0.0)       # Delta chi = -S~ 1, mean zero
    chi = chi - chi[0, 0]                          # the corner node is exterior: value 0
    if regularized:
        return chi
    return (chi >= 0.5).astype(np.float64)


def nearest_markers(X, p, k=3):
    """Indices of the k markers nearest to p, by (squared distance dx^2 + dy^2, index)."""
    dx = X[:, 0] - p[0]
    dy = X[:, 1] - p[1]
    d2 = dx * dx + dy * dy
    order = np.lexsort((np.arange(len(d2)), d2))
    return order[:k], d2[order[:k]]


def segment_point(p, x1, x2):
    """Closest point to p on the segment [x1, x2] and the unclamped line parameter t (x_A =
    x2 + t (x1 - x2)), in plain scalar arithmetic."""
    d0, d1 = float(x1[0] - x2[0]), float(x1[1] - x2[1])
    num = (float(p[0]) - float(x2[0])) * d0 + (float(p[1]) - float(x2[1])) * d1
    t = num / (d0 * d0 + d1 * d1)
    tc = min(max(t, 0.0), 1.0)
    return np.array([x2[0] + tc * d0, x2[1] + tc * d1]), t


def bilinear(grid: Grid, u, xb):
    """Bilinear interpolation of u ([y][x], periodic) at the point xb."""
    h = grid.h
    fx = (xb[0] - grid.origin[0]) / h
    fy = (xb[1] - grid.origin[1]) / h
    i0, j0 = int(np.floor(fx)), int(np.floor(fy))
    ax, ay = fx - i0, fy - j0
    nx, ny = grid.n[0], grid.n[1]
    u00 = u[j0 % ny, i0 % nx]
    u10 = u[j0 % ny, (i0 + 1) % nx]
    u01 = u[(j0 + 1) % ny, i0 % nx]
    u11 = u[(j0 + 1) % ny, (i0 + 1) % nx]
    return ax * ay * u11 + ay * (1.0 - ax) * u01 + ax * (1.0 - ay) * u10 + (1.0 - ax - ay + ax * ay) * u00


def correct_point(grid: Grid, X, Ub, u, p, m2):
    """The interpolated value at grid point p (steps 1-4 above)."""
    idx, _ = nearest_markers(X, p, 3)
    a, b = idx[0], idx[1]
    xa, t = segment_point(p, X[a], X[b])
    if not (0.0 <= t <= 1.0) and len(idx) >= 3:
        pairs = [(idx[0], idx[1]), (idx[0], idx[2]), (idx[1], idx[2])]
        sep = [np.sum((X[i] - X[j]) ** 2) for i, j in pairs]
        a, b = pairs[int(np.argmax(sep))]
        xa, t = segment_point(p, X[a], X[b])
    x1, x2 = X[a], X[b]
    L12 = np.linalg.norm(x2 - x1)
    uA = Ub[a] * np.linalg.norm(xa - x2) / L12 + Ub[b] * np.linalg.norm(xa - x1) / L12
    dpa = np.linalg.norm(p - xa)
    if dpa == 0.0:
        return uA
    xb = xa + (p - xa) / dpa * (m2 * grid.h)
    uB = bilinear(grid, u, xb)
    dab = np.linalg.norm(xb - xa)
    return uA * np.linalg.norm(xb - p) / dab + uB * dpa / dab


def near_points(grid: Grid, X, chi, m1):
    """Grid points of Omega (chi = 1) within m1 h of the nearest marker: list of (j, i)."""
    xs, ys = grid.nodes()
    out = []
    for j in range(grid.n[1]):
        for i in range(grid.n[0]):
            if chi[j, i] != 1.0:
                continue
            p = np.array([xs[j, i], ys[j, i]])
            dx = X[:, 0] - p[0]
            dy = X[:, 1] - p[1]
            d2 = np.min(dx * dx + dy * dy)
            if d2 <= (m1 * grid.h) ** 2:
                out.append((j, i))
    return out


def near_boundary(grid: Grid, X, Ub, chi, u, m1, m2):
    """u with every near-boundary point of Omega replaced by its interpolated value."""
    X = np.asarray(X, dtype=np.float64)
    Ub = np.asarray(Ub, dtype=np.float64)
    xs, ys = grid.nodes()
    out = np.array(u, dtype=np.float64, copy=True)
    for j, i in near_points(grid, X, chi, m1):
        out[j, i] = correct_point(grid, X, Ub, u, np.array([xs[j, i], ys[j, i]]), m2)
    return out
