"""Eulerian grid and Lagrangian-Eulerian coupling operators S, S* and S~.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Definitions restated from the thesis:
  * grid: periodic box, nodes at origin + j h, h equal on every axis (Sec. 2.2.1);
  * spread (SF)(x) = sum_i F_i delta_h(x - X_i) ds_i (Sec. 2.2.2, eq. spread operator again2);
  * interpolate (S*u)_i = sum_x u(x) delta_h(x - X_i) h^D (Sec. 2.2.2, eq. interpolation again);
  * dipole spread S~Q = div(S(Q n)) with the divergence of the PDE discretisation (Sec. 5.3.1).
Periodicity enters through the index wrap j mod N (the box is a torus).
Grid arrays are indexed [z][y][x] (x fastest); marker coordinates are (x, y[, z]).
"""
from __future__ import annotations

import itertools

import numpy as np

from .delta import dkernel as _dkernel, kernel as _kernel


class Grid:
    def __init__(self, dim, n, L, origin):
        self.dim = int(dim)
        self.n = tuple(int(v) for v in n)
        self.L = tuple(float(v) for v in L)
        self.origin = tuple(float(v) for v in origin)
        hs = [self.L[d] / self.n[d] for d in range(self.dim)]
        if max(hs) - min(hs) > 1e-12 * max(hs):
            raise ValueError("the grid spacing must be equal on every axis")
        self.h = hs[0]

    @property
    def shape(self):
        return tuple(reversed(self.n))

    def axis(self, d):
        """numpy axis of spatial direction d in a [z][y][x] array."""
        return self.dim - 1 - d

    def nodes(self):
        axes = [self.origin[d] + self.h * np.arange(self.n[d]) for d in range(self.dim)]
        mesh = np.meshgrid(*reversed(axes), indexing="ij")
        return list(reversed(mesh))


def stencil(grid: Grid, X, kname):
    """Per marker and direction: wrapped node indices and kernel weights phi((x_j - X)/h).

    Taps j = floor(xi) - S + 1 ... floor(xi) + S with xi = (X - origin)/h and S the
    half support; every node with |x_j - X| < S h is among them.
    """
    phi, S = _kernel(kname)
    idx, w = [], []
    offs = np.arange(-S + 1, S + 1)
    for d in range(grid.dim):
        xi = (X[:, d] - grid.origin[d]) / grid.h
        b = np.floor(xi).astype(np.int64)
        j = b[:, None] + offs[None, :]
        w.append(phi(j - xi[:, None]))
        idx.append(np.mod(j, grid.n[d]))
    return idx, w


def spread(grid: Grid, X, ds, F, kname):
    """S: marker values F (n_ib,) or (n_ib, nc) -> grid field(s) (grid.shape) or (nc,)+shape."""
    F = np.asarray(F, dtype=np.float64)
    vec = F.ndim == 2
    F2 = F if vec else F[:, None]
    nc = F2.shape[1]
    idx, w = stencil(grid, X, kname)
    out = np.zeros((nc,) + grid.shape)
    ntap = idx[0].shape[1]
    scale = ds / grid.h ** grid.dim
    for taps in itertools.product(range(ntap), repeat=grid.dim):
        wt = scale.copy()
        for d, t in enumerate(taps):
            wt = wt * w[d][:, t]
        where = tuple(idx[d][:, taps[d]] for d in reversed(range(grid.dim)))
        for c in range(nc):
            np.add.at(out[c], where, F2[:, c] * wt)
    return out if vec else out[0]


def interp(grid: Grid, X, u, kname):
    """S*: grid field(s) -> marker values; h^D of the quadrature cancels h^-D of delta_h."""
    u = np.asarray(u, dtype=np.float64)
    vec = u.ndim == grid.dim + 1
    u2 = u if vec else u[None]
    idx, w = stencil(grid, X, kname)
    out = np.zeros((X.shape[0], u2.shape[0]))
    ntap = idx[0].shape[1]
    for taps in itertools.product(range(ntap), repeat=grid.dim):
        wt = np.ones(X.shape[0])
        for d, t in enumerate(taps):
            wt = wt * w[d][:, t]
        where = tuple(idx[d][:, taps[d]] for d in reversed(range(grid.dim)))
        for c in range(u2.shape[0]):
            out[:, c] += u2[c][where] * wt
    return out if vec else out[:, 0]


def _weights_dX(grid: Grid, X, kname):
    """Stencil of `stencil` plus d/dX_d of each weight: d phi((x_j - X)/h) / dX = -phi'(r) / h."""
    idx, w = stencil(grid, X, kname)
    dphi = _dkernel(kname)
    _, S = _kernel(kname)
    offs = np.arange(-S + 1, S + 1)
    dw = []
    for d in range(grid.dim):
        xi = (X[:, d] - grid.origin[d]) / grid.h
        j = np.floor(xi).astype(np.int64)[:, None] + offs[None, :]
        dw.append(-dphi(j - xi[:, None]) / grid.h)
    return idx, w, dw


def spread_dX(grid: Grid, X, ds, F, kname, dX):
    """Directional derivative d/dt S(X + t dX) F at t = 0 (S as in `spread`, ds held fixed)."""
    F = np.asarray(F, dtype=np.float64)
    vec = F.ndim == 2
    F2 = F if vec else F[:, None]
    nc = F2.shape[1]
    idx, w, dw = _weights_dX(grid, X, kname)
    out = np.zeros((nc,) + grid.shape)
    ntap = idx[0].shape[1]
    scale = ds / grid.h ** grid.dim
    for taps in itertools.product(range(ntap), repeat=grid.dim):
        dwt = np.zeros(X.shape[0])
        for e in range(grid.dim):          # product rule over the D factors
            t = np.ones(X.shape[0])
            for d, k in enumerate(taps):
                t = t * (dw[d][:, k] if d == e else w[d][:, k])
            dwt = dwt + dX[:, e] * t
        where = tuple(idx[d][:, taps[d]] for d in reversed(range(grid.dim)))
        for c in range(nc):
            np.add.at(out[c], where, F2[:, c] * scale * dwt)
    return out if vec else out[0]


def interp_dX(grid: Grid, X, u, kname, dX):
    """Directional derivative d/dt S*(X + t dX) u at t = 0."""
    u = np.asarray(u, dtype=np.float64)
    vec = u.ndim == grid.dim + 1
    u2 = u if vec else u[None]
    idx, w, dw = _weights_dX(grid, X, kname)
    out = np.zeros((X.shape[0], u2.shape[0]))
    ntap = idx[0].shape[1]
    for taps in itertools.product(range(ntap), repeat=grid.dim):
        dwt = np.zeros(X.shape[0])
        for e in range(grid.dim):
            t = np.ones(X.shape[0])
            for d, k in enumerate(taps):
                t = t * (dw[d][:, k] if d == e else w[d][:, k])
            dwt = dwt + dX[:, e] * t
        where = tuple(idx[d][:, taps[d]] for d in reversed(range(grid.dim)))
        for c in range(u2.shape[0]):
            out[:, c] += u2[c][where] * dwt
    return out if vec else out[:, 0]
