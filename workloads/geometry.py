"""Seeded, synthetic immersed-boundary geometries.

Input generators only: marker positions X, unit normals n and quadrature
weights ds for closed curves (2-D) and a closed surface (3-D).  Nothing here
evaluates the IBDL operator; both the CPU oracle and the HIP path receive
these arrays as inputs.

Conventions (thesis Sec. 2.2.2 and Sec. 5.3.1): boundary points are equally
spaced in arclength, ds = (curve length) / N_IB, and the normal of a closed
curve is its outward normal.  A caller solving an exterior problem negates it
so that n points out of the PDE domain Omega.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Markers:
    X: np.ndarray      # (n_ib, dim) positions
    nrm: np.ndarray    # (n_ib, dim) unit normals (outward of the closed curve/surface)
    ds: np.ndarray     # (n_ib,) arclength (2-D) or area (3-D) weights
    length: float      # total curve length / surface area

    @property
    def n_ib(self) -> int:
        return self.X.shape[0]

    def flipped(self) -> "Markers":
        """Same markers with the normal reversed (exterior PDE domain)."""
        return Markers(self.X.copy(), -self.nrm, self.ds.copy(), self.length)


# ---------------------------------------------------------------- 2-D curves
class PolarCurve:
    """Closed star-shaped curve r(t) = r0 * (1 + a*cos(m t + p) + b*sin(m t + p)) about c."""

    def __init__(self, center, r0, m=0, a=0.0, b=0.0, phase=0.0):
        self.c = np.asarray(center, dtype=np.float64)
        self.r0, self.m, self.a, self.b, self.p = float(r0), int(m), float(a), float(b), float(phase)

    def r(self, t):
        arg = self.m * t + self.p
        return self.r0 * (1.0 + self.a * np.cos(arg) + self.b * np.sin(arg))

    def dr(self, t):
        arg = self.m * t + self.p
        return self.r0 * self.m * (-self.a * np.sin(arg) + self.b * np.cos(arg))

    def point(self, t):
        r = self.r(t)
        return np.stack([self.c[0] + r * np.cos(t), self.c[1] + r * np.sin(t)], axis=-1)

    def tangent(self, t):
        r, dr = self.r(t), self.dr(t)
        return np.stack([dr * np.cos(t) - r * np.sin(t), dr * np.sin(t) + r * np.cos(t)], axis=-1)

    def speed(self, t):
        return np.hypot(self.r(t), self.dr(t))

    def inside(self, x, y):
        dx, dy = x - self.c[0], y - self.c[1]
        return np.hypot(dx, dy) < self.r(np.arctan2(dy, dx))

    def _arclength_table(self, nq=1 << 15):
        # trapezoid rule on a smooth periodic integrand: spectrally accurate
        t = np.arange(nq) * (2 * math.pi / nq)
        sp = self.speed(t)
        cum = np.concatenate([[0.0], np.cumsum(0.5 * (sp[1:] + sp[:-1]) * (2 * math.pi / nq))])
        total = float(np.sum(sp) * (2 * math.pi / nq))
        return t, cum, total

    def perimeter(self) -> float:
        return self._arclength_table()[2]

    def arclength(self, t):
        """s(t) by Gauss-Legendre on [0, t] (vectorised)."""
        t = np.atleast_1d(np.asarray(t, dtype=np.float64))
        xg, wg = np.polynomial.legendre.leggauss(64)
        # split [0, t] into 16 panels for accuracy on wiggly curves
        out = np.zeros_like(t)
        npan = 16
        for k in range(npan):
            a = t * k / npan
            b = t * (k + 1) / npan
            tt = 0.5 * (b - a)[:, None] * xg[None, :] + 0.5 * (a + b)[:, None]
            out += 0.5 * (b - a) * (self.speed(tt) @ wg)
        return out

    def markers(self, n_ib: int, s0: float = 0.0) -> Markers:
        """n_ib points equally spaced in arclength starting at parameter t=s0-offset 0."""
        t_tab, s_tab, P = self._arclength_table()
        s_target = (np.arange(n_ib) + s0) * (P / n_ib)
        # initial guess from the table, then Newton on s(t) = s_target
        t = np.interp(s_target, s_tab, np.concatenate([t_tab, [2 * math.pi]])[: s_tab.size])
        for _ in range(8):
            f = self.arclength(t) - s_target
            t = t - f / self.speed(t)
        X = self.point(t)
        T = self.tangent(t)
        T /= np.linalg.norm(T, axis=1, keepdims=True)
        nrm = np.stack([T[:, 1], -T[:, 0]], axis=1)      # outward for counter-clockwise t
        ds = np.full(n_ib, P / n_ib)
        return Markers(X, nrm, ds, P)


def circle(center, radius, n_ib, s0=0.0) -> Markers:
    return PolarCurve(center, radius).markers(n_ib, s0)


def star(center, r0, amp, lobes, n_ib, phase=0.0) -> Markers:
    """r(t) = r0 (1 + amp cos(lobes t + phase))."""
    return PolarCurve(center, r0, lobes, amp, 0.0, phase).markers(n_ib)


def starfish(n_ib, scale=1.0) -> Markers:
    """Thesis starfish, Sec. 5.4.2, eq. (starfish eqn): r = 1 + sin(5t)/4 about the origin."""
    return PolarCurve((0.0, 0.0), scale, 5, 0.0, 0.25).markers(n_ib)


def n_ib_for_spacing(perimeter: float, h: float, alpha: float) -> int:
    """N_IB with ds ~ alpha*h (Sec. 2.2.2)."""
    return max(8, int(round(perimeter / (alpha * h))))


# ---------------------------------------------------------------- 3-D surface
def icosphere(center, radius, freq: int) -> Markers:
    """Class-I geodesic icosphere with 10*freq^2+2 vertices projected to the sphere.

    ds_i = one third of the flat areas of the triangles around vertex i,
    rescaled so that sum(ds) = 4 pi r^2.  Normals are radial (outward).
    """
    phi = (1 + 5 ** 0.5) / 2
    V = np.array([[-1, phi, 0], [1, phi, 0], [-1, -phi, 0], [1, -phi, 0],
                  [0, -1, phi], [0, 1, phi], [0, -1, -phi], [0, 1, -phi],
                  [phi, 0, -1], [phi, 0, 1], [-phi, 0, -1], [-phi, 0, 1]], dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]])
    nu = int(freq)
    # barycentric lattice per face: points (i, j) with i + j <= nu
    ii, jj = np.meshgrid(np.arange(nu + 1), np.arange(nu + 1), indexing="ij")
    keep = ii + jj <= nu
    ii, jj = ii[keep], jj[keep]
    lat_index = -np.ones((nu + 1, nu + 1), dtype=np.int64)
    lat_index[ii, jj] = np.arange(ii.size)
    # small triangles of the lattice
    tri = []
    for i in range(nu):
        for j in range(nu - i):
            tri.append((lat_index[i, j], lat_index[i + 1, j], lat_index[i, j + 1]))
            if i + j + 1 < nu:
                tri.append((lat_index[i + 1, j], lat_index[i + 1, j + 1], lat_index[i, j + 1]))
    tri = np.array(tri, dtype=np.int64)
    pts, tris = [], []
    for f, (a, b, c) in enumerate(F):
        P = (V[a][None, :] * (nu - ii - jj)[:, None] + V[b][None, :] * ii[:, None]
             + V[c][None, :] * jj[:, None]) / nu
        pts.append(P)
        tris.append(tri + f * ii.size)
    P = np.concatenate(pts)
    T = np.concatenate(tris)
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    key = np.round(P * 1e9).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    # order unique vertices by first appearance for a stable layout
    order = np.argsort(first)
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    Pu = P[first[order]]
    Tu = rank[inv[T]]
    nv = Pu.shape[0]
    assert nv == 10 * nu * nu + 2, nv
    Xs = Pu * radius
    a, b, c = Xs[Tu[:, 0]], Xs[Tu[:, 1]], Xs[Tu[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    ds = np.zeros(nv)
    for k in range(3):
        np.add.at(ds, Tu[:, k], area / 3.0)
    total = 4 * math.pi * radius ** 2
    ds *= total / ds.sum()
    X = Xs + np.asarray(center, dtype=np.float64)[None, :]
    return Markers(X, Pu.copy(), ds, total)
