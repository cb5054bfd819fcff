"""The Immersed Boundary Single Layer (IBSL) method: Schur complements of Chapter 2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Unknowns q = [F_0, ..., F_{n-1}] (scalars, or [n_ib][D] for Brinkman / Stokes), followed by u_bar
(1 or D values) when the grid operator is the singular periodic one (kappa = 0).  With
L = Delta - kappa^2 (scalar) or mu Delta - k^2 (vector) and the mean-zero inverse where L is
singular:
  * scalar, Sec. 2.2.3 eq. (schur complement again):  -S* L^-1 S F = U_b - S* L^-1 g~;
  * Poisson, Sec. 2.2.4 eq. (poisson schur system 2):
      [-S* Delta_0^-1 S F + u_bar 1;  1^T F] = [U_b - S* Delta_0^-1 g~;  (h^D / ds) 1^T g~];
  * Brinkman, Sec. 2.3.1 eq. (brink schur): -S* L^-1 P S F = U_b - S* L^-1 P g~;
  * Stokes, Sec. 2.3.2 eq. (stokes schur): the Poisson pattern with -(1/mu) S* Delta_0^-1 P S and
    D border rows.
The thesis has equal spacings ds; for unequal ones the border rows weigh F_i by ds_i / mean(ds)
(and the right-hand side divides by mean(ds)), which keeps the system self-adjoint in the
inner product with those weights (1 on u_bar), the one MINRES then uses.
Grid solution: u = L^-1 (g~ - S F) (P in front for the vector cases) + u_bar.
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from .ib import Grid, interp, spread


class IBSL:
    def __init__(self, dim, n, L, origin, X, ds, pde, kappa, mu, kernel, disc):
        self.grid = Grid(dim, n, L, origin)
        self.dim = dim
        self.X = np.asarray(X, dtype=np.float64)
        self.ds = np.asarray(ds, dtype=np.float64)
        self.pde, self.kappa, self.mu = pde, float(kappa), float(mu)
        self.kernel, self.disc = kernel, disc

    @classmethod
    def from_spec(cls, s):
        return cls(s.dim, s.n, s.L, s.origin, s.markers.X, s.markers.ds, s.pde, s.kappa, s.mu, s.kernel, s.disc)

    @property
    def n_ib(self):
        return self.X.shape[0]

    @property
    def nq(self):
        return self.dim if self.pde == "stokes" else 1

    @property
    def has_ubar(self):
        return self.kappa == 0.0

    @property
    def n_aug(self):
        return self.n_ib * self.nq + (self.nq if self.has_ubar else 0)

    @property
    def wt(self):
        """MINRES inner-product weights: ds_i / mean(ds) per marker entry, 1 per u_bar entry."""
        w = np.repeat(self.ds / np.mean(self.ds), self.nq)
        return np.concatenate([w, np.ones(self.nq if self.has_ubar else 0)])

    def split(self, q):
        q = np.asarray(q, dtype=np.float64)
        F = q[: self.n_ib * self.nq]
        F = F.reshape(self.n_ib, self.nq) if self.nq > 1 else F.copy()
        ub = q[self.n_ib * self.nq:] if self.has_ubar else np.zeros(self.nq)
        return F, ub

    def Linv(self, f):
        c0 = self.kappa ** 2
        c2 = self.mu if self.pde == "stokes" else 1.0
        if f.ndim == self.dim + 1:
            return np.stack([G.solve(self.grid, fc, self.disc, c0, c2) for fc in f])
        return G.solve(self.grid, f, self.disc, c0, c2)

    def response(self, f):
        """L^-1 f (scalar) or L^-1 P f (vector)."""
        if self.pde == "stokes":
            return self.Linv(G.project(self.grid, f, self.disc))
        return self.Linv(f)

    def S(self, F):
        return spread(self.grid, self.X, self.ds, F, self.kernel)

    def apply(self, q):
        F, ub = self.split(q)
        y = -interp(self.grid, self.X, self.response(self.S(F)), self.kernel)
        if self.has_ubar:
            y = y + (ub[None, :] if self.nq > 1 else ub[0])
        out = [np.asarray(y).reshape(-1)]
        if self.has_ubar:
            w = self.ds / np.mean(self.ds)
            out.append(np.sum(w[:, None] * F, axis=0) if self.nq > 1 else np.array([np.sum(w * F)]))
        return np.concatenate(out)

    def rhs(self, data, g=None):
        b = np.asarray(data, dtype=np.float64).copy()
        if g is not None:
            b = b - interp(self.grid, self.X, self.response(g), self.kernel)
        out = [b.reshape(-1)]
        if self.has_ubar:
            gs = np.zeros(self.nq) if g is None else (
                g.reshape(self.nq, -1).sum(axis=1) if self.nq > 1 else np.array([g.sum()]))
            out.append(self.grid.h ** self.dim / np.mean(self.ds) * gs)
        return np.concatenate(out)

    def recover(self, q, g=None):
        F, ub = self.split(q)
        f = -self.S(F)
        if g is not None:
            f = f + g
        u = self.response(f)
        if self.has_ubar:
            u = u + (ub.reshape((-1,) + (1,) * self.dim) if self.nq > 1 else ub[0])
        return u

    def assemble(self):
        n = self.n_aug
        A = np.empty((n, n))
        e = np.zeros(n)
        for j in range(n):
            e[j] = 1.0
            A[:, j] = self.apply(e)
            e[j] = 0.0
        return A
