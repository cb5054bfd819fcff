"""IBDL boundary operators, right-hand sides and grid recovery, written from the thesis.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Unknown vector layout: q = [Q_0, ..., Q_{n-1}] with Q_i a scalar (Helmholtz,
Poisson) or a D-vector (Stokes, stored [n_ib][D]), followed by u_bar (1 or D
values) when the completed method meets a singular grid operator
(eta > 0 and kappa = 0).

Operators (n points out of Omega, arclength weights ds):
  * scalar Dirichlet, Sec. 5.3.2 eq. (ibdl schur again):
      A Q = -S* L^-1 S~ Q + Q/2,  b = U_b - S* L^-1 g~,  L = Delta - kappa^2;
  * completed scalar, Sec. 5.3.3 (system after eq. ibdl completed again):
      A [Q; ub] = [-S* L^-1 (S~ + eta S) Q + ub 1 + Q/2;  eta sum_i ds_i Q_i],
      b = [U_b - S* L^-1 g~;  h^D sum_x g~];
  * Neumann, Sec. 5.2 eq. (Neumann saddle point):
      A U = -S* L^-1 S~ U - U/2,  b = S* L^-1 S V_b - S* L^-1 g~;
  * Brinkman/Stokes, Sec. 6.3.2 eq. (brink ibdl eqn), Sec. 6.3.3 and eq. (discrete operator for Q):
      u[Q] = -grad Delta_0^-1 S(Q.n) - L^-1 P (eta S Q + mu div(S A)),  A_ij = Q_i n_j + Q_j n_i,
      A Q = S* u[Q] + Q/2 (+ ub 1),  b = U_b - S* L^-1 P g~,  L = mu Delta - k^2,
      border rows eta sum_i ds_i Q_i = h^D sum_x g~ when k = 0.
Grid recovery: Sec. 5.3.2 (ibdl again 1), eq. following Sec. 5.3.3's system, Sec. 6.3.2 eq. (onC).
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from .ib import Grid, interp, spread


class Setup:
    """One IBDL problem: grid, markers and PDE parameters (plain arrays and scalars)."""

    def __init__(self, dim, n, L, origin, X, nrm, ds, pde, kappa, mu, bc, eta, kernel, disc):
        self.grid = Grid(dim, n, L, origin)
        self.dim = int(dim)
        self.X = np.asarray(X, dtype=np.float64)
        self.nrm = np.asarray(nrm, dtype=np.float64)
        self.ds = np.asarray(ds, dtype=np.float64)
        self.pde, self.bc = pde, bc
        self.kappa, self.mu, self.eta = float(kappa), float(mu), float(eta)
        self.kernel, self.disc = kernel, disc
        if pde not in ("screened", "poisson", "stokes"):
            raise ValueError(pde)
        if pde == "poisson" and self.kappa != 0.0:
            raise ValueError("poisson means kappa = 0")
        if bc == "neumann" and (pde == "stokes" or self.eta != 0.0):
            raise ValueError("Neumann is implemented for the plain scalar operator only")

    @classmethod
    def from_spec(cls, s):
        """Build from any object carrying the problem's plain fields (duck-typed)."""
        m = s.markers
        return cls(s.dim, s.n, s.L, s.origin, m.X, m.nrm, m.ds, s.pde, s.kappa, s.mu, s.bc,
                   s.eta, s.kernel, s.disc)

    # ------------------------------------------------------------ sizes
    @property
    def n_ib(self):
        return self.X.shape[0]

    @property
    def nq(self):
        return self.dim if self.pde == "stokes" else 1

    @property
    def has_ubar(self):
        return self.eta > 0.0 and self.kappa == 0.0

    @property
    def n_aug(self):
        return self.n_ib * self.nq + (self.nq if self.has_ubar else 0)

    def split(self, q):
        q = np.asarray(q, dtype=np.float64)
        Q = q[: self.n_ib * self.nq]
        Q = Q.reshape(self.n_ib, self.nq) if self.nq > 1 else Q.copy()
        ub = q[self.n_ib * self.nq:] if self.has_ubar else np.zeros(self.nq)
        return Q, ub

    # ------------------------------------------------------------ building blocks
    def S(self, F):
        return spread(self.grid, self.X, self.ds, F, self.kernel)

    def Sstar(self, u):
        return interp(self.grid, self.X, u, self.kernel)

    def Stilde(self, Q):
        """div(S(Q n)) (Sec. 5.3.1, eq. Stilde)."""
        return G.div(self.grid, self.S(Q[:, None] * self.nrm), self.disc)

    def Linv(self, f):
        """L^-1 (Delta_0^-1 where L has a null space) applied componentwise."""
        if self.pde == "stokes":
            c0, c2 = self.kappa ** 2, self.mu
        else:
            c0, c2 = self.kappa ** 2, 1.0
        if f.ndim == self.dim + 1:
            return np.stack([G.solve(self.grid, fc, self.disc, c0, c2) for fc in f])
        return G.solve(self.grid, f, self.disc, c0, c2)

    def P(self, F):
        return G.project(self.grid, F, self.disc)

    def tensor_A(self, Q):
        """A_ij = Q_i n_j + Q_j n_i per marker, shape (n_ib, D, D)."""
        return Q[:, :, None] * self.nrm[:, None, :] + Q[:, None, :] * self.nrm[:, :, None]

    # ------------------------------------------------------------ density -> grid
    def u_of_q(self, Q):
        """Grid field induced by the boundary density alone (no forcing, no u_bar)."""
        if self.pde != "stokes":
            f = self.Stilde(Q)
            if self.eta != 0.0:
                f = f + self.eta * self.S(Q)
            return -self.Linv(f)
        D = self.dim
        s = self.S(np.sum(Q * self.nrm, axis=1))
        t1 = -G.grad(self.grid, G.solve(self.grid, s, self.disc, 0.0), self.disc)
        A = self.tensor_A(Q)
        SA = self.S(A.reshape(self.n_ib, D * D)).reshape((D, D) + self.grid.shape)
        divSA = np.stack([sum(G.deriv(self.grid, SA[i, j], j, self.disc) for j in range(D))
                          for i in range(D)])
        f = self.mu * divSA
        if self.eta != 0.0:
            f = f + self.eta * self.S(Q)
        t2 = -self.Linv(self.P(f))
        return t1 + t2

    # ------------------------------------------------------------ operator
    def apply(self, q):
        Q, ub = self.split(q)
        u = self.u_of_q(Q)
        su = self.Sstar(u)
        if self.bc == "neumann":
            y = su - 0.5 * Q
        else:
            y = su + 0.5 * Q
            if self.has_ubar:
                y = y + (ub[None, :] if self.nq > 1 else ub[0])
        out = [np.asarray(y).reshape(-1)]
        if self.has_ubar:
            if self.nq > 1:
                out.append(self.eta * np.sum(self.ds[:, None] * Q, axis=0))
            else:
                out.append(np.array([self.eta * np.sum(self.ds * Q)]))
        return np.concatenate(out)

    def _g_response(self, g):
        """L^-1 g~ (scalar) or L^-1 P g~ (Stokes)."""
        if self.pde == "stokes":
            return self.Linv(self.P(g))
        return self.Linv(g)

    def rhs(self, data, g=None):
        data = np.asarray(data, dtype=np.float64)
        if self.bc == "neumann":
            b = self.Sstar(self.Linv(self.S(data)))
        else:
            b = data.copy()
        if g is not None:
            b = b - self.Sstar(self._g_response(g))
        out = [np.asarray(b).reshape(-1)]
        if self.has_ubar:
            gsum = np.zeros(self.nq) if g is None else (
                g.reshape(self.nq, -1).sum(axis=1) if self.nq > 1 else np.array([g.sum()]))
            out.append(self.grid.h ** self.dim * gsum)
        return np.concatenate(out)

    def recover(self, q, data=None, g=None):
        """Grid solution u on the whole box from the solved density."""
        Q, ub = self.split(q)
        u = self.u_of_q(Q)
        if self.bc == "neumann":
            u = u - self.Linv(self.S(np.asarray(data, dtype=np.float64)))
        if g is not None:
            u = u + self._g_response(g)
        if self.has_ubar:
            u = u + (ub.reshape((-1,) + (1,) * self.dim) if self.nq > 1 else ub[0])
        return u

    # ------------------------------------------------------------ dense reference
    def assemble(self):
        n = self.n_aug
        A = np.empty((n, n))
        e = np.zeros(n)
        for j in range(n):
            e[j] = 1.0
            A[:, j] = self.apply(e)
            e[j] = 0.0
        return A
