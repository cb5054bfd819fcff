"""Exact gradients of a loss of the recovered grid solution with respect to the markers and the
boundary data, by forward-mode differentiation of the oracle's own forward map.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The forward map, for fixed normals n and weights ds, is
    X, data  ->  q = A(X)^-1 b(X, data)  ->  u = recover(q, data)        (Sec. 5.3.2, 5.3.3, 6.3.3)
and a loss L(u) enters only through psi = dL/du (a grid array of u's shape; the pairing
<psi, u> is the plain sum over grid values).  Returned: dL/dX [n_ib][D] and dL/ddata [n_ib(*nq)].

Every marker dependence of A, b and recover is carried by the spread S and the interpolation S*
(Sec. 2.2.2), and each term of those maps contains S at most once and S* at most once.  The
directional derivative along dX therefore follows from the product rule by re-evaluating the
same oracle code with S (or S*) replaced by its derivative, minus the same code with that
operator replaced by zero (which removes the terms that do not contain it):
    dE = [E(S*, dS) - E(S*, 0)] + [E(dS*, S) - E(0, S)].
The solves use a dense LU factorisation of the assembled A, so the result carries no iteration
error.  Cost: one derivative evaluation per component of X and one solve per data value, so
this is meant for small problems (a few hundred unknowns).
"""
from __future__ import annotations

import copy

import numpy as np
import scipy.linalg as sla

from .ib import interp_dX, spread_dX


def _variant(setup, s_mode, sstar_mode, dX):
    """Copy of `setup` whose S / S* are the operator ('op'), its derivative along dX ('d'), or 0."""
    v = copy.copy(setup)
    g, X, ds, k = setup.grid, setup.X, setup.ds, setup.kernel
    if s_mode == "d":
        v.S = lambda F: spread_dX(g, X, ds, F, k, dX)
    elif s_mode == "0":
        def zero_S(F):
            F = np.asarray(F)
            return np.zeros((F.shape[1],) + g.shape) if F.ndim == 2 else np.zeros(g.shape)
        v.S = zero_S
    if sstar_mode == "d":
        v.Sstar = lambda u: interp_dX(g, X, u, k, dX)
    elif sstar_mode == "0":
        def zero_Sstar(u):
            u = np.asarray(u)
            return np.zeros((X.shape[0], u.shape[0])) if u.ndim == g.dim + 1 else np.zeros(X.shape[0])
        v.Sstar = zero_Sstar
    return v


def directional(setup, fn, dX):
    """d/dt fn(setup with markers X + t dX) at t = 0, for fn using S and S* at most once per term."""
    a = fn(_variant(setup, "d", "op", dX)) - fn(_variant(setup, "0", "op", dX))
    b = fn(_variant(setup, "op", "d", dX)) - fn(_variant(setup, "op", "0", dX))
    return a + b


def forward(setup, data, g=None):
    """Dense solve of the forward problem: (q, u, LU factors of A)."""
    A = setup.assemble()
    lu = sla.lu_factor(A)
    q = sla.lu_solve(lu, setup.rhs(data, g))
    return q, setup.recover(q, data, g), lu


def gradients(setup, data, g, psi):
    """dL/dX [n_ib][D] and dL/ddata [n_ib * nq] for dL/du = psi, by forward mode."""
    data = np.asarray(data, dtype=np.float64)
    q, u, lu = forward(setup, data, g)
    zeros = np.zeros_like(data)
    n_ib, D = setup.X.shape

    def pair(du):
        return float(np.sum(np.asarray(psi) * du))

    gX = np.zeros((n_ib, D))
    for i in range(n_ib):
        for e in range(D):
            dX = np.zeros((n_ib, D))
            dX[i, e] = 1.0
            dA_q = directional(setup, lambda s: s.apply(q), dX)
            db = directional(setup, lambda s: s.rhs(data, g), dX)
            du_q = directional(setup, lambda s: s.recover(q, data, g), dX)
            dq = sla.lu_solve(lu, db - dA_q)
            gX[i, e] = pair(du_q + setup.recover(dq, zeros, None))
    flat = data.reshape(-1)
    gd = np.zeros(flat.size)
    for j in range(flat.size):
        e = np.zeros(flat.size)
        e[j] = 1.0
        ej = e.reshape(data.shape)
        dq = sla.lu_solve(lu, setup.rhs(ej, None))
        gd[j] = pair(setup.recover(dq, ej, None))
    return gX, gd


def loss_value(setup, data, g, psi):
    """<psi, u(X, data)> with a dense solve (the linear loss whose gradient `gradients` returns)."""
    return float(np.sum(np.asarray(psi) * forward(setup, data, g)[1]))
