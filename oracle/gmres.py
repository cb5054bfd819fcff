"""Textbook GMRES (Saad & Schultz): modified Gram-Schmidt Arnoldi, Givens rotations.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The thesis solves the non-symmetric IBDL systems with GMRES to a tolerance of
1e-8 unless stated otherwise (Sec. 5.3.2).  Reading used here: x0 = 0, no
restart, stop when the Arnoldi residual estimate ||b - A x_k|| / ||b|| <= tol;
the iteration count is the number of Arnoldi steps k.
"""
from __future__ import annotations

import numpy as np


def gmres(apply, b, tol=1e-8, maxit=100):
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    beta = float(np.linalg.norm(b))
    hist = []
    if beta == 0.0:
        return np.zeros(n), 0, hist
    m = min(maxit, n)
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    V[0] = b / beta
    k = 0
    for j in range(m):
        w = np.asarray(apply(V[j]), dtype=np.float64).copy()
        for i in range(j + 1):
            H[i, j] = np.dot(w, V[i])
            w -= H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        breakdown = H[j + 1, j] == 0.0
        if not breakdown:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        r = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / r, H[j + 1, j] / r
        H[j, j], H[j + 1, j] = r, 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]) / beta)
        if hist[-1] <= tol or breakdown:
            break
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):      # back substitution on the rotated Hessenberg
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    x = V[:k].T @ y
    return x, k, hist
