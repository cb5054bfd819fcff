"""Textbook MINRES (Paige and Saunders), no preconditioner.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 2.2.3 (solution to the discrete system for invertible L) solves the symmetric Schur
complement with MINRES to a relative residual of 1e-8.  The iteration: Lanczos vectors
v_{k+1} beta_{k+1} = A v_k - alpha_k v_k - beta_k v_{k-1}, alpha_k = <v_k, A v_k>; the growing
tridiagonal matrix is reduced by Givens rotations (the two previous ones act on the new column,
a new one removes beta_{k+1}); the iterate is updated along w_k = (v_k - delta_k w_{k-1} -
epsilon_k w_{k-2}) / gamma_k and the residual norm is the running product |beta_1 s_1 ... s_k|.
The inner product is <a, b> = sum_i wt_i a_i b_i (wt = 1: the Euclidean one); the operator must be
self-adjoint in it.  Stops when the recurrence residual is at most tol times |b|.
"""
from __future__ import annotations

import math

import numpy as np


def minres(apply, b, tol, maxit, wt=None):
    """Returns (x, iterations, residual history |r_k| / |b| (recurrence), converged)."""
    b = np.asarray(b, dtype=np.float64)
    wt = np.ones_like(b) if wt is None else np.asarray(wt, dtype=np.float64)

    def dot(a, c):
        return float(np.sum(wt * a * c))

    x = np.zeros_like(b)
    beta1 = math.sqrt(dot(b, b))
    if beta1 == 0.0:
        return x, 0, [], True
    v_prev = np.zeros_like(b)
    v = b / beta1
    w1 = np.zeros_like(b)   # w_{k-1}
    w2 = np.zeros_like(b)   # w_{k-2}
    beta = 0.0              # beta_k (couples v_k to v_{k-1})
    c1, s1 = 1.0, 0.0       # rotation k-1
    c2, s2 = 1.0, 0.0       # rotation k-2
    eta = beta1
    hist = []
    for k in range(1, maxit + 1):
        p = apply(v)
        alpha = dot(v, p)
        p = p - alpha * v - beta * v_prev
        beta_next = math.sqrt(dot(p, p))
        # the previous two rotations on the new column (beta_k, alpha_k, beta_{k+1})
        eps = s2 * beta
        d0 = c2 * beta
        delta = c1 * d0 + s1 * alpha
        g0 = -s1 * d0 + c1 * alpha
        gamma = math.hypot(g0, beta_next)
        c, s = (g0 / gamma, beta_next / gamma) if gamma > 0.0 else (1.0, 0.0)
        w = (v - delta * w1 - eps * w2) / gamma if gamma > 0.0 else np.zeros_like(b)
        x = x + (c * eta) * w
        eta = -s * eta
        hist.append(abs(eta) / beta1)
        if abs(eta) <= tol * beta1 or beta_next == 0.0:
            return x, k, hist, True
        w2, w1 = w1, w
        c2, s2, c1, s1 = c1, s1, c, s
        v_prev, v = v, p / beta_next
        beta = beta_next
    return x, maxit, hist, False
