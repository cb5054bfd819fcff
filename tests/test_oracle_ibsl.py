"""Pins of the oracle's MINRES and single layer (IBSL) Schur complements (Chapter 2).

* MINRES against GMRES: for a symmetric matrix both minimise the residual over the same Krylov
  space, so their residual histories agree; both reach the dense solution;
* the weighted inner product: MINRES on an operator self-adjoint in it follows the Euclidean
  MINRES of the symmetrised system step for step;
* the Schur complements are symmetric with equal spacings (Sec. 2.2.3, 2.2.4), and -S* L^-1 S is
  positive semidefinite for L = Delta - 1;
* iteration counts against the thesis's table for the Helmholtz circle (N = 64 and 128, all four
  spacings): never fewer, and at most 15 % + 2 more (marker phase and the stopping test of the
  thesis's MINRES are not printed);
* the same for the Brinkman circle (Sec. 2.4.2's table; N = 64 and 128, ds ~ 2 dx and 1.5 dx);
* solutions converge at first order, on the nodes with r < 0.15, to the closed forms: I_2(r) sin 2 theta / I_2(1/4) (Helmholtz) and 32 x y
  (Poisson, with the border row 1^T F = 0 that g~ = 0 imposes).
"""
import json
import pathlib

import numpy as np
import pytest
from scipy.special import iv

from oracle.gmres import gmres
from oracle.ibsl import IBSL
from oracle.minres import minres
from workloads import problems as P

TABLE = json.loads((pathlib.Path(__file__).parent / "golden" / "ibsl_iterations.json").read_text())
BRINK = json.loads((pathlib.Path(__file__).parent / "golden" / "ibsl_iterations_brinkman.json").read_text())


def _sym(n, seed, indefinite=True):
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = rng.uniform(0.5, 5.0, n) * (np.where(rng.random(n) < 0.5, -1.0, 1.0) if indefinite else 1.0)
    return Qm @ np.diag(ev) @ Qm.T


@pytest.mark.parametrize("indefinite", [False, True])
def test_minres_matches_gmres_and_solves(indefinite):
    A = _sym(40, 1 + indefinite, indefinite)
    b = np.random.default_rng(5).standard_normal(40)
    x, it, hist, ok = minres(lambda v: A @ v, b, 1e-12, 200)
    _, _, ghist = gmres(lambda v: A @ v, b, 1e-12, 200)
    assert ok
    k = min(20, len(hist), len(ghist))
    assert np.allclose(hist[:k], ghist[:k], rtol=1e-6, atol=1e-14)
    assert np.all(np.diff(hist) <= 1e-14)                  # MINRES residuals never grow
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_minres_weighted_inner_product():
    n = 30
    K = _sym(n, 7)
    w = np.random.default_rng(8).uniform(0.5, 2.0, n)
    A = K / w[:, None]                                      # W A = K: self-adjoint in <., .>_W
    b = np.random.default_rng(9).standard_normal(n)
    x, it, hist, ok = minres(lambda v: A @ v, b, 1e-12, 200, wt=w)
    r = np.sqrt(w)
    At = r[:, None] * A / r[None, :]                        # W^1/2 A W^-1/2, symmetric
    assert np.allclose(At, At.T, atol=1e-12)
    xt, itt, histt, _ = minres(lambda v: At @ v, r * b, 1e-12, 200)
    assert abs(it - itt) <= 1
    k = min(15, len(hist), len(histt))
    assert np.allclose(hist[:k], histt[:k], rtol=1e-8, atol=1e-15)
    assert np.allclose(x, xt / r, rtol=1e-8, atol=1e-12)
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


def _poisson_circle(N, alpha):
    s = P.helmholtz_circle(N, alpha)
    return P.ProblemSpec(**{**s.__dict__, "pde": "poisson", "kappa": 0.0,
                            "exact": lambda x, y: 32.0 * x * y})


@pytest.mark.parametrize("case", ["helmholtz", "poisson"])
def test_schur_complement_symmetric(case):
    s = P.helmholtz_circle(32, 1.0) if case == "helmholtz" else _poisson_circle(32, 1.0)
    o = IBSL.from_spec(s)
    M = o.assemble()
    assert np.max(np.abs(M - M.T)) < 1e-12 * np.max(np.abs(M))
    if case == "helmholtz":
        assert np.min(np.linalg.eigvalsh(0.5 * (M + M.T))) > -1e-12 * np.max(np.abs(M))
    else:
        assert o.has_ubar and M.shape[0] == o.n_ib + 1
        assert np.allclose(M[-1, :-1], 1.0) and M[-1, -1] == 0.0


@pytest.mark.parametrize("N", [64, 128])
def test_iteration_counts_against_table(N):
    want = TABLE["rows"][str(N)]
    for a, w in zip(TABLE["alpha"], want):
        s = P.helmholtz_circle(N, a)
        o = IBSL.from_spec(s)
        _, it, _, ok = minres(o.apply, o.rhs(s.data, s.g), 1e-8, 20000, o.wt)
        assert ok
        assert w <= it <= 1.15 * w + 2, (N, a, it, w)


@pytest.mark.parametrize("N,alpha", [(64, 2.0), (64, 1.5), (128, 2.0)])
def test_brinkman_iteration_counts_against_table(N, alpha):
    w = BRINK["rows"][str(N)][BRINK["alpha"].index(alpha)]
    s = P.brinkman_circle(N, alpha)
    o = IBSL.from_spec(s)
    _, it, _, ok = minres(o.apply, o.rhs(s.data, s.g), 1e-8, 20000, o.wt)
    assert ok
    assert w <= it <= 1.15 * w + 2, (N, alpha, it, w)


def _interior_error(s, o, q):
    u = o.recover(q, s.g)
    xs, ys = o.grid.nodes()
    r = np.hypot(xs, ys)
    inner = r < 0.15
    return np.max(np.abs(u - s.exact(xs, ys))[inner]), q


@pytest.mark.parametrize("case", ["helmholtz", "poisson"])
def test_solution_converges_to_closed_form(case):
    errs = []
    for N in (64, 128):
        s = P.helmholtz_circle(N, 1.0) if case == "helmholtz" else _poisson_circle(N, 1.0)
        if case == "helmholtz":
            xs, ys = np.meshgrid([0.1], [0.05])
            th = np.arctan2(0.05, 0.1)
            assert abs(s.exact(0.1, 0.05) - iv(2, np.hypot(0.1, 0.05)) * np.sin(2 * th) / iv(2, 0.25)) < 1e-12
        o = IBSL.from_spec(s)
        q, it, _, ok = minres(o.apply, o.rhs(s.data, s.g), 1e-10, 20000, o.wt)
        assert ok
        e, q = _interior_error(s, o, q)
        errs.append(e)
        if case == "poisson":
            F, _ = o.split(q)
            assert abs(np.sum(F)) < 1e-8 * np.sum(np.abs(F))
    assert errs[1] < 0.6 * errs[0], errs                   # first order away from the circle
    assert errs[1] < 0.025
