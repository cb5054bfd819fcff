"""GPU parity of the 2-D near-boundary tools (ibdl_indicator, ibdl_near_boundary) against the oracle.

Tolerances: the regularized indicator 1e-11 (FP64) / 2e-5 (mixed) absolute (it is O(1)); the
thresholded indicator equal wherever the oracle's regularized value is not within that tolerance
of 1/2 (and consistent with the GPU's own regularized value there); the interpolated field
1e-12 (FP64) / 1e-6 (mixed) relative to its max-norm, on every node.  The oracle receives the
same inputs as the GPU (grid values rounded to the grid type first).
"""
import numpy as np
import pytest
import torch

import paper_2210_07403_amd as ibdl
from oracle import nearbdry as NB
from oracle.gmres import gmres
from oracle.ib import Grid
from workloads import problems as P

from _helpers import make_oracle, make_problem, to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]

TOL_REG = {"fp64": 1e-11, "mixed": 2e-5}
TOL_U = {"fp64": 1e-12, "mixed": 1e-6}


def _grid(spec):
    return Grid(spec.dim, spec.n, spec.L, spec.origin)


CASES = {
    "circle64_fd": lambda: P.helmholtz_circle(64, 0.75, data="linear"),
    "circle64_spectral": lambda: P.helmholtz_circle(64, 0.75, data="linear", disc="spectral"),
    "circle128_cos4": lambda: P.ProblemSpec(**{**P.helmholtz_circle(128, 0.75).__dict__, "kernel": "cos4"}),
    "star256": lambda: P.cfg2_star_poisson(256, 1024),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_indicator_matches_oracle(name, precision):
    spec = CASES[name]()
    m = spec.markers
    pr = make_problem(spec, precision)
    chi, reg = pr.indicator(regularized=True)
    chi, reg = to_np(chi), to_np(reg)
    want_reg = NB.indicator(_grid(spec), m.X, m.nrm, m.ds, spec.kernel, spec.disc, regularized=True)
    tol = TOL_REG[precision]
    assert np.max(np.abs(reg - want_reg)) < tol
    clear = np.abs(want_reg - 0.5) > 2 * tol
    assert np.array_equal(chi[clear], (want_reg[clear] >= 0.5).astype(chi.dtype))
    assert np.array_equal(chi, (reg >= 0.5).astype(chi.dtype))
    pr.close()


def _field(spec, precision, seed):
    """A smooth field with noise, rounded to the grid type (the oracle gets the same values)."""
    g = _grid(spec)
    xs, ys = g.nodes()
    u = np.sin(3 * xs + 1) * np.cos(2 * ys) + 0.05 * np.random.default_rng(seed).standard_normal(xs.shape)
    dt = np.float64 if precision == "fp64" else np.float32
    return u.astype(dt).astype(np.float64)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["circle64_fd", "circle128_cos4", "star256"])
@pytest.mark.parametrize("m1,m2", [(6, 8), (3, 5)])
def test_near_boundary_matches_oracle(name, precision, m1, m2):
    spec = CASES[name]()
    g = _grid(spec)
    xs, ys = g.nodes()
    omega = spec.inside(xs, ys).astype(np.float64)
    u = _field(spec, precision, 7)
    Ub = np.sin(3 * spec.markers.X[:, 0] + 1) * np.cos(2 * spec.markers.X[:, 1])
    pr = make_problem(spec, precision)
    got = to_np(pr.near_boundary(Ub, omega, u, m1, m2))
    want = NB.near_boundary(g, spec.markers.X, Ub, omega, u, m1, m2)
    npts = len(NB.near_points(g, spec.markers.X, omega, m1))
    assert npts > 50
    err = np.abs(got - want) / np.max(np.abs(want))
    assert np.max(err) < TOL_U[precision], (np.max(err), int(np.sum(err > TOL_U[precision])), npts)
    pr.close()


@pytest.mark.parametrize("N,disc", [(64, "fd2"), (64, "spectral"), (128, "spectral"), (256, "spectral")])
def test_near_widths_match_oracle(N, disc):
    pr = make_problem(P.helmholtz_circle(N, 0.75, disc=disc), "fp64")
    assert pr.near_widths() == NB.widths(disc, N)
    pr.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_near_boundary_default_widths_spectral(precision):
    """Spectral symbols at 128^2: the default widths (m1 = 6, m2 = 8 by the logarithmic rule)."""
    spec = P.helmholtz_circle(128, 0.75, data="linear", disc="spectral")
    g = _grid(spec)
    xs, ys = g.nodes()
    omega = spec.inside(xs, ys).astype(np.float64)
    u = _field(spec, precision, 11)
    Ub = np.cos(2 * spec.markers.X[:, 0]) + spec.markers.X[:, 1]
    pr = make_problem(spec, precision)
    got = to_np(pr.near_boundary(Ub, omega, u))
    m1, m2 = NB.widths("spectral", 128)
    want = NB.near_boundary(g, spec.markers.X, Ub, omega, u, m1, m2)
    assert np.max(np.abs(got - want)) / np.max(np.abs(want)) < TOL_U[precision]
    pr.close()


def test_pipeline_reduces_max_error():
    """The thesis's linear-solution problem (Sec. 5.5) end to end on the GPU in FP64: solve,
    recover, indicator, interpolation with m1 = 6, m2 = 8; against the oracle's own pipeline."""
    spec = P.helmholtz_circle(128, 0.75, data="linear")
    pr = make_problem(spec, "fp64")
    q, u, info = pr.solve(spec.data, spec.g, tol=1e-12, maxit=200)
    assert info.status == 0
    chi = pr.indicator()
    fixed = to_np(pr.near_boundary(spec.data, chi, u, 6, 8))
    o = make_oracle(spec)
    qo, _, _ = gmres(o.apply, o.rhs(spec.data, spec.g), 1e-12, 200)
    uo = o.recover(qo, spec.data, spec.g)
    g = o.grid
    chio = NB.indicator(g, spec.markers.X, spec.markers.nrm, spec.markers.ds, spec.kernel, spec.disc)
    assert np.array_equal(to_np(chi), chio)
    fixo = NB.near_boundary(g, spec.markers.X, spec.data, chio, uo, 6, 8)
    assert np.max(np.abs(fixed - fixo)) < 1e-10
    xs, ys = g.nodes()
    exact = spec.exact(xs, ys)
    om = chio == 1
    before = np.max(np.abs(to_np(u) - exact)[om])
    after = np.max(np.abs(fixed - exact)[om])
    assert after < 0.5 * before, (before, after)
    pr.close()


@pytest.mark.parametrize("N,n_ib", [(1024, 4096), (2048, 8192)])
def test_full_size_star_sampled(N, n_ib):
    """1024^2 star (4096 markers), and 2048^2 (8192; its y lines go through the four-step
    transform), FP64: the indicator against the oracle on every node, the interpolation on a
    sample of 400 corrected nodes computed one by one by the oracle."""
    spec = P.cfg2_star_poisson(N, n_ib)
    g = _grid(spec)
    m = spec.markers
    pr = make_problem(spec, "fp64")
    chi, reg = pr.indicator(regularized=True)
    want_reg = NB.indicator(g, m.X, m.nrm, m.ds, spec.kernel, spec.disc, regularized=True)
    assert np.max(np.abs(to_np(reg) - want_reg)) < 1e-11
    xs, ys = g.nodes()
    omega = spec.inside(xs, ys).astype(np.float64)
    u = _field(spec, "fp64", 8)
    Ub = np.sin(3 * m.X[:, 0] + 1) * np.cos(2 * m.X[:, 1])
    got = to_np(pr.near_boundary(Ub, omega, u, 6, 8))
    changed = np.argwhere(got != u)
    assert len(changed) > 1000
    rng = np.random.default_rng(9)
    for j, i in changed[rng.choice(len(changed), 400, replace=False)]:
        p = np.array([xs[j, i], ys[j, i]])
        want = NB.correct_point(g, m.X, Ub, u, p, 8)
        assert abs(got[j, i] - want) < 1e-12 * np.max(np.abs(u)), (j, i, got[j, i], want)
    pr.close()


def test_rejects_unsupported():
    pr3 = make_problem(P.cfg3_sphere(16, 2), "fp64")
    with pytest.raises(ibdl.IBDLError):
        pr3.indicator()
    pr3.close()
    spec = CASES["circle64_fd"]()
    pr = make_problem(spec, "fp64")
    g = _grid(spec)
    u = np.zeros(g.shape)
    with pytest.raises(ibdl.IBDLError):
        pr.near_boundary(spec.data, np.ones(g.shape), u, 8, 6)
    pr.close()


def test_degenerate_masks():
    """An empty domain mask changes nothing; a full mask with the smallest width changes only the
    nodes within h of a marker, as the oracle says."""
    spec = CASES["circle64_fd"]()
    g = _grid(spec)
    u = _field(spec, "fp64", 3)
    Ub = np.ones(spec.markers.X.shape[0])
    pr = make_problem(spec, "fp64")
    got = to_np(pr.near_boundary(Ub, np.zeros(g.shape), u, 6, 8))
    assert np.array_equal(got, u)
    full = np.ones(g.shape)
    got = to_np(pr.near_boundary(Ub, full, u, 1, 2))
    want = NB.near_boundary(g, spec.markers.X, Ub, full, u, 1, 2)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
    assert 0 < np.sum(got != u) == len(NB.near_points(g, spec.markers.X, full, 1))
    pr.close()
