"""Pins of the oracle's grid coupling: S, S* and S~ (thesis Sec. 2.2.2, 5.3.1).

* brute force: S computed by visiting every (node, marker) pair with the
  minimum-image separation on the torus, independent of the tap indexing;
* adjointness h^D <S F, u> = sum_i ds_i F_i (S* u)_i (Sec. 2.1, eq. adjoint);
* S* of a constant is that constant (Sec. 2.2.4, eq. interp of constant);
* total mass h^D sum_x S F = sum_i F_i ds_i (Sec. 2.2.4);
* the dipole spread S~ Q = div(S Q n) has zero grid sum.
"""
import numpy as np
import pytest

from oracle import delta
from oracle.grid import div
from oracle.ib import Grid, interp, spread


def _markers(grid, n, seed, near_edge=True):
    rng = np.random.default_rng(seed)
    X = np.array(grid.origin) + rng.uniform(0, 1, (n, grid.dim)) * np.array(grid.L)
    if near_edge:  # force a few markers onto the periodic seam and onto nodes
        X[0, :] = grid.origin
        X[1, 0] = grid.origin[0] + grid.L[0] - 1e-3 * grid.h
        X[2, :] = np.array(grid.origin) + 3 * grid.h
    ds = rng.uniform(0.5, 1.5, n) * grid.h ** (grid.dim - 1)
    nrm = rng.standard_normal((n, grid.dim))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return X, nrm, ds


GRIDS = [Grid(2, (16, 16), (1.0, 1.0), (0.0, 0.0)),
         Grid(2, (12, 20), (0.6, 1.0), (-0.3, -0.5)),
         Grid(3, (8, 8, 8), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))]


@pytest.mark.parametrize("kname", ["peskin4", "cos4", "bspline6"])
@pytest.mark.parametrize("gi", [0, 1, 2])
def test_spread_brute_force(kname, gi):
    grid = GRIDS[gi]
    X, _, ds = _markers(grid, 5, 3 + gi)
    F = np.random.default_rng(5).standard_normal(5)
    phi, _ = delta.kernel(kname)
    ref = np.zeros(grid.shape)
    nodes = grid.nodes()
    for i in range(5):
        w = np.ones(grid.shape)
        for d in range(grid.dim):
            sep = nodes[d] - X[i, d]
            sep = (sep + grid.L[d] / 2) % grid.L[d] - grid.L[d] / 2   # minimum image
            w = w * phi(sep / grid.h)
        ref += F[i] * ds[i] * w / grid.h ** grid.dim
    np.testing.assert_allclose(spread(grid, X, ds, F, kname), ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("kname", ["peskin4", "cos4", "bspline6"])
@pytest.mark.parametrize("gi", [0, 1, 2])
def test_adjoint_constant_and_mass(kname, gi):
    grid = GRIDS[gi]
    X, _, ds = _markers(grid, 37, 7 + gi)
    rng = np.random.default_rng(9)
    F = rng.standard_normal(37)
    u = rng.standard_normal(grid.shape)
    lhs = grid.h ** grid.dim * np.sum(spread(grid, X, ds, F, kname) * u)
    rhs = np.sum(ds * F * interp(grid, X, u, kname))
    assert lhs == pytest.approx(rhs, rel=1e-13, abs=1e-13)
    np.testing.assert_allclose(interp(grid, X, np.full(grid.shape, 2.5), kname), 2.5, atol=1e-13)
    mass = grid.h ** grid.dim * spread(grid, X, ds, F, kname).sum()
    assert mass == pytest.approx(np.sum(F * ds), rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("disc", ["fd2", "spectral"])
@pytest.mark.parametrize("gi", [0, 2])
def test_dipole_spread_zero_sum(disc, gi):
    grid = GRIDS[gi]
    X, nrm, ds = _markers(grid, 23, 13)
    Q = np.random.default_rng(2).standard_normal(23)
    st = div(grid, spread(grid, X, ds, Q[:, None] * nrm, "peskin4"), disc)
    assert abs(st.sum()) < 1e-12 * np.abs(st).sum()


def test_vector_spread_matches_components():
    grid = GRIDS[0]
    X, nrm, ds = _markers(grid, 11, 1)
    F = np.random.default_rng(3).standard_normal((11, 3))
    out = spread(grid, X, ds, F, "peskin4")
    for c in range(3):
        np.testing.assert_array_equal(out[c], spread(grid, X, ds, F[:, c], "peskin4"))
    u = np.random.default_rng(4).standard_normal((3,) + grid.shape)
    v = interp(grid, X, u, "peskin4")
    for c in range(3):
        np.testing.assert_array_equal(v[:, c], interp(grid, X, u[c], "peskin4"))
