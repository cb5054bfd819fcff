"""Pins of the oracle's periodic grid operators (thesis Sec. 2.2.1, 2.2.4, 2.3.1, 2.3.2).

* the FD inverse, computed through its Fourier symbol, is checked by applying
  the real-space 5/7-point stencil written out node by node in the test;
* spectral operators: Fourier modes are eigenfunctions with eigenvalue -|k|^2;
* Delta_0^{-1} returns the mean-zero solution;
* first derivatives converge to the analytic derivative (2nd order FD, exact spectral);
* the Leray projection is idempotent, divergence-free (off the Nyquist lines)
  and annihilates gradients.
"""
import itertools

import numpy as np
import pytest

from oracle import grid as G
from oracle.ib import Grid


def _stencil_loops(u, h):
    """(Delta u)_{i,j} = (u_{i-1,j} + u_{i,j-1} + u_{i+1,j} + u_{i,j+1} - 4 u_{i,j}) / h^2, wrapped."""
    out = np.zeros_like(u)
    shape = u.shape
    D = len(shape)
    for idx in itertools.product(*[range(s) for s in shape]):
        acc = -2 * D * u[idx]
        for ax in range(D):
            for sgn in (-1, 1):
                j = list(idx)
                j[ax] = (j[ax] + sgn) % shape[ax]
                acc += u[tuple(j)]
        out[idx] = acc / h ** 2
    return out


@pytest.mark.parametrize("shape,kappa", [((8, 12), 1.0), ((10, 6), 0.0), ((4, 6, 8), 10.0), ((6, 4, 4), 0.0)])
def test_fd_inverse_against_stencil(shape, kappa):
    dim = len(shape)
    n = tuple(reversed(shape))
    h = 0.1
    grid = Grid(dim, n, tuple(h * v for v in n), (0.0,) * dim)
    rhs = np.random.default_rng(1).standard_normal(shape)
    u = G.solve(grid, rhs, "fd2", kappa ** 2)
    back = _stencil_loops(u, h) - kappa ** 2 * u
    want = rhs - (rhs.mean() if kappa == 0 else 0.0)
    np.testing.assert_allclose(back, want, atol=1e-11 * np.abs(rhs).max())
    if kappa == 0:
        assert abs(u.mean()) < 1e-14
    np.testing.assert_allclose(G.laplacian(grid, u, "fd2"), _stencil_loops(u, h), atol=1e-10)


def test_spectral_eigenfunctions():
    grid = Grid(2, (16, 8), (2.0, 1.0), (-1.0, 0.0))
    x, y = grid.nodes()
    k1, k2 = 2 * np.pi * 3 / 2.0, 2 * np.pi * 2 / 1.0
    f = np.cos(k1 * x + 0.3) * np.sin(k2 * y - 0.1)
    np.testing.assert_allclose(G.laplacian(grid, f, "spectral"), -(k1 ** 2 + k2 ** 2) * f, atol=1e-11)
    np.testing.assert_allclose(G.solve(grid, f, "spectral", 4.0), f / (-(k1 ** 2 + k2 ** 2) - 4.0), atol=1e-14)
    np.testing.assert_allclose(G.deriv(grid, f, 0, "spectral"),
                               -k1 * np.sin(k1 * x + 0.3) * np.sin(k2 * y - 0.1), atol=1e-11)


def test_derivative_orders():
    errs = []
    for N in (32, 64):
        grid = Grid(2, (N, N), (1.0, 1.0), (0.0, 0.0))
        x, y = grid.nodes()
        f = np.exp(np.sin(2 * np.pi * x)) * np.cos(2 * np.pi * y)
        fx = 2 * np.pi * np.cos(2 * np.pi * x) * f
        errs.append(np.abs(G.deriv(grid, f, 0, "fd2") - fx).max())
        assert np.abs(G.deriv(grid, f, 0, "spectral") - fx).max() < 1e-9
    assert 3.6 < errs[0] / errs[1] < 4.4


def _no_nyquist(f):
    fh = np.fft.fft2(f)
    fh[..., 8, :] = 0.0
    fh[..., :, 8] = 0.0
    return np.real(np.fft.ifft2(fh))


def test_projection():
    """Exact off the Nyquist lines, where the derivative symbol is zeroed but |k|^2 is not."""
    grid = Grid(2, (16, 16), (1.0, 1.0), (0.0, 0.0))
    rng = np.random.default_rng(4)
    F = _no_nyquist(rng.standard_normal((2, 16, 16)))
    PF = G.project(grid, F, "spectral")
    np.testing.assert_allclose(G.project(grid, PF, "spectral"), PF, atol=1e-12)
    assert np.abs(G.div(grid, PF, "spectral")).max() < 1e-10
    phi = _no_nyquist(rng.standard_normal((16, 16)))
    gphi = G.grad(grid, phi, "spectral")
    assert np.abs(G.project(grid, gphi, "spectral")).max() < 1e-10


def test_fd_symbol_low_modes_on_long_lines():
    """The FD symbol (2 cos(2 pi m / N) - 2) / h^2 of the 5-point Laplacian at the lowest modes of an
    8192-point axis, against the same formula evaluated in extended precision (64-bit significand):
    relative 1e-12, which the formula evaluated directly in double misses by more than an order (the
    cancellation leaves 2.5e-11 at m = 1)."""
    g = Grid(2, (16, 8192), (1.0 / 64, 8.0), (0.0, 0.0))
    sig = G.laplacian_symbol(g, "fd2")
    col = sig[:, 0] - sig[0, 0]           # the y component (x index 0 adds nothing)
    m = np.arange(1, 9, dtype=np.longdouble)
    th = 2 * np.pi * m / np.longdouble(8192)
    want = (2 * np.cos(th) - 2) / np.longdouble(g.h) ** 2
    assert np.all(np.abs(col[1:9] / want.astype(np.float64) - 1) < 1e-12)
