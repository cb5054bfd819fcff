"""Periodic-grid differential operators and their inverses.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Finite differences (Sec. 2.2.1, eq. standard laplacian; Sec. 2.3.1): the
5-point (7-point in 3-D) Laplacian and the centred first difference, applied
in real space by index shifts.  Fourier spectral (Sec. 2.2.1, 2.3.1):
Laplacian -|k|^2, derivative i k_d.  Inverses of (c2 Delta - c0) are taken
with the FFT, the Laplacian replaced by its Fourier symbol; where that symbol
vanishes (the k = 0 mode when c0 = 0) the inverse returns the mean-zero
solution, i.e. Delta_0^{-1} of Sec. 2.2.4.

Reading where the thesis is silent: at the Nyquist index N/2 the spectral
first-derivative symbol is set to zero (so derivatives of real fields stay
real and D^T = -D), while the spectral Laplacian keeps -(2 pi (N/2) / L)^2.
"""
from __future__ import annotations

import numpy as np

from .ib import Grid

# Threads of the FFTs: None uses numpy.fft (one thread); a count uses scipy.fft with that many
# workers (the same pocketfft transforms, for timing the oracle on all host cores).
FFT_WORKERS = None


def _fftn(f):
    if FFT_WORKERS is None:
        return np.fft.fftn(f)
    import scipy.fft
    return scipy.fft.fftn(f, workers=FFT_WORKERS)


def _ifftn(f):
    if FFT_WORKERS is None:
        return np.fft.ifftn(f)
    import scipy.fft
    return scipy.fft.ifftn(f, workers=FFT_WORKERS)


def _wavenumber_index(n):
    """Signed mode index m for FFT position j: 0, 1, ..., N/2-1, -N/2, ..., -1."""
    return np.fft.fftfreq(n) * n


def laplacian_symbol(grid: Grid, disc: str):
    """Fourier symbol sigma(k) of the discrete Laplacian on the full FFT grid ([z][y][x])."""
    out = np.zeros(grid.shape)
    for d in range(grid.dim):
        m = _wavenumber_index(grid.n[d])
        if disc == "fd2":
            # the 5-point symbol (2 cos(k h) - 2) / h^2, written as -4 sin^2(k h / 2) / h^2: the same
            # value without the cancellation that costs the lowest modes ten digits at N = 8192
            s = -4.0 * np.sin(np.pi * m / grid.n[d]) ** 2 / grid.h ** 2
        else:
            s = -(2 * np.pi * m / grid.L[d]) ** 2
        shape = [1] * grid.dim
        shape[grid.axis(d)] = grid.n[d]
        out = out + s.reshape(shape)
    return out


def deriv_symbol(grid: Grid, disc: str, d: int):
    """Real k~_d with D_d <-> i k~_d: sin(k h)/h (centred difference) or k (0 at Nyquist)."""
    n = grid.n[d]
    m = _wavenumber_index(n)
    if disc == "fd2":
        s = np.sin(2 * np.pi * m / n) / grid.h
    else:
        s = 2 * np.pi * m / grid.L[d]
        s[n // 2] = 0.0
    shape = [1] * grid.dim
    shape[grid.axis(d)] = n
    return s.reshape(shape)


def deriv(grid: Grid, f, d: int, disc: str):
    """First derivative along direction d."""
    if disc == "fd2":
        ax = grid.axis(d)
        return (np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) / (2.0 * grid.h)
    fh = _fftn(f)
    return np.real(_ifftn(1j * deriv_symbol(grid, disc, d) * fh))


def laplacian(grid: Grid, f, disc: str):
    if disc == "fd2":
        out = -2.0 * grid.dim * f
        for d in range(grid.dim):
            ax = grid.axis(d)
            out = out + np.roll(f, -1, axis=ax) + np.roll(f, 1, axis=ax)
        return out / grid.h ** 2
    return np.real(_ifftn(laplacian_symbol(grid, disc) * _fftn(f)))


def solve(grid: Grid, rhs, disc: str, c0: float, c2: float = 1.0):
    """u with (c2 Delta - c0) u = rhs; mean-zero branch where the symbol vanishes."""
    lam = c2 * laplacian_symbol(grid, disc) - c0
    rh = _fftn(rhs)
    safe = np.where(lam == 0.0, 1.0, lam)
    uh = np.where(lam == 0.0, 0.0, rh / safe)
    return np.real(_ifftn(uh))


def div(grid: Grid, F, disc: str):
    """Divergence of a vector field F[(d,) + shape]."""
    return sum(deriv(grid, F[d], d, disc) for d in range(grid.dim))


def grad(grid: Grid, f, disc: str):
    return np.stack([deriv(grid, f, d, disc) for d in range(grid.dim)])


def project(grid: Grid, F, disc: str):
    """P = I - grad Delta_0^{-1} div (Sec. 2.3.2)."""
    phi = solve(grid, div(grid, F, disc), disc, 0.0)
    return F - grad(grid, phi, disc)
