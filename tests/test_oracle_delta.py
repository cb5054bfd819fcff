"""Pins of the oracle's delta kernels: identities the kernels are built to satisfy.

Peskin's 4-point kernel (thesis Sec. 2.2.2) satisfies the discrete partition of
unity, zero first moment, sum of squares 3/8 and the even/odd condition; the
cosine kernel satisfies all but the first moment; the quintic B-spline
(Sec. 6.3.1) has unit mass, zero first moment and second moment 1/2.  Each
piecewise formula must also be continuous at its breakpoints and vanish at the
edge of its support.  A wrong coefficient or sign fails one of these.
"""
import numpy as np
import pytest

from oracle import delta

R = np.random.default_rng(11).uniform(0.0, 1.0, 257)
J = np.arange(-4, 5)


def sums(phi, power=1, moment=0, parity=None):
    rr = R[:, None] - J[None, :]
    w = phi(rr) ** power * rr ** moment
    if parity is not None:
        w = w[:, (J % 2) == parity]
    return w.sum(axis=1)


def test_peskin4_identities():
    phi = delta.phi_peskin4
    np.testing.assert_allclose(sums(phi), 1.0, atol=1e-14)
    np.testing.assert_allclose(sums(phi, moment=1), 0.0, atol=1e-14)
    np.testing.assert_allclose(sums(phi, power=2), 3.0 / 8.0, atol=1e-14)
    np.testing.assert_allclose(sums(phi, parity=0), 0.5, atol=1e-14)
    np.testing.assert_allclose(sums(phi, parity=1), 0.5, atol=1e-14)
    assert phi(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-15)


def test_cos4_identities():
    phi = delta.phi_cos4
    np.testing.assert_allclose(sums(phi), 1.0, atol=1e-14)
    np.testing.assert_allclose(sums(phi, power=2), 3.0 / 8.0, atol=1e-14)
    np.testing.assert_allclose(sums(phi, parity=0), 0.5, atol=1e-14)
    # not first-moment exact: the reading that keeps both kernels distinct
    assert np.max(np.abs(sums(phi, moment=1))) > 1e-3


def test_bspline6_identities():
    phi = delta.phi_bspline6
    np.testing.assert_allclose(sums(phi), 1.0, atol=1e-13)
    np.testing.assert_allclose(sums(phi, moment=1), 0.0, atol=1e-13)
    np.testing.assert_allclose(sums(phi, moment=2), 0.5, atol=1e-13)


@pytest.mark.parametrize("name", ["peskin4", "cos4", "bspline6"])
def test_continuity_and_support(name):
    phi, S = delta.kernel(name)
    eps = 1e-9
    for b in range(1, S + 1):
        lo, hi = phi(np.array([b - eps]))[0], phi(np.array([b + eps]))[0]
        assert abs(lo - hi) < 1e-7, (b, lo, hi)
    assert abs(phi(np.array([float(S)]))[0]) < 1e-12
    assert np.all(phi(np.linspace(S, S + 3, 50)) == 0.0)
    r = np.linspace(-S, S, 1001)
    np.testing.assert_allclose(phi(r), phi(-r), atol=0)      # even
    assert np.all(phi(r) >= -1e-15)
