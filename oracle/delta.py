"""Regularized delta kernels phi(r), with delta_h(x) = h^-D prod_d phi(x_d / h).

TEST INFRASTRUCTURE ONLY: the oracle is a plain FP64 CPU restatement of the
thesis used to check the HIP library.  Only tests, the smoke check and the
benchmark's CPU-baseline leg may import it.
"""
from __future__ import annotations

import numpy as np


def phi_peskin4(r):
    """Peskin 4-point kernel, Sec. 2.2.2 (equation following `delta_h = h^-2 phi phi`)."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a < 2.0)
    out[m1] = (3.0 - 2.0 * a[m1] + np.sqrt(1.0 + 4.0 * a[m1] - 4.0 * a[m1] ** 2)) / 8.0
    out[m2] = (5.0 - 2.0 * a[m2] - np.sqrt(np.maximum(-7.0 + 12.0 * a[m2] - 4.0 * a[m2] ** 2, 0.0))) / 8.0
    return out


def phi_cos4(r):
    """Peskin's cosine kernel: (1 + cos(pi r / 2)) / 4 for |r| < 2, else 0."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    return np.where(a < 2.0, 0.25 * (1.0 + np.cos(0.5 * np.pi * a)), 0.0)


def phi_bspline6(r):
    """6-point quintic B-spline kernel, Sec. 6.3.1 (pieces evaluated at |r|)."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a <= 2.0)
    m3 = (a > 2.0) & (a < 3.0)
    x = a[m1]
    out[m1] = 11 / 20 - x ** 2 / 2 + x ** 4 / 4 - x ** 5 / 12
    x = a[m2]
    out[m2] = 17 / 40 + 5 * x / 8 - 7 * x ** 2 / 4 + 5 * x ** 3 / 4 - 3 * x ** 4 / 8 + x ** 5 / 24
    x = a[m3]
    out[m3] = 81 / 40 - 27 * x / 8 + 9 * x ** 2 / 4 - 3 * x ** 3 / 4 + x ** 4 / 8 - x ** 5 / 120
    return out


def dphi_peskin4(r):
    """d phi / d r of the 4-point kernel (derivative of each piece in |r|, times sign r)."""
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(r)
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a < 2.0)
    x = a[m1]
    out[m1] = (-2.0 + (4.0 - 8.0 * x) / (2.0 * np.sqrt(1.0 + 4.0 * x - 4.0 * x ** 2))) / 8.0
    x = a[m2]
    out[m2] = (-2.0 - (12.0 - 8.0 * x) / (2.0 * np.sqrt(np.maximum(-7.0 + 12.0 * x - 4.0 * x ** 2, 1e-300)))) / 8.0
    return np.sign(r) * out


def dphi_cos4(r):
    r = np.asarray(r, dtype=np.float64)
    return np.where(np.abs(r) < 2.0, -0.125 * np.pi * np.sin(0.5 * np.pi * r), 0.0)


def dphi_bspline6(r):
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(r)
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a <= 2.0)
    m3 = (a > 2.0) & (a < 3.0)
    x = a[m1]
    out[m1] = -x + x ** 3 - 5 * x ** 4 / 12
    x = a[m2]
    out[m2] = 5 / 8 - 7 * x / 2 + 15 * x ** 2 / 4 - 3 * x ** 3 / 2 + 5 * x ** 4 / 24
    x = a[m3]
    out[m3] = -27 / 8 + 9 * x / 2 - 9 * x ** 2 / 4 + x ** 3 / 2 - x ** 4 / 24
    return np.sign(r) * out


DERIVATIVES = {"peskin4": dphi_peskin4, "cos4": dphi_cos4, "bspline6": dphi_bspline6}


def dkernel(name):
    """phi' of the named kernel (used for derivatives with respect to marker positions)."""
    return DERIVATIVES[name]


KERNELS = {
    "peskin4": (phi_peskin4, 2),
    "cos4": (phi_cos4, 2),
    "bspline6": (phi_bspline6, 3),
}


def kernel(name):
    """Return (phi, half_support)."""
    return KERNELS[name]
