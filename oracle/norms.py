"""Discrete error norms rescaled by the area (volume) of the PDE domain (Sec. 2.2.1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

||u||_1 = (h^D / |Omega|) sum_x |u(x)| chi_Omega(x) and
||u||_2 = ((h^D / |Omega|) sum_x u(x)^2 chi_Omega(x))^(1/2), with |Omega| the measure of
Omega.  The thesis states the 1-norm without the absolute value; an error norm takes
|u|.  When the caller does not know |Omega| in closed form, the node count times h^D
stands in for it.  ||u||_inf is the largest |u| over the nodes of Omega.
"""
from __future__ import annotations

import numpy as np


def _measure(mask, h, dim, area):
    return float(area) if area is not None else h ** dim * float(np.count_nonzero(mask))


def l1(err, mask, h, dim, area=None):
    m = np.asarray(mask, dtype=bool)
    return float(h ** dim * np.sum(np.abs(np.asarray(err))[m]) / _measure(m, h, dim, area))


def l2(err, mask, h, dim, area=None):
    m = np.asarray(mask, dtype=bool)
    return float(np.sqrt(h ** dim * np.sum(np.asarray(err)[m] ** 2) / _measure(m, h, dim, area)))


def linf(err, mask):
    return float(np.max(np.abs(np.asarray(err)[np.asarray(mask, dtype=bool)])))
