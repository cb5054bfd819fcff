"""Discrete error norms rescaled by the domain size (Sec. 2.2.1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np


def l1(err, mask, h, dim):
    vol = h ** dim * mask.sum()
    return float(h ** dim * np.sum(np.abs(err) * mask) / vol)


def l2(err, mask, h, dim):
    vol = h ** dim * mask.sum()
    return float(np.sqrt(h ** dim * np.sum(err ** 2 * mask) / vol))


def linf(err, mask):
    return float(np.max(np.abs(err[mask.astype(bool)])))
