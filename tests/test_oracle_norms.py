"""Pins of the oracle's error norms (Sec. 2.2.1): a case worked by hand and closed-form
integrals over a disk that the rescaled norms approach under refinement."""
import math

import numpy as np

from oracle import norms


def test_hand_worked_case():
    # 3 x 3 grid, h = 0.5, Omega = three nodes with errors 1, -2, 2; |Omega| = 0.75.
    err = np.array([[1.0, -2.0, 5.0], [0.0, 2.0, 0.0], [9.0, 0.0, 0.0]])
    mask = np.array([[1, 1, 0], [0, 1, 0], [0, 0, 0]], dtype=bool)
    # h^2 = 0.25: l1 = 0.25 * (1 + 2 + 2) / 0.75 = 5/3; l2 = sqrt(0.25 * 9 / 0.75) = sqrt(3)
    assert abs(norms.l1(err, mask, 0.5, 2, area=0.75) - 5.0 / 3.0) < 1e-15
    assert abs(norms.l2(err, mask, 0.5, 2, area=0.75) - math.sqrt(3.0)) < 1e-15
    assert norms.linf(err, mask) == 2.0          # the 5 and the 9 lie outside Omega
    # without |Omega| the node count times h^2 (0.75 here) stands in for it
    assert abs(norms.l1(err, mask, 0.5, 2) - 5.0 / 3.0) < 1e-15


def test_disk_integrals():
    """On the unit disk: mean |x| = 4/(3 pi), rms of x = 1/2, max |x| -> 1."""
    n = 1024
    h = 2.0 / n
    t = -1.0 + h * (np.arange(n) + 0.5)
    x, y = np.meshgrid(t, t, indexing="ij")
    mask = x * x + y * y < 1.0
    assert abs(norms.l1(x, mask, h, 2, area=math.pi) - 4.0 / (3.0 * math.pi)) < 2e-3
    assert abs(norms.l2(x, mask, h, 2, area=math.pi) - 0.5) < 2e-3
    assert abs(norms.linf(x, mask) - 1.0) < 2 * h
    # the rescaling makes a constant's norms equal to the constant
    c = np.full_like(x, -3.0)
    assert abs(norms.l1(c, mask, h, 2) - 3.0) < 1e-12 and abs(norms.l2(c, mask, h, 2) - 3.0) < 1e-12
