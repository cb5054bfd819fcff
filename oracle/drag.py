"""Net force, torque, flux and dimensionless drag of a Stokes solution (2-D).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 6.5 (Stokes flow around a periodic array of cylinders) with Sec. 6.1 (exterior domains):
  * for the completed method the single layer of strength eta Q carries the whole net force on
    the body, B = -eta sum_i ds_i Q_i (the double layer carries none); the net torque about the
    coordinate origin is, by the same argument, L = -eta sum_i ds_i (X_i x Q_i), the z component
    of the cross product in 2-D;
  * U = the integral of the x velocity over the left face x = -1/2 of the periodic box, taken
    over the grid line by the rectangle rule (h times the sum of the nodes: exact for
    trigonometric polynomials the grid resolves);
  * D = B_1 / (mu U);
  * the asymptotic expressions the thesis compares with: the dilute form
    D_dil = 8 pi / (log(1/c) - 1.47633597 + 2c - 1.77428264 c^2 + 4.07770444 c^3 - 4.84227402 c^4)
    and the dense form D_den = 9 pi / (2 sqrt 2) (1 - sqrt(c / c_max))^(-5/2), c_max = pi/4.

Parity: pinned by tests/test_oracle_drag.py (the asymptotic forms against the printed columns of
the drag table; the solvability condition B = -(box integral of g); flux independent of the
line away from the body; first-order convergence of D to the printed reference values and its
extrapolation within 0.1 % of them; torque under a shift of the origin).
"""
from __future__ import annotations

import math

import numpy as np

from .ib import Grid


def net_force(Q, ds, eta):
    """B = -eta sum_i ds_i Q_i; Q is [n_ib][D]."""
    Q = np.asarray(Q, dtype=np.float64)
    return -eta * np.sum(np.asarray(ds, dtype=np.float64)[:, None] * Q, axis=0)


def torque(X, Q, ds, eta):
    """L = -eta sum_i ds_i (X_i,x Q_i,y - X_i,y Q_i,x) (2-D)."""
    X = np.asarray(X, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    ds = np.asarray(ds, dtype=np.float64)
    total = 0.0
    for i in range(X.shape[0]):
        total += ds[i] * (X[i, 0] * Q[i, 1] - X[i, 1] * Q[i, 0])
    return -eta * total


def line_integral(grid: Grid, u, axis, index):
    """h times the sum of the 2-D field u ([y][x]) over the grid line where coordinate `axis`
    has node index `index` (axis 0: the line x = x_index, summed over y)."""
    u = np.asarray(u, dtype=np.float64)
    line = u[:, index] if axis == 0 else u[index, :]
    return grid.h * float(np.sum(line))


def drag(B1, U, mu=1.0):
    return B1 / (mu * U)


def drag_dilute(c):
    return 8.0 * math.pi / (math.log(1.0 / c) - 1.47633597 + 2.0 * c - 1.77428264 * c ** 2
                            + 4.07770444 * c ** 3 - 4.84227402 * c ** 4)


def drag_dense(c):
    cmax = math.pi / 4.0
    return 9.0 * math.pi / (2.0 * math.sqrt(2.0)) * (1.0 - math.sqrt(c / cmax)) ** (-2.5)
