"""GPU parity of the net force / torque (ibdl_net_force) and grid line integrals
(ibdl_line_integral) against the oracle, and the periodic-cylinder-array drag of Sec. 6.5 end to
end (solve, recovery, force, flux) against the oracle's pipeline and the thesis's drag table.

Tolerances: the reductions 1e-13 relative (FP64 sums in another order); the mixed path's line
integral sums the same float values in double, 1e-12; the drag from GPU solves at tol 1e-10,
1e-8 relative to the oracle's (FP64) and 2e-5 (mixed, whose grid work is float)."""
import json
import pathlib

import numpy as np
import pytest
import torch

import paper_2210_07403_amd as ibdl
import oracle
from oracle import drag as Dr
from oracle.gmres import gmres
from oracle.ib import Grid
from workloads import problems as P

from _helpers import make_problem, to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]

TABLE = json.loads((pathlib.Path(__file__).parent / "golden" / "drag_table.json").read_text())
GK = {r[0]: r[3] for r in TABLE["rows"]}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_net_force_matches_oracle(precision):
    spec = P.cylinder_array(256, 0.3)
    pr = make_problem(spec, precision)
    m = spec.markers
    rng = np.random.default_rng(21)
    for _ in range(3):
        q = rng.standard_normal(pr.n_aug)
        got = to_np(pr.net_force(q))
        Q = q[: 2 * m.X.shape[0]].reshape(-1, 2)
        B = Dr.net_force(Q, m.ds, spec.eta)
        L = Dr.torque(m.X, Q, m.ds, spec.eta)
        want = np.array([B[0], B[1], L])
        assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))
    pr.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("N", [64, 1024])
def test_line_integral_matches_oracle(precision, N):
    spec = P.cylinder_array(N, 0.2)
    pr = make_problem(spec, precision)
    g = Grid(spec.dim, spec.n, spec.L, spec.origin)
    dt = np.float64 if precision == "fp64" else np.float32
    u = (np.random.default_rng(N).standard_normal((2, N, N)) + 0.3).astype(dt).astype(np.float64)
    ut = pr._as_grid(u, 2)
    tol = 1e-13 if precision == "fp64" else 1e-12
    for comp in (0, 1):
        for axis in (0, 1):
            for index in (0, 1, N // 2 + 3, N - 1):
                got = float(to_np(pr.line_integral(ut, comp, axis, index))[0])
                want = Dr.line_integral(g, u[comp], axis, index)
                line = u[comp][:, index] if axis == 0 else u[comp][index, :]
                assert abs(got - want) < tol * g.h * np.sum(np.abs(line)), (comp, axis, index)
    pr.close()


def _gpu_drag(spec, precision):
    pr = make_problem(spec, precision)
    q, u, info = pr.solve(spec.data, spec.g, tol=1e-10, maxit=200)
    assert info.status == 0
    F = to_np(pr.net_force(q))
    U = float(to_np(pr.line_integral(u, 0, 0, 0))[0])
    pr.close()
    return F, U, info


@pytest.mark.parametrize("c", [0.1, 0.4])
def test_cylinder_array_drag_matches_oracle(c):
    spec = P.cylinder_array(128, c)
    o = oracle.Setup.from_spec(spec)
    qo, _, _ = gmres(o.apply, o.rhs(spec.data, spec.g), 1e-12, 300)
    uo = o.recover(qo, spec.data, spec.g)
    Qo, _ = o.split(qo)
    Bo = Dr.net_force(Qo, o.ds, o.eta)
    Uo = Dr.line_integral(o.grid, uo[0], 0, 0)
    Do = Dr.drag(Bo[0], Uo)
    F, U, info = _gpu_drag(spec, "fp64")
    assert abs(F[0] - Bo[0]) < 1e-9 and abs(F[1] - Bo[1]) < 1e-9
    assert abs(F[2]) < 1e-9                                      # symmetric flow: no torque
    assert abs(U / Uo - 1) < 1e-8
    assert abs(Dr.drag(F[0], U) / Do - 1) < 1e-8
    Fm, Um, _ = _gpu_drag(spec, "mixed")
    assert abs(Dr.drag(Fm[0], Um) / Do - 1) < 2e-5


def test_cylinder_array_drag_extrapolates_to_the_reference():
    """c = 0.1 on 512^2 and 1024^2 (FP64): first-order error against the Greengard-Kropinski value
    of the drag table, and the extrapolation 2 D_1024 - D_512 within 3e-4 of it."""
    gk = GK[0.1]
    d = {}
    for N in (512, 1024):
        F, U, info = _gpu_drag(P.cylinder_array(N, 0.1), "fp64")
        assert info.iters <= 18
        d[N] = Dr.drag(F[0], U)
    e512, e1024 = d[512] - gk, d[1024] - gk
    assert 1.7 < e512 / e1024 < 2.3
    assert abs((2 * d[1024] - d[512]) / gk - 1) < 3e-4


def test_rejects():
    pr = make_problem(P.helmholtz_circle(64, 0.75), "fp64")
    with pytest.raises(ibdl.IBDLError):
        pr.net_force(np.zeros(pr.n_aug))
    pr.close()
    pr = make_problem(P.cylinder_array(64, 0.1), "fp64")
    u = np.zeros((2, 64, 64))
    for comp, axis, index in ((2, 0, 0), (0, 2, 0), (0, 0, 64), (0, 1, -1)):
        with pytest.raises(ibdl.IBDLError):
            pr.line_integral(u, comp, axis, index)
    pr.close()
