"""GPU parity of the adjoint: A^T through ibdl_apply_transpose against the oracle's assembled A,
and ibdl_backward against the oracle's forward-mode gradients (dense solves), element by element.

Tolerances (relative to the max-norm of the oracle result): A^T p 1e-12 (FP64) / 2e-5 (mixed);
gradients 1e-8 (FP64, forward and adjoint GMRES both at 1e-13, so the Krylov error is far below
it) and 2e-4 (mixed).  Markers are moved off the lattice by a small seeded jitter, as in the
oracle's own pins, so that no kernel breakpoint sits exactly on a marker.
"""
import numpy as np
import pytest
import torch

import paper_2210_07403_amd as ibdl
from oracle import Setup
from oracle import adjoint as ADJ
from workloads import geometry as geo
from workloads import problems as P

from _helpers import make_problem, relerr, to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]


def _jitter(spec, seed=7):
    m = spec.markers
    h = spec.L[0] / spec.n[0]
    X = m.X + np.random.default_rng(seed).uniform(-1e-3, 1e-3, m.X.shape) * h
    return P.ProblemSpec(**{**spec.__dict__, "markers": geo.Markers(X, m.nrm, m.ds, m.length)})


CASES = {
    "helmholtz_fd": lambda: P.helmholtz_circle(32, 1.5),
    "helmholtz_spectral": lambda: P.helmholtz_circle(32, 1.5, disc="spectral"),
    "cos4_circle": lambda: P.ProblemSpec(**{**P.helmholtz_circle(32, 1.5).__dict__, "kernel": "cos4"}),
    "completed_poisson": lambda: P.completed_poisson_exterior(32, 2.0, 10.0, "trig"),
    "completed_screened": lambda: P.ProblemSpec(**{**P.helmholtz_circle(32, 1.5).__dict__, "eta": 3.0}),
    "brinkman": lambda: P.brinkman_circle(16, 1.5),
    "stokes_exterior": lambda: P.stokes_exterior_circle(16, 10.0),
    "brinkman_bspline": lambda: P.ProblemSpec(**{**P.brinkman_circle(16, 1.5).__dict__, "kernel": "bspline6"}),
    "brinkman_eta": lambda: P.ProblemSpec(**{**P.brinkman_circle(16, 1.5).__dict__, "eta": 2.0}),
    "sphere_3d": lambda: P.cfg3_sphere(16, 2),
    "sphere_3d_completed": lambda: P.ProblemSpec(**{**P.cfg3_sphere(16, 2).__dict__, "eta": 2.0}),
}


def _oracle(spec):
    m = spec.markers
    return Setup(spec.dim, spec.n, spec.L, spec.origin, m.X, m.nrm, m.ds, spec.pde, spec.kappa, spec.mu, spec.bc,
                 spec.eta, spec.kernel, spec.disc)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", sorted(CASES) + ["neumann"])
def test_apply_transpose(name, precision):
    spec = _jitter(P.neumann_circle(32) if name == "neumann" else CASES[name]())
    o = _oracle(spec)
    A = o.assemble()
    pr = make_problem(spec, precision)
    p = np.random.default_rng(4).standard_normal(o.n_aug)
    got = to_np(pr.apply_transpose(p))
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert relerr(got, A.T @ p) < tol, relerr(got, A.T @ p)
    pr.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_apply_transpose_long_axis(precision):
    """A 16 x 1024 Brinkman grid (completed): the transposed fused pass on 1024-point lines."""
    base = P.brinkman_circle(16, 1.5)
    spec = _jitter(P.ProblemSpec(**{**base.__dict__, "n": (16, 1024), "L": (2.0, 128.0), "g": None, "eta": 2.0}))
    o = _oracle(spec)
    A = o.assemble()
    pr = make_problem(spec, precision)
    p = np.random.default_rng(6).standard_normal(o.n_aug)
    got = to_np(pr.apply_transpose(p))
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert relerr(got, A.T @ p) < tol, relerr(got, A.T @ p)
    assert relerr(to_np(pr.apply(p)), A @ p) < tol
    pr.close()


@pytest.mark.parametrize("name", sorted(CASES))
def test_backward_fp64(name):
    spec = _jitter(CASES[name]())
    o = _oracle(spec)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((o.nq,) + o.grid.shape if o.nq > 1 else o.grid.shape)
    gX, gd = ADJ.gradients(o, spec.data, spec.g, psi)
    pr = make_problem(spec, "fp64")
    q, u, info = pr.solve(spec.data, spec.g, tol=1e-13, maxit=200)
    assert info.status == 0
    dX, dd, ainfo = pr.backward(q, u, torch.as_tensor(psi), tol=1e-13, maxit=200)
    assert ainfo.status == 0 and ainfo.true_relres_fp64 < 1e-12
    assert relerr(to_np(dd), gd) < 1e-9, relerr(to_np(dd), gd)
    assert relerr(to_np(dX), gX) < 1e-8, relerr(to_np(dX), gX)
    pr.close()


@pytest.mark.parametrize("name", ["helmholtz_fd", "stokes_exterior", "sphere_3d"])
def test_backward_mixed(name):
    spec = _jitter(CASES[name]())
    o = _oracle(spec)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((o.nq,) + o.grid.shape if o.nq > 1 else o.grid.shape)
    gX, gd = ADJ.gradients(o, spec.data, spec.g, psi)
    pr = make_problem(spec, "mixed")
    q, u, _ = pr.solve(spec.data, spec.g, tol=1e-7, maxit=200)
    dX, dd, _ = pr.backward(q, u, torch.as_tensor(psi), tol=1e-7, maxit=200)
    assert relerr(to_np(dd), gd) < 2e-4, relerr(to_np(dd), gd)
    assert relerr(to_np(dX), gX) < 2e-4, relerr(to_np(dX), gX)
    pr.close()


def test_backward_central_difference_3d():
    """At a size the forward-mode oracle does not reach (32^3, 1212 markers): the adjoint
    gradient against central differences of the GPU's own FP64 forward map, solved to 1e-13."""
    spec = _jitter(P.cfg3_sphere(32, 11))
    pr = make_problem(spec, "fp64")
    m = spec.markers
    rng = np.random.default_rng(5)
    psi = torch.as_tensor(rng.standard_normal(tuple(reversed(spec.n))), device="cuda")
    q, u, _ = pr.solve(spec.data, spec.g, tol=1e-13, maxit=200)
    dX, dd, _ = pr.backward(q, u, psi, tol=1e-13, maxit=200)
    dX = to_np(dX)

    def loss(X):
        pr.set_markers(X, m.nrm, m.ds)
        _, uu, _ = pr.solve(spec.data, spec.g, tol=1e-13, maxit=200)
        return float(torch.sum(psi * uu))

    eps = 1e-6
    dirs = [rng.standard_normal(m.X.shape)]
    for k in rng.choice(m.X.size, 3, replace=False):
        v = np.zeros(m.X.size)
        v[k] = 1.0
        dirs.append(v.reshape(m.X.shape))
    for v in dirs:
        fd = (loss(m.X + eps * v) - loss(m.X - eps * v)) / (2 * eps)
        an = float(np.sum(dX * v))
        assert abs(an - fd) < 1e-6 * max(abs(fd), np.abs(dX).max()), (an, fd)
    pr.close()


def test_autograd_function_matches_backward():
    """ibdl_solve as a torch.autograd.Function: X.grad and data.grad of a quadratic loss equal
    ibdl_backward with psi = dL/du, and a second forward with other markers does not disturb
    the first one's backward."""
    spec = _jitter(CASES["helmholtz_fd"]())
    pr = make_problem(spec, "fp64")
    m = spec.markers
    dev = torch.device("cuda")
    X = torch.tensor(m.X, device=dev, requires_grad=True)
    data = torch.tensor(np.asarray(spec.data, dtype=np.float64), device=dev, requires_grad=True)
    g = torch.as_tensor(spec.g, device=dev) if spec.g is not None else None
    target = torch.zeros(tuple(reversed(spec.n)), dtype=torch.float64, device=dev)
    h2 = (spec.L[0] / spec.n[0]) ** 2
    u = ibdl.ibdl_solve(pr, X, m.nrm, m.ds, data, g, 1e-13, 200)
    loss = 0.5 * h2 * torch.sum((u - target) ** 2)
    # a forward with other markers between this forward and its backward
    ibdl.ibdl_solve(pr, X.detach() + 0.01, m.nrm, m.ds, data.detach(), g, 1e-10, 200)
    loss.backward()
    pr.set_markers(m.X, m.nrm, m.ds)
    q, u2, _ = pr.solve(spec.data, spec.g, tol=1e-13, maxit=200)
    dX, dd, _ = pr.backward(q, u2, h2 * (u2 - target), tol=1e-13, maxit=200)
    assert relerr(to_np(X.grad), to_np(dX)) < 1e-10
    assert relerr(to_np(data.grad), to_np(dd)) < 1e-10
    pr.close()


def test_backward_rejects_neumann():
    spec = P.neumann_circle(32)
    pr = make_problem(spec, "fp64")
    q, u, _ = pr.solve(spec.data, spec.g, tol=1e-8)
    with pytest.raises(ibdl.IBDLError):
        pr.backward(q, u, torch.zeros_like(u))
    pr.close()
