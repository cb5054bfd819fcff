"""GPU parity at the workloads' full sizes, in the configuration the benchmark times.

* 256^3 sphere (73,962 markers), mixed precision: the operator apply against the FP64 oracle on
  every marker (2e-5), the FP64 apply (1e-12), and the mixed solve at 1e-8 against the oracle's
  solution (1e-5); the recovered grid solution on a sample of nodes; the transposed apply on
  sampled entries and by adjointness against the oracle's forward apply.
* 1024^2 star (4,096 markers), Dirichlet and Neumann: FP64 apply (1e-12) and solve (1e-10); the
  mixed path (float grid work, double GMRES) apply (2e-5) and solve at 1e-8 (1e-5).
* 512^2 exterior Stokes star (1,024 markers, eta = 10, spectral), FP64: apply (1e-12) and solve
  (1e-10, with ubar), and the 1e-8 iteration count against the oracle's; the gradients of
  L = sum_x |w|^2 h^2 (w the disturbance velocity, so the target is the background shear) with
  respect to the marker positions and the boundary data against central differences of the
  GPU's own FP64 forward map.
The oracle runs the same operators in numpy; its GMRES (textbook MGS) is run to 1e-12.
"""
import numpy as np
import pytest
import torch

from oracle.gmres import gmres
from workloads import problems as P

from _helpers import make_oracle, make_problem, relerr, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]


def test_sphere256_apply_and_solve():
    spec = P.cfg3_sphere(256, 86)
    o = make_oracle(spec)
    q = P.random_density(spec, seed=0)
    want = o.apply(q)
    pr = make_problem(spec, "mixed")
    assert relerr(to_np(pr.apply(q)), want) < 2e-5
    pr64 = make_problem(spec, "fp64")
    assert relerr(to_np(pr64.apply(q)), want) < 1e-12
    pr64.close()
    # solve: the mixed path at the benchmark tolerance against the oracle's solution
    b = o.rhs(spec.data, spec.g)
    xo, ko, _ = gmres(o.apply, b, 1e-12, 60)
    qg, ug, info = pr.solve(spec.data, spec.g, tol=1e-8, maxit=100)
    assert info.status == 0 and info.true_relres_fp64 < 2e-7, info
    assert relerr(to_np(qg), xo) < 1e-5, relerr(to_np(qg), xo)
    # grid recovery on a sample of 4096 nodes (the oracle recovers the whole grid once)
    uo = o.recover(xo, spec.data, spec.g)
    rng = np.random.default_rng(1)
    idx = tuple(rng.integers(0, 256, (3, 4096)))
    ugn = to_np(ug)
    assert np.max(np.abs(ugn[idx] - uo[idx])) / np.max(np.abs(uo)) < 1e-5
    pr.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sphere256_apply_transpose(precision):
    """A^T p at full size (the backward's transposed apply), against the oracle's forward apply:
    sampled entries (A^T p)_i = p . (A e_i), one oracle apply per sample, and the adjointness
    <A^T p, q> = <p, A q> for a random q."""
    spec = P.cfg3_sphere(256, 86)
    o = make_oracle(spec)
    pr = make_problem(spec, precision)
    rng = np.random.default_rng(11)
    p = rng.standard_normal(pr.n_aug)
    q = P.random_density(spec, seed=0)
    got = to_np(pr.apply_transpose(p))
    tol = 1e-12 if precision == "fp64" else 2e-5
    scale = np.linalg.norm(got) / np.sqrt(got.size)
    for i in rng.integers(0, pr.n_aug, 3):
        e = np.zeros(pr.n_aug)
        e[i] = 1.0
        want_i = float(p @ o.apply(e))
        assert abs(got[i] - want_i) < tol * scale, (i, got[i], want_i)
    lhs, rhs = float(got @ q), float(p @ o.apply(q))
    assert abs(lhs - rhs) < tol * np.linalg.norm(got) * np.linalg.norm(q), (lhs, rhs)
    pr.close()


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_star1024_fp64(bc):
    spec = P.cfg2_star_poisson(1024, 4096, bc=bc)
    o = make_oracle(spec)
    pr = make_problem(spec, "fp64")
    q = P.random_density(spec, seed=3)
    assert relerr(to_np(pr.apply(q)), o.apply(q)) < 1e-12
    b = o.rhs(spec.data, spec.g)
    xo, ko, _ = gmres(o.apply, b, 1e-12, 100)
    qg, ug, info = pr.solve(spec.data, spec.g, tol=1e-12, maxit=150)
    assert info.status == 0
    assert relerr(to_np(qg), xo) < 1e-10, relerr(to_np(qg), xo)
    uo = o.recover(xo, spec.data, spec.g)
    assert relerr(to_np(ug), uo) < 1e-10
    pr.close()


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_star1024_mixed(bc):
    spec = P.cfg2_star_poisson(1024, 4096, bc=bc)
    o = make_oracle(spec)
    pr = make_problem(spec, "mixed")
    q = P.random_density(spec, seed=3)
    assert relerr(to_np(pr.apply(q)), o.apply(q)) < 2e-5
    b = o.rhs(spec.data, spec.g)
    xo, _, _ = gmres(o.apply, b, 1e-12, 100)
    qg, ug, info = pr.solve(spec.data, spec.g, tol=1e-8, maxit=150)
    assert info.status == 0
    print(f"# star1024 mixed {bc}: {info.iters} its, true relres {info.true_relres_fp64:.2e}, "
          f"|q - q_oracle| {relerr(to_np(qg), xo):.2e}")
    assert relerr(to_np(qg), xo) < 1e-5, relerr(to_np(qg), xo)
    uo = o.recover(xo, spec.data, spec.g)
    assert relerr(to_np(ug), uo) < 1e-5
    pr.close()


def _off_breakpoints(X, h, margin):
    """Coordinates at least margin (in units of h) away from a grid line, where the 4-point
    kernel's second derivative jumps (central differences are exact to O(eps^2) only there)."""
    f = np.abs(X / h - np.round(X / h))
    return f > margin


def test_stokes512_gradient_central_difference():
    """dL/dX and dL/ddata of L = sum_x |w|^2 h^2 on the 512^2 Stokes star, from ibdl_backward,
    against central differences (eps = 1e-6) of the GPU's FP64 forward map solved to 1e-13:
    one random direction and 16 single components each, relative 1e-6 of the gradient's size.
    The five-point central difference is used: L varies on the kernel's width h = 1/512, and the
    three-point difference's O(eps^2) truncation error is 3e-5 of the directional derivative at
    eps = 1e-6 on this grid (measured: 2.85e-3, 2.85e-5, 3.6e-7 at eps = 1e-5, 1e-6, 1e-7).
    Coordinates within 5e-3 h of a grid line are left out of the X directions: the 4-point
    kernel's second derivative jumps there, so no difference quotient converges at its order."""
    spec = P.cfg5_stokes_star(512, 1024)
    pr = make_problem(spec, "fp64")
    m = spec.markers
    h = spec.L[0] / spec.n[0]
    h2 = h * h
    data = np.asarray(spec.data, dtype=np.float64)
    q, w, info = pr.solve(data, None, tol=1e-13, maxit=200)
    assert info.true_relres_fp64 < 1e-11, info
    dX, dd, ainfo = pr.backward(q, w, 2.0 * h2 * w, tol=1e-13, maxit=200)
    assert ainfo.true_relres_fp64 < 1e-11, ainfo
    dX, dd = to_np(dX), to_np(dd).reshape(data.shape)

    def loss(X, dat):
        pr.set_markers(X, m.nrm, m.ds)
        _, ww, _ = pr.solve(dat, None, tol=1e-13, maxit=200)
        return float(h2 * torch.sum(ww.double() ** 2))

    def central(f, eps):   # fourth-order central difference of f(t) at t = 0
        return (f(-2 * eps) - 8 * f(-eps) + 8 * f(eps) - f(2 * eps)) / (12 * eps)

    eps = 1e-6
    rng = np.random.default_rng(5)
    ok = _off_breakpoints(m.X, h, 5e-3)
    dirs = [rng.standard_normal(m.X.shape) * ok]
    for k in rng.choice(np.flatnonzero(ok.reshape(-1)), 16, replace=False):
        v = np.zeros(m.X.size)
        v[k] = 1.0
        dirs.append(v.reshape(m.X.shape))
    scale = np.abs(dX).max()
    for v in dirs:
        fd = central(lambda t: loss(m.X + t * v, data), eps)
        an = float(np.sum(dX * v))
        assert abs(an - fd) < 1e-6 * max(abs(fd), scale), (an, fd)
    pr.set_markers(m.X, m.nrm, m.ds)
    dirs = [rng.standard_normal(data.shape)]
    for k in rng.choice(data.size, 16, replace=False):
        v = np.zeros(data.size)
        v[k] = 1.0
        dirs.append(v.reshape(data.shape))
    scale = np.abs(dd).max()
    for v in dirs:
        fd = central(lambda t: loss(m.X, data + t * v), eps)
        an = float(np.sum(dd * v))
        assert abs(an - fd) < 1e-6 * max(abs(fd), scale), (an, fd)
    pr.close()


def test_stokes512_fp64():
    spec = P.cfg5_stokes_star(512, 1024)
    o = make_oracle(spec)
    pr = make_problem(spec, "fp64")
    q = P.random_density(spec, seed=4)
    assert relerr(to_np(pr.apply(q)), o.apply(q)) < 1e-12
    b = o.rhs(spec.data, spec.g)
    xo, _, _ = gmres(o.apply, b, 1e-12, 200)
    qg, ug, info = pr.solve(spec.data, spec.g, tol=1e-12, maxit=200)
    assert info.status == 0
    assert relerr(to_np(qg), xo) < 1e-10, relerr(to_np(qg), xo)
    uo = o.recover(xo, spec.data, spec.g)
    assert relerr(to_np(ug).reshape(uo.shape), uo) < 1e-10
    _, k8, _ = gmres(o.apply, b, 1e-8, 200)
    _, _, i8 = pr.solve(spec.data, spec.g, tol=1e-8, maxit=200, want_u=False)
    assert abs(i8.iters - k8) <= 1, (i8.iters, k8)
    pr.close()
