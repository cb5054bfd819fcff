"""GPU parity at the workloads' full sizes, in the configuration the benchmark times.

* 256^3 sphere (73,962 markers), mixed precision: the operator apply against the FP64 oracle on
  every marker (2e-5), the FP64 apply (1e-12), and the mixed solve at 1e-8 against the oracle's
  solution (1e-5); the recovered grid solution on a sample of nodes; the transposed apply on
  sampled entries and by adjointness against the oracle's forward apply.
* 1024^2 star (4,096 markers), Dirichlet and Neumann, FP64: apply (1e-12) and solve (1e-10).
* 512^2 exterior Stokes star (1,024 markers, eta = 10, spectral), FP64: apply (1e-12) and solve
  (1e-10, with ubar), and the 1e-8 iteration count against the oracle's.
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
