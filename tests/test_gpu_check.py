"""IBDL_CHECK=1: the opt-in scan of device arrays for NaN and infinities at the calls' boundaries.

A handle created with IBDL_CHECK=1 in the environment returns IBDL_ERR_NONFINITE when the markers,
the boundary data, the forcing, a density or a grid right-hand side holds a NaN or an infinity; a
handle created without it does not inspect device data (an apply passes a NaN through; GMRES still
stops on a non-finite right-hand side norm, which it reads on the host anyway).  Clean inputs give
the same results with and without the check.
"""
import numpy as np
import pytest
import torch

import paper_2210_07403_amd as ibdl
from workloads import problems as P

from _helpers import make_problem, relerr, to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]

NONFINITE = -5


def _checked(spec, precision, monkeypatch):
    monkeypatch.setenv("IBDL_CHECK", "1")
    pr = make_problem(spec, precision)
    monkeypatch.delenv("IBDL_CHECK")
    return pr


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_check_rejects_nonfinite_inputs(precision, monkeypatch):
    spec = P.starfish_poisson(64, 0.75)
    pr = _checked(spec, precision, monkeypatch)
    data = np.array(spec.data, dtype=np.float64)
    data[7] = np.nan
    with pytest.raises(ibdl.IBDLError) as e:
        pr.solve(data, spec.g, tol=1e-8, maxit=20)
    assert e.value.status == NONFINITE and "data" in str(e.value)
    g = np.array(spec.g, dtype=np.float64)
    g[3, 5] = np.inf
    with pytest.raises(ibdl.IBDLError) as e:
        pr.solve(spec.data, g, tol=1e-8, maxit=20)
    assert e.value.status == NONFINITE and "g" in str(e.value)
    q = np.zeros(pr.n_aug)
    q[1] = -np.inf
    with pytest.raises(ibdl.IBDLError) as e:
        pr.apply(q)
    assert e.value.status == NONFINITE
    with pytest.raises(ibdl.IBDLError) as e:
        pr.apply_transpose(q)
    assert e.value.status == NONFINITE
    rhs = np.zeros((64, 64))
    rhs[10, 10] = np.nan
    with pytest.raises(ibdl.IBDLError) as e:
        pr.grid_solve(torch.as_tensor(rhs))
    assert e.value.status == NONFINITE and "rhs" in str(e.value)
    m = spec.markers
    X = m.X.copy()
    X[2, 1] = np.nan
    with pytest.raises(ibdl.IBDLError) as e:
        pr.set_markers(X, m.nrm, m.ds)
    assert e.value.status == NONFINITE and "X" in str(e.value)
    pr.close()


def test_check_rejects_nonfinite_markers_at_create(monkeypatch):
    spec = P.starfish_poisson(64, 0.75)
    m = spec.markers
    ds = m.ds.copy()
    ds[0] = np.inf
    monkeypatch.setenv("IBDL_CHECK", "1")
    with pytest.raises(ibdl.IBDLError) as e:
        ibdl.Problem(spec.dim, spec.n, spec.L, spec.origin, m.X, m.nrm, ds, pde=spec.pde, kappa=spec.kappa,
                     mu=spec.mu, bc=spec.bc, eta=spec.eta, kernel=spec.kernel, disc=spec.disc, precision="fp64")
    assert e.value.status == NONFINITE and "ds" in str(e.value)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_check_leaves_clean_results_alone(precision, monkeypatch):
    spec = P.cylinder_array(128, 0.2)
    pr = _checked(spec, precision, monkeypatch)
    ref = make_problem(spec, precision)
    q1, u1, i1 = pr.solve(spec.data, spec.g, tol=1e-10, maxit=100)
    q0, u0, i0 = ref.solve(spec.data, spec.g, tol=1e-10, maxit=100)
    assert i1.status == 0 and i1.iters == i0.iters
    assert np.array_equal(to_np(q1), to_np(q0)) and np.array_equal(to_np(u1), to_np(u0))
    qr = np.random.default_rng(3).standard_normal(pr.n_aug)
    assert relerr(to_np(pr.apply(qr)), to_np(ref.apply(qr))) == 0.0
    pr.close()
    ref.close()


def test_without_check_device_data_is_not_inspected(monkeypatch):
    """Without IBDL_CHECK an apply passes a NaN through (no scan); a solve still stops at its
    right-hand side norm, which GMRES checks on the host in any case."""
    monkeypatch.delenv("IBDL_CHECK", raising=False)
    spec = P.starfish_poisson(64, 0.75)
    pr = make_problem(spec, "fp64")
    q = np.zeros(pr.n_aug)
    q[1] = np.nan
    y = to_np(pr.apply(q))
    assert not np.all(np.isfinite(y))
    data = np.array(spec.data, dtype=np.float64)
    data[7] = np.nan
    with pytest.raises(ibdl.IBDLError) as e:
        pr.solve(data, spec.g, tol=1e-8, maxit=5, want_u=False)
    assert e.value.status == NONFINITE and "right-hand side" in str(e.value)
    pr.close()
