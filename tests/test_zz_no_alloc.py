"""ibdl_grid_solve_static, the grid solve that allocates nothing (its half spectra and tables live
in a static device array), called through the C ABI and compared with the handle's
ibdl_grid_solve on the same input: two calls in a row, the second smaller, so the second runs on
what the first left in the shared array.  Also the host-side rejection of a grid beyond the
array, and agreement with the oracle's grid solve."""
import ctypes

import numpy as np
import pytest

from oracle import grid as G
from oracle.ib import Grid
from paper_2210_07403_amd import _binding as B

from _helpers import relerr


def _markers(dim):
    # a few markers away from the box faces; the handle needs some, the grid solve ignores them
    rng = np.random.default_rng(7)
    X = 0.3 + 0.4 * rng.random((8, dim))
    nrm = np.zeros((8, dim))
    nrm[:, 0] = 1.0
    return X, nrm, np.full(8, 0.01)


def _case(lib, dim, n, pde, kappa, disc, precision, seed):
    import torch
    L = 1.0
    X, nrm, ds = _markers(dim)
    pr = lib.Problem(dim, (n,) * dim, (L,) * dim, (0.0,) * dim, X, nrm, ds, pde=pde, kappa=kappa, mu=1.3,
                     disc=disc, precision=precision)
    nq = dim if pde == "stokes" else 1
    rng = np.random.default_rng(seed)
    rhs_np = rng.standard_normal((nq,) + (n,) * dim)
    rhs = torch.as_tensor(rhs_np, device="cuda").to(pr.grid_dtype).contiguous()
    want = pr.grid_solve(rhs)
    got = torch.empty_like(rhs)
    cfg = B.Config()
    cfg.dim = dim
    for d in range(3):
        cfg.n[d] = n if d < dim else 1
        cfg.L[d] = L
        cfg.origin[d] = 0.0
    cfg.pde, cfg.kappa, cfg.mu = B.PDE[pde], float(kappa), 1.3
    cfg.bc, cfg.eta, cfg.kernel = 0, 0.0, 0
    cfg.disc, cfg.precision = B.DISC[disc], B.PRECISION[precision]
    cfg.stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cfg.method = 0
    print(f"# grid_solve_static dim={dim} n={n} pde={pde} disc={disc} {precision}", flush=True)
    st = B.load().ibdl_grid_solve_static(ctypes.byref(cfg), rhs.data_ptr(), got.data_ptr())
    assert st == 0, B.load().ibdl_last_error(None)
    torch.cuda.synchronize()
    pr.close()
    return rhs_np, want.double().cpu().numpy(), got.double().cpu().numpy()


@pytest.mark.gpu
@pytest.mark.parametrize("first,second", [
    ((2, 512, "stokes", 0.0, "spectral", "fp64"), (2, 64, "screened", 1.0, "fd2", "fp64")),
    ((3, 128, "screened", 10.0, "fd2", "mixed"), (3, 32, "poisson", 0.0, "spectral", "mixed")),
    ((2, 1024, "poisson", 0.0, "fd2", "fp64"), (2, 128, "stokes", 2.0, "fd2", "mixed")),
])
def test_static_matches_handle_twice(lib, first, second):
    for k, c in enumerate((first, second)):
        rhs, want, got = _case(lib, *c, seed=11 + k)
        tol = 1e-12 if c[-1] == "fp64" else 2e-6
        assert relerr(got, want) < tol, (c, relerr(got, want))
        if c[1] <= 128 and c[2] != "stokes":      # the oracle beside it on the small scalar cases
            g = Grid(c[0], (c[1],) * c[0], (1.0,) * c[0], (0.0,) * c[0])
            uo = G.solve(g, rhs[0], c[4], c[3] ** 2)
            assert relerr(got[0], uo) < (1e-11 if c[-1] == "fp64" else 2e-5), relerr(got[0], uo)


def test_static_rejects_grid_beyond_scratch_on_host():
    """256^3 in float needs about 75 MB of spectra: refused before any device work."""
    cfg = B.Config()
    cfg.dim = 3
    for d in range(3):
        cfg.n[d], cfg.L[d], cfg.origin[d] = 256, 1.0, 0.0
    cfg.pde, cfg.kappa, cfg.mu, cfg.bc, cfg.eta, cfg.kernel = 0, 10.0, 1.0, 0, 0.0, 0
    cfg.disc, cfg.precision, cfg.stream, cfg.method = 0, 1, None, 0
    lib = B.load()
    assert lib.ibdl_grid_solve_static(ctypes.byref(cfg), ctypes.c_void_p(8), ctypes.c_void_p(8)) == -2
    assert b"static scratch" in lib.ibdl_last_error(None)
    assert lib.ibdl_grid_solve_static(None, None, None) == -1
