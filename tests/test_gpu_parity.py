"""GPU parity: the HIP library through its C ABI against the FP64 CPU oracle, element by element.

Tolerances (relative to the max-norm of the oracle result):
  * FP64 path: spread / interp / grid solves / operator applies 1e-12 (rounding of a few FFT
    passes of length <= 1024 and of 16-64-term stencil sums);
  * mixed path (float grid work): 2e-5 for single applies, 1e-5 for solved densities;
  * solves: 1e-10 with the GPU and the oracle both iterated to 1e-13.
"""
import numpy as np
import pytest
import torch

from oracle.gmres import gmres
from oracle.ib import Grid, interp as o_interp, spread as o_spread
from oracle import grid as G
from workloads import problems as P
from workloads import geometry as geo

from _helpers import make_oracle, make_problem, relerr, to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]


def _markers(dim, n, L, origin, count, seed):
    rng = np.random.default_rng(seed)
    X = np.array(origin) + rng.uniform(0, 1, (count, dim)) * np.array(L)
    h = L[0] / n[0]
    X[0] = origin                                    # on a node and on the periodic seam
    X[1, 0] = origin[0] + L[0] - 1e-7 * h            # just below the seam
    X[2] = np.array(origin) + 5 * h                  # exactly on a node
    X[3, 0] = origin[0] - 0.3 * h                    # outside the box (wraps)
    nrm = rng.standard_normal((count, dim))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    ds = rng.uniform(0.5, 1.5, count) * h ** (dim - 1)
    return X, nrm, ds


def _spec_like(dim, n, L, origin, X, nrm, ds, **kw):
    mk = geo.Markers(X, nrm, ds, float(ds.sum()))
    base = dict(pde="screened", kappa=1.0, mu=1.0, bc="dirichlet", eta=0.0, kernel="peskin4", disc="fd2")
    base.update(kw)
    return P.ProblemSpec("adhoc", dim, tuple(n), tuple(L), tuple(origin), base["pde"], base["kappa"],
                         base["mu"], base["bc"], base["eta"], base["kernel"], base["disc"], mk,
                         np.zeros(len(ds)), None)


GEOMS = [
    (2, (64, 32), (1.0, 0.5), (0.0, 0.0), 301),
    (2, (16, 16), (2.0, 2.0), (-1.0, -1.0), 7),
    (3, (32, 16, 16), (2.0, 1.0, 1.0), (0.0, -0.5, 0.0), 517),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kernel", ["peskin4", "cos4", "bspline6"])
@pytest.mark.parametrize("gi", range(len(GEOMS)))
def test_spread_interp(gi, kernel, precision):
    dim, n, L, origin, count = GEOMS[gi]
    X, nrm, ds = _markers(dim, n, L, origin, count, 10 + gi)
    spec = _spec_like(dim, n, L, origin, X, nrm, ds, kernel=kernel,
                      disc="spectral" if kernel == "bspline6" else "fd2")
    pr = make_problem(spec, precision)
    grid = Grid(dim, n, L, origin)
    rng = np.random.default_rng(3)
    F = rng.standard_normal((count, 3))
    want = o_spread(grid, X, ds, F, kernel)
    got = to_np(pr.spread(F))
    tol = 1e-13 if precision == "fp64" else 2e-6
    assert relerr(got, want) < tol
    u = rng.standard_normal((2,) + grid.shape)
    assert relerr(to_np(pr.interp(torch.as_tensor(u))), o_interp(grid, X, u, kernel)) < tol
    pr.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", [
    dict(dim=2, n=(64, 32), L=(1.0, 0.5), pde="screened", kappa=3.0, disc="fd2"),
    dict(dim=2, n=(32, 64), L=(0.5, 1.0), pde="poisson", kappa=0.0, disc="fd2"),
    dict(dim=2, n=(64, 64), L=(2.0, 2.0), pde="screened", kappa=1.0, disc="spectral"),
    dict(dim=3, n=(16, 32, 64), L=(0.25, 0.5, 1.0), pde="screened", kappa=10.0, disc="fd2"),
    dict(dim=3, n=(32, 32, 16), L=(1.0, 1.0, 0.5), pde="poisson", kappa=0.0, disc="spectral"),
    dict(dim=2, n=(64, 64), L=(2.0, 2.0), pde="stokes", kappa=0.0, disc="spectral"),
    dict(dim=2, n=(32, 64), L=(1.0, 2.0), pde="stokes", kappa=2.0, disc="spectral"),
    dict(dim=2, n=(64, 64), L=(1.0, 1.0), pde="stokes", kappa=0.0, disc="fd2"),
    # long last axes: the fused passes that hold 8 elements per thread (two accumulators, or
    # 1024-point lines in double)
    dict(dim=2, n=(16, 1024), L=(0.125, 8.0), pde="stokes", kappa=1.0, disc="spectral"),
    dict(dim=2, n=(32, 256), L=(0.5, 4.0), pde="stokes", kappa=0.0, disc="spectral"),
    dict(dim=2, n=(16, 128), L=(0.125, 1.0), pde="stokes", kappa=0.0, disc="fd2"),
    dict(dim=2, n=(16, 1024), L=(0.125, 8.0), pde="screened", kappa=3.0, disc="fd2"),
    dict(dim=2, n=(16, 1024), L=(0.125, 8.0), pde="screened", kappa=3.0, disc="spectral"),
])
def test_grid_solve(case, precision):
    dim, n, L = case["dim"], case["n"], case["L"]
    origin = (0.0,) * dim
    X, nrm, ds = _markers(dim, n, L, origin, 20, 1)
    spec = _spec_like(dim, n, L, origin, X, nrm, ds, pde=case["pde"], kappa=case["kappa"],
                      disc=case["disc"], mu=1.3)
    pr = make_problem(spec, precision)
    o = make_oracle(spec)
    nq = dim if case["pde"] == "stokes" else 1
    rhs = np.random.default_rng(5).standard_normal((nq,) + o.grid.shape)
    got = to_np(pr.grid_solve(torch.as_tensor(rhs)))
    want = o._g_response(rhs if nq > 1 else rhs[0])
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert relerr(got.reshape(want.shape), want) < tol
    pr.close()


OPERATORS = {
    "helmholtz_fd": lambda: P.helmholtz_circle(64, 0.75),
    "helmholtz_cos4": lambda: P.cfg1_circle_cos4(),
    "helmholtz_spectral": lambda: P.helmholtz_circle(64, 1.0, disc="spectral"),
    "starfish_poisson": lambda: P.starfish_poisson(64, 0.75),
    "neumann": lambda: P.neumann_circle(64),
    "completed_poisson": lambda: P.completed_poisson_exterior(64, 2.0, 10.0, "trig"),
    "completed_spectral": lambda: P.ProblemSpec(**{**P.completed_poisson_exterior(64, 2.0, 10.0, "trig").__dict__,
                                                 "disc": "spectral"}),
    "brinkman": lambda: P.brinkman_circle(32, 1.0),
    "stokes_exterior": lambda: P.stokes_exterior_circle(32, 10.0),
    "stokes_exterior_fd": lambda: P.ProblemSpec(**{**P.stokes_exterior_circle(32, 10.0).__dict__, "disc": "fd2"}),
    "sphere_3d": lambda: P.cfg3_sphere(32, 11),
    "sphere_3d_spectral": lambda: P.ProblemSpec(**{**P.cfg3_sphere(16, 5).__dict__, "disc": "spectral",
                                                  "n": (16, 16, 16)}),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", sorted(OPERATORS))
def test_apply(name, precision):
    spec = OPERATORS[name]()
    pr = make_problem(spec, precision)
    o = make_oracle(spec)
    q = P.random_density(spec, seed=2)
    got = to_np(pr.apply(q))
    want = o.apply(q)
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert relerr(got, want) < tol, relerr(got, want)
    # bitwise deterministic: no atomics on floating-point data anywhere in the apply
    again = to_np(pr.apply(q))
    assert np.array_equal(got, again)
    pr.close()


SOLVES = ["helmholtz_fd", "helmholtz_cos4", "starfish_poisson", "neumann", "completed_poisson", "brinkman",
          "stokes_exterior", "sphere_3d"]


@pytest.mark.parametrize("name", SOLVES)
def test_solve_fp64(name):
    spec = OPERATORS[name]()
    pr = make_problem(spec, "fp64")
    o = make_oracle(spec)
    b = o.rhs(spec.data, spec.g)
    xo, ko, _ = gmres(o.apply, b, 1e-13, 300)
    q, u, info = pr.solve(spec.data, spec.g, tol=1e-13, maxit=200)
    assert info.status == 0 and info.true_relres_fp64 < 1e-12
    assert relerr(to_np(q), xo) < 1e-10
    uo = o.recover(xo, spec.data, spec.g)
    assert relerr(to_np(u).reshape(uo.shape), uo) < 1e-10
    # same Krylov process: iteration counts at the thesis tolerance agree
    _, k8, _ = gmres(o.apply, b, spec.tol, 300)
    _, _, info8 = pr.solve(spec.data, spec.g, tol=spec.tol, maxit=200, want_u=False)
    assert abs(info8.iters - k8) <= 1, (info8.iters, k8)
    pr.close()


@pytest.mark.parametrize("name", ["helmholtz_fd", "starfish_poisson", "neumann", "stokes_exterior", "sphere_3d"])
def test_solve_mixed(name):
    spec = OPERATORS[name]()
    pr = make_problem(spec, "mixed")
    o = make_oracle(spec)
    xo, _, _ = gmres(o.apply, o.rhs(spec.data, spec.g), 1e-13, 300)
    q, u, info = pr.solve(spec.data, spec.g, tol=1e-6, maxit=200)
    assert info.status == 0
    assert relerr(to_np(q), xo) < 1e-5, relerr(to_np(q), xo)
    uo = o.recover(xo, spec.data, spec.g)
    assert relerr(to_np(u).reshape(uo.shape), uo) < 1e-5
    pr.close()


def test_zero_rhs_and_single_marker():
    spec = P.helmholtz_circle(16, 1.0)
    spec.markers = geo.Markers(spec.markers.X[:1], spec.markers.nrm[:1], spec.markers.ds[:1], 1.0)
    spec.data = spec.data[:1]
    pr = make_problem(spec)
    o = make_oracle(spec)
    q = np.array([0.7])
    assert relerr(to_np(pr.apply(q)), o.apply(q)) < 1e-12
    qz, uz, info = pr.solve(np.zeros(1), None, tol=1e-10)
    assert info.iters == 0 and np.all(to_np(qz) == 0) and np.all(to_np(uz) == 0)
    pr.close()


def test_invalid_arguments_raise():
    import paper_2210_07403_amd as ibdl
    spec = P.helmholtz_circle(16, 1.0)
    pr = make_problem(spec)
    with pytest.raises(ValueError):
        pr.apply(np.zeros(3))
    with pytest.raises(ibdl.IBDLError):
        pr.solve(spec.data, None, tol=1e-8, maxit=0)
    pr.close()


@pytest.mark.parametrize("name", ["helmholtz_fd", "completed_poisson", "neumann", "stokes_exterior", "sphere_3d"])
def test_solve_refined_mixed_reaches_fp64_accuracy(name):
    """Iterative refinement on a mixed handle: float-grid GMRES corrections, double residuals,
    down to a double-precision true residual far below what the float operator resolves.  Both
    sides are solved to 1e-13, as in the FP64 solve test; the solution error is bounded by the
    condition number times the residual (the completed operator's is the largest here)."""
    spec = OPERATORS[name]()
    pr = make_problem(spec, "mixed")
    o = make_oracle(spec)
    # a mixed handle receives g~ in float: the oracle solves with the same rounded forcing
    g32 = None if spec.g is None else np.asarray(spec.g, dtype=np.float32).astype(np.float64)
    xo, _, _ = gmres(o.apply, o.rhs(spec.data, g32), 1e-13, 300)
    q, u, info = pr.solve_refined(spec.data, spec.g, tol=1e-13, maxit=100, inner_tol=1e-4, max_rounds=30)
    assert info.status == 0 and info.true_relres_fp64 <= 1e-13, info
    assert relerr(to_np(q), xo) < 1e-9, relerr(to_np(q), xo)
    pr.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["helmholtz_fd", "stokes_exterior", "sphere_3d"])
def test_gmres_graph_replays_match_direct_launches(name, precision):
    """GMRES replays the captured graph of the operator apply once per iteration.  Several solves
    and a backward solve, with direct applies and synchronisations between them, give the same
    bits as the same calls with the graph off."""
    spec = OPERATORS[name]()
    pr = make_problem(spec, precision)
    qin = P.random_density(spec, seed=9)
    pr.set_graph(False)
    q0, u0, i0 = pr.solve(spec.data, spec.g, tol=1e-9, maxit=200)
    y0 = to_np(pr.apply(qin))
    q0, u0 = to_np(q0), to_np(u0)
    psi = torch.as_tensor(np.random.default_rng(2).standard_normal(u0.shape), device="cuda").to(
        torch.float64 if precision == "fp64" else torch.float32)
    can_adjoint = spec.bc != "neumann"
    if can_adjoint:
        dX0, dd0, _ = pr.backward(torch.as_tensor(q0, device="cuda"), torch.as_tensor(u0, device="cuda"), psi,
                                  tol=1e-9, maxit=200)
        dX0, dd0 = to_np(dX0), to_np(dd0)
    pr.set_graph(True)
    for rep in range(3):
        q1, u1, i1 = pr.solve(spec.data, spec.g, tol=1e-9, maxit=200)
        assert i1.iters == i0.iters, rep
        assert np.array_equal(to_np(q1), q0), rep
        assert np.array_equal(to_np(u1), u0), rep
        assert np.array_equal(to_np(pr.apply(qin)), y0), rep
        torch.cuda.synchronize()
        if can_adjoint:
            dX1, dd1, _ = pr.backward(torch.as_tensor(q0, device="cuda"), torch.as_tensor(u0, device="cuda"), psi,
                                      tol=1e-9, maxit=200)
            assert np.array_equal(to_np(dX1), dX0), rep
            assert np.array_equal(to_np(dd1), dd0), rep
    pr.close()


def _tiles_reference(spec):
    """Busy tiles, active rows and busy row segments from the markers' 6-node windows (node
    s = floor((x - origin) / h) - 2 and the five after it on each axis, periodic)."""
    n = spec.n
    dim = spec.dim
    h = spec.L[0] / n[0]
    X = np.asarray(spec.markers.X, dtype=np.float64)
    xi = (X - np.asarray(spec.origin)) / h
    xi = xi - np.asarray(n) * np.floor(xi / np.asarray(n))
    s = (np.floor(xi).astype(np.int64) - 2) % np.asarray(n)
    tile = (16, 4, 8) if dim == 3 else (16, 16)
    nt = [n[d] // tile[d] for d in range(dim)]
    busy = np.zeros(tuple(reversed(nt)), dtype=bool)     # [tz][ty][tx] or [ty][tx]
    nplanes = n[2] if dim == 3 else 1
    lo = np.full(nplanes, n[1], dtype=np.int64)
    hi = np.full(nplanes, -1, dtype=np.int64)
    off = np.arange(6)
    for m in range(len(X)):
        nodes = [(s[m, d] + off) % n[d] for d in range(dim)]
        tiles = [np.unique(nodes[d] // tile[d]) for d in range(dim)]
        if dim == 3:
            busy[np.ix_(tiles[2], tiles[1], tiles[0])] = True
            for z in nodes[2]:
                lo[z] = min(lo[z], nodes[1].min())
                hi[z] = max(hi[z], nodes[1].max())
        else:
            busy[np.ix_(tiles[1], tiles[0])] = True
            lo[0] = min(lo[0], nodes[1].min())
            hi[0] = max(hi[0], nodes[1].max())
    nact, nseg = 0, 0
    for z in range(nplanes):
        for y in range(lo[z], hi[z] + 1):
            nact += 1
            nseg += int(busy[z // tile[2], y // tile[1]].sum()) if dim == 3 else int(busy[y // tile[1]].sum())
    # span along the last axis: the z planes holding an active row (3-D), the active rows (2-D)
    if dim == 3:
        zs = np.nonzero(lo <= hi)[0]
        span = (int(zs.min()), int(zs.max())) if len(zs) else (nplanes, -1)
    else:
        span = (int(lo[0]), int(hi[0]))
    return int(busy.sum()), nact, nseg, tile, span


@pytest.mark.parametrize("name", ["sphere_3d", "helmholtz_fd", "stokes_exterior"])
def test_spread_tiles_and_active_rows(name):
    """The tile binning and the row bookkeeping the apply's x passes rely on, recounted on the host."""
    spec = OPERATORS[name]()
    pr = make_problem(spec, "mixed")
    nbusy, nact, nseg, tile, span = _tiles_reference(spec)
    got_busy, got_seg, got_tile = pr.spread_tiles()
    assert got_tile[:spec.dim] == tile
    assert (got_busy, pr.active_rows()[0], got_seg) == (nbusy, nact, nseg)
    assert pr.active_span() == span
    pr.close()


def _bodies_3d(centres, r, freq, disc):
    """Icospheres on a 32^3 unit grid (kappa 10), for the z-plane bookkeeping of the apply."""
    sph = [geo.icosphere(c, r, freq) for c in centres]
    X = np.vstack([m.X for m in sph])
    nrm = np.vstack([m.nrm for m in sph])
    ds = np.concatenate([m.ds for m in sph])
    return _spec_like(3, (32, 32, 32), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), X, nrm, ds, kappa=10.0, disc=disc)


PLANE_CASES = {
    # two bodies apart in z: planes without an active row between the first and the last
    "gap": ([(0.5, 0.5, 0.22), (0.45, 0.55, 0.72)], 0.08, 3),
    # a body across the periodic seam in z: active planes at both ends of the axis
    "wrap": ([(0.5, 0.5, 0.02)], 0.15, 5),
    # one body off the centre: a range starting well inside the axis
    "offset": ([(0.3, 0.6, 0.7)], 0.15, 5),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("disc", ["fd2", "spectral"])
@pytest.mark.parametrize("case", sorted(PLANE_CASES))
def test_apply_plane_range(case, disc, precision):
    """The 3-D apply runs its y passes over the z planes between the first and the last holding
    an active row and masks the last-axis pass to them: the span against a host recount, A q and
    A^T p against the oracle (one spread field with FD symbols, several with spectral ones)."""
    centres, r, freq = PLANE_CASES[case]
    spec = _bodies_3d(centres, r, freq, disc)
    pr = make_problem(spec, precision)
    *_, span = _tiles_reference(spec)
    assert pr.active_span() == span
    if case == "wrap":
        assert span == (0, 31)
    else:
        assert 0 < span[0] and span[1] < 31
    o = make_oracle(spec)
    tol = 1e-12 if precision == "fp64" else 2e-5
    q = np.random.default_rng(6).standard_normal(o.n_aug)
    assert relerr(to_np(pr.apply(q)), o.apply(q)) < tol
    A = o.assemble()
    p = np.random.default_rng(8).standard_normal(o.n_aug)
    assert relerr(to_np(pr.apply_transpose(p)), A.T @ p) < tol
    pr.close()


def test_spread_tiles_seam_crossing():
    """Markers on and across the periodic seams (windows that wrap) in 3-D."""
    X, nrm, ds = _markers(3, (32, 16, 16), (2.0, 1.0, 1.0), (0.0, -0.5, 0.0), 517, 5)
    spec = _spec_like(3, (32, 16, 16), (2.0, 1.0, 1.0), (0.0, -0.5, 0.0), X, nrm, ds)
    pr = make_problem(spec, "fp64")
    nbusy, nact, nseg, _, span = _tiles_reference(spec)
    got_busy, got_seg, _ = pr.spread_tiles()
    assert (got_busy, pr.active_rows()[0], got_seg) == (nbusy, nact, nseg)
    assert pr.active_span() == span
    pr.close()
