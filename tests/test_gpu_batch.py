"""GPU parity of batched solves (ibdl_batch_*): every problem of a batch against the oracle and
against the single-problem path, graph replays against direct launches.

Tolerances as for single problems: applies 1e-12 (FP64) / 2e-5 (mixed) relative to the oracle;
solved densities 1e-10 (FP64 at tol 1e-13) / 1e-5 (mixed).
"""
import numpy as np
import pytest
import torch

import paper_2210_07403_amd as ibdl
from oracle.gmres import gmres
from workloads import problems as P

from _helpers import make_oracle, make_problem, relerr, to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")]


def _as_dict(spec):
    m = spec.markers
    return dict(dim=spec.dim, n=spec.n, L=spec.L, origin=spec.origin, X=m.X, nrm=m.nrm, ds=m.ds, pde=spec.pde,
                kappa=spec.kappa, kernel=spec.kernel)


def _small_batch():
    """Uneven grids and marker counts, two PDEs, repeated grids (so groups hold several problems)."""
    specs = P.cfg4_batch(nprob=7, seed=11, sizes=(32, 64, 128))
    specs.append(P.helmholtz_circle(64, 1.0))               # screened, its own group (box, kappa)
    specs.append(P.helmholtz_circle(64, 0.75))
    specs.append(P.starfish_poisson(64, 0.75))              # Poisson on another box
    # batches solve with g~ = 0
    return [P.ProblemSpec(**{**s.__dict__, "g": None}) for s in specs]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_apply_matches_oracle(precision):
    specs = _small_batch()
    bt = ibdl.Batch([_as_dict(s) for s in specs], precision=precision)
    qs = [np.random.default_rng(100 + k).standard_normal(s.n_ib) for k, s in enumerate(specs)]
    ys = bt.apply(qs)
    tol = 1e-12 if precision == "fp64" else 2e-5
    for s, q, y in zip(specs, qs, ys):
        want = make_oracle(s).apply(q)
        assert relerr(to_np(y), want) < tol, (s.name, relerr(to_np(y), want))
    assert len(bt.groups()) >= 3
    bt.close()


def test_batch_solve_fp64_matches_oracle_and_single():
    specs = _small_batch()
    bt = ibdl.Batch([_as_dict(s) for s in specs], precision="fp64")
    qs, us, infos = bt.solve([s.data for s in specs], tol=1e-13, maxit=200)
    for s, q, u, info in zip(specs, qs, us, infos):
        o = make_oracle(s)
        b = o.rhs(s.data, s.g)
        xo, _, _ = gmres(o.apply, b, 1e-13, 300)
        assert info.status == 0 and info.true_relres_fp64 < 1e-12, (s.name, info)
        assert relerr(to_np(q), xo) < 1e-10, (s.name, relerr(to_np(q), xo))
        uo = o.recover(xo, s.data, s.g)
        assert relerr(to_np(u), uo) < 1e-10
    # the same GMRES as the single-problem path: iteration counts at the workload tolerance agree
    _, _, infos8 = bt.solve([s.data for s in specs], tol=1e-8, maxit=200, want_u=False)
    for s, info in zip(specs, infos8):
        pr = make_problem(s, "fp64")
        _, _, one = pr.solve(s.data, s.g, tol=1e-8, maxit=200, want_u=False)
        assert abs(one.iters - info.iters) <= 1, (s.name, one.iters, info.iters)
        pr.close()
    bt.close()


def test_batch_solve_mixed():
    specs = _small_batch()
    bt = ibdl.Batch([_as_dict(s) for s in specs], precision="mixed")
    qs, us, infos = bt.solve([s.data for s in specs], tol=1e-6, maxit=200)
    for s, q, info in zip(specs, qs, infos):
        o = make_oracle(s)
        xo, _, _ = gmres(o.apply, o.rhs(s.data, s.g), 1e-13, 300)
        assert info.status == 0
        assert relerr(to_np(q), xo) < 1e-5, (s.name, relerr(to_np(q), xo))
    bt.close()


def test_graph_replays_match_direct_launches():
    """Replays of the captured graph, with direct launches and synchronisations in between, give
    the same bits as the directly launched batch every time."""
    specs = _small_batch()
    data = [s.data for s in specs]
    bt = ibdl.Batch([_as_dict(s) for s in specs], precision="mixed")
    bt.set_graph(False)
    q0, _, i0 = bt.solve(data, tol=1e-8, maxit=100, want_u=False)
    ref = [to_np(q) for q in q0]
    qs_in = [np.random.default_rng(7 + k).standard_normal(s.n_ib) for k, s in enumerate(specs)]
    y_direct = [to_np(y) for y in bt.apply(qs_in)]
    for rep in range(3):
        bt.set_graph(True)
        q1, _, i1 = bt.solve(data, tol=1e-8, maxit=100, want_u=False)
        for a, b in zip(q1, ref):
            assert np.array_equal(to_np(a), b), rep
        assert [x.iters for x in i1] == [x.iters for x in i0]
        y_graph = [to_np(y) for y in bt.apply(qs_in)]
        for a, b in zip(y_graph, y_direct):
            assert np.array_equal(a, b), rep
        bt.set_graph(False)
        torch.cuda.synchronize()
        y_again = [to_np(y) for y in bt.apply(qs_in)]
        for a, b in zip(y_again, y_direct):
            assert np.array_equal(a, b), rep
    bt.close()


def test_full_size_batch_sampled():
    """The 64-problem workload (grids 128, 256, 512; 256-2048 markers): every problem solved in one
    batch, mixed precision; sampled problems of each grid size against a single-problem FP64 solve,
    and the operator of one problem per grid size against the oracle."""
    specs = P.cfg4_batch()
    bt = ibdl.Batch([_as_dict(s) for s in specs], precision="mixed")
    qs, _, infos = bt.solve([s.data for s in specs], tol=1e-8, maxit=100, want_u=False)
    assert all(i.status == 0 and i.true_relres_fp64 < 1e-6 for i in infos)
    assert max(i.iters for i in infos) <= 40
    seen = set()
    for k, s in enumerate(specs):
        if s.n[0] in seen:
            continue
        seen.add(s.n[0])
        pr = make_problem(s, "fp64")
        q1, _, _ = pr.solve(s.data, None, tol=1e-10, maxit=200, want_u=False)
        assert relerr(to_np(qs[k]), to_np(q1)) < 1e-5, (s.name, relerr(to_np(qs[k]), to_np(q1)))
        qr = np.random.default_rng(k).standard_normal(s.n_ib)
        y = bt.apply([qr if j == k else np.zeros(t.n_ib) for j, t in enumerate(specs)])[k]
        assert relerr(to_np(y), make_oracle(s).apply(qr)) < 2e-5
        pr.close()
    assert seen == {128, 256, 512}
    assert len(bt.groups()) == 3
    bt.close()


def test_batch_rejects_unsupported():
    s = P.brinkman_circle(16, 1.5)
    with pytest.raises(ibdl.IBDLError):
        ibdl.Batch([dict(_as_dict(s), pde="stokes")], precision="fp64")


_CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import paper_2210_07403_amd as ibdl
from workloads import problems as P
from test_gpu_batch import _as_dict
specs = [P.ProblemSpec(**{**s.__dict__, "g": None}) for s in P.cfg4_batch(nprob=6, seed=3, sizes=(64, 128))]
bt = ibdl.Batch([_as_dict(s) for s in specs], precision="mixed")
print(json.dumps(bt.groups()))
"""


def test_batch_tuning_persists_in_json_cache(tmp_path):
    """The measured tile and launch shapes are written to the JSON file named by IBDL_TUNE_CACHE; a
    second process reads them back and makes the same choices."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.json"
    env = dict(os.environ, IBDL_TUNE_CACHE=str(cache))
    run = lambda: subprocess.run([sys.executable, "-c", _CHILD, root], env=env, capture_output=True, text=True,
                                 timeout=240)
    r1 = run()
    assert r1.returncode == 0, r1.stderr[-2000:]
    doc = json.loads(cache.read_text())
    assert doc["format"] == "ibdl-tune-3" and doc["device"]
    tiles = [e for e in doc["entries"] if e["key"][0] == 3]
    assert len(tiles) == 2 and all(e["tile"] in (16, 32, 64) for e in tiles)
    first = json.loads(r1.stdout.strip().splitlines()[-1])
    before = cache.read_text()
    r2 = run()
    assert r2.returncode == 0, r2.stderr[-2000:]
    assert json.loads(r2.stdout.strip().splitlines()[-1]) == first
    assert cache.read_text() == before          # nothing measured again, nothing rewritten
