"""Host-side parts of bench.py (no GPU): the spread's candidate pair count against a brute-force
count of the tiles each marker's 6-node window meets, and the refusal of more than one GPU."""
import numpy as np

import bench
from workloads import geometry as geo
from workloads import problems as P


def _brute_pairs(spec, tile):
    n = spec.n
    h = spec.L[0] / n[0]
    total = 0
    for x in np.asarray(spec.markers.X, dtype=np.float64):
        s = [int(np.floor((x[d] - spec.origin[d]) / h)) - 2 for d in range(spec.dim)]
        tiles = set()
        for k0 in range(6):
            for k1 in range(6):
                for k2 in range(6):
                    k = (k0, k1, k2)
                    tiles.add(tuple(((s[d] + k[d]) % n[d]) // tile[d] for d in range(spec.dim)))
        total += len(tiles)
    return total


def test_candidate_pairs_match_brute_force():
    rng = np.random.default_rng(11)
    X = rng.uniform(0.0, 1.0, (300, 3))
    X[0] = (0.0, 0.0, 0.0)            # windows across every periodic seam
    X[1] = (1.0 - 1e-9, 0.5, 0.999)
    nrm = rng.standard_normal((300, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    mk = geo.Markers(X, nrm, np.full(300, 1e-3), 0.3)
    spec = P.ProblemSpec("pairs", 3, (32, 16, 64), (1.0, 0.5, 2.0), (0.0, 0.0, 0.0), "screened", 1.0, 1.0,
                         "dirichlet", 0.0, "peskin4", "fd2", mk, np.zeros(300), None)
    tile = (16, 4, 8)
    assert bench.candidate_pairs(spec, tile) == _brute_pairs(spec, tile)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits non-zero with a message, before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
