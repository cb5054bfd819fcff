"""Shared test helpers: build library problems and oracle setups from the same seeded spec."""
import numpy as np

import oracle


def make_problem(spec, precision="fp64"):
    import paper_2210_07403_amd as ibdl
    m = spec.markers
    return ibdl.Problem(spec.dim, spec.n, spec.L, spec.origin, m.X, m.nrm, m.ds, pde=spec.pde,
                        kappa=spec.kappa, mu=spec.mu, bc=spec.bc, eta=spec.eta, kernel=spec.kernel,
                        disc=spec.disc, precision=precision)


def make_oracle(spec):
    return oracle.Setup.from_spec(spec)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)
