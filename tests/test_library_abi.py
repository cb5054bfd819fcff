"""The C-ABI library loads, exports every entry point its header declares, and rejects invalid
arguments on the host (no GPU needed: validation precedes any device call)."""
import ctypes

import pytest

from paper_2210_07403_amd import _binding as B


def test_exports_every_declared_symbol():
    lib = B.load()
    names = B.header_symbols()
    assert {"ibdl_create", "ibdl_apply", "ibdl_solve", "ibdl_spread", "ibdl_interp",
            "ibdl_grid_solve", "ibdl_destroy"} <= set(names)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_argument_counts_match_the_header():
    """Every declaration's parameter count equals the binding's argtypes (a wrong count would pass
    arguments into the wrong slots)."""
    import re
    text = open(B.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    decls = dict(re.findall(r"\b(ibdl_[a-z_]+)\s*\(([^;{]*?)\)\s*;", text))
    assert len(decls) >= 30
    for name, params in decls.items():
        params = params.strip()
        n = 0 if params in ("", "void") else params.count(",") + 1
        assert name in B._SIGS, name
        assert len(B._SIGS[name][1]) == n, (name, n, len(B._SIGS[name][1]))


def _cfg(**kw):
    c = B.Config()
    c.dim = kw.get("dim", 2)
    for d in range(3):
        c.n[d] = kw.get("n", (64, 64, 64))[d]
        c.L[d] = kw.get("L", (1.0, 1.0, 1.0))[d]
        c.origin[d] = 0.0
    c.pde = kw.get("pde", 0)
    c.kappa = kw.get("kappa", 1.0)
    c.mu = kw.get("mu", 1.0)
    c.bc = kw.get("bc", 0)
    c.eta = kw.get("eta", 0.0)
    c.kernel = kw.get("kernel", 0)
    c.disc = kw.get("disc", 0)
    c.precision = kw.get("precision", 0)
    c.stream = None
    c.method = kw.get("method", 0)
    return c


@pytest.mark.parametrize("kw,code", [
    (dict(dim=4), -1),
    (dict(n=(63, 64, 64)), -2),
    (dict(n=(16384, 16384, 1)), -2),          # 2-D grids go up to 8192
    (dict(dim=3, n=(2048, 2048, 2048)), -2),  # 3-D up to 1024
    (dict(L=(1.0, 2.0, 1.0)), -1),
    (dict(kappa=-1.0), -1),
    (dict(kappa=0.0), -1),                    # screened needs kappa > 0
    (dict(pde=2, dim=3), -2),                 # 3-D Stokes not implemented
    (dict(bc=1, eta=1.0), -2),                # Neumann + completed
    (dict(bc=1, pde=2), -2),
    (dict(kernel=2, disc=0), -2),             # B-spline with FD scalar
    (dict(kernel=7), -1),
    (dict(precision=3), -1),
    (dict(eta=float("nan")), -1),
    (dict(method=2), -1),
    (dict(method=1, eta=1.0), -2),            # the single layer takes no completion
    (dict(method=1, bc=1), -2),
    (dict(method=1, dim=3), -2),
])
def test_create_rejects_invalid_config(kw, code):
    lib = B.load()
    h = ctypes.c_void_p()
    cfg = _cfg(**kw)
    dummy = ctypes.c_void_p(8)
    st = lib.ibdl_create(ctypes.byref(cfg), 10, dummy, dummy, dummy, ctypes.byref(h))
    assert st == code, (st, lib.ibdl_last_error(None))
    assert h.value is None
    assert lib.ibdl_last_error(None)


def test_null_pointers_rejected():
    lib = B.load()
    h = ctypes.c_void_p()
    cfg = _cfg()
    assert lib.ibdl_create(ctypes.byref(cfg), 10, None, None, None, ctypes.byref(h)) == -1
    assert lib.ibdl_create(None, 10, None, None, None, ctypes.byref(h)) == -1
    assert lib.ibdl_apply(None, None, None) == -1
    assert lib.ibdl_destroy(None) == -1
    # the entry points beyond the operator reject a NULL handle before touching anything
    assert lib.ibdl_indicator(None, None, None) == -1
    assert lib.ibdl_near_boundary(None, None, None, None, 6.0, 8.0, None) == -1
    assert lib.ibdl_near_widths(None, None, None) == -1
    assert lib.ibdl_net_force(None, None, None) == -1
    assert lib.ibdl_line_integral(None, None, 0, 0, 0, None) == -1
    assert lib.ibdl_advection(None, None, None) == -1
    p = B.NSParams(1.0, 0.01, 0.0, 0.0, 0, 0.0, 1e-8, 10)
    assert lib.ibdl_ns_step(None, ctypes.byref(p), None, None, None, None, None, None, None, None, None) == -1
    assert lib.ibdl_pressure(None, None, None, None) == -1
    box = (ctypes.c_int32 * 4)(1, 2, 1, 2)
    assert lib.ibdl_cv_force(None, None, None, 0.0, None, None, 1.0, box, None) == -1
