"""MI355X-native Immersed Boundary Double Layer (IBDL) operator library.

Python surface over the C ABI of include/ibdl.h.  PyTorch supplies device memory and the
stream; the spread, FFT passes, Fourier multipliers, interpolation and Krylov vectors all run
in the HIP library (libibdl.so, built in-tree for gfx950).  There is no CPU fallback: without
the library every call raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _binding as B

__all__ = ["Problem", "Batch", "SolveInfo", "IBDLError", "IBDLSolve", "ibdl_solve"]

IBDLError = B.IBDLError


def _dev_f64(a, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)


@dataclass
class SolveInfo:
    iters: int
    status: int
    krylov_relres: float
    true_relres_fp64: float
    history: list


class Problem:
    """One IBDL problem on a periodic grid: ibdl_create / ibdl_destroy around a handle.

    X, nrm: (n_ib, dim) marker positions and unit normals pointing out of Omega; ds: (n_ib,)
    quadrature weights.  Grid tensors are (ncomp, [nz,] ny, nx) of float64 (precision="fp64") or
    float32 (precision="mixed").  method="sl" makes a single layer (IBSL) handle, solved with
    MINRES; its normals are not used (nrm may be None).
    """

    def __init__(self, dim, n, L, origin, X, nrm, ds, pde="screened", kappa=0.0, mu=1.0, bc="dirichlet",
                 eta=0.0, kernel="peskin4", disc="fd2", precision="fp64", device="cuda", method="dl"):
        lib = B.load()
        self.device = torch.device(device)
        self.dim = int(dim)
        self.n = tuple(int(v) for v in n)
        self.precision = precision
        self.grid_dtype = torch.float64 if precision == "fp64" else torch.float32
        cfg = B.Config()
        cfg.dim = self.dim
        for d in range(3):
            cfg.n[d] = self.n[d] if d < self.dim else 1
            cfg.L[d] = float(L[d]) if d < self.dim else 1.0
            cfg.origin[d] = float(origin[d]) if d < self.dim else 0.0
        cfg.pde = B.PDE[pde]
        cfg.kappa = float(kappa)
        cfg.mu = float(mu)
        cfg.bc = B.BC[bc]
        cfg.eta = float(eta)
        cfg.kernel = B.KERNEL[kernel]
        cfg.disc = B.DISC[disc]
        cfg.precision = B.PRECISION[precision]
        cfg.method = B.METHOD[method]
        self.method = method
        self.stream = torch.cuda.current_stream(self.device)
        cfg.stream = ctypes.c_void_p(self.stream.cuda_stream)
        self._cfg = cfg
        Xd, Dd = _dev_f64(X, self.device), _dev_f64(ds, self.device)
        Nd = _dev_f64(nrm, self.device) if nrm is not None else None
        self.n_ib = int(Dd.shape[0])
        self._h = ctypes.c_void_p()
        B.check(lib.ibdl_create(ctypes.byref(cfg), self.n_ib, Xd.data_ptr(), Nd.data_ptr() if Nd is not None else None,
                                Dd.data_ptr(), ctypes.byref(self._h)), None)
        n_aug, pts, nq = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        B.check(lib.ibdl_query(self._h, ctypes.byref(n_aug), ctypes.byref(pts), ctypes.byref(nq)), self._h)
        self.n_aug, self.grid_points, self.nq = int(n_aug.value), int(pts.value), int(nq.value)
        self.grid_shape = tuple(reversed(self.n))

    # ---------------------------------------------------------------- helpers
    def _grid(self, ncomp):
        return torch.empty((ncomp,) + self.grid_shape, dtype=self.grid_dtype, device=self.device)

    def _as_grid(self, g, ncomp):
        t = g if isinstance(g, torch.Tensor) else torch.as_tensor(np.asarray(g))
        t = t.to(device=self.device, dtype=self.grid_dtype).contiguous()
        if t.numel() != ncomp * self.grid_points:
            raise ValueError(f"grid array must hold {ncomp} x {self.grid_shape}")
        return t

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            B.load().ibdl_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------------- operations
    def set_markers(self, X, nrm, ds):
        Xd, Nd, Dd = _dev_f64(X, self.device), _dev_f64(nrm, self.device), _dev_f64(ds, self.device)
        B.check(B.load().ibdl_set_markers(self._h, Xd.data_ptr(), Nd.data_ptr(), Dd.data_ptr()), self._h)
        self._markers_token = object()

    def spread(self, f):
        """S: marker values (n_ib,) or (n_ib, nc) -> grid (nc, ...)."""
        ft = _dev_f64(f, self.device)
        nc = 1 if ft.dim() == 1 else int(ft.shape[1])
        out = self._grid(nc)
        B.check(B.load().ibdl_spread(self._h, ft.data_ptr(), nc, out.data_ptr()), self._h)
        return out

    def interp(self, grid, nc=None):
        """S*: grid (nc, ...) -> marker values (n_ib, nc)."""
        nc = nc or (grid.shape[0] if grid.dim() == self.dim + 1 else 1)
        g = self._as_grid(grid, nc)
        out = torch.empty((self.n_ib, nc), dtype=torch.float64, device=self.device)
        B.check(B.load().ibdl_interp(self._h, g.data_ptr(), nc, out.data_ptr()), self._h)
        return out

    def grid_solve(self, rhs):
        """L^-1 rhs (scalar) or L^-1 P rhs (Stokes)."""
        g = self._as_grid(rhs, self.nq)
        out = self._grid(self.nq)
        B.check(B.load().ibdl_grid_solve(self._h, g.data_ptr(), out.data_ptr()), self._h)
        return out

    def apply(self, q):
        qt = _dev_f64(q, self.device).reshape(-1)
        if qt.numel() != self.n_aug:
            raise ValueError(f"q must have n_aug = {self.n_aug} entries")
        y = torch.empty_like(qt)
        B.check(B.load().ibdl_apply(self._h, qt.data_ptr(), y.data_ptr()), self._h)
        return y

    def solve_refined(self, data, g=None, tol=1e-8, maxit=100, inner_tol=1e-4, max_rounds=10, want_u=True):
        """Iterative refinement to a double-precision true residual <= tol (working-precision
        GMRES corrections, double residuals); returns (q, u or None, SolveInfo)."""
        dt = _dev_f64(data, self.device).reshape(-1)
        if dt.numel() != self.n_ib * self.nq:
            raise ValueError("data must have n_ib * nq entries")
        gt = self._as_grid(g, self.nq) if g is not None else None
        q = torch.empty(self.n_aug, dtype=torch.float64, device=self.device)
        u = self._grid(self.nq) if want_u else None
        info = B.Info()
        st = B.load().ibdl_solve_refined(self._h, dt.data_ptr(), gt.data_ptr() if gt is not None else None,
                                         float(tol), int(maxit), float(inner_tol), int(max_rounds), q.data_ptr(),
                                         u.data_ptr() if u is not None else None, ctypes.byref(info))
        B.check(st, self._h)
        res = SolveInfo(info.iters, info.status, info.krylov_relres, info.true_relres_fp64, [])
        if u is not None and self.nq == 1:
            u = u[0]
        return q, u, res

    def apply_transpose(self, p):
        pt = _dev_f64(p, self.device).reshape(-1)
        if pt.numel() != self.n_aug:
            raise ValueError(f"p must have n_aug = {self.n_aug} entries")
        y = torch.empty_like(pt)
        B.check(B.load().ibdl_apply_transpose(self._h, pt.data_ptr(), y.data_ptr()), self._h)
        return y

    def backward(self, q, u, dL_du, tol=1e-8, maxit=100):
        """Adjoint gradients (dL/dX (n_ib, dim), dL/ddata (n_ib * nq,), SolveInfo of the adjoint
        GMRES) for the forward solution q, u of the current markers and dL/du on the grid."""
        qt = _dev_f64(q, self.device).reshape(-1)
        if qt.numel() != self.n_aug:
            raise ValueError(f"q must have n_aug = {self.n_aug} entries")
        ut = self._as_grid(u, self.nq)
        gt = self._as_grid(dL_du, self.nq)
        dX = torch.empty((self.n_ib, self.dim), dtype=torch.float64, device=self.device)
        dd = torch.empty(self.n_ib * self.nq, dtype=torch.float64, device=self.device)
        info = B.Info()
        st = B.load().ibdl_backward(self._h, qt.data_ptr(), ut.data_ptr(), gt.data_ptr(), float(tol), int(maxit),
                                    dX.data_ptr(), dd.data_ptr(), ctypes.byref(info))
        B.check(st, self._h)
        return dX, dd, SolveInfo(info.iters, info.status, info.krylov_relres, info.true_relres_fp64, [])

    def active_rows(self):
        """(rows the markers' windows meet, all rows) of one grid field."""
        a, t = ctypes.c_int64(), ctypes.c_int64()
        B.check(B.load().ibdl_active_rows(self._h, ctypes.byref(a), ctypes.byref(t)), self._h)
        return int(a.value), int(t.value)

    def active_span(self):
        """(first, last) index along the last grid axis holding an active row: the part of the
        spectra the operator apply's last-axis pass loads and stores."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        B.check(B.load().ibdl_active_span(self._h, ctypes.byref(a), ctypes.byref(b)), self._h)
        return int(a.value), int(b.value)

    def indicator(self, regularized=False):
        """Indicator of the interior of the markers' curve (2-D): chi [ny][nx] of the grid type,
        and the regularized field before the threshold when regularized=True."""
        chi = self._grid(1)[0]
        reg = self._grid(1)[0] if regularized else None
        B.check(B.load().ibdl_indicator(self._h, chi.data_ptr(), reg.data_ptr() if reg is not None else None),
                self._h)
        return (chi, reg) if regularized else chi

    def advection(self, u):
        """(u . grad) u of a 2-D velocity field [2][ny][nx] (Sec. 6.5)."""
        ut = self._as_grid(u, 2)
        out = self._grid(2)
        B.check(B.load().ibdl_advection(self._h, ut.data_ptr(), out.data_ptr()), self._h)
        return out

    def ns_step(self, state, Ub, rho, dt, omega=None, m1=0.0, m2=0.0, strip=0, u_inf=0.0, tol=1e-8, maxit=100,
                g_out=None):
        """One Navier-Stokes IMEX step (Sec. 6.5) on state = [u_prev, u, n_prev, n] (four grid
        tensors of shape (2, ny, nx), updated in place; g_out, if given, receives the step's
        forcing); returns (q, SolveInfo)."""
        p = B.NSParams(float(rho), float(dt), float(m1), float(m2), int(strip), float(u_inf), float(tol), int(maxit))
        ub = _dev_f64(Ub, self.device).reshape(-1)
        if ub.numel() != 2 * self.n_ib:
            raise ValueError("Ub must have 2 n_ib entries")
        for t in list(state) + ([g_out] if g_out is not None else []):
            if not (isinstance(t, torch.Tensor) and t.dtype == self.grid_dtype and t.is_contiguous()
                    and t.numel() == 2 * self.grid_points and t.device.type == self.device.type):
                raise ValueError("state tensors must be contiguous (2, ny, nx) grid tensors on the device")
        om = self._as_grid(omega, 1) if omega is not None else None
        q = torch.empty(self.n_aug, dtype=torch.float64, device=self.device)
        info = B.Info()
        st = B.load().ibdl_ns_step(self._h, ctypes.byref(p), ub.data_ptr(), om.data_ptr() if om is not None else None,
                                   *[t.data_ptr() for t in state], q.data_ptr(),
                                   g_out.data_ptr() if g_out is not None else None, ctypes.byref(info))
        B.check(st, self._h)
        return q, SolveInfo(info.iters, info.status, info.krylov_relres, info.true_relres_fp64, [])

    def pressure(self, q, g=None):
        """Mean-zero pressure of a 2-D Brinkman / Stokes solution (density q, forcing g)."""
        qt = _dev_f64(q, self.device).reshape(-1)
        gt = self._as_grid(g, 2) if g is not None else None
        out = self._grid(1)[0]
        B.check(B.load().ibdl_pressure(self._h, qt.data_ptr(), gt.data_ptr() if gt is not None else None,
                                       out.data_ptr()), self._h)
        return out

    def cv_force(self, u, u_prev, dt, p, omega, rho, box):
        """Control-volume force (Sec. 6.5) over the grid box (i0, i1, j0, j1), u_t = (u - u_prev) / dt
        (no volume term for u_prev None): device double [2]."""
        up_ = self._as_grid(u_prev, 2) if u_prev is not None else None
        u_ = self._as_grid(u, 2)
        p_ = self._as_grid(p, 1)
        om = self._as_grid(omega, 1)
        bx = (ctypes.c_int32 * 4)(*[int(v) for v in box])
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        B.check(B.load().ibdl_cv_force(self._h, u_.data_ptr(), up_.data_ptr() if up_ is not None else None, float(dt),
                                       p_.data_ptr(), om.data_ptr(), float(rho), bx, out.data_ptr()), self._h)
        return out

    def net_force(self, q):
        """(B_x, B_y, L) of a 2-D completed Stokes solution q (Sec. 6.1, Sec. 6.5): device double [3]."""
        qt = _dev_f64(q, self.device).reshape(-1)
        if qt.numel() != self.n_aug:
            raise ValueError(f"q must have n_aug = {self.n_aug} entries")
        out = torch.empty(3, dtype=torch.float64, device=self.device)
        B.check(B.load().ibdl_net_force(self._h, qt.data_ptr(), out.data_ptr()), self._h)
        return out

    def line_integral(self, u, comp=0, axis=0, index=0):
        """h times the sum of component comp of the 2-D grid field u over the grid line on which
        coordinate `axis` has node index `index`: device double [1]."""
        ut = self._as_grid(u, self.nq)
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        B.check(B.load().ibdl_line_integral(self._h, ut.data_ptr(), int(comp), int(axis), int(index),
                                            out.data_ptr()), self._h)
        return out

    def near_widths(self):
        """(m1, m2) of the thesis's width rules (Sec. 5.5) for this handle's discretisation."""
        a, b = ctypes.c_double(), ctypes.c_double()
        B.check(B.load().ibdl_near_widths(self._h, ctypes.byref(a), ctypes.byref(b)), self._h)
        return float(a.value), float(b.value)

    def near_boundary(self, Ub, omega, u, m1=None, m2=None):
        """u with its near-boundary nodes of omega replaced by the interpolation of Sec. 5.3.3 (2-D);
        m1, m2 default to near_widths()."""
        if m1 is None or m2 is None:
            d1, d2 = self.near_widths()
            m1 = d1 if m1 is None else m1
            m2 = d2 if m2 is None else m2
        ub = _dev_f64(Ub, self.device).reshape(-1)
        if ub.numel() != self.n_ib * self.nq:
            raise ValueError("Ub must have n_ib * nq entries")
        om = self._as_grid(omega, 1)
        ut = self._as_grid(u, self.nq)
        out = self._grid(self.nq)
        if self.nq == 1:
            out = out[0]
        B.check(B.load().ibdl_near_boundary(self._h, ub.data_ptr(), om.data_ptr(), ut.data_ptr(), float(m1),
                                            float(m2), out.data_ptr()), self._h)
        return out

    def spread_tiles(self):
        """(busy tiles, busy row segments the apply's forward x pass reads per field, tile shape)."""
        nb, ns = ctypes.c_int64(), ctypes.c_int64()
        t = (ctypes.c_int32 * 3)()
        B.check(B.load().ibdl_spread_tiles(self._h, ctypes.byref(nb), ctypes.byref(ns), t), self._h)
        return int(nb.value), int(ns.value), tuple(int(v) for v in t)

    def launch_shape(self):
        """Measured launch shapes of the apply's FFT passes: (rows per block, y lines, last-axis lines)."""
        r, y, z = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        B.check(B.load().ibdl_launch_shape(self._h, ctypes.byref(r), ctypes.byref(y), ctypes.byref(z)), self._h)
        return int(r.value), int(y.value), int(z.value)

    def set_graph(self, enable=True):
        """Replay the Krylov solvers' operator applies from a captured HIP graph or launch them
        directly (the default is the graph below 2^20 grid points)."""
        B.check(B.load().ibdl_set_graph(self._h, 1 if enable else 0), self._h)

    def set_timing(self, enable=True):
        B.check(B.load().ibdl_set_timing(self._h, 1 if enable else 0), self._h)

    def timing(self):
        """{stage: (total_ms, launches)} accumulated since set_timing(True)."""
        ms = (ctypes.c_double * 9)()
        cnt = (ctypes.c_int64 * 9)()
        B.check(B.load().ibdl_get_timing(self._h, ms, cnt, 9), self._h)
        return {B.STAGES[i]: (ms[i], cnt[i]) for i in range(9)}

    def solve(self, data, g=None, tol=1e-8, maxit=100, want_u=True):
        """GMRES solve of the IBDL system; returns (q, u or None, SolveInfo)."""
        dt = _dev_f64(data, self.device).reshape(-1)
        if dt.numel() != self.n_ib * self.nq:
            raise ValueError("data must have n_ib * nq entries")
        gt = self._as_grid(g, self.nq) if g is not None else None
        q = torch.empty(self.n_aug, dtype=torch.float64, device=self.device)
        u = self._grid(self.nq) if want_u else None
        cap = max(256, min(int(maxit), 1 << 20))
        hist = (ctypes.c_double * cap)()
        info = B.Info()
        info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        info.history_cap = cap
        st = B.load().ibdl_solve(self._h, dt.data_ptr(), gt.data_ptr() if gt is not None else None, float(tol),
                                 int(maxit), q.data_ptr(), u.data_ptr() if u is not None else None,
                                 ctypes.byref(info))
        B.check(st, self._h)
        res = SolveInfo(info.iters, info.status, info.krylov_relres, info.true_relres_fp64,
                        [hist[i] for i in range(min(info.iters, cap))])
        if u is not None and self.nq == 1:
            u = u[0]
        return q, u, res


class Batch:
    """Many independent plain scalar Dirichlet problems solved together (ibdl_batch_*).

    problems: sequence of dicts with keys dim, n, L, origin, X, nrm, ds, pde ("screened" or
    "poisson"), kappa and optionally kernel ("peskin4" / "cos4"); all share dim, kernel and the
    precision given here.  Finite-difference symbols, eta = 0."""

    def __init__(self, problems, precision="mixed", device="cuda"):
        lib = B.load()
        self.device = torch.device(device)
        self.precision = precision
        self.grid_dtype = torch.float64 if precision == "fp64" else torch.float32
        self.nprob = len(problems)
        cfgs = (B.Config * self.nprob)()
        self.stream = torch.cuda.current_stream(self.device)
        keep = []
        self.n_ib, self.grid_shapes = [], []
        for k, pb in enumerate(problems):
            c = cfgs[k]
            dim = int(pb["dim"])
            c.dim = dim
            for d in range(3):
                c.n[d] = int(pb["n"][d]) if d < dim else 1
                c.L[d] = float(pb["L"][d]) if d < dim else 1.0
                c.origin[d] = float(pb["origin"][d]) if d < dim else 0.0
            c.pde = B.PDE[pb.get("pde", "poisson")]
            c.kappa = float(pb.get("kappa", 0.0))
            c.mu = 1.0
            c.bc = B.BC["dirichlet"]
            c.eta = 0.0
            c.kernel = B.KERNEL[pb.get("kernel", "peskin4")]
            c.disc = B.DISC["fd2"]
            c.precision = B.PRECISION[precision]
            c.stream = ctypes.c_void_p(self.stream.cuda_stream)
            Xd, Nd, Dd = (_dev_f64(pb["X"], self.device), _dev_f64(pb["nrm"], self.device),
                          _dev_f64(pb["ds"], self.device))
            keep += [Xd, Nd, Dd]
            self.n_ib.append(int(Dd.shape[0]))
            self.grid_shapes.append(tuple(reversed([int(v) for v in pb["n"]][:dim])))
        ptr = lambda ts: (ctypes.c_void_p * self.nprob)(*[t.data_ptr() for t in ts])
        nib = (ctypes.c_int64 * self.nprob)(*self.n_ib)
        self._h = ctypes.c_void_p()
        B.check_batch(lib.ibdl_batch_create(self.nprob, cfgs, nib, ptr(keep[0::3]), ptr(keep[1::3]),
                                            ptr(keep[2::3]), ctypes.byref(self._h)), None)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            B.load().ibdl_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vecs(self, vs):
        ts = [_dev_f64(v, self.device).reshape(-1) for v in vs]
        for t, n in zip(ts, self.n_ib):
            if t.numel() != n:
                raise ValueError("each vector must have n_ib entries of its problem")
        return ts

    def set_graph(self, enable=True):
        B.check_batch(B.load().ibdl_batch_set_graph(self._h, 1 if enable else 0), self._h)

    def groups(self):
        """[{nprob, n, rows_per_block, lines_per_block, tile_x}] of the grid groups."""
        lib = B.load()
        ng = ctypes.c_int32()
        B.check_batch(lib.ibdl_batch_query(self._h, -1, ctypes.byref(ng), None, None, None, None, None), self._h)
        out = []
        for g in range(ng.value):
            npg, rpb, w, tx = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            n = (ctypes.c_int32 * 3)()
            B.check_batch(lib.ibdl_batch_query(self._h, g, None, ctypes.byref(npg), n, ctypes.byref(rpb),
                                               ctypes.byref(w), ctypes.byref(tx)), self._h)
            out.append(dict(nprob=npg.value, n=tuple(n), rows_per_block=rpb.value, lines_per_block=w.value,
                            tile_x=tx.value))
        return out

    def apply(self, qs):
        qt = self._vecs(qs)
        ys = [torch.empty_like(t) for t in qt]
        P = lambda ts: (ctypes.c_void_p * self.nprob)(*[t.data_ptr() for t in ts])
        B.check_batch(B.load().ibdl_batch_apply(self._h, P(qt), P(ys)), self._h)
        return ys

    def solve(self, data, tol=1e-8, maxit=100, want_u=True):
        """Returns (q list, u list or None, [SolveInfo])."""
        dt = self._vecs(data)
        qs = [torch.empty(n, dtype=torch.float64, device=self.device) for n in self.n_ib]
        us = [torch.empty(s, dtype=self.grid_dtype, device=self.device) for s in self.grid_shapes] if want_u else None
        infos = (B.Info * self.nprob)()
        hists = [(ctypes.c_double * 256)() for _ in range(self.nprob)]
        for k in range(self.nprob):
            infos[k].history = ctypes.cast(hists[k], ctypes.POINTER(ctypes.c_double))
            infos[k].history_cap = 256
        P = lambda ts: (ctypes.c_void_p * self.nprob)(*[t.data_ptr() for t in ts])
        st = B.load().ibdl_batch_solve(self._h, P(dt), float(tol), int(maxit), P(qs), P(us) if us else None, infos)
        B.check_batch(st, self._h)
        res = [SolveInfo(infos[k].iters, infos[k].status, infos[k].krylov_relres, infos[k].true_relres_fp64,
                         [hists[k][i] for i in range(min(infos[k].iters, 256))]) for k in range(self.nprob)]
        return qs, us, res


class IBDLSolve(torch.autograd.Function):
    """u = the IBDL grid solution for markers X and boundary data (normals, weights and forcing
    held fixed), differentiable in X and data through ibdl_backward.

    Call as IBDLSolve.apply(problem, X, nrm, ds, data, g, tol, maxit) or via ibdl_solve(...)."""

    @staticmethod
    def forward(ctx, problem, X, nrm, ds, data, g, tol, maxit):
        problem.set_markers(X.detach(), nrm, ds)
        q, u, _ = problem.solve(data.detach(), g, tol=tol, maxit=maxit)
        ctx.problem, ctx.tol, ctx.maxit = problem, tol, maxit
        ctx.token = problem._markers_token
        ctx.shapes = (X.shape, data.shape)
        ctx.save_for_backward(X.detach().to(torch.float64), torch.as_tensor(nrm, dtype=torch.float64),
                              torch.as_tensor(ds, dtype=torch.float64), q, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        X, nrm, ds, q, u = ctx.saved_tensors
        pr = ctx.problem
        if getattr(pr, "_markers_token", None) is not ctx.token:
            pr.set_markers(X, nrm, ds)
            ctx.token = pr._markers_token
        dX, dd, _ = pr.backward(q, u, grad_u.contiguous(), tol=ctx.tol, maxit=ctx.maxit)
        xs, ds_shape = ctx.shapes
        return (None, dX.reshape(xs) if ctx.needs_input_grad[1] else None, None, None,
                dd.reshape(ds_shape) if ctx.needs_input_grad[4] else None, None, None, None)


def ibdl_solve(problem, X, nrm, ds, data, g=None, tol=1e-8, maxit=100):
    """Differentiable IBDL solve: returns the grid solution u (see IBDLSolve)."""
    return IBDLSolve.apply(problem, X, nrm, ds, data, g, tol, maxit)
