#!/usr/bin/env python
"""IBDL throughput on one MI355X: GMRES solves/s at a double-precision residual of 1e-8 and
operator applies/s, with the roofline of the apply's dominant kernel and the FP64 CPU oracle
timed on the host beside them.

A step is one whole IBDL solve through the C ABI on the 256^3 sphere workload with float grid
work and double-precision Krylov vectors: ibdl_solve_refined, i.e. the right-hand side
b = U_b - S* L^-1 g~ in double, GMRES on the float-applied operator (every iteration one operator
apply: spread -> FFT passes with the fused multiplier -> interpolation; Arnoldi, Givens rotations
and least squares in double on the device), double-precision residuals b - A q with corrections
until ||b - A q|| / ||b|| <= 1e-8, and the grid recovery u = L^-1 (g~ - S~ q).  `value` is solves
per second at that true residual.  Inputs are resident on the GPU before the timed region starts.

Beside it on the same JSON line: single operator applies, the stages' rates, the plain mixed and
FP64 solves, every other workload of the method (the 64^2 circle, the 1024^2 star, the 512^2
Stokes star with its gradient, the batch of 64) and the measurements beyond the hot path.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MATRIX_PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}   # MI355X dense MFMA FP32 / FP64
METRIC = "IBDL operator applies/sec + GMRES solves/sec at 1e-8 residual; % HBM peak"


def workload(name):
    from workloads import problems as P
    if name == "sphere256":
        return P.cfg3_sphere(256, 86), "mixed", (
            "3-D IBDL screened Poisson kappa=10, 256^3 periodic grid, sphere r=0.3, 73962 icosphere markers, "
            "Peskin 4-point, FD2, float grid/spread/FFT + double GMRES and residuals, double-precision residual 1e-8")
    if name == "star1024":
        return P.cfg2_star_poisson(1024, 4096), "fp64", (
            "2-D IBDL Poisson Dirichlet, 1024^2 grid, star r=0.3(1+0.2cos5t), 4096 markers, Peskin 4-point, FD2, "
            "double precision, tol 1e-8")
    if name == "circle64":
        return P.cfg1_circle_cos4(), "fp64", (
            "2-D IBDL screened Poisson kappa=1, 64^2 grid, circle r=0.25, 200 markers, cosine 4-point, FD2, "
            "double precision, tol 1e-10")
    raise SystemExit(f"unknown workload {name}")


def stage_cost(spec, prec, pr):
    """Algorithmic cost per launch of each stage of one operator apply: HBM bytes for the
    memory-bound passes (the x passes touch only the rows the markers' windows meet, the forward
    one only their busy tile segments; the forward y pass reads only those rows, the inverse
    writes only those; in 3-D the y passes and the last-axis pass touch only the z planes from
    the first to the last holding such a row), floating-point operations for the spread (a
    per-tile contraction on the matrix cores)."""
    t = 4 if prec == "mixed" else 8
    ntot = pr.grid_points
    nxh = spec.n[0] // 2 + 1
    nspec = ntot // spec.n[0] * nxh
    C = nspec * 2 * t
    nact, _ = pr.active_rows()
    Ra, Ca = nact * spec.n[0] * t, nact * nxh * 2 * t
    scalar_fd = spec.pde != "stokes" and spec.disc == "fd2"
    c = 1 if scalar_fd else (5 if spec.pde == "stokes" else spec.dim + (1 if spec.eta > 0 else 0))
    o = pr.nq
    taps = 4 ** spec.dim
    # the forward x pass reads only the busy tile segments of the active rows (the rest is zero)
    _, nseg, tile = pr.spread_tiles()
    Rb = nseg * tile[0] * t
    b = {
        "fft_x_fwd": ("hbm", c * (Rb + Ca)),
        "fft_x_inv": ("hbm", o * (Ca + Ra)),
        "interp": ("hbm", spec.n_ib * (taps * t * o + 36 + 8 * pr.nq * 2)),
    }
    if spec.dim == 3:
        z0, z1 = pr.active_span()
        Cz = C * max(0, z1 - z0 + 1) // spec.n[2]   # half spectra of the planes in the span
        b["fft_y_fwd"] = ("hbm", c * (Ca + Cz))
        b["fused_last_axis"] = ("hbm", (c + o) * Cz)
        b["fft_y_inv"] = ("hbm", o * (Cz + Ca))
    else:
        b["fused_last_axis"] = ("hbm", (c + o) * Ca)
    # spread: per marker and window node, D-1 products per term and one add per term; the
    # finite-difference dipole spread has D derivative terms (+ mass), other modes c fields
    if scalar_fd:
        flops = spec.n_ib * 6 ** spec.dim * ((spec.dim + 1) * spec.dim)
    else:
        flops = spec.n_ib * taps * c * spec.dim
    b["spread"] = ("mfma", flops)
    if spec.dim == 3 and scalar_fd:
        # its bytes: each marker's weight row (24 (W, G) pairs), density, normal and spacing, each
        # candidate pair's list entry and window offsets, the busy tiles written; below the matrix
        # ridge (flop per byte) the roofline that bounds it is the HBM one
        nbusy, _, tile = pr.spread_tiles()
        sb = spec.n_ib * (24 * 2 * t + 8 + 8 * spec.dim + 8) + 8 * candidate_pairs(spec, tile) + nbusy * 512 * t
        ridge = MATRIX_PEAK_TFLOPS[prec] * 1e12 / (HBM_PEAK_GBS * 1e9)
        if flops / sb < ridge:
            b["spread"] = ("hbm", sb)
    return b


def candidate_pairs(spec, tile):
    """(tile, marker) pairs of the spread: the tiles each marker's 6-node window meets, counted on
    the host from the window starts floor((X - origin) / h) - 2 (periodic)."""
    import numpy as np
    n = np.asarray(spec.n)
    h = spec.L[0] / spec.n[0]
    xi = (np.asarray(spec.markers.X, dtype=np.float64) - np.asarray(spec.origin)) / h
    s = (np.floor(xi).astype(np.int64) - 2) % n
    count = np.ones(len(s), dtype=np.int64)
    for d in range(spec.dim):
        tiles = np.sort(((s[:, d:d + 1] + np.arange(6)) % n[d]) // tile[d], axis=1)
        count *= 1 + (np.diff(tiles, axis=1) != 0).sum(axis=1)
    return int(count.sum())


def model_bytes(spec, prec, pr):
    """Bytes of one apply when every stage is materialised in HBM with the unfused field counts
    (c spread fields: D divergence components (+1 mass), Stokes 5; o = nq inverse fields), and
    the fused floor that keeps only the FFT passes over the half spectra."""
    t = 4 if prec == "mixed" else 8
    ntot = pr.grid_points
    nspec = ntot // spec.n[0] * (spec.n[0] // 2 + 1)
    R, C = ntot * t, nspec * 2 * t
    c = 5 if spec.pde == "stokes" else spec.dim + (1 if spec.eta > 0 else 0)
    o = pr.nq
    if spec.dim == 3:
        return (2 * c + o) * R + (4 * c + 4 * o) * C, (4 * c + 4 * o) * C
    return (2 * c + o) * R + (2 * c + 2 * o) * C, (2 * c + 2 * o) * C


# The sources the operator apply's grid passes are compiled from (the FFT passes with the fused
# multiplier, and the declarations and helpers they include); the traffic counters in profiles/
# stand only while these are unchanged.
DIGEST_SOURCES = ("fft.hip", "kernels.h", "common.h", "tables.h")


def sources_digest():
    """Digest of the code in DIGEST_SOURCES: comments and whitespace are dropped first, so that a
    reworded comment keeps the counters while any change to the code itself discards them."""
    import hashlib
    import re
    hsh = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2210_07403_amd", "csrc")
    for f in DIGEST_SOURCES:
        text = open(os.path.join(csrc, f), encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        hsh.update(" ".join(text.split()).encode())
    return hsh.hexdigest()[:16]


def load_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, if it was
    taken on the current kernel sources; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("sources") != sources_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def _timed(fn, reps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def measure_extras(spec, prec, pr, data, g, tol, dev):
    """The other workloads of the method (the 64^2 circle, the 1024^2 star, the 512^2 Stokes star
    with its gradient), the adjoint on this workload, 64 problems batched vs one after another,
    and the measurements beyond the hot path."""
    import numpy as np
    import torch
    import paper_2210_07403_amd as ibdl
    from workloads import problems as P
    out = {}
    m = spec.markers
    print("# extras: the 64^2 circle, the 1024^2 star, the 512^2 Stokes star", file=sys.stderr, flush=True)
    out["cfg1_circle64"] = _cfg1_circle(dev)
    out["cfg2_star1024"] = _cfg2_star(dev)
    out["cfg5_stokes512"] = _cfg5_stokes(dev)
    print("# extras: adjoint", file=sys.stderr, flush=True)
    q, u, _ = pr.solve(data, g, tol=tol, maxit=100)
    psi = torch.randn(u.shape, dtype=u.dtype, device=dev, generator=torch.Generator(device=dev).manual_seed(0))
    t_fw, _ = _timed(lambda: pr.solve(data, g, tol=tol, maxit=100), 2)
    t_bw, (_, _, ib) = _timed(lambda: pr.backward(q, u, psi, tol=tol, maxit=100), 2)
    out["adjoint"] = {"forward_solve_ms": round(1e3 * t_fw, 3), "backward_ms": round(1e3 * t_bw, 3),
                      "adjoint_iters": ib.iters, "adjoint_true_relres": ib.true_relres_fp64}
    print("# extras: batch of 64", file=sys.stderr, flush=True)
    out["batch64"] = _batch_timing(dev)
    print("# extras: near-boundary tools", file=sys.stderr, flush=True)
    out["near_boundary_star1024"] = _near_boundary_timing(dev)
    print("# extras: cylinder array drag", file=sys.stderr, flush=True)
    out["cylinder_array_drag"] = _cylinder_drag(dev)
    print("# extras: single vs double layer", file=sys.stderr, flush=True)
    out["ibsl_vs_ibdl_helmholtz1024"] = _ibsl_vs_ibdl(dev)
    print("# extras: Navier-Stokes cylinder", file=sys.stderr, flush=True)
    out["ns_cylinder_re100"] = ns_cylinder(dev, 100.0, 200, 5)
    return out


def _batch_timing(dev):
    """Config 4: 64 independent 2-D Poisson problems batched (mixed and FP64) against the same
    problems solved one after another in FP64."""
    import numpy as np
    import torch
    import paper_2210_07403_amd as ibdl
    from workloads import problems as P
    specs = P.cfg4_batch()
    dicts = [dict(dim=s.dim, n=s.n, L=s.L, origin=s.origin, X=s.markers.X, nrm=s.markers.nrm, ds=s.markers.ds,
                  pde=s.pde, kappa=s.kappa, kernel=s.kernel) for s in specs]
    bdata = [torch.as_tensor(np.asarray(s.data, dtype=np.float64), device=dev) for s in specs]
    res = {}
    for bp in ("mixed", "fp64"):
        bt = ibdl.Batch(dicts, precision=bp, device=dev)
        bt.solve(bdata, tol=1e-8, maxit=100, want_u=False)
        tb, (_, _, binfo) = _timed(lambda: bt.solve(bdata, tol=1e-8, maxit=100, want_u=False), 3)
        res[bp] = {"ms": round(1e3 * tb, 3), "solves_per_sec": round(len(specs) / tb, 1),
                   "max_iters": max(i.iters for i in binfo),
                   "max_true_relres": max(i.true_relres_fp64 for i in binfo), "groups": bt.groups()}
        bt.close()
    probs = [ibdl.Problem(s.dim, s.n, s.L, s.origin, s.markers.X, s.markers.nrm, s.markers.ds, pde=s.pde,
                          kappa=s.kappa, kernel=s.kernel, precision="fp64", device=dev) for s in specs]
    for p_, d_ in zip(probs, bdata):
        p_.solve(d_, None, tol=1e-8, maxit=100, want_u=False)
    tseq, _ = _timed(lambda: [p_.solve(d_, None, tol=1e-8, maxit=100, want_u=False) for p_, d_ in zip(probs, bdata)], 2)
    for p_ in probs:
        p_.close()
    return {"workload": "64 2-D Poisson Dirichlet problems, grids 128/256/512, 256-2048 markers, tol 1e-8",
            "batched_mixed": res["mixed"], "batched_fp64": res["fp64"],
            "sequential_fp64_ms": round(1e3 * tseq, 3),
            "speedup_batched_mixed_vs_sequential_fp64": round(tseq / (res["mixed"]["ms"] * 1e-3), 2),
            "speedup_batched_fp64_vs_sequential_fp64": round(tseq / (res["fp64"]["ms"] * 1e-3), 2)}


def ns_cylinder(dev, re, steps, warm, report_every=0, precision="fp64"):
    """Flow past a cylinder with the Navier-Stokes IMEX scheme (Sec. 6.5's setting): periodic box
    [0, 8]^2 on 1024^2 (dx = 2^-7), cylinder r = 0.15 at (1.85, 4), rho = 1, u_inf = 1 on a 4-column
    inflow strip, Re = 2 r rho u_inf / mu, dt = 1.8e-3, completed IBDL (eta = 10), spectral,
    near-boundary interpolation with the thesis's widths for each case (m1 = 3, m2 = 4 at Re = 10;
    m1 = 6, m2 = 8 at Re = 100); starts from the uniform flow.  Times `steps` steps after `warm`,
    and reports the drag coefficient C_D = B_1 / (rho u_inf^2 r) by the control volume
    [0.5, 3.203125] x [2.8125, 5.1875]: at the last step, and averaged over the samples with
    54 <= t <= 144 (the thesis's averaging window at Re = 10) when the run covers them."""
    import math
    import numpy as np
    import torch
    import paper_2210_07403_amd as ibdl
    from workloads import geometry as geo
    N, L, r, c0 = 1024, 8.0, 0.15, (1.85, 4.0)
    rho, u_inf, dt, eta = 1.0, 1.0, 1.8e-3, 10.0
    mu = 2 * r * rho * u_inf / re
    m1, m2 = (3, 4) if re <= 10 else (6, 8)
    h = L / N
    curve = geo.PolarCurve(c0, r)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), h, 1.0)).flipped()
    pr = ibdl.Problem(2, (N, N), (L, L), (0.0, 0.0), mk.X, mk.nrm, mk.ds, pde="stokes",
                      kappa=math.sqrt(1.5 * rho / dt), mu=mu, eta=eta, kernel="peskin4", disc="spectral",
                      precision=precision, device=dev)
    ax = h * np.arange(N)
    ys, xs = np.meshgrid(ax, ax, indexing="ij")
    omega = torch.as_tensor((np.hypot(xs - c0[0], ys - c0[1]) >= r).astype(np.float64), device=dev).to(pr.grid_dtype)
    u0 = torch.zeros((2, N, N), dtype=pr.grid_dtype, device=dev)
    u0[0] = u_inf
    state = [u0.clone(), u0.clone(), torch.zeros_like(u0), torch.zeros_like(u0)]
    g = torch.empty_like(u0)
    Ub = np.zeros((mk.X.shape[0], 2))
    box = (int(round(0.5 / h)), int(round(3.203125 / h)), int(round(2.8125 / h)), int(round(5.1875 / h)))
    iters = []
    hist = []

    def cd():
        p = pr.pressure(q, g)
        B = pr.cv_force(state[1], state[0], dt, p, omega, rho, box).cpu().numpy()
        return float(B[0] / (rho * u_inf ** 2 * r)), float(B[1] / (rho * u_inf ** 2 * r))

    for _ in range(warm):
        q, info = pr.ns_step(state, Ub, rho, dt, omega, m1, m2, 4, u_inf, tol=1e-8, maxit=100, g_out=g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        q, info = pr.ns_step(state, Ub, rho, dt, omega, m1, m2, 4, u_inf, tol=1e-8, maxit=100, g_out=g)
        iters.append(info.iters)
        if report_every and (k + 1) % report_every == 0:
            cdx, cdy = cd()
            hist.append((round((warm + k + 1) * dt, 4), round(cdx, 5), round(cdy, 5)))
            print(f"# t = {hist[-1][0]}: C_D = {hist[-1][1]}, C_L = {hist[-1][2]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    cdx, cdy = cd()
    pr.close()
    st = strouhal(hist, 2 * r / u_inf)
    win = [c for t, c, _ in hist if 54.0 <= t <= 144.0]
    return {"workload": "flow past a cylinder, Re = %g, [0, 8]^2 on 1024^2, %d markers, dt = 1.8e-3, eta = 10, "
                        "m1 = %d, m2 = %d, spectral, %s, GMRES tol 1e-8" % (re, mk.X.shape[0], m1, m2, precision),
            "steps": steps, "ms_per_step": round(1e3 * el / steps, 3), "steps_per_sec": round(steps / el, 1),
            "mean_gmres_iters": round(float(np.mean(iters)), 2), "t_end": round((warm + steps) * dt, 4),
            "C_D": round(cdx, 5), "C_L": round(cdy, 5),
            "C_D_mean_t54_144": round(float(np.mean(win)), 5) if win else None,
            "strouhal_second_half": st, "history": hist}


def strouhal(hist, d_over_u):
    """St = D / (u_inf T) from the mean spacing T of the upward zero crossings of C_L - mean(C_L)
    over the second half of a (t, C_D, C_L) history; None without at least three crossings or with
    a lift amplitude below 1e-3."""
    if len(hist) < 8:
        return None
    h2 = hist[len(hist) // 2:]
    t = [a for a, _, _ in h2]
    cl = [c for _, _, c in h2]
    m = sum(cl) / len(cl)
    if max(abs(c - m) for c in cl) < 1e-3:
        return None
    ups = []
    for k in range(1, len(cl)):
        a, b = cl[k - 1] - m, cl[k] - m
        if a < 0 <= b:
            ups.append(t[k - 1] + (t[k] - t[k - 1]) * (-a) / (b - a))
    if len(ups) < 3:
        return None
    period = (ups[-1] - ups[0]) / (len(ups) - 1)
    return round(d_over_u / period, 4)


def _ibsl_vs_ibdl(dev):
    """The thesis's central contrast on its Helmholtz circle (Delta u - u = 0 in r < 1/4,
    u = sin 2 theta), 1024^2, ds ~ dx, FD, FP64, tol 1e-8: the single layer Schur complement with
    MINRES against the double layer operator with GMRES; iterations, solve time, time per
    iteration, and the interior error of each grid solution against the closed form."""
    import numpy as np
    import paper_2210_07403_amd as ibdl
    from workloads import problems as P
    s = P.helmholtz_circle(1024, 1.0)
    m = s.markers
    h = s.L[0] / s.n[0]
    ax = [s.origin[d] + h * np.arange(s.n[d]) for d in range(2)]
    ys, xs = np.meshgrid(ax[1], ax[0], indexing="ij")
    inner = np.hypot(xs, ys) < 0.15
    exact = s.exact(xs, ys)
    res = {"workload": "Helmholtz circle r = 0.25, 1024^2, %d markers (ds ~ dx), FD, FP64, tol 1e-8" % m.X.shape[0]}
    for meth, maxit in (("sl", 100000), ("dl", 100)):
        pr = ibdl.Problem(s.dim, s.n, s.L, s.origin, m.X, m.nrm, m.ds, pde=s.pde, kappa=s.kappa, kernel=s.kernel,
                          disc=s.disc, precision="fp64", device=dev, method=meth)
        pr.solve(s.data, None, tol=1e-8, maxit=maxit)
        reps = 1 if meth == "sl" else 5
        t, (_, u, info) = _timed(lambda: pr.solve(s.data, None, tol=1e-8, maxit=maxit), reps)
        err = float(np.max(np.abs(u.cpu().numpy() - exact)[inner]))
        res[meth] = {"iters": info.iters, "solve_ms": round(1e3 * t, 3),
                     "ms_per_iteration": round(1e3 * t / max(info.iters, 1), 4),
                     "true_relres": info.true_relres_fp64, "max_error_r_lt_0.15": err}
        pr.close()
    res["time_ratio_sl_over_dl"] = round(res["sl"]["solve_ms"] / res["dl"]["solve_ms"], 1)
    return res


def _adjoint_timing(dev):
    """Forward solve and adjoint backward on the 256^3 sphere, mixed path (the adjoint row alone)."""
    import numpy as np
    import torch
    import paper_2210_07403_amd as ibdl
    spec, prec, _ = workload("sphere256")
    m = spec.markers
    pr = ibdl.Problem(spec.dim, spec.n, spec.L, spec.origin, m.X, m.nrm, m.ds, pde=spec.pde, kappa=spec.kappa,
                      mu=spec.mu, bc=spec.bc, eta=spec.eta, kernel=spec.kernel, disc=spec.disc, precision=prec,
                      device=dev)
    data = torch.as_tensor(np.asarray(spec.data, dtype=np.float64), device=dev)
    g = torch.as_tensor(spec.g, device=dev).to(pr.grid_dtype) if spec.g is not None else None
    q, u, _ = pr.solve(data, g, tol=spec.tol, maxit=100)
    psi = torch.randn(u.shape, dtype=u.dtype, device=dev, generator=torch.Generator(device=dev).manual_seed(0))
    pr.backward(q, u, psi, tol=spec.tol, maxit=100)
    t_fw, _ = _timed(lambda: pr.solve(data, g, tol=spec.tol, maxit=100), 3)
    t_bw, (_, _, ib) = _timed(lambda: pr.backward(q, u, psi, tol=spec.tol, maxit=100), 3)
    pr.close()
    return {"forward_solve_ms": round(1e3 * t_fw, 3), "backward_ms": round(1e3 * t_bw, 3), "adjoint_iters": ib.iters}


def _cylinder_drag(dev):
    """Stokes flow past the periodic cylinder array (area fraction 0.1, 1024^2, spectral,
    ds ~ h, eta = 10, tol 1e-10): solve + recovery time, GMRES iterations, net force, flux and
    the drag D against the reference value of the thesis's drag table (24.8317); and the FP64 solve
    on 8192^2, the size of the thesis's own IBDL column (24.8368)."""
    import paper_2210_07403_amd as ibdl
    from workloads import problems as P
    s = P.cylinder_array(1024, 0.1)
    m = s.markers
    res = {"workload": "periodic cylinder array, c = 0.1, 1024^2, %d markers, spectral, eta = 10, tol 1e-10"
           % m.X.shape[0]}
    for prec in ("fp64", "mixed"):
        pr = ibdl.Problem(s.dim, s.n, s.L, s.origin, m.X, m.nrm, m.ds, pde=s.pde, kappa=s.kappa, mu=s.mu,
                          eta=s.eta, kernel=s.kernel, disc=s.disc, precision=prec, device=dev)
        g = pr._as_grid(s.g, 2)
        pr.solve(s.data, g, tol=1e-10, maxit=200)
        t, (q, u, info) = _timed(lambda: pr.solve(s.data, g, tol=1e-10, maxit=200), 3)
        tf, F = _timed(lambda: pr.net_force(q), 20)
        tu, U = _timed(lambda: pr.line_integral(u, 0, 0, 0), 20)
        F = F.cpu().tolist()
        U = float(U.cpu()[0])
        D = F[0] / (s.mu * U)
        res[prec] = {"solve_ms": round(1e3 * t, 3), "iters": info.iters, "true_relres": info.true_relres_fp64,
                     "B": [round(F[0], 12), F[1]], "torque": F[2], "U": U, "D": round(D, 4),
                     "D_rel_err_vs_reference": round(D / 24.8317 - 1, 6),
                     "net_force_us": round(1e6 * tf, 1), "line_integral_us": round(1e6 * tu, 1)}
        pr.close()
    s = P.cylinder_array(8192, 0.1)
    m = s.markers
    pr = ibdl.Problem(s.dim, s.n, s.L, s.origin, m.X, m.nrm, m.ds, pde=s.pde, kappa=s.kappa, mu=s.mu,
                      eta=s.eta, kernel=s.kernel, disc=s.disc, precision="fp64", device=dev)
    g = pr._as_grid(s.g, 2)
    pr.solve(s.data, g, tol=1e-10, maxit=200)
    t, (q, u, info) = _timed(lambda: pr.solve(s.data, g, tol=1e-10, maxit=200), 2)
    F = pr.net_force(q).cpu().tolist()
    U = float(pr.line_integral(u, 0, 0, 0).cpu()[0])
    D = F[0] / (s.mu * U)
    res["fp64_8192"] = {"workload": "c = 0.1 on 8192^2, %d markers" % m.X.shape[0],
                        "solve_ms": round(1e3 * t, 2), "iters": info.iters, "true_relres": info.true_relres_fp64,
                        "D": round(D, 6), "D_rel_err_vs_thesis_ibdl_8192": round(D / 24.8368 - 1, 7),
                        "D_rel_err_vs_reference": round(D / 24.8317 - 1, 6)}
    pr.close()
    del q, u, g
    return res


def _near_boundary_timing(dev):
    """Indicator function and near-boundary interpolation (m1 = 6, m2 = 8) on the 1024^2 star
    (4096 markers), FP64: times and nodes corrected (each searches the marker cells around it for
    its three nearest markers)."""
    import numpy as np
    import torch
    import paper_2210_07403_amd as ibdl
    from workloads import problems as P
    s = P.cfg2_star_poisson(1024, 4096)
    m = s.markers
    pr = ibdl.Problem(s.dim, s.n, s.L, s.origin, m.X, m.nrm, m.ds, pde=s.pde, kappa=s.kappa, kernel=s.kernel,
                      disc=s.disc, precision="fp64", device=dev)
    data = torch.as_tensor(np.asarray(s.data, dtype=np.float64), device=dev)
    _, u, _ = pr.solve(data, None, tol=1e-8, maxit=100)
    chi = pr.indicator()
    pr.near_boundary(data, chi, u)
    t_ind, _ = _timed(lambda: pr.indicator(), 5)
    t_nb, fixed = _timed(lambda: pr.near_boundary(data, chi, u), 5)
    ncorr = int(torch.count_nonzero(fixed != u))
    pr.close()
    return {"indicator_ms": round(1e3 * t_ind, 3), "near_boundary_ms": round(1e3 * t_nb, 3),
            "nodes_corrected": ncorr}


def _problem(spec, prec, dev):
    import paper_2210_07403_amd as ibdl
    m = spec.markers
    return ibdl.Problem(spec.dim, spec.n, spec.L, spec.origin, m.X, m.nrm, m.ds, pde=spec.pde, kappa=spec.kappa,
                        mu=spec.mu, bc=spec.bc, eta=spec.eta, kernel=spec.kernel, disc=spec.disc, precision=prec,
                        device=dev)


def _cfg1_circle(dev):
    """The 64^2 circle (cosine kernel, FP64, tol 1e-10): one solve in seconds, on the GPU and by
    the oracle (right-hand side and textbook GMRES to the same tolerance)."""
    import numpy as np
    import oracle
    from oracle.gmres import gmres
    from workloads import problems as P
    s = P.cfg1_circle_cos4()
    pr = _problem(s, "fp64", dev)
    g = pr._as_grid(s.g, 1)
    pr.solve(s.data, g, tol=1e-10, maxit=100)
    t, (_, _, info) = _timed(lambda: pr.solve(s.data, g, tol=1e-10, maxit=100), 20)
    pr.close()
    o = oracle.Setup.from_spec(s)

    def osolve():
        x, k, _ = gmres(o.apply, o.rhs(s.data, s.g), 1e-10, 100)
        o.recover(x, s.data, s.g)
        return k
    t_o, _ = _per_call(osolve, 3, 10.0)
    return {"workload": "2-D screened Poisson kappa=1, 64^2, circle r=0.25, 200 markers, cosine 4-point, FD2, FP64, "
                        "tol 1e-10", "gpu_solve_s": round(t, 6), "iters": info.iters,
            "true_relres": info.true_relres_fp64,
            "cpu_baseline": {"oracle_solve_s": round(t_o, 4), "cores": 1, "kind": "oracle",
                             "sample": "right-hand side, GMRES to 1e-10 and recovery, single-threaded numpy"}}


def _cfg2_star(dev):
    """The 1024^2 star (Poisson, 4096 markers, FD2), Dirichlet and Neumann: FP64 GMRES at 1e-8,
    the mixed path at a Krylov residual of 1e-8, and refinement to a double-precision residual of
    1e-8 (solves/s, iterations, true residual)."""
    import numpy as np
    import torch
    from workloads import problems as P
    out = {"workload": "2-D Poisson, 1024^2, star r=0.3(1+0.2cos5t), 4096 markers, Peskin 4-point, FD2, tol 1e-8"}
    for bc in ("dirichlet", "neumann"):
        s = P.cfg2_star_poisson(1024, 4096, bc=bc)
        data = torch.as_tensor(np.asarray(s.data, dtype=np.float64), device=dev)
        row = {}
        for prec, kind in (("fp64", "solve"), ("mixed", "solve"), ("mixed", "refined")):
            pr = _problem(s, prec, dev)
            run = (lambda: pr.solve(data, None, tol=1e-8, maxit=150)) if kind == "solve" else \
                (lambda: pr.solve_refined(data, None, tol=1e-8, maxit=150, inner_tol=3e-4))
            run()
            t, (_, _, info) = _timed(run, 10)
            name = prec if kind == "solve" else "mixed_refined"
            row[name] = {"solves_per_sec": round(1.0 / t, 1), "ms": round(1e3 * t, 4), "iters": info.iters,
                         "true_relres": info.true_relres_fp64}
            pr.close()
        row["mixed_refined_vs_fp64_at_1e-8"] = round(row["fp64"]["ms"] / row["mixed_refined"]["ms"], 3)
        out[bc] = row
    return out


def _cfg5_stokes(dev):
    """The 512^2 exterior Stokes star (1024 markers, eta = 10, spectral, FP64): the forward solve at
    1e-8 with the grid recovery, and the backward (adjoint GMRES and marker gradients) of
    L = sum_x |w|^2 h^2."""
    import numpy as np
    import torch
    from workloads import problems as P
    s = P.cfg5_stokes_star(512, 1024)
    pr = _problem(s, "fp64", dev)
    data = torch.as_tensor(np.asarray(s.data, dtype=np.float64), device=dev)
    h2 = (s.L[0] / s.n[0]) ** 2
    q, w, _ = pr.solve(data, None, tol=1e-8, maxit=200)
    psi = 2.0 * h2 * w
    pr.backward(q, w, psi, tol=1e-8, maxit=200)
    t_fw, (q, w, info) = _timed(lambda: pr.solve(data, None, tol=1e-8, maxit=200), 10)
    t_bw, (_, _, ib) = _timed(lambda: pr.backward(q, w, psi, tol=1e-8, maxit=200), 10)
    loss = float(h2 * torch.sum(w.double() ** 2))
    pr.close()
    return {"workload": "2-D exterior Stokes, 512^2, star r=0.25(1+0.15cos4t), 1024 markers, eta=10, spectral, FP64, "
                        "tol 1e-8", "forward_ms": round(1e3 * t_fw, 4), "backward_ms": round(1e3 * t_bw, 4),
            "forward_iters": info.iters, "adjoint_iters": ib.iters, "true_relres": info.true_relres_fp64,
            "adjoint_true_relres": ib.true_relres_fp64, "loss": loss}


def host_cpu():
    """CPU model and logical CPU count of this host (lscpu when present)."""
    import subprocess
    model, count = platform.processor() or platform.machine(), os.cpu_count()
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() == "Model name":
                model = v.strip()
            elif k.strip() == "CPU(s)":
                count = int(v.strip())
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return model, count


def cpu_baseline(spec):
    """The FP64 numpy oracle's whole solve of the headline workload on this host: the right-hand
    side, textbook GMRES to a residual of 1e-8 (MGS Arnoldi in exact double arithmetic, so the
    Krylov residual is the true one) and the grid recovery, with the FFTs on every core the process
    may use (scipy.fft workers); beside it one single-threaded operator apply, scaled by the
    solve's apply count (iterations + right-hand side + recovery) to a single-threaded solve."""
    import numpy as np
    import oracle
    from oracle import grid as G
    from oracle.gmres import gmres
    from workloads.problems import random_density
    o = oracle.Setup.from_spec(spec)
    model, ncpu = host_cpu()
    workers = max(1, min(int(os.environ.get("OMP_NUM_THREADS", ncpu) or ncpu), ncpu))
    iters = []

    def osolve():
        x, k, _ = gmres(o.apply, o.rhs(spec.data, spec.g), spec.tol, 100)
        o.recover(x, spec.data, spec.g)
        iters.append(k)
    G.FFT_WORKERS = workers
    try:
        tn, _ = _per_call(osolve, 1)
    finally:
        G.FFT_WORKERS = None
    k = iters[-1]
    q = random_density(spec, seed=0)
    t1, _ = _per_call(lambda: o.apply(q), 1)
    est1 = t1 * (k + 2)
    return {"value": round(1.0 / tn, 5), "unit": "solves/s", "cores": workers, "kind": "oracle",
            "solve_s": round(tn, 2), "oracle_iters": k,
            "single_thread": {"value": round(1.0 / est1, 5), "unit": "solves/s", "cores": 1,
                              "apply_s": round(t1, 2), "solve_s_estimate": round(est1, 2)},
            "sample": f"one whole solve of the same workload (right-hand side, GMRES to 1e-8 in {k} iterations, "
                      f"recovery) by the numpy oracle with its FFTs on {workers} threads (scipy.fft workers; the rest "
                      f"is single-threaded numpy); single_thread: one apply on one thread times {k + 2}; host {model}, "
                      f"{ncpu} logical CPUs"}


def _per_call(fn, max_reps=3, budget_s=4.0):
    """Seconds per call of fn over a bounded sample (at least one call)."""
    reps, t0 = 0, time.perf_counter()
    while True:
        fn()
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= max_reps:
            return el / reps, reps


def cpu_baseline_extras(extras):
    """The FP64 numpy oracle beside the measurements beyond the hot path, each on a bounded sample
    of its workload (one or a few applies, or a sample of nodes), scaled to the GPU figure it sits
    next to; single-threaded numpy / pocketfft."""
    import math
    import numpy as np
    import oracle
    from oracle import nearbdry as NB
    from oracle.ibsl import IBSL
    from oracle.ib import Grid
    from workloads import geometry as geo
    from workloads import problems as P
    out = {}
    if "near_boundary_star1024" in extras:
        s = P.cfg2_star_poisson(1024, 4096)
        m = s.markers
        g = Grid(s.dim, s.n, s.L, s.origin)
        t_ind, _ = _per_call(lambda: NB.indicator(g, m.X, m.nrm, m.ds, s.kernel, s.disc), 1)
        xs, ys = g.nodes()
        u = np.sin(3 * xs + 1) * np.cos(2 * ys)
        nodes = np.argwhere((np.abs(np.hypot(xs - 0.5, ys - 0.5) - 0.3) < 0.02))[:200]
        t_node, _ = _per_call(lambda: [NB.correct_point(g, m.X, s.data, u, np.array([xs[j, i], ys[j, i]]), 8)
                                       for j, i in nodes], 1)
        n_corr = extras["near_boundary_star1024"]["nodes_corrected"]
        out["near_boundary_star1024"] = {
            "indicator_ms": round(1e3 * t_ind, 1),
            "near_boundary_ms": round(1e3 * t_node / len(nodes) * n_corr, 1),
            "sample": f"one indicator; the interpolation of {len(nodes)} nodes scaled to {n_corr}"}
    if "cfg2_star1024" in extras:
        from oracle.gmres import gmres
        s = P.cfg2_star_poisson(1024, 4096)
        o = oracle.Setup.from_spec(s)

        def osolve():
            x, k, _ = gmres(o.apply, o.rhs(s.data, s.g), 1e-8, 150)
            o.recover(x, s.data, s.g)
        t, _ = _per_call(osolve, 1)
        out["cfg2_star1024"] = {"dirichlet_solve_ms": round(1e3 * t, 1), "cores": 1,
                                "sample": "one whole FP64 Dirichlet solve (right-hand side, GMRES to 1e-8, recovery)"}
    if "cfg5_stokes512" in extras:
        s = P.cfg5_stokes_star(512, 1024)
        o = oracle.Setup.from_spec(s)
        q = np.random.default_rng(0).standard_normal(o.n_aug)
        t_app, _ = _per_call(lambda: o.apply(q), 1)
        it = extras["cfg5_stokes512"]["forward_iters"]
        out["cfg5_stokes512"] = {"apply_ms": round(1e3 * t_app, 1),
                                 "forward_ms_estimate": round(1e3 * t_app * (it + 3), 1), "cores": 1,
                                 "sample": f"one FP64 apply, times {it} GMRES iterations + 3 (right-hand side, "
                                           "true residual, recovery)"}
    if "cylinder_array_drag" in extras:
        s = P.cylinder_array(1024, 0.1)
        o = oracle.Setup.from_spec(s)
        q = np.random.default_rng(0).standard_normal(o.n_aug)
        t_app, _ = _per_call(lambda: o.apply(q), 1)
        it = extras["cylinder_array_drag"]["fp64"]["iters"]
        out["cylinder_array_drag"] = {"apply_ms": round(1e3 * t_app, 1),
                                      "solve_ms_estimate": round(1e3 * t_app * (it + 3), 1),
                                      "sample": f"one FP64 apply, times {it} GMRES iterations + 3 (right-hand side, "
                                                "true residual, recovery)"}
    if "ibsl_vs_ibdl_helmholtz1024" in extras:
        s = P.helmholtz_circle(1024, 1.0)
        o = IBSL.from_spec(s)
        q = np.random.default_rng(0).standard_normal(o.n_aug)
        t_app, _ = _per_call(lambda: o.apply(q), 1)
        it = extras["ibsl_vs_ibdl_helmholtz1024"]["sl"]["iters"]
        out["ibsl_vs_ibdl_helmholtz1024"] = {"sl_apply_ms": round(1e3 * t_app, 1),
                                             "sl_solve_ms_estimate": round(1e3 * t_app * it, 1),
                                             "sample": f"one FP64 single-layer apply, times {it} MINRES iterations"}
    if "ns_cylinder_re100" in extras:
        N, L, r, rho, dt = 1024, 8.0, 0.15, 1.0, 1.8e-3
        curve = geo.PolarCurve((1.85, 4.0), r)
        mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), L / N, 1.0)).flipped()
        o = oracle.Setup(2, (N, N), (L, L), (0.0, 0.0), mk.X, mk.nrm, mk.ds, "stokes", math.sqrt(1.5 * rho / dt),
                         2 * r / 100.0, "dirichlet", 10.0, "peskin4", "spectral")
        q = np.random.default_rng(0).standard_normal(o.n_aug)
        t_app, _ = _per_call(lambda: o.apply(q), 1)
        it = extras["ns_cylinder_re100"]["mean_gmres_iters"]
        out["ns_cylinder_re100"] = {"apply_ms": round(1e3 * t_app, 1),
                                    "step_ms_estimate": round(1e3 * t_app * (it + 3), 1),
                                    "sample": f"one FP64 apply, times {it} GMRES iterations + 3 (right-hand side, "
                                              "recovery, nonlinear term)"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sphere256", choices=["sphere256", "star1024", "circle64"])
    ap.add_argument("--apply-reps", type=int, default=100)
    ap.add_argument("--inner-tol", type=float, default=3e-4,
                    help="Krylov tolerance of each float GMRES round of the refined solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-vs-FP64, adjoint and batched measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain device copy of known size (counter calibration runs)")
    ap.add_argument("--ns-cylinder", type=int, default=0, metavar="STEPS",
                    help="only run the Navier-Stokes cylinder for STEPS steps and print its JSON line")
    ap.add_argument("--ns-re", type=float, default=10.0)
    ap.add_argument("--ns-every", type=int, default=0, help="drag/lift sample interval in steps (0: STEPS / 40)")
    ap.add_argument("--only", choices=["near_boundary", "cylinder_array", "ibsl", "ns", "adjoint", "batch"],
                    default=None,
                    help="only run one of the measurements beyond the hot path and print its JSON line")
    args = ap.parse_args()
    if args.only:
        import torch
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        run = {"near_boundary": _near_boundary_timing, "cylinder_array": _cylinder_drag, "ibsl": _ibsl_vs_ibdl,
               "ns": lambda d: ns_cylinder(d, 100.0, 200, 5), "adjoint": _adjoint_timing,
               "batch": _batch_timing}[args.only]
        print(json.dumps(run(dev)))
        return
    if args.ns_cylinder > 0:
        import torch
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        every = args.ns_every if args.ns_every > 0 else max(args.ns_cylinder // 40, 1)
        print(json.dumps(ns_cylinder(dev, args.ns_re, args.ns_cylinder, 0, report_every=every)))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the IBDL library has no multi-GPU path (see the design notes); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2210_07403_amd as ibdl
    from workloads.problems import random_density

    spec, prec, desc = workload(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    m = spec.markers
    print(f"# workload {args.workload}: {desc}", file=sys.stderr, flush=True)
    pr = ibdl.Problem(spec.dim, spec.n, spec.L, spec.origin, m.X, m.nrm, m.ds, pde=spec.pde, kappa=spec.kappa,
                      mu=spec.mu, bc=spec.bc, eta=spec.eta, kernel=spec.kernel, disc=spec.disc, precision=prec,
                      device=dev)
    gdt = torch.float32 if prec == "mixed" else torch.float64
    data = torch.as_tensor(np.asarray(spec.data, dtype=np.float64), device=dev)
    g = torch.as_tensor(spec.g, device=dev).to(gdt).reshape((pr.nq,) + pr.grid_shape) if spec.g is not None else None
    tol = spec.tol

    step = lambda: pr.solve_refined(data, g, tol=tol, maxit=100, inner_tol=args.inner_tol)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} solves)", file=sys.stderr, flush=True)

    iters, relres = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, info = step()
        iters.append(info.iters)
        relres.append(info.true_relres_fp64)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(f"# timed {args.steps} solves in {el:.3f} s, inner iterations {iters}, worst true residual "
          f"{max(relres):.2e}", file=sys.stderr, flush=True)
    # the same workload solved plainly: the mixed path stopped on its own Krylov residual of 1e-8 (its
    # true residual stays at the float operator's level), and FP64 GMRES at 1e-8
    t_mix, (_, _, im) = _timed(lambda: pr.solve(data, g, tol=tol, maxit=100), 5)
    p64 = ibdl.Problem(spec.dim, spec.n, spec.L, spec.origin, m.X, m.nrm, m.ds, pde=spec.pde, kappa=spec.kappa,
                       mu=spec.mu, bc=spec.bc, eta=spec.eta, kernel=spec.kernel, disc=spec.disc, precision="fp64",
                       device=dev)
    g64 = g.double() if g is not None else None
    p64.solve(data, g64, tol=tol, maxit=100)
    t64, (_, _, i64) = _timed(lambda: p64.solve(data, g64, tol=tol, maxit=100), 5)
    p64.close()
    plain = {"mixed_krylov_1e-8": {"solves_per_sec": round(1.0 / t_mix, 2), "ms": round(1e3 * t_mix, 4),
                                   "iters": im.iters, "true_relres": im.true_relres_fp64},
             "fp64_1e-8": {"solves_per_sec": round(1.0 / t64, 2), "ms": round(1e3 * t64, 4), "iters": i64.iters,
                           "true_relres": i64.true_relres_fp64},
             "refined_vs_fp64_speedup": round(t64 / (el / args.steps), 3)}

    # operator applies alone, and per-stage HIP-event timing on the handle's stream
    q = torch.as_tensor(random_density(spec, seed=0), device=dev)
    for _ in range(5):
        pr.apply(q)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(pr.stream)
    for _ in range(args.apply_reps):
        pr.apply(q)
    ev1.record(pr.stream)
    ev1.synchronize()
    apply_ms = ev0.elapsed_time(ev1) / args.apply_reps
    # the distribution of single applies (an event pair around each, same stream)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.apply_reps)]
    for e0, e1 in evs:
        e0.record(pr.stream)
        pr.apply(q)
        e1.record(pr.stream)
    evs[-1][1].synchronize()
    single = np.sort([e0.elapsed_time(e1) for e0, e1 in evs])
    apply_pct = {"p10": float(np.percentile(single, 10)), "median": float(np.median(single)),
                 "p90": float(np.percentile(single, 90))}
    pr.set_timing(True)
    for _ in range(args.apply_reps):
        pr.apply(q)
    stages = pr.timing()
    pr.set_timing(False)
    cost = stage_cost(spec, prec, pr)
    per = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items() if v[1]}
    dom = max(per, key=per.get)
    stage_report = {}
    for k in per:
        kind, amount = cost.get(k, ("hbm", 0))
        rate = amount / (per[k] * 1e-3) if per[k] > 0 else 0.0
        stage_report[k] = {"ms": round(per[k], 5), "bound": kind,
                           ("GB" if kind == "hbm" else "GFLOP"): round(amount / 1e9, 5),
                           ("GB_s" if kind == "hbm" else "TFLOP_s"): round(rate / (1e9 if kind == "hbm" else 1e12), 3)}
    kind, amount = cost[dom]
    if kind == "hbm":
        ach = amount / (per[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4)}
    else:
        ach = amount / (per[dom] * 1e-3) / 1e12
        peak = MATRIX_PEAK_TFLOPS[prec]
        roof = {"bound": kind, "kernel": dom, "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 5)}
    roof["traffic"] = load_traffic(args.workload, dom)
    apply_bytes = sum(v[1] for k, v in cost.items() if v[0] == "hbm")
    mu, mf = model_bytes(spec, prec, pr)
    if args.calibrate_copy:
        # a device copy of 256 MiB each way, and a second kernel of known size (a float to bfloat16
        # cast: 256 MiB read, 128 MiB written) to cross-check the counters' scale
        x = torch.empty(64 * 2 ** 20, dtype=torch.float32, device=dev).fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        z = torch.empty(64 * 2 ** 20, dtype=torch.bfloat16, device=dev)
        for _ in range(3):
            z.copy_(x)
        torch.cuda.synchronize()

    extras = {} if args.no_extras else measure_extras(spec, prec, pr, data, g, tol, dev)
    out = {
        "metric": METRIC,
        "value": round(args.steps / el, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 grid + f64 Krylov" if prec == "mixed" else "f64",
        "data": "synthetic (seeded geometry and manufactured boundary data; no dataset)",
        "config": {"workload": desc, "grid": list(spec.n), "n_ib": spec.n_ib, "n_aug": pr.n_aug,
                   "tol": tol, "residual": "double-precision ||b - A q|| / ||b||", "precision": prec,
                   "solver": f"GMRES on the float-applied operator, double-precision residual corrections "
                             f"(inner tolerance {args.inner_tol:g})"},
        "solves_per_sec": round(args.steps / el, 3),
        "inner_gmres_iterations": iters,
        "true_relres_fp64": max(relres),
        "applies_per_sec": round(1e3 / apply_ms, 2),
        "plain_solves": plain,
        "apply_ms": round(apply_ms, 5),
        "apply_single_ms": {k: round(v, 5) for k, v in apply_pct.items()},
        "apply_effective_GB_s": round(apply_bytes / (apply_ms * 1e-3) / 1e9, 1),
        "apply_frac_hbm_peak": round(apply_bytes / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "model_U_GB": round(mu / 1e9, 4),
        "model_U_effective_GB_s": round(mu / (apply_ms * 1e-3) / 1e9, 1),
        "model_U_frac_hbm_peak": round(mu / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "model_F_effective_GB_s": round(mf / (apply_ms * 1e-3) / 1e9, 1),
        "active_rows": list(pr.active_rows()),
        "launch_shape": dict(zip(("rows_per_block", "lines_y", "lines_last"), pr.launch_shape())),
        "stages": stage_report,
        "roofline": roof,
        **extras,
    }
    pr.close()
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on the same workload", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(spec)
        if extras:
            print("# timing the CPU oracle beside the other measurements", file=sys.stderr, flush=True)
            for k, v in cpu_baseline_extras(extras).items():
                out[k]["cpu_baseline"] = v
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
