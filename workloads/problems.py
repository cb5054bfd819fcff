"""Seeded synthetic IBDL problems: grid, markers, boundary data, forcing.

Each builder returns a `ProblemSpec` holding plain arrays.  Both the CPU
oracle and the HIP library take these as inputs; no builder evaluates the
IBDL operator itself.  Manufactured data follow the thesis's test problems
(Sec. 5.4, 5.7, 6.4) and the workload recipes stated in the design notes.

Grid conventions: nodes at origin + j*h (Sec. 2.2.1), arrays indexed
[z][y][x] (x fastest); 2-D arrays are [y][x].  Vector fields carry a leading
component axis.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from . import geometry as geo


@dataclass
class ProblemSpec:
    name: str
    dim: int
    n: tuple                    # grid points per axis, (nx, ny[, nz])
    L: tuple                    # box lengths per axis
    origin: tuple               # box origin per axis
    pde: str                    # "screened" | "poisson" | "stokes"
    kappa: float                # screening constant (scalar) or Brinkman k (Stokes)
    mu: float                   # viscosity (Stokes); 1 for scalar problems
    bc: str                     # "dirichlet" | "neumann"
    eta: float                  # completion constant (0 = plain IBDL)
    kernel: str                 # "peskin4" | "cos4" | "bspline6"
    disc: str                   # "fd2" | "spectral"
    markers: geo.Markers
    data: np.ndarray            # U_b (Dirichlet) or V_b (Neumann); (n_ib,) or (n_ib, dim)
    g: Optional[np.ndarray]     # extended forcing on the grid, or None for zero
    tol: float = 1e-8
    exact: Optional[Callable] = None        # exact solution u(x, y[, z]) for error checks
    inside: Optional[Callable] = None       # indicator of the PDE domain Omega at nodes
    meta: dict = field(default_factory=dict)

    @property
    def h(self) -> float:
        return self.L[0] / self.n[0]

    @property
    def n_ib(self) -> int:
        return self.markers.n_ib

    @property
    def nq(self) -> int:
        return self.dim if self.pde == "stokes" else 1

    @property
    def has_ubar(self) -> bool:
        return self.eta > 0 and self.kappa == 0

    @property
    def n_aug(self) -> int:
        return self.n_ib * self.nq + (self.nq if self.has_ubar else 0)

    def grid_shape(self) -> tuple:
        return tuple(reversed(self.n))

    def nodes(self):
        """Node coordinates as arrays of grid_shape, in (x, y[, z]) order."""
        axes = [self.origin[d] + self.h * np.arange(self.n[d]) for d in range(self.dim)]
        mesh = np.meshgrid(*reversed(axes), indexing="ij")
        return list(reversed(mesh))


def _grid(dim, n, L, origin):
    n = (n,) * dim if np.isscalar(n) else tuple(n)
    L = (L,) * dim if np.isscalar(L) else tuple(L)
    origin = (origin,) * dim if np.isscalar(origin) else tuple(origin)
    return n, L, origin


def _nodes(dim, n, L, origin):
    h = L[0] / n[0]
    axes = [origin[d] + h * np.arange(n[d]) for d in range(dim)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(mesh))


# --------------------------------------------------------------- thesis pins
def helmholtz_circle(N, alpha, kernel="peskin4", disc="fd2", tol=1e-8, data="sin2theta"):
    """Sec. 5.4.1, eq. (pde again again): Delta u - u = 0 inside r<0.25, u = sin 2theta on Gamma,
    box [-1/2, 1/2]^2.  Exact u = I_2(r) sin(2 theta) / I_2(1/4).  `data="linear"` gives
    eq. (pde again 2): Delta u - u = -(x+y), u = x + y."""
    from scipy.special import iv
    n, L, o = _grid(2, N, 1.0, -0.5)
    h = 1.0 / N
    curve = geo.PolarCurve((0.0, 0.0), 0.25)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), h, alpha))
    x, y = _nodes(2, n, L, o)
    inside = np.hypot(x, y) < 0.25
    if data == "sin2theta":
        def exact(x, y):
            r, t = np.hypot(x, y), np.arctan2(y, x)
            return iv(2, r) * np.sin(2 * t) / iv(2, 0.25)
        g = None
    else:
        def exact(x, y):
            return x + y
        g = np.where(inside, -(x + y), 0.0)
    Ub = exact(mk.X[:, 0], mk.X[:, 1])
    return ProblemSpec(f"helmholtz_circle_N{N}_a{alpha}", 2, n, L, o, "screened", 1.0, 1.0,
                       "dirichlet", 0.0, kernel, disc, mk, Ub, g, tol, exact,
                       lambda x, y: np.hypot(x, y) < 0.25,
                       meta=dict(curve=curve, alpha=alpha))


def starfish_poisson(N, alpha, tol=1e-8):
    """Sec. 5.4.2, eq. (pde again 3): exterior of the starfish in [-2, 2]^2, Poisson,
    u = sin(pi x/2) - cos(pi y/2).  g_e inside the star makes the grid sum of g~ vanish
    (solvability choice of Sec. 5.3.3)."""
    n, L, o = _grid(2, N, 4.0, -2.0)
    h = 4.0 / N
    curve = geo.PolarCurve((0.0, 0.0), 1.0, 5, 0.0, 0.25)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), h, alpha)).flipped()
    x, y = _nodes(2, n, L, o)
    star_in = curve.inside(x, y)
    gfun = (math.pi ** 2 / 4) * (np.cos(math.pi * y / 2) - np.sin(math.pi * x / 2))
    g = np.where(star_in, 0.0, gfun)
    g_e = -g.sum() / star_in.sum()
    g = np.where(star_in, g_e, g)

    def exact(x, y):
        return np.sin(math.pi * x / 2) - np.cos(math.pi * y / 2)
    Ub = exact(mk.X[:, 0], mk.X[:, 1])
    return ProblemSpec(f"starfish_poisson_N{N}_a{alpha}", 2, n, L, o, "poisson", 0.0, 1.0,
                       "dirichlet", 0.0, "peskin4", "fd2", mk, Ub, g, tol, exact,
                       lambda x, y: ~curve.inside(x, y), meta=dict(curve=curve, alpha=alpha))


def completed_poisson_exterior(N, Lbox, eta, which="exp", alpha=0.75, tol=1e-8):
    """Sec. 5.4.3: exterior of the circle r=1/4 in [-L/2, L/2]^2, Poisson.
    which="exp": u = exp(sin(2 pi x / L)) (eq. poisson shit pde exp);
    which="trig": u = sin(2 pi x/L) - cos(2 pi y/L) (eq. poisson shit pde fine)."""
    n, L, o = _grid(2, N, Lbox, -Lbox / 2)
    h = Lbox / N
    curve = geo.PolarCurve((0.0, 0.0), 0.25)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), h, alpha)).flipped()
    x, y = _nodes(2, n, L, o)
    w = 2 * math.pi / Lbox
    if which == "exp":
        def exact(x, y):
            return np.exp(np.sin(w * x))
        gfun = w ** 2 * np.exp(np.sin(w * x)) * (np.cos(w * x) ** 2 - np.sin(w * x))
    else:
        def exact(x, y):
            return np.sin(w * x) - np.cos(w * y)
        gfun = -w ** 2 * (np.sin(w * x) - np.cos(w * y))
    body = np.hypot(x, y) < 0.25
    g = np.where(body, 0.0, gfun)
    if eta == 0:
        g = np.where(body, -g.sum() / body.sum(), g)
    Ub = exact(mk.X[:, 0], mk.X[:, 1])
    return ProblemSpec(f"completed_poisson_{which}_N{N}_L{Lbox}_eta{eta}", 2, n, L, o, "poisson",
                       0.0, 1.0, "dirichlet", float(eta), "peskin4", "fd2", mk, Ub, g, tol, exact,
                       lambda x, y: np.hypot(x, y) >= 0.25, meta=dict(curve=curve, alpha=alpha))


def neumann_circle(N, alpha=0.75, tol=1e-8):
    """Sec. 5.7, eq. (pde again 4): Delta u - u = -(x^2 - y^2) inside r<1/4,
    du/dn = 8 (x^2 - y^2) on Gamma; exact u = x^2 - y^2."""
    n, L, o = _grid(2, N, 1.0, -0.5)
    h = 1.0 / N
    curve = geo.PolarCurve((0.0, 0.0), 0.25)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), h, alpha))
    x, y = _nodes(2, n, L, o)
    inside = np.hypot(x, y) < 0.25
    g = np.where(inside, -(x ** 2 - y ** 2), 0.0)
    Vb = 8.0 * (mk.X[:, 0] ** 2 - mk.X[:, 1] ** 2)

    def exact(x, y):
        return x ** 2 - y ** 2
    return ProblemSpec(f"neumann_circle_N{N}_a{alpha}", 2, n, L, o, "screened", 1.0, 1.0,
                       "neumann", 0.0, "peskin4", "fd2", mk, Vb, g, tol, exact,
                       lambda x, y: np.hypot(x, y) < 0.25, meta=dict(curve=curve, alpha=alpha))


def _brinkman_fields(x, y, s, k):
    """Sec. 6.4.1/6.4.2 manufactured flow, frequency s: u = e^{sin sx} cos sy,
    v = -cos sx e^{sin sx} sin sy, p = e^{cos sy}; forcing g = Delta u - k^2 u - grad p."""
    es = np.exp(np.sin(s * x))
    u = es * np.cos(s * y)
    v = -np.cos(s * x) * es * np.sin(s * y)
    g1 = s ** 2 * es * np.cos(s * y) * (np.cos(s * x) ** 2 - np.sin(s * x) - 1 - k ** 2 / s ** 2)
    g2 = (-s ** 2 * np.cos(s * x) * es * np.sin(s * y)
          * (np.cos(s * x) ** 2 - 3 * np.sin(s * x) - 2 - k ** 2 / s ** 2)
          + s * np.sin(s * y) * np.exp(np.cos(s * y)))
    return u, v, g1, g2


def brinkman_circle(N, alpha, tol=1e-8):
    """Sec. 6.4.1, eq. (brink pde again): Delta u - u - grad p = g inside r<3/4,
    box [-1, 1]^2, spectral.  Iteration counts in table (iteration table 6.1)."""
    n, L, o = _grid(2, N, 2.0, -1.0)
    h = 2.0 / N
    curve = geo.PolarCurve((0.0, 0.0), 0.75)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), h, alpha))
    x, y = _nodes(2, n, L, o)
    inside = np.hypot(x, y) < 0.75
    _, _, g1, g2 = _brinkman_fields(x, y, 1.0, 1.0)
    g = np.stack([np.where(inside, g1, 0.0), np.where(inside, g2, 0.0)])
    u, v, _, _ = _brinkman_fields(mk.X[:, 0], mk.X[:, 1], 1.0, 1.0)
    Ub = np.stack([u, v], axis=1)

    def exact(x, y):
        uu, vv, _, _ = _brinkman_fields(x, y, 1.0, 1.0)
        return np.stack([uu, vv])
    return ProblemSpec(f"brinkman_circle_N{N}_a{alpha}", 2, n, L, o, "stokes", 1.0, 1.0,
                       "dirichlet", 0.0, "peskin4", "spectral", mk, Ub, g, tol, exact,
                       lambda x, y: np.hypot(x, y) < 0.75, meta=dict(curve=curve, alpha=alpha))


def stokes_exterior_circle(N, eta=10.0, k=0.0, alpha=1.0, tol=1e-8):
    """Sec. 6.4.2, eq. (brink pde ext): exterior of r=3/4 in [-1, 1]^2, completed IBDL,
    spectral, ds ~ dx, pi-scaled manufactured flow.  g_e = 0 inside the body."""
    n, L, o = _grid(2, N, 2.0, -1.0)
    h = 2.0 / N
    curve = geo.PolarCurve((0.0, 0.0), 0.75)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), h, alpha)).flipped()
    x, y = _nodes(2, n, L, o)
    body = np.hypot(x, y) < 0.75
    _, _, g1, g2 = _brinkman_fields(x, y, math.pi, k)
    g = np.stack([np.where(body, 0.0, g1), np.where(body, 0.0, g2)])
    u, v, _, _ = _brinkman_fields(mk.X[:, 0], mk.X[:, 1], math.pi, k)
    Ub = np.stack([u, v], axis=1)

    def exact(x, y):
        uu, vv, _, _ = _brinkman_fields(x, y, math.pi, k)
        return np.stack([uu, vv])
    return ProblemSpec(f"stokes_exterior_N{N}_eta{eta}_k{k}", 2, n, L, o, "stokes", float(k), 1.0,
                       "dirichlet", float(eta), "peskin4", "spectral", mk, Ub, g, tol, exact,
                       lambda x, y: np.hypot(x, y) >= 0.75, meta=dict(curve=curve, alpha=alpha))


def cylinder_array(N, c, eta=10.0, alpha=1.0, tol=1e-10):
    """Sec. 6.5 (Stokes flow around a periodic array of cylinders): Stokes (mu = 1, k = 0) in the
    periodic box [-0.5, 0.5]^2 outside the disk of area fraction c at the origin, u = 0 on the
    circle, driven by g = (-1, 0); completed IBDL, spectral, ds ~ alpha h.  The forcing is
    extended by the same constant inside the disk."""
    n, L, o = _grid(2, N, 1.0, -0.5)
    h = 1.0 / N
    r = math.sqrt(c / math.pi)
    curve = geo.PolarCurve((0.0, 0.0), r)
    mk = curve.markers(geo.n_ib_for_spacing(curve.perimeter(), h, alpha)).flipped()
    g = np.stack([-np.ones((N, N)), np.zeros((N, N))])
    return ProblemSpec(f"cylinder_array_N{N}_c{c}", 2, n, L, o, "stokes", 0.0, 1.0, "dirichlet", float(eta),
                       "peskin4", "spectral", mk, np.zeros((mk.X.shape[0], 2)), g, tol, None,
                       lambda x, y: np.hypot(x, y) >= r, meta=dict(curve=curve, c=c, r=r, alpha=alpha))


# ---------------------------------------------------------------- workloads
def harmonic_poly_2d(rng, center=(0.5, 0.5), degree=4):
    """u = sum_k a_k * {Re, Im}(z - c)^n, n = 1..degree, a_k ~ N(0, 1): harmonic."""
    coef = rng.standard_normal(2 * degree)
    c = complex(*center)

    def u(x, y):
        z = (x + 1j * y) - c
        out = np.zeros(np.shape(z))
        for m in range(1, degree + 1):
            zm = z ** m
            out = out + coef[2 * m - 2] * zm.real + coef[2 * m - 1] * zm.imag
        return out

    def grad(x, y):
        z = (x + 1j * y) - c
        gx = np.zeros(np.shape(z))
        gy = np.zeros(np.shape(z))
        for m in range(1, degree + 1):
            dz = m * z ** (m - 1)
            # d/dx Re f = Re f', d/dy Re f = -Im f'; d/dx Im f = Im f', d/dy Im f = Re f'
            gx = gx + coef[2 * m - 2] * dz.real + coef[2 * m - 1] * dz.imag
            gy = gy - coef[2 * m - 2] * dz.imag + coef[2 * m - 1] * dz.real
        return gx, gy
    return u, grad, coef


def cfg1_circle_cos4(N=64, n_ib=200, tol=1e-10):
    """2-D interior Dirichlet screened Poisson (kappa=1), unit box, circle r=1/4 at the centre,
    cosine 4-point kernel, u = e^x sin y (harmonic), so g = -u inside and 0 outside."""
    n, L, o = _grid(2, N, 1.0, 0.0)
    mk = geo.circle((0.5, 0.5), 0.25, n_ib)
    x, y = _nodes(2, n, L, o)
    inside = np.hypot(x - 0.5, y - 0.5) < 0.25

    def exact(x, y):
        return np.exp(x) * np.sin(y)
    g = np.where(inside, -exact(x, y), 0.0)
    Ub = exact(mk.X[:, 0], mk.X[:, 1])
    return ProblemSpec(f"cfg1_circle_N{N}", 2, n, L, o, "screened", 1.0, 1.0, "dirichlet", 0.0,
                       "cos4", "fd2", mk, Ub, g, tol, exact,
                       lambda x, y: np.hypot(x - 0.5, y - 0.5) < 0.25)


def cfg2_star_poisson(N=1024, n_ib=4096, bc="dirichlet", seed=2, tol=1e-8):
    """2-D interior Poisson, unit box, star r = 0.3 (1 + 0.2 cos 5t), harmonic-polynomial data."""
    n, L, o = _grid(2, N, 1.0, 0.0)
    curve = geo.PolarCurve((0.5, 0.5), 0.3, 5, 0.2, 0.0)
    mk = curve.markers(n_ib)
    u, grad, coef = harmonic_poly_2d(np.random.default_rng(seed))
    if bc == "dirichlet":
        data = u(mk.X[:, 0], mk.X[:, 1])
    else:
        gx, gy = grad(mk.X[:, 0], mk.X[:, 1])
        data = gx * mk.nrm[:, 0] + gy * mk.nrm[:, 1]
    return ProblemSpec(f"cfg2_star_{bc}_N{N}", 2, n, L, o, "poisson", 0.0, 1.0, bc, 0.0,
                       "peskin4", "fd2", mk, data, None, tol, u,
                       lambda x, y: curve.inside(x, y), meta=dict(curve=curve, coef=coef))


def cfg3_sphere(N=256, freq=86, tol=1e-8, kappa=10.0):
    """3-D interior Dirichlet screened Poisson (kappa=10), unit box, sphere r=0.3 at the centre
    (icosphere of 10 freq^2 + 2 markers), u = e^{x+y} cos(sqrt 2 z) (harmonic), g = -kappa^2 u
    inside and 0 outside."""
    n, L, o = _grid(3, N, 1.0, 0.0)
    mk = geo.icosphere((0.5, 0.5, 0.5), 0.3, freq)

    def exact(x, y, z):
        return np.exp(x + y) * np.cos(math.sqrt(2.0) * z)
    x, y, z = _nodes(3, n, L, o)
    inside = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2 < 0.09
    g = np.where(inside, -kappa ** 2 * exact(x, y, z), 0.0)
    Ub = exact(mk.X[:, 0], mk.X[:, 1], mk.X[:, 2])
    return ProblemSpec(f"cfg3_sphere_N{N}", 3, n, L, o, "screened", kappa, 1.0, "dirichlet", 0.0,
                       "peskin4", "fd2", mk, Ub, g, tol, exact,
                       lambda x, y, z: (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2 < 0.09)


def cfg4_batch(nprob=64, seed=4, sizes=(128, 256, 512)):
    """Batch of independent 2-D interior Poisson problems on random stars (uneven grids)."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(nprob):
        N = int(rng.choice(sizes))
        lobes = int(rng.integers(3, 8))
        amp = float(rng.uniform(0.05, 0.25))
        r0 = float(rng.uniform(0.2, 0.35))
        a = float(rng.uniform(0.5, 1.0))
        curve = geo.PolarCurve((0.5, 0.5), r0, lobes, amp, 0.0)
        P = curve.perimeter()
        n_ib = int(np.clip(round(P / (a * (1.0 / N))), 256, 2048))
        mk = curve.markers(n_ib)
        u, _, coef = harmonic_poly_2d(np.random.default_rng((seed, p)))
        n, L, o = _grid(2, N, 1.0, 0.0)
        out.append(ProblemSpec(f"cfg4_p{p}_N{N}", 2, n, L, o, "poisson", 0.0, 1.0, "dirichlet",
                               0.0, "peskin4", "fd2", mk, u(mk.X[:, 0], mk.X[:, 1]), None, 1e-8, u,
                               lambda x, y, c=curve: c.inside(x, y), meta=dict(curve=curve)))
    return out


def cfg5_stokes_star(N=512, n_ib=1024, eta=10.0, seed=5, tol=1e-8):
    """2-D exterior Stokes (mu=1, k=0), completed IBDL, star body r = 0.25 (1 + 0.15 cos 4t),
    spectral.  Disturbance form: w = -u_bg on Gamma with u_bg = (a sin 2 pi y, b sin 2 pi x)."""
    rng = np.random.default_rng(seed)
    a = float(rng.uniform(0.5, 1.5))
    b = float(rng.uniform(-0.5, 0.5))
    n, L, o = _grid(2, N, 1.0, 0.0)
    curve = geo.PolarCurve((0.5, 0.5), 0.25, 4, 0.15, 0.0)
    mk = curve.markers(n_ib).flipped()
    ubg = np.stack([a * np.sin(2 * math.pi * mk.X[:, 1]), b * np.sin(2 * math.pi * mk.X[:, 0])], 1)
    return ProblemSpec(f"cfg5_stokes_star_N{N}", 2, n, L, o, "stokes", 0.0, 1.0, "dirichlet", eta,
                       "peskin4", "spectral", mk, -ubg, None, tol, None,
                       lambda x, y: ~curve.inside(x, y), meta=dict(curve=curve, a=a, b=b))


def random_density(spec: ProblemSpec, seed=0):
    """q ~ N(0, 1) of length n_aug (apply benchmarks and parity)."""
    return np.random.default_rng(seed).standard_normal(spec.n_aug)


def random_grid(spec: ProblemSpec, ncomp=1, seed=0):
    shape = ((ncomp,) if ncomp > 1 else ()) + spec.grid_shape()
    return np.random.default_rng(seed).standard_normal(shape)
