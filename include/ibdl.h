/*
 * ibdl.h -- C ABI of the MI355X (gfx950) Immersed Boundary Double Layer library.
 *
 * The library applies and inverts the IBDL boundary operator of
 * B. J. Leathers, "The Immersed Boundary Double Layer (IBDL) Method" (2022, arXiv 2210.07403):
 *
 *   scalar Dirichlet   A Q = -S* L^-1 S~ Q + Q/2                 (Sec. 5.3.2, eq. ibdl schur again)
 *   scalar Neumann     A U = -S* L^-1 S~ U - U/2                 (Sec. 5.2, eq. Neumann saddle point)
 *   completed scalar   + eta S in the dipole spread, + u_bar and a border row (Sec. 5.3.3)
 *   Brinkman / Stokes  A Q = S* u[Q] + Q/2 (+ u_bar),             (Sec. 6.3.2 eq. brink ibdl eqn,
 *                      u[Q] = -grad D0^-1 S(Q.n) - L^-1 P (eta S Q + mu div S A)    Sec. 6.3.3)
 *
 * with S the spread (Sec. 2.2.2, eq. spread operator again2), S* the interpolation
 * (eq. interpolation again), S~ Q = div(S(Q n)) (Sec. 5.3.1, eq. Stilde), L = Delta - kappa^2
 * (scalar) or mu Delta - k^2 (Stokes) on a periodic grid, D0^-1 the mean-zero inverse Laplacian
 * (Sec. 2.2.4) and P = I - grad D0^-1 div (Sec. 2.3.2).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller (e.g. a PyTorch tensor's
 *     data pointer).  The handle owns only its internal workspaces.
 *   - Grid arrays are row-major [component][z][y][x] (x fastest; 2-D: [component][y][x]).  Their
 *     element type is double under IBDL_FP64 and float under IBDL_MIXED.
 *   - Marker arrays are double: X and nrm are [n_ib][dim]; ds is [n_ib].  Densities and boundary
 *     data are double [n_ib][nq] (nq = 1 scalar, nq = dim Stokes) followed, in the unknown vector
 *     only, by u_bar ([nq]) when the method carries it: n_aug = n_ib*nq + (has_ubar ? nq : 0),
 *     has_ubar = (eta > 0 && kappa == 0).
 *   - nrm is the unit normal pointing out of the PDE domain Omega (Sec. 5.1.1); ds are the
 *     quadrature weights (arclength in 2-D, area in 3-D).
 *   - All calls are asynchronous on cfg.stream (a hipStream_t; NULL = the default stream), except
 *     ibdl_create / ibdl_set_markers (which synchronise once) and ibdl_solve, which synchronises to
 *     run the Krylov iteration and to fill ibdl_info_t.
 *   - One host thread per handle at a time.  Calls that overlap on one handle race.
 *   - Errors: a negative status; outputs are then unspecified and ibdl_last_error() describes the
 *     failure.  Arguments are validated on the host.  Device data are inspected only when the
 *     environment holds IBDL_CHECK=1 as the handle is created: then ibdl_create,
 *     ibdl_set_markers, ibdl_apply, ibdl_apply_transpose, ibdl_grid_solve, ibdl_solve,
 *     ibdl_solve_refined and ibdl_backward scan the arrays they take and return for NaN and
 *     infinities (one device pass and one stream synchronisation per array; not for use under
 *     graph capture) and return IBDL_ERR_NONFINITE on a hit.
 */
#ifndef IBDL_H
#define IBDL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibdl_s* ibdl_t;

typedef enum {
  IBDL_OK = 0,
  IBDL_NOT_CONVERGED = 1,      /* warning: maxit reached; outputs hold the best iterate      */
  IBDL_ERR_ARG = -1,           /* invalid argument (null pointer, size, enum value)          */
  IBDL_ERR_UNSUPPORTED = -2,   /* valid but not implemented (e.g. 3-D Stokes, N not 2^k)     */
  IBDL_ERR_NOMEM = -3,         /* device allocation failed                                   */
  IBDL_ERR_HIP = -4,           /* a HIP runtime call failed                                  */
  IBDL_ERR_NONFINITE = -5,     /* non-finite value: a residual, or device data under IBDL_CHECK=1 */
  IBDL_ERR_STATE = -6          /* call not valid in the handle's state                       */
} ibdl_status_t;

enum { IBDL_PDE_SCREENED = 0, IBDL_PDE_POISSON = 1, IBDL_PDE_STOKES = 2 };
enum { IBDL_BC_DIRICHLET = 0, IBDL_BC_NEUMANN = 1 };
enum { IBDL_K_PESKIN4 = 0, IBDL_K_COS4 = 1, IBDL_K_BSPLINE6 = 2 };
enum { IBDL_DISC_FD2 = 0, IBDL_DISC_SPECTRAL = 1 };
enum { IBDL_FP64 = 0, IBDL_MIXED = 1 };
enum { IBDL_METHOD_DL = 0, IBDL_METHOD_SL = 1 };

typedef struct {
  int32_t dim;        /* 2 or 3                                                             */
  int64_t n[3];       /* grid points per axis (x, y, z): powers of two in [16, 1024]; in 2-D
                         up to 8192 (the handle entry points; batches and the allocation-free
                         grid solve keep 1024)                                               */
  double  L[3];       /* box lengths; h = L[d]/n[d] must be equal on every axis (Sec. 2.2.1) */
  double  origin[3];  /* nodes at origin + j*h                                              */
  int32_t pde;        /* IBDL_PDE_SCREENED (L = Delta - kappa^2, kappa > 0),
                         IBDL_PDE_POISSON (L = Delta, mean-zero inverse),
                         IBDL_PDE_STOKES (L = mu Delta - kappa^2; kappa = 0 is Stokes; 2-D only) */
  double  kappa;      /* screening constant, or the Brinkman k for Stokes                   */
  double  mu;         /* viscosity (Stokes); ignored for scalar problems                    */
  int32_t bc;         /* IBDL_BC_DIRICHLET or IBDL_BC_NEUMANN (scalar, eta = 0 only)        */
  double  eta;        /* 0 = plain IBDL; > 0 = completed IBDL (Sec. 5.3.3, 6.1.3)           */
  int32_t kernel;     /* IBDL_K_PESKIN4 (Sec. 2.2.2), IBDL_K_COS4, IBDL_K_BSPLINE6 (Sec. 6.3.1;
                         spectral discretisation only)                                      */
  int32_t disc;       /* IBDL_DISC_FD2 (5/7-point Laplacian, centred differences) or
                         IBDL_DISC_SPECTRAL (Fourier; derivative symbol 0 at Nyquist)       */
  int32_t precision;  /* IBDL_FP64, or IBDL_MIXED: float grid, spread, FFT and interpolation;
                         double marker data and Krylov iteration                            */
  void*   stream;     /* hipStream_t                                                        */
  int32_t method;     /* IBDL_METHOD_DL (0): the double layer method, everything above.
                         IBDL_METHOD_SL: the single layer method of Chapter 2 (IBSL): the Schur
                         complement -S* L^-1 S (Sec. 2.2.3), with u_bar and the border rows
                         sum_i (ds_i / mean ds) F_i = (h^D / mean ds) sum_x g~ when L is singular
                         (Poisson, Sec. 2.2.4; Stokes, Sec. 2.3.2), and L^-1 P for Brinkman and
                         Stokes (Sec. 2.3.1); 2-D, Dirichlet data, eta = 0; the normals are not used
                         (nrm may be NULL).  ibdl_solve then runs MINRES.  With equal spacings the
                         border rows are the thesis's 1^T F.  Not available: the transposed
                         operator, the adjoint, refinement, batches, the indicator function. */
} ibdl_config_t;

typedef struct {
  int32_t iters;              /* Arnoldi steps taken                                          */
  int32_t status;             /* IBDL_OK or IBDL_NOT_CONVERGED                                */
  double  krylov_relres;      /* GMRES residual estimate ||b - A q|| / ||b|| at exit          */
  double  true_relres_fp64;   /* ||b - A q|| / ||b|| recomputed with a double-precision apply */
  double* history;            /* optional HOST array: relative residual per iteration, or NULL */
  int32_t history_cap;        /* capacity of history                                          */
} ibdl_info_t;

/* Create a handle for one problem (grid, PDE, markers).  X, nrm, ds: device double arrays as
 * above; they are copied, so the caller may free them afterwards.  Builds the per-marker stencil
 * data and the tile bins used by the spread.  Returns IBDL_ERR_UNSUPPORTED for combinations not
 * implemented (3-D Stokes, Neumann with Stokes or eta > 0, B-spline with FD2). */
ibdl_status_t ibdl_create(const ibdl_config_t* cfg, int64_t n_ib, const double* X,
                          const double* nrm, const double* ds, ibdl_t* out);

/* Replace the markers (same n_ib) and rebuild stencils and bins. */
ibdl_status_t ibdl_set_markers(ibdl_t h, const double* X, const double* nrm, const double* ds);

/* Release the handle and its workspaces (synchronises its stream first). */
ibdl_status_t ibdl_destroy(ibdl_t h);

/* Spread S (Sec. 2.2.2): grid[c][x] = sum_i f[i][c] delta_h(x - X_i) ds_i, c < nc <= 5.
 * f: device double [n_ib][nc]; grid: device [nc][grid] of the handle's grid type. */
ibdl_status_t ibdl_spread(ibdl_t h, const double* f, int32_t nc, void* grid);

/* Interpolation S* (Sec. 2.2.2): f[i][c] = sum_x grid[c][x] delta_h(x - X_i) h^dim, c < nc <= 5. */
ibdl_status_t ibdl_interp(ibdl_t h, const void* grid, int32_t nc, double* f);

/* Periodic grid solve: scalar u = L^-1 rhs (mean-zero branch when L has a null space);
 * Stokes u = L^-1 P rhs with rhs, u of dim components.  rhs and u may alias. */
ibdl_status_t ibdl_grid_solve(ibdl_t h, const void* rhs, void* u);

/* ibdl_grid_solve without a handle and without allocating: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same operator and layouts as ibdl_grid_solve for the grid, PDE, discretisation and precision
 * that cfg describes (dim, n, L, pde, kappa, mu, disc, precision, stream; markers, bc, eta and
 * kernel are ignored): scalar u = L^-1 rhs (mean-zero branch for Poisson), Stokes u = L^-1 P rhs.
 * rhs and u are device arrays owned by the caller ([nq][grid] of the grid type) and may alias.
 * The half spectra and the FFT tables live in a fixed static device array of 32 MiB per GPU, held
 * until the process ends: grids that need more (for example 3-D 256^3) return
 * IBDL_ERR_UNSUPPORTED before any device work.  Calls no hipMalloc, hipFree or other allocating
 * routine.  Asynchronous on cfg->stream, on the current device.  Every call on one GPU shares that
 * array and leaves its contents behind: calls that overlap on one GPU (two streams, two host
 * threads) race.  ibdl_last_error(NULL) describes a failure. */
ibdl_status_t ibdl_grid_solve_static(const ibdl_config_t* cfg, const void* rhs, void* u);

/* y = A q for the handle's operator; q, y: device double [n_aug] (must not alias). */
ibdl_status_t ibdl_apply(ibdl_t h, const double* q, double* y);

/* Solve A q = b with GMRES (x0 = 0, no restart, double-precision Arnoldi with classical
 * Gram-Schmidt applied twice, Givens rotations) to ||b - A q|| / ||b|| <= tol, maxit <= 200.
 *   data: Dirichlet U_b or Neumann V_b, device double [n_ib][nq];
 *   g_grid: extended forcing g~ on the grid ([nq][grid], grid type) or NULL for zero;
 *   q: output density (device double [n_aug]); u_grid: output grid solution ([nq][grid], grid
 *   type, Sec. 5.3.2 and 5.3.3 grid recovery) or NULL; info: optional host struct.
 * The right-hand side is b = U_b - S* L^-1 g~ (Dirichlet; Stokes with P), b = S* L^-1 (S V_b - g~)
 * (Neumann), plus h^dim sum(g~) in the border rows.  Returns IBDL_NOT_CONVERGED if maxit is
 * reached (outputs hold the last iterate).
 * Single layer handles (IBDL_METHOD_SL) run MINRES instead (Sec. 2.2.3; x0 = 0, the Lanczos
 * three-term recurrence without reorthogonalisation, Givens rotations, all on the device), in the
 * inner product with weights ds_i / mean(ds) per marker entry and 1 per u_bar entry, to the
 * recurrence residual |r| <= tol |b| in that norm; maxit <= 1000000; info->iters counts MINRES
 * iterations, info->krylov_relres is the recurrence residual and the history its values; the
 * grid solution is u = L^-1 (g~ - S F) (P in front for Stokes) + u_bar. */
ibdl_status_t ibdl_solve(ibdl_t h, const double* data, const void* g_grid, double tol,
                         int32_t maxit, double* q, void* u_grid, ibdl_info_t* info);

/* Solve A q = b to a double-precision true residual ||b - A q|| / ||b|| <= tol by iterative
 * refinement: b and every residual are formed with double-precision applies, and each round adds
 * the GMRES solution (working precision: float grid work on a mixed handle) of A d = r to
 * inner_tol (0 < inner_tol < 1).  At most max_rounds rounds of at most maxit iterations.
 * Arguments as in ibdl_solve; info->iters is the total of inner iterations, info->krylov_relres
 * the last round's Krylov residual, info->true_relres_fp64 the final true residual.
 * IBDL_NOT_CONVERGED if tol is not met within max_rounds. */
ibdl_status_t ibdl_solve_refined(ibdl_t h, const double* data, const void* g_grid, double tol, int32_t maxit,
                                 double inner_tol, int32_t max_rounds, double* q, void* u_grid, ibdl_info_t* info);

/* y = A^T p, the transpose of the operator of ibdl_apply (same layout and precision rules).
 * With Phi the interpolation matrix (S* = Phi, Sec. 2.2.2), S = h^-D Phi^T diag(ds) and the grid
 * operators' transposes (L^-1 symmetric, D_d^T = -D_d with the Nyquist reading of the spectral
 * derivative), A^T p = J p/2 + K^T Phi^T p (+ eta ds p_ubar; u_bar rows: sum_i p_i), where K is the
 * density-to-grid map of the operator.  With finite-difference symbols the scalar K^T is applied
 * as the exact transpose of the forward map's fused divergence spread (one grid field).
 * p, y: device double [n_aug], must not alias. */
ibdl_status_t ibdl_apply_transpose(ibdl_t h, const double* p, double* y);

/* Gradients of a loss L(u) of the grid solution of ibdl_solve with respect to the marker positions
 * and the boundary data, normals and weights held fixed (the thesis's forward map, Sec. 5.3.2,
 * 5.3.3, 6.3.3, differentiated by the adjoint method):
 *   solve A^T mu = (du/dq)^T psi with GMRES (tol, maxit as in ibdl_solve), dL/ddata = mu,
 *   dL/dX_ie = -sum_c mu_ic (Phi'_e u_c)_i + (kernel-derivative gathers of the adjoint fields),
 * where Phi'_e holds the derivatives of the interpolation weights, -phi'(r_e)/h prod_{d!=e} phi(r_d).
 *   q: the forward solution (device double [n_aug]); u_grid: the forward grid solution
 *   ([nq][grid], grid type) for the handle's current markers; dL_du: psi, the gradient of L with
 *   respect to the grid values ([nq][grid], grid type); dL_dX: output device double [n_ib][dim]
 *   or NULL; dL_ddata: output device double [n_ib][nq] or NULL; info: the adjoint GMRES.
 * Dirichlet problems (scalar, completed, Brinkman/Stokes); IBDL_ERR_UNSUPPORTED for Neumann.
 * Synchronises like ibdl_solve. */
ibdl_status_t ibdl_backward(ibdl_t h, const double* q, const void* u_grid, const void* dL_du, double tol,
                            int32_t maxit, double* dL_dX, double* dL_ddata, ibdl_info_t* info);

/* ---------------------------------------------------------------- batches of problems
 * Many independent plain scalar Dirichlet problems (Sec. 5.3.2: screened Poisson or Poisson,
 * eta = 0, finite-difference symbols, a 4-point kernel), of any grid sizes and marker counts,
 * solved together.  Problems with the same grid (sizes, box, origin, kappa) form a group.  In 2-D
 * the spread of every group is one persistent launch over a single work queue of busy tiles and
 * the interpolation of every group one launch; the FFT passes run once per group.  The batched
 * operator is replayed from a HIP graph every GMRES iteration, and each iteration's Arnoldi step,
 * Givens rotations and convergence test run on the device for every problem in one launch, so the
 * host only watches the published residuals.  The FFT passes' launch shapes and the 2-D spread's
 * tile shape are chosen by timing per (dim, grid, precision, problem count, markers per problem)
 * and kept in a JSON file ($IBDL_TUNE_CACHE, else ~/.cache/ibdl/tune.json; an empty
 * IBDL_TUNE_CACHE keeps them in memory only).  All problems share dim, precision and kernel. */
typedef struct ibdl_batch_s* ibdl_batch_t;

/* cfgs[p], n_ib[p]: host arrays of nprob configurations and marker counts; X[p], nrm[p], ds[p]:
 * host arrays of device pointers to each problem's markers (layouts as in ibdl_create; copied).
 * The batch works on its own stream, ordered after cfgs[0].stream at every call. */
ibdl_status_t ibdl_batch_create(int32_t nprob, const ibdl_config_t* cfgs, const int64_t* n_ib,
                                const double* const* X, const double* const* nrm, const double* const* ds,
                                ibdl_batch_t* out);
ibdl_status_t ibdl_batch_destroy(ibdl_batch_t b);

/* y[p] = A_p q[p] for every problem (host arrays of device pointers to double [n_ib[p]]). */
ibdl_status_t ibdl_batch_apply(ibdl_batch_t b, const double* const* q, double* const* y);

/* Solve every problem with boundary data data[p] (device double [n_ib[p]]) and g~ = 0 to
 * ||b - A q|| / ||b|| <= tol (GMRES as in ibdl_solve, per problem), q[p] the densities, u[p] the
 * grid solutions ([grid] of the grid type, or NULL entries / u = NULL to skip), infos[p] per
 * problem (or NULL).  Returns IBDL_NOT_CONVERGED if any problem did not converge.  Synchronises. */
ibdl_status_t ibdl_batch_solve(ibdl_batch_t b, const double* const* data, double tol, int32_t maxit,
                               double* const* q, void* const* u, ibdl_info_t* infos);

/* Replay the batched apply from a captured HIP graph (1, the default) or launch it directly (0). */
ibdl_status_t ibdl_batch_set_graph(ibdl_batch_t b, int32_t enable);

/* Number of grid groups; for group >= 0 also its problem count, grid sizes n[3], the launch shapes
 * chosen for its FFT passes (rows per block of the x passes, lines per block of the fused pass) and
 * the tile width along x of its 2-D spread (16, 32 or 64 nodes, tiles of 256 nodes; 16 in 3-D).
 * Any output pointer may be NULL. */
ibdl_status_t ibdl_batch_query(ibdl_batch_t b, int32_t group, int32_t* ngroups, int32_t* nprob_in_group,
                               int32_t* n, int32_t* rows_per_block, int32_t* lines_per_block, int32_t* tile_x);

/* Message of the last failure on the batch (or of the last failed ibdl_batch_create for NULL). */
const char* ibdl_batch_last_error(ibdl_batch_t b);

/* Indicator function of the interior of the markers' closed curve(s), two-dimensional handles
 * only (Sec. 5.3.4, flagging interior and exterior points).  chi is the mean-zero solution of
 * Delta chi + S~ 1 = 0 (S~: the dipole spread of the unit density with the handle's kernel,
 * normals and discretisation; the normals point out of the interior), shifted so that the node at
 * the origin corner is 0; the curve then carries about 1/2, and chi = 1 where the shifted field is
 * at least 1/2, else 0.  chi and regularized (the shifted field before the threshold; may be NULL)
 * are [ny][nx] of the grid type, device, owned by the caller.  Asynchronous on the handle's
 * stream. */
ibdl_status_t ibdl_indicator(ibdl_t h, void* chi, void* regularized);

/* Near-boundary interpolation, two-dimensional handles (Sec. 5.3.3, interpolation for
 * near-boundary points); Stokes handles interpolate each velocity component the same way.
 * out = u, except at the nodes p with omega != 0 whose nearest marker is
 * within m1 h: there x_A = the point closest to p on the segment between the two nearest markers
 * (if the projection leaves it, the two of the three nearest markers farthest apart, projection
 * clamped), u(x_A) = the linear interpolation of Ub (device double [n_ib][nq]) between them,
 * x_B = x_A + m2 h (p - x_A) / |p - x_A|, u(x_B) = the bilinear interpolation of u, and
 * out(p) = the linear interpolation between u(x_A) and u(x_B) at p.  Distances are plain
 * Euclidean (the curve keeps clear of the box faces); ties between markers go to the lower index.
 * omega (the nodes of the PDE domain, e.g. ibdl_indicator's chi or 1 - chi): [ny][nx]; u, out:
 * [nq][ny][nx]; both of the grid type, device; out must not alias u.  Needs 1 <= m1 < m2 <= 64 (ibdl_near_widths gives
 * the thesis's values) and at least two markers.  Asynchronous on the handle's stream. */
ibdl_status_t ibdl_near_boundary(ibdl_t h, const double* Ub, const void* omega, const void* u, double m1, double m2,
                                 void* out);

/* The interpolation widths of Sec. 5.5 (interpolation widths) for the handle's discretisation:
 * with finite-difference symbols m1 = 6, m2 = 8; with Fourier spectral symbols
 * m1 = 2 (log2 nx - 4), at least 2, and m2 = m1 + 2.  Host only, synchronous; two-dimensional
 * handles; either pointer may be NULL. */
ibdl_status_t ibdl_near_widths(ibdl_t h, double* m1, double* m2);

/* The nonlinear term (u . grad) u of a two-dimensional velocity field (Sec. 6.5, Navier-Stokes:
 * numerical implementation), 2-D Stokes handles: out[c] = u_0 d_x u_c + u_1 d_y u_c with the
 * handle's derivative symbols (Fourier: i k, 0 at the Nyquist index; finite differences:
 * centred).  u, out: device [2][ny][nx] of the grid type, owned by the caller, not aliased.
 * Asynchronous on the handle's stream. */
ibdl_status_t ibdl_advection(ibdl_t h, const void* u, void* out);

typedef struct {
  double  rho;        /* density                                                            */
  double  dt;         /* time step; the handle's kappa^2 must equal 3 rho / (2 dt)           */
  double  m1, m2;     /* near-boundary interpolation widths (m1 = 0: no interpolation)        */
  int32_t strip;      /* width in grid columns of the inflow strip along x = origin (0: none) */
  double  u_inf;      /* strip velocity (u_inf, 0)                                           */
  double  tol;        /* GMRES tolerance of the Brinkman solve                               */
  int32_t maxit;      /* GMRES iteration limit (<= 200)                                      */
} ibdl_ns_params_t;

/* One step of the Navier-Stokes IMEX scheme with the completed IBDL method (Sec. 6.5): BDF2 in
 * time for the viscous and boundary terms, the nonlinear term extrapolated from the two previous
 * steps.  u^{n+1} solves the Brinkman problem of the handle (2-D Stokes, mu, kappa^2 =
 * 3 rho / (2 dt), eta) with the forcing g~ = rho ((-4 u^n + u^{n-1}) / (2 dt) + 2 N^n - N^{n-1}),
 * N = (u . grad) u, and the boundary data Ub = U_b^{n+1} (device double [n_ib][2]); it is then
 * recovered on the grid, near-boundary interpolated on the nodes of omega (device [ny][nx] of the
 * grid type; may be NULL when m1 = 0), reset to (u_inf, 0) on the inflow strip, and its nonlinear
 * term is formed from the interpolated field.  State (device [2][ny][nx] of the grid type, owned
 * by the caller, four distinct buffers): on entry u = u^n, u_prev = u^{n-1}, n = N(u^n),
 * n_prev = N(u^{n-1}); on return u = u^{n+1}, u_prev = u^n, n = N(u^{n+1}), n_prev = N(u^n).
 * q: device double [n_aug], the density of the step; g_out (optional, [2][ny][nx] of the grid
 * type): the step's forcing g~, which ibdl_pressure needs.  info (optional host struct): the GMRES
 * iterations and residual of the step; true_relres_fp64 is -1 (not computed).  Synchronises the
 * handle's stream once per GMRES iteration, like ibdl_solve. */
ibdl_status_t ibdl_ns_step(ibdl_t h, const ibdl_ns_params_t* p, const double* Ub, const void* omega, void* u_prev,
                           void* u, void* n_prev, void* n, double* q, void* g_out, ibdl_info_t* info);

/* Pressure of a two-dimensional Brinkman / Stokes solution (Sec. 6.5, with the system of Sec. 6.1
 * and 6.3): taking the divergence of (mu Delta - k^2) u - grad p + eta S Q + mu div(S A) = g~ with
 * div u = -S(Q.n) gives p = Delta_0^-1 [div(eta S Q + mu div(S A) - g~) - (mu Delta - k^2) S(Q.n)],
 * the mean-zero solution.  q: device double [n_aug] (ibdl_solve's); g_grid: the forcing
 * ([2][ny][nx], grid type) or NULL; p: device [ny][nx] of the grid type, owned by the caller.
 * Asynchronous on the handle's stream. */
ibdl_status_t ibdl_pressure(ibdl_t h, const double* q, const void* g_grid, void* p);

/* Force on a body by a control volume (Sec. 6.5): over the grid box R of node indices
 * box = {i0, i1, j0, j1} (x from i0 to i1, y from j0 to j1, inclusive; 0 <= i0 < i1 < nx,
 * 0 <= j0 < j1 < ny) around the body,
 *   B = -rho int_{R'} u_t dx + oint_{dR} (sigma - rho u u^T) . n_R dl,  sigma = -p I + mu (grad u + grad u^T),
 * R' = the nodes of R with omega != 0 (the fluid), u_t = (u - u_prev) / dt (the volume term is
 * left out when u_prev is NULL: steady flow), the velocity gradients by the handle's derivative
 * symbols, both integrals by the trapezoidal rule on the nodes.  u, u_prev: [2][ny][nx], p, omega:
 * [ny][nx], device, grid type.  out: device double [2].  2-D Stokes handles (mu from the handle).
 * Asynchronous on the handle's stream. */
ibdl_status_t ibdl_cv_force(ibdl_t h, const void* u, const void* u_prev, double dt, const void* p, const void* omega,
                            double rho, const int32_t* box, double* out);

/* Net force and torque of a two-dimensional Stokes solution with the completed method (Sec. 6.1,
 * exterior domains; Sec. 6.5, Stokes flow around a periodic array of cylinders).  The single layer
 * of strength eta Q carries the whole net force, B = -eta sum_i ds_i Q_i, and the torque about the
 * coordinate origin, L = -eta sum_i ds_i (X_i,x Q_i,y - X_i,y Q_i,x), with X as the handle was given
 * it.  q: device double [n_aug], the unknowns of ibdl_solve (Q as [n_ib][2] first).  out: device
 * double [3] = (B_x, B_y, L), owned by the caller.  Summed in a fixed order (the same bits every
 * call).  Without the completion (eta = 0) all three are 0.  Asynchronous on the handle's
 * stream; IBDL_ERR_UNSUPPORTED for scalar or three-dimensional handles. */
ibdl_status_t ibdl_net_force(ibdl_t h, const double* q, double* out);

/* Line integral of one component of a two-dimensional grid field over a grid line: h times the sum
 * of the line's nodes (the rectangle rule, exact for the trigonometric polynomials the periodic
 * grid resolves).  axis 0 takes the line on which x has node index `index` (summed over y), axis 1
 * the line on which y has node index `index`.  Sec. 6.5 takes the x velocity over the box face
 * x = origin_x (comp 0, axis 0, index 0) as the flux U of its drag D = B_x / (mu U).  u: device,
 * grid type, [nq][ny][nx] as ibdl_solve writes it; 0 <= comp < nq; 0 <= index < n[axis].  out:
 * device double [1], owned by the caller; the sum is in double in a fixed order.  Asynchronous on
 * the handle's stream. */
ibdl_status_t ibdl_line_integral(ibdl_t h, const void* u, int32_t comp, int32_t axis, int64_t index, double* out);

/* Sizes of the handle: n_aug (unknowns), grid points per component, grid components of the
 * solution (nq).  Any output pointer may be NULL. */
ibdl_status_t ibdl_query(ibdl_t h, int64_t* n_aug, int64_t* grid_points, int32_t* nq);

/* Rows (x-lines) that the markers' 6-node windows meet, nact, out of rows_total = grid points / nx.
 * The operator apply runs its x passes over those rows only: the spread field is zero on the
 * others and the interpolation does not read them.  Either pointer may be NULL. */
ibdl_status_t ibdl_active_rows(ibdl_t h, int64_t* nact, int64_t* rows_total);

/* Range [first, last] of indices along the last grid axis (z in 3-D, y in 2-D) that hold an active
 * row.  The operator apply's last-axis pass loads and stores only those elements of its lines, and
 * in 3-D its y passes run over those z planes only; the rest of the spectra is zero on the way in
 * and not needed on the way out.  2-D grids over 1024 points along y report the whole axis (their
 * four-step last-axis pass does not mask).  last < first when no row is active.  Either pointer
 * may be NULL. */
ibdl_status_t ibdl_active_span(ibdl_t h, int32_t* first, int32_t* last);

/* Tiling of the spread: nbusy = tiles (tile[0] x tile[1] (x tile[2]) nodes) that a marker window
 * meets, which the spread writes whole; segments_read = (active row, busy tile) pairs, i.e. the
 * tile[0]-node row segments the operator apply's forward x pass reads per spread field (it takes
 * every other value of an active row as zero).  Any pointer may be NULL. */
ibdl_status_t ibdl_spread_tiles(ibdl_t h, int64_t* nbusy, int64_t* segments_read, int32_t* tile);

/* Launch shapes of the operator apply's FFT passes in the working precision, chosen by timing at
 * the first apply (rows per block of the x passes, lines per block of the y passes and of the fused
 * last-axis pass; 0 = not measured yet, the largest shape is used).  Any pointer may be NULL. */
ibdl_status_t ibdl_launch_shape(ibdl_t h, int32_t* rows_per_block, int32_t* lines_y, int32_t* lines_last);

/* GMRES and MINRES in ibdl_solve, ibdl_solve_refined, ibdl_backward and ibdl_ns_step replay each
 * operator apply from a HIP graph captured at the first apply (1) or launch its kernels directly
 * (0).  The default is 1 below 2^20 grid points, where an apply is shorter than its launches, and
 * 0 from there on.  Both give the same bits.  Disabling drops the captured graphs. */
ibdl_status_t ibdl_set_graph(ibdl_t h, int32_t enable);

/* Profiling: enable (1) or disable (0) per-stage timing with HIP events recorded on the handle's
 * stream around every kernel stage (resets the accumulated times).  Costs a few microseconds per
 * stage; leave it off outside profiling. */
ibdl_status_t ibdl_set_timing(ibdl_t h, int32_t enable);

/* Accumulated milliseconds and launch counts per stage since ibdl_set_timing(h, 1), stage ids:
 * 0 spread, 1 x-axis forward FFT, 2 y-axis forward FFT (3-D), 3 fused last-axis FFT + multiplier,
 * 4 y-axis inverse FFT (3-D), 5 x-axis inverse FFT, 6 interpolation, 7 Krylov vectors (not
 * instrumented), 8 zero fill (none in the current operator apply: always 0).
 * ms and count are host arrays of cap entries (cap >= 9 returns every stage).  Synchronises on the
 * recorded events. */
ibdl_status_t ibdl_get_timing(ibdl_t h, double* ms, int64_t* count, int32_t cap);

/* Message of the last failure on this handle (or, when h is NULL, of the last failed ibdl_create or
 * ibdl_grid_solve_static).
 * The string stays valid until the next call on the handle. */
const char* ibdl_last_error(ibdl_t h);

#ifdef __cplusplus
}
#endif

#endif /* IBDL_H */
