// Navier-Stokes IMEX pieces (Sec. 6.5): elementwise grid kernels of one time step.
#pragma once

#include "common.h"

namespace ibdl {

// g = rho ((-4 un + unm1) / (2 dt) + 2 Nn - Nnm1) over n values (all velocity components)
template <typename T>
void ns_forcing(const T* un, const T* unm1, const T* Nn, const T* Nnm1, double rho, double dt, int64_t n, T* g,
                hipStream_t st);
// out[c] = u[0] G[2c] + u[1] G[2c + 1] (c = 0, 1): the nonlinear term (u . grad) u from the
// gradients G = (d_x u_0, d_y u_0, d_x u_1, d_y u_1), fields of n values
template <typename T>
void ns_advect_combine(const T* u, const T* G, int64_t n, T* out, hipStream_t st);
// u[0] = u_inf, u[1] = 0 on the grid columns x index < width of a [2][ny][nx] field
template <typename T>
void ns_strip(T* u, int nx, int ny, int width, double u_inf, hipStream_t st);

// Control-volume force over the grid box box = (i0, i1, j0, j1) (inclusive node indices):
// out[2] = oint (sigma - rho u u^T) . n dl - rho int omega u_t dx, sigma = -p I + mu (grad u +
// grad u^T), G[2c + d] = d_d u_c, u_t = (u - uprev) / dt (no volume term when uprev is NULL);
// trapezoidal weights on the nodes.
template <typename T>
void cv_force(const T* u, const T* uprev, double dt, const T* p, const T* omega, const T* G, int nx, int ny,
              const int* box, double h, double rho, double mu, double* out, hipStream_t st);

}  // namespace ibdl
