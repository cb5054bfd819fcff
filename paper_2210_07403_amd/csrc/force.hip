// Net force and torque of the completed Stokes density, and line integrals of a grid field
// (2-D): the quantities Sec. 6.5 (Stokes flow around a periodic array of cylinders) forms the
// dimensionless drag from, with the force of the completed density from Sec. 6.1 (exterior
// domains).  Both are single-workgroup reductions in a fixed order, so results do not depend on
// scheduling.
#include "kernels.h"
#include "ns.h"

namespace ibdl {
namespace {

constexpr int kRB = 256;

// tree sum of v[kRB] in LDS; the result is in v[0] for every thread after the final barrier
__device__ __forceinline__ void block_tree(double* v) {
  for (int s = kRB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) v[threadIdx.x] += v[threadIdx.x + s];
    __syncthreads();
  }
}

// out = (B_x, B_y, L): B = -eta sum_i ds_i Q_i, L = -eta sum_i ds_i (X_i,x Q_i,y - X_i,y Q_i,x)
__global__ __launch_bounds__(kRB) void k_net_force(const double* __restrict__ X, const double* __restrict__ Q,
                                                   const double* __restrict__ ds, int64_t n, double eta,
                                                   double* __restrict__ out) {
  __shared__ double sb0[kRB], sb1[kRB], sl[kRB];
  double b0 = 0.0, b1 = 0.0, l = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kRB) {
    const double w = ds[i], q0 = Q[2 * i], q1 = Q[2 * i + 1];
    b0 += w * q0;
    b1 += w * q1;
    l += w * (X[2 * i] * q1 - X[2 * i + 1] * q0);
  }
  sb0[threadIdx.x] = b0;
  sb1[threadIdx.x] = b1;
  sl[threadIdx.x] = l;
  __syncthreads();
  block_tree(sb0);
  block_tree(sb1);
  block_tree(sl);
  if (threadIdx.x == 0) {
    out[0] = -eta * sb0[0];
    out[1] = -eta * sb1[0];
    out[2] = -eta * sl[0];
  }
}

// out[0] = h * sum_k u[k * stride], k < n
template <typename T>
__global__ __launch_bounds__(kRB) void k_line_sum(const T* __restrict__ u, int64_t stride, int64_t n, double h,
                                                  double* __restrict__ out) {
  __shared__ double sv[kRB];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += kRB) s += (double)u[k * stride];
  sv[threadIdx.x] = s;
  __syncthreads();
  block_tree(sv);
  if (threadIdx.x == 0) out[0] = h * sv[0];
}

// Control-volume force over the grid box [i0, i1] x [j0, j1] (trapezoidal weights):
// out = oint (sigma - rho u u^T) . n dl - rho int omega u_t dx, sigma = -p I + mu (grad u + grad u^T),
// with the velocity gradients G[2c + d] = d_d u_c and u_t = (u - u_prev) / dt (no volume term
// without u_prev).
template <typename T>
__global__ __launch_bounds__(kRB) void k_cv_force(const T* __restrict__ u, const T* __restrict__ uprev, double dt,
                                                  const T* __restrict__ p, const T* __restrict__ om,
                                                  const T* __restrict__ G, int nx, int64_t n, int i0, int i1, int j0,
                                                  int j1, double h, double rho, double mu, double* __restrict__ out) {
  __shared__ double s0[kRB], s1[kRB];
  auto flux = [&](int c, int d, int64_t e) -> double {
    const double sig = mu * ((double)G[(2 * c + d) * n + e] + (double)G[(2 * d + c) * n + e]) - (c == d ? (double)p[e] : 0.0);
    return sig - rho * (double)u[c * n + e] * (double)u[d * n + e];
  };
  const int ny_ = j1 - j0 + 1, nx_ = i1 - i0 + 1;
  double b0 = 0.0, b1 = 0.0;
  for (int k = threadIdx.x; k < ny_; k += kRB) {   // right (n = +x) and left (n = -x) sides
    const double w = (k == 0 || k == ny_ - 1) ? 0.5 * h : h;
    const int64_t er = (int64_t)(j0 + k) * nx + i1, el = (int64_t)(j0 + k) * nx + i0;
    b0 += w * (flux(0, 0, er) - flux(0, 0, el));
    b1 += w * (flux(1, 0, er) - flux(1, 0, el));
  }
  for (int k = threadIdx.x; k < nx_; k += kRB) {   // top (n = +y) and bottom (n = -y) sides
    const double w = (k == 0 || k == nx_ - 1) ? 0.5 * h : h;
    const int64_t et = (int64_t)j1 * nx + i0 + k, eb = (int64_t)j0 * nx + i0 + k;
    b0 += w * (flux(0, 1, et) - flux(0, 1, eb));
    b1 += w * (flux(1, 1, et) - flux(1, 1, eb));
  }
  const int64_t area = (int64_t)nx_ * ny_;
  for (int64_t k = uprev ? threadIdx.x : area; k < area; k += kRB) {   // -rho int over the fluid part of u_t
    const int kj = (int)(k / nx_), ki = (int)(k % nx_);
    const double wy = (kj == 0 || kj == ny_ - 1) ? 0.5 * h : h;
    const double wx = (ki == 0 || ki == nx_ - 1) ? 0.5 * h : h;
    const int64_t e = (int64_t)(j0 + kj) * nx + i0 + ki;
    const double w = wy * wx * (double)om[e] * rho / dt;
    b0 -= w * ((double)u[e] - (double)uprev[e]);
    b1 -= w * ((double)u[n + e] - (double)uprev[n + e]);
  }
  s0[threadIdx.x] = b0;
  s1[threadIdx.x] = b1;
  __syncthreads();
  block_tree(s0);
  block_tree(s1);
  if (threadIdx.x == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
  }
}

}  // namespace

template <typename T>
void cv_force(const T* u, const T* uprev, double dt, const T* p, const T* omega, const T* G, int nx, int ny,
              const int* box, double h, double rho, double mu, double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_cv_force<T>), dim3(1), dim3(kRB), 0, st, u, uprev, dt, p, omega, G, nx, (int64_t)nx * ny, box[0],
                     box[1], box[2], box[3], h, rho, mu, out);
  IBDL_LAUNCH_CHECK();
}
template void cv_force<float>(const float*, const float*, double, const float*, const float*, const float*, int, int,
                              const int*, double, double, double, double*, hipStream_t);
template void cv_force<double>(const double*, const double*, double, const double*, const double*, const double*, int,
                               int, const int*, double, double, double, double*, hipStream_t);

void net_force(const double* X, const double* Q, const double* ds, int64_t n_ib, double eta, double* out,
               hipStream_t st) {
  hipLaunchKernelGGL(k_net_force, dim3(1), dim3(kRB), 0, st, X, Q, ds, n_ib, eta, out);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void line_sum(const T* u, int64_t stride, int64_t n, double h, double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_line_sum<T>), dim3(1), dim3(kRB), 0, st, u, stride, n, h, out);
  IBDL_LAUNCH_CHECK();
}

template void line_sum<float>(const float*, int64_t, int64_t, double, double*, hipStream_t);
template void line_sum<double>(const double*, int64_t, int64_t, double, double*, hipStream_t);

}  // namespace ibdl
