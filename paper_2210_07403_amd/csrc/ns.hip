// Navier-Stokes IMEX pieces (Sec. 6.5, Navier-Stokes: numerical implementation): the forcing of
// the implicit Brinkman solve (the BDF2 history terms and the extrapolated nonlinear term), the
// nonlinear term from the spectral velocity gradients, and the inflow strip that drives the flow.
#include "ns.h"

namespace ibdl {
namespace {

constexpr int kNS = 256;

inline unsigned ns_blocks(int64_t n) {
  const int64_t b = (n + kNS - 1) / kNS;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

template <typename T>
__global__ __launch_bounds__(kNS) void k_ns_forcing(const T* __restrict__ un, const T* __restrict__ unm1,
                                                    const T* __restrict__ Nn, const T* __restrict__ Nnm1, double rho,
                                                    double dt, int64_t n, T* __restrict__ g) {
  const double a = rho / (2.0 * dt);
  for (int64_t e = (int64_t)blockIdx.x * kNS + threadIdx.x; e < n; e += (int64_t)gridDim.x * kNS) {
    const double hist = -4.0 * (double)un[e] + (double)unm1[e];
    const double adv = 2.0 * (double)Nn[e] - (double)Nnm1[e];
    g[e] = (T)(a * hist + rho * adv);
  }
}

template <typename T>
__global__ __launch_bounds__(kNS) void k_ns_advect(const T* __restrict__ u, const T* __restrict__ G, int64_t n,
                                                   T* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * kNS + threadIdx.x; e < n; e += (int64_t)gridDim.x * kNS) {
    const double u0 = u[e], u1 = u[n + e];
    out[e] = (T)(u0 * (double)G[e] + u1 * (double)G[n + e]);
    out[n + e] = (T)(u0 * (double)G[2 * n + e] + u1 * (double)G[3 * n + e]);
  }
}

template <typename T>
__global__ __launch_bounds__(kNS) void k_ns_strip(T* __restrict__ u, int nx, int ny, int width, double u_inf) {
  const int64_t m = (int64_t)ny * width;
  const int64_t n = (int64_t)nx * ny;
  for (int64_t k = (int64_t)blockIdx.x * kNS + threadIdx.x; k < m; k += (int64_t)gridDim.x * kNS) {
    const int64_t e = (k / width) * nx + (k % width);
    u[e] = (T)u_inf;
    u[n + e] = (T)0;
  }
}

}  // namespace

template <typename T>
void ns_forcing(const T* un, const T* unm1, const T* Nn, const T* Nnm1, double rho, double dt, int64_t n, T* g,
                hipStream_t st) {
  hipLaunchKernelGGL((k_ns_forcing<T>), dim3(ns_blocks(n)), dim3(kNS), 0, st, un, unm1, Nn, Nnm1, rho, dt, n, g);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void ns_advect_combine(const T* u, const T* G, int64_t n, T* out, hipStream_t st) {
  hipLaunchKernelGGL((k_ns_advect<T>), dim3(ns_blocks(n)), dim3(kNS), 0, st, u, G, n, out);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void ns_strip(T* u, int nx, int ny, int width, double u_inf, hipStream_t st) {
  if (width <= 0) return;
  hipLaunchKernelGGL((k_ns_strip<T>), dim3(ns_blocks((int64_t)ny * width)), dim3(kNS), 0, st, u, nx, ny, width,
                     u_inf);
  IBDL_LAUNCH_CHECK();
}

#define IBDL_NS_INST(T)                                                                                         \
  template void ns_forcing<T>(const T*, const T*, const T*, const T*, double, double, int64_t, T*, hipStream_t); \
  template void ns_advect_combine<T>(const T*, const T*, int64_t, T*, hipStream_t);                           \
  template void ns_strip<T>(T*, int, int, int, double, hipStream_t);
IBDL_NS_INST(float)
IBDL_NS_INST(double)

}  // namespace ibdl
