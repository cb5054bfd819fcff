// Net force and torque of the completed Stokes density, and line integrals of a grid field
// (2-D): the quantities Sec. 6.5 (Stokes flow around a periodic array of cylinders) forms the
// dimensionless drag from, with the force of the completed density from Sec. 6.1 (exterior
// domains).  Both are single-workgroup reductions in a fixed order, so results do not depend on
// scheduling.
#include "kernels.h"

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

}  // namespace

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
