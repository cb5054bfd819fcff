// Double-precision Krylov vector kernels (GMRES Arnoldi with classical Gram-Schmidt twice).
// Reductions are two-level with a fixed order (per-block partial sums, then one pass over the
// partials), so every dot product is deterministic.
#include "kernels.h"

namespace ibdl {
namespace {

constexpr int kB = 256;
constexpr int kElemsPerBlock = 2048;

// partial[j * nblk + b] = sum over block b's chunk of V_j . w, for j < k
__global__ __launch_bounds__(kB) void k_multidot(const double* __restrict__ V, int64_t ldv, int k,
                                                 const double* __restrict__ w, int64_t n, int nblk,
                                                 double* __restrict__ partial) {
  __shared__ double red[kB];
  const int64_t beg = (int64_t)blockIdx.x * kElemsPerBlock;
  const int64_t end = beg + kElemsPerBlock < n ? beg + kElemsPerBlock : n;
  for (int j = 0; j < k; ++j) {
    const double* vj = V + j * ldv;
    double s = 0.0;
    for (int64_t e = beg + threadIdx.x; e < end; e += kB) s += vj[e] * w[e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = kB / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[j * nblk + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ void k_reduce(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
  const int j = blockIdx.x;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[j * nblk + b];
    out[j] = s;
  }
}

__global__ void k_gemv_sub(const double* __restrict__ V, int64_t ldv, int k, const double* __restrict__ h,
                           double* __restrict__ w, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double s = w[e];
    for (int j = 0; j < k; ++j) s -= V[j * ldv + e] * h[j];
    w[e] = s;
  }
}

__global__ void k_lincomb(const double* __restrict__ V, int64_t ldv, int k, const double* __restrict__ y,
                          double* __restrict__ x, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += V[j * ldv + e] * y[j];
    x[e] = s;
  }
}

__global__ void k_scale(const double* __restrict__ src, double s, double* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e] * s;
}

__global__ void k_axpby_d(double* __restrict__ y, double a, const double* __restrict__ x, double b, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = a * x[e] + b * y[e];
}

__global__ void k_add_small(double* __restrict__ dst, const double* __restrict__ a, const double* __restrict__ b, int n) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = a[e] + b[e];
}

// partial sums of eta * ds_i * q[i][c] over markers, per component c
__global__ __launch_bounds__(kB) void k_border_partial(const double* __restrict__ q, const double* __restrict__ ds,
                                                       int64_t n_ib, int nq, int nblk, double* __restrict__ partial) {
  __shared__ double red[kB];
  const int c = blockIdx.y;
  const int64_t beg = (int64_t)blockIdx.x * kElemsPerBlock;
  const int64_t end = beg + kElemsPerBlock < n_ib ? beg + kElemsPerBlock : n_ib;
  double s = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kB) s += ds[i] * q[i * nq + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kB / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[c * nblk + blockIdx.x] = red[0];
}

__global__ void k_border_final(const double* __restrict__ partial, int nblk, double eta, double* __restrict__ out) {
  const int c = blockIdx.x;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[c * nblk + b];
    out[c] = eta * s;
  }
}

inline unsigned blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

}  // namespace

int kr_nblk(int64_t n) { return (int)((n + kElemsPerBlock - 1) / kElemsPerBlock) > 0 ? (int)((n + kElemsPerBlock - 1) / kElemsPerBlock) : 1; }

void kr_multidot(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* partial, int nblk,
                 double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_multidot, dim3(nblk), dim3(kB), 0, st, V, ldv, k, w, n, nblk, partial);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce, dim3(k), dim3(64), 0, st, partial, nblk, out);
  IBDL_LAUNCH_CHECK();
}

void kr_gemv_sub(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_sub, dim3(blocks_for(n)), dim3(256), 0, st, V, ldv, k, h, w, n);
  IBDL_LAUNCH_CHECK();
}

void kr_lincomb(const double* V, int64_t ldv, int k, const double* y, double* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb, dim3(blocks_for(n)), dim3(256), 0, st, V, ldv, k, y, x, n);
  IBDL_LAUNCH_CHECK();
}

void kr_scale(const double* src, double s, double* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(256), 0, st, src, s, dst, n);
  IBDL_LAUNCH_CHECK();
}

void kr_axpby(double* y, double a, const double* x, double b, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby_d, dim3(blocks_for(n)), dim3(256), 0, st, y, a, x, b, n);
  IBDL_LAUNCH_CHECK();
}

void kr_add(double* dst, const double* a, const double* b, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_add_small, dim3(1), dim3(256), 0, st, dst, a, b, n);
  IBDL_LAUNCH_CHECK();
}

void kr_border(const double* q, const double* ds, int64_t n_ib, int nq, double eta, double* out, double* partial,
               int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_border_partial, dim3(nblk, nq), dim3(kB), 0, st, q, ds, n_ib, nq, nblk, partial);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_border_final, dim3(nq), dim3(64), 0, st, partial, nblk, eta, out);
  IBDL_LAUNCH_CHECK();
}

}  // namespace ibdl
