// MINRES (Paige and Saunders) on the device, for the symmetric Schur complements of the single
// layer method (Sec. 2.2.3: solved with MINRES to a relative residual of 1e-8).
//
// Per iteration, after the operator apply p = A v_k: (1) block partials of alpha_k = <v_k, p>;
// (2) every workgroup reduces them in the same fixed order, p -= alpha_k v_k + beta_k v_{k-1},
// block partials of <p, p>; (3) every workgroup reduces those to beta_{k+1}, applies the two
// previous Givens rotations to the new tridiagonal column, forms the new rotation, and updates
// w_k = (v_k - delta w_{k-1} - epsilon w_{k-2}) / gamma, x += c eta w_k, v_{k+1} = p / beta_{k+1}
// element by element.  The inner product carries weights wt (self-adjointness of the operator
// with unequal spacings).  The scalar recurrence state lives in device memory, double-buffered
// (each iteration reads one copy and writes the other), so the host never has to take part in an
// iteration; once the recurrence residual reaches tol |b| the state's done flag freezes x, and the
// later kernels of iterations the host had queued return at once.
#include <math.h>

#include "kernels.h"

namespace ibdl {
namespace {

constexpr int kMB = 256;
constexpr int kMElems = 2048;   // elements per workgroup (8 per thread)

__device__ __forceinline__ double block_sum(double v, double* lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int s = kMB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

// sum of p[0 .. nblk) in a fixed order (the same bits in every workgroup)
__device__ __forceinline__ double reduce_partials(const double* __restrict__ p, int nblk, double* lds) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kMB) s += p[b];
  return block_sum(s, lds);
}

// workgroup blk's part of <a, b>_wt
__device__ __forceinline__ double mr_wdot_part(const double* __restrict__ a, const double* __restrict__ b,
                                               const double* __restrict__ wt, int64_t n, int blk, double* lds) {
  const int64_t e0 = (int64_t)blk * kMElems;
  double s = 0.0;
  for (int k = threadIdx.x; k < kMElems; k += kMB) {
    const int64_t e = e0 + k;
    if (e < n) s += wt[e] * a[e] * b[e];
  }
  return block_sum(s, lds);
}

__global__ __launch_bounds__(kMB) void k_mr_wdot(const double* __restrict__ a, const double* __restrict__ b,
                                                 const double* __restrict__ wt, int64_t n,
                                                 const double* __restrict__ state, double* __restrict__ partial) {
  __shared__ double lds[kMB];
  if (state && state[MR_DONE] != 0.0) return;
  const double s = mr_wdot_part(a, b, wt, n, blockIdx.x, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kMB) void k_mr_start(const double* __restrict__ b, int64_t n,
                                                  const double* __restrict__ partial, int nblk, double tol,
                                                  double* __restrict__ v, double* __restrict__ vprev,
                                                  double* __restrict__ w1, double* __restrict__ w2,
                                                  double* __restrict__ x, double* __restrict__ state) {
  __shared__ double lds[kMB];
  const double beta1 = sqrt(fmax(reduce_partials(partial, nblk, lds), 0.0));
  const double inv = beta1 > 0.0 ? 1.0 / beta1 : 0.0;
  const int64_t e0 = (int64_t)blockIdx.x * kMElems;
  for (int k = threadIdx.x; k < kMElems; k += kMB) {
    const int64_t e = e0 + k;
    if (e < n) {
      v[e] = b[e] * inv;
      vprev[e] = 0.0;
      w1[e] = 0.0;
      w2[e] = 0.0;
      x[e] = 0.0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    state[MR_BETA] = 0.0;
    state[MR_C1] = 1.0;
    state[MR_S1] = 0.0;
    state[MR_C2] = 1.0;
    state[MR_S2] = 0.0;
    state[MR_ETA] = beta1;
    state[MR_BETA1] = beta1;
    state[MR_DONE] = beta1 > 0.0 ? 0.0 : 1.0;
    state[MR_ITERS] = 0.0;
    state[MR_ALPHA] = 0.0;
    state[MR_TOL] = tol;
  }
}

// p -= alpha v + beta vprev on workgroup blk's elements; returns their part of <p, p>_wt
__device__ __forceinline__ double mr_lanczos_part(const double* __restrict__ v, const double* __restrict__ vprev,
                                                  double* __restrict__ p, const double* __restrict__ wt, int64_t n,
                                                  double alpha, double beta, int blk, double* lds) {
  const int64_t e0 = (int64_t)blk * kMElems;
  double s = 0.0;
  for (int k = threadIdx.x; k < kMElems; k += kMB) {
    const int64_t e = e0 + k;
    if (e < n) {
      const double pe = p[e] - alpha * v[e] - beta * vprev[e];
      p[e] = pe;
      s += wt[e] * pe * pe;
    }
  }
  return block_sum(s, lds);
}

// alpha = <v, p>; p -= alpha v + beta vprev; partial2 = block partials of <p, p>
__global__ __launch_bounds__(kMB) void k_mr_lanczos(const double* __restrict__ v, const double* __restrict__ vprev,
                                                    double* __restrict__ p, const double* __restrict__ wt, int64_t n,
                                                    const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ partial2, const double* __restrict__ in,
                                                    double* __restrict__ out) {
  __shared__ double lds[kMB];
  if (in[MR_DONE] != 0.0) return;
  const double alpha = reduce_partials(partial, nblk, lds);
  const double s = mr_lanczos_part(v, vprev, p, wt, n, alpha, in[MR_BETA], blockIdx.x, lds);
  if (threadIdx.x == 0) partial2[blockIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) out[MR_ALPHA] = alpha;
}

// The two previous rotations on the new column (beta_k, alpha_k, beta_{k+1}), then a new one.
struct MrRot {
  double eps, delta, ginv, step, binv, c, s, eta_new;
  bool done;
};
__device__ __forceinline__ MrRot mr_rotation(const double* __restrict__ in, double beta_next, double alpha) {
  const double beta = in[MR_BETA], c1 = in[MR_C1], s1 = in[MR_S1], c2 = in[MR_C2], s2 = in[MR_S2];
  const double eta = in[MR_ETA], beta1 = in[MR_BETA1], tol = in[MR_TOL];
  MrRot r;
  r.eps = s2 * beta;
  const double d0 = c2 * beta;
  r.delta = c1 * d0 + s1 * alpha;
  const double g0 = -s1 * d0 + c1 * alpha;
  const double gamma = hypot(g0, beta_next);
  r.c = gamma > 0.0 ? g0 / gamma : 1.0;
  r.s = gamma > 0.0 ? beta_next / gamma : 0.0;
  r.ginv = gamma > 0.0 ? 1.0 / gamma : 0.0;
  r.step = r.c * eta;
  r.eta_new = -r.s * eta;
  r.done = fabs(r.eta_new) <= tol * beta1 || !(beta_next > 0.0);
  r.binv = beta_next > 0.0 ? 1.0 / beta_next : 0.0;
  return r;
}

// the new state (one thread)
__device__ __forceinline__ void mr_store_state(const double* __restrict__ in, double* __restrict__ out,
                                               const MrRot& r, double beta_next, double* __restrict__ hist,
                                               int64_t hist_cap) {
  const double beta1 = in[MR_BETA1];
  out[MR_BETA] = beta_next;
  out[MR_C1] = r.c;
  out[MR_S1] = r.s;
  out[MR_C2] = in[MR_C1];
  out[MR_S2] = in[MR_S1];
  out[MR_ETA] = r.eta_new;
  out[MR_BETA1] = beta1;
  out[MR_DONE] = r.done ? 1.0 : 0.0;
  out[MR_ITERS] = in[MR_ITERS] + 1.0;
  out[MR_TOL] = in[MR_TOL];
  const int64_t j = (int64_t)in[MR_ITERS];
  if (j < hist_cap) hist[j] = beta1 > 0.0 ? fabs(r.eta_new) / beta1 : 0.0;
}

// the element updates of workgroup blk, from beta_{k+1} and alpha_k; workgroup 0 writes the state
__device__ __forceinline__ void mr_update_part(double* __restrict__ v, double* __restrict__ vprev,
                                               const double* __restrict__ p, double* __restrict__ w1,
                                               double* __restrict__ w2, double* __restrict__ x, int64_t n,
                                               double beta_next, double alpha, const double* __restrict__ in,
                                               double* __restrict__ out, double* __restrict__ hist, int64_t hist_cap,
                                               int blk) {
  const MrRot r = mr_rotation(in, beta_next, alpha);
  const int64_t e0 = (int64_t)blk * kMElems;
  for (int k = threadIdx.x; k < kMElems; k += kMB) {
    const int64_t e = e0 + k;
    if (e < n) {
      const double ve = v[e], a1 = w1[e];
      const double we = (ve - r.delta * a1 - r.eps * w2[e]) * r.ginv;
      x[e] += r.step * we;
      w2[e] = a1;
      w1[e] = we;
      vprev[e] = ve;
      v[e] = p[e] * r.binv;
    }
  }
  if (blk == 0 && threadIdx.x == 0) mr_store_state(in, out, r, beta_next, hist, hist_cap);
}

__global__ __launch_bounds__(kMB) void k_mr_update(double* __restrict__ v, double* __restrict__ vprev,
                                                   const double* __restrict__ p, double* __restrict__ w1,
                                                   double* __restrict__ w2, double* __restrict__ x, int64_t n,
                                                   const double* __restrict__ partial2, int nblk,
                                                   const double* __restrict__ in, double* __restrict__ out,
                                                   double* __restrict__ hist, int64_t hist_cap) {
  __shared__ double lds[kMB];
  if (in[MR_DONE] != 0.0) {
    if (blockIdx.x == 0 && threadIdx.x < MR_NSTATE) out[threadIdx.x] = in[threadIdx.x];
    return;
  }
  const double beta_next = sqrt(fmax(reduce_partials(partial2, nblk, lds), 0.0));
  mr_update_part(v, vprev, p, w1, w2, x, n, beta_next, out[MR_ALPHA], in, out, hist, hist_cap, blockIdx.x);
}

// A whole iteration in one workgroup when the vectors fit one (n <= kMElems): the three kernels
// above in sequence, with the same sums in the same order (each partial is reduced from the one
// value, as reduce_partials does over a single block), so the same bits in one launch.  Each
// thread loads its entries of every vector once, at the start, and keeps them in registers.
constexpr int kME = kMElems / kMB;   // entries per thread
__global__ __launch_bounds__(kMB) void k_mr_iter1(double* __restrict__ v, double* __restrict__ vprev,
                                                  double* __restrict__ p, double* __restrict__ w1,
                                                  double* __restrict__ w2, double* __restrict__ x,
                                                  const double* __restrict__ wt, int64_t n,
                                                  const double* __restrict__ in, double* __restrict__ out,
                                                  double* __restrict__ hist, int64_t hist_cap) {
  __shared__ double lds[kMB];
  if (in[MR_DONE] != 0.0) {
    if (threadIdx.x < MR_NSTATE) out[threadIdx.x] = in[threadIdx.x];
    return;
  }
  double rv[kME], rp[kME], rw[kME], rq[kME], r1[kME], r2[kME], rx[kME];
#pragma unroll
  for (int i = 0; i < kME; ++i) {
    const int64_t e = threadIdx.x + (int64_t)i * kMB;
    const bool ok = e < n;
    rv[i] = ok ? v[e] : 0.0;
    rp[i] = ok ? p[e] : 0.0;
    rw[i] = ok ? wt[e] : 0.0;
    rq[i] = ok ? vprev[e] : 0.0;
    r1[i] = ok ? w1[e] : 0.0;
    r2[i] = ok ? w2[e] : 0.0;
    rx[i] = ok ? x[e] : 0.0;
  }
  // alpha = <v, p>
  double sa = 0.0;
#pragma unroll
  for (int i = 0; i < kME; ++i)
    if (threadIdx.x + (int64_t)i * kMB < n) sa += rw[i] * rv[i] * rp[i];
  sa = block_sum(sa, lds);
  const double alpha = block_sum(threadIdx.x == 0 ? sa : 0.0, lds);
  // p -= alpha v + beta vprev; <p, p>
  const double beta = in[MR_BETA];
  double sb = 0.0;
#pragma unroll
  for (int i = 0; i < kME; ++i) {
    const int64_t e = threadIdx.x + (int64_t)i * kMB;
    if (e < n) {
      const double pe = rp[i] - alpha * rv[i] - beta * rq[i];
      rp[i] = pe;
      p[e] = pe;
      sb += rw[i] * pe * pe;
    }
  }
  if (threadIdx.x == 0) out[MR_ALPHA] = alpha;
  sb = block_sum(sb, lds);
  const double beta_next = sqrt(fmax(block_sum(threadIdx.x == 0 ? sb : 0.0, lds), 0.0));
  const MrRot r = mr_rotation(in, beta_next, alpha);
#pragma unroll
  for (int i = 0; i < kME; ++i) {
    const int64_t e = threadIdx.x + (int64_t)i * kMB;
    if (e < n) {
      const double ve = rv[i], a1 = r1[i];
      const double we = (ve - r.delta * a1 - r.eps * r2[i]) * r.ginv;
      x[e] = rx[i] + r.step * we;
      w2[e] = a1;
      w1[e] = we;
      vprev[e] = ve;
      v[e] = rp[i] * r.binv;
    }
  }
  if (threadIdx.x == 0) mr_store_state(in, out, r, beta_next, hist, hist_cap);
}

}  // namespace

int mr_nblk(int64_t n) { return n > 0 ? (int)((n + kMElems - 1) / kMElems) : 1; }

void mr_start(const double* b, const double* wt, int64_t n, double tol, double* v, double* vprev, double* w1,
              double* w2, double* x, double* partial, double* state, hipStream_t st) {
  const int nblk = mr_nblk(n);
  hipLaunchKernelGGL(k_mr_wdot, dim3(nblk), dim3(kMB), 0, st, b, b, wt, n, (const double*)nullptr, partial);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_mr_start, dim3(nblk), dim3(kMB), 0, st, b, n, partial, nblk, tol, v, vprev, w1, w2, x, state);
  IBDL_LAUNCH_CHECK();
}

void mr_iteration(double* v, double* vprev, double* p, double* w1, double* w2, double* x, const double* wt,
                  int64_t n, double* partial, const double* in, double* out, double* hist, int64_t hist_cap,
                  hipStream_t st) {
  const int nblk = mr_nblk(n);
  if (nblk == 1) {
    hipLaunchKernelGGL(k_mr_iter1, dim3(1), dim3(kMB), 0, st, v, vprev, p, w1, w2, x, wt, n, in, out, hist,
                       hist_cap);
    IBDL_LAUNCH_CHECK();
    return;
  }
  double* partial2 = partial + nblk;
  hipLaunchKernelGGL(k_mr_wdot, dim3(nblk), dim3(kMB), 0, st, v, p, wt, n, in, partial);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_mr_lanczos, dim3(nblk), dim3(kMB), 0, st, v, vprev, p, wt, n, partial, nblk, partial2, in,
                     out);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_mr_update, dim3(nblk), dim3(kMB), 0, st, v, vprev, p, w1, w2, x, n, partial2, nblk, in, out,
                     hist, hist_cap);
  IBDL_LAUNCH_CHECK();
}

}  // namespace ibdl
