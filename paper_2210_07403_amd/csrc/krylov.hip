// Double-precision Krylov vector kernels (GMRES Arnoldi with classical Gram-Schmidt twice).
// Reductions are two-level with a fixed order (per-block partial sums, then one pass over the
// partials), so every dot product is deterministic.
#include <algorithm>

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

// x = sum_j y_j V_j (k <= 256); y is read once per workgroup into LDS (it may live in host memory)
__global__ void k_lincomb(const double* __restrict__ V, int64_t ldv, int k, const double* __restrict__ y,
                          double* __restrict__ x, int64_t n) {
  __shared__ double ys[256];
  for (int j = threadIdx.x; j < k; j += blockDim.x) ys[j] = y[j];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += V[j * ldv + e] * ys[j];
    x[e] = s;
  }
}

// x = V y over the k = gs[GM_K] steps of a GMRES state; gate as in k_gmres_y
__global__ void k_lincomb_state(const double* __restrict__ V, int64_t ldv, const double* __restrict__ gs,
                                const double* __restrict__ y, double* __restrict__ x, int64_t n, int gate) {
  __shared__ double ys[256];
  if (gate && gs[GM_DONE] == 0.0) return;
  const int k = (int)gs[GM_K];
  for (int j = threadIdx.x; j < k; j += blockDim.x) ys[j] = y[j];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += V[j * ldv + e] * ys[j];
    x[e] = s;
  }
}

__global__ void k_scale(const double* __restrict__ src, double s, double* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e] * s;
}

// dst (and dst2 if set) = src / sqrt(max(*nrm2, 0)); 0 where that norm is not above floor (the
// Arnoldi breakdown, which the host detects from the same value).  Norms clamp a negative rounding
// residue to 0 but keep a NaN, so that the host sees non-finite data rather than a zero vector.
__global__ void k_scale_norm(const double* src, const double* __restrict__ nrm2, double floor, double* dst,
                             double* dst2, int64_t n) {
  const double v = *nrm2;
  const double h = sqrt(v < 0.0 ? 0.0 : v);
  const double s = (h > floor && h < INFINITY) ? 1.0 / h : 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const double x = src[e] * s;
    dst[e] = x;
    if (dst2) dst2[e] = x;
  }
}

__global__ void k_axpby_d(double* __restrict__ y, double a, const double* __restrict__ x, double b, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = a * x[e] + b * y[e];
}

__global__ void k_add_small(double* __restrict__ dst, const double* __restrict__ a, const double* __restrict__ b, int n) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = a[e] + b[e];
}

// partial sums of eta * ds_i * q[i][c] over markers, per component c (ds = NULL: unit weights)
__global__ __launch_bounds__(kB) void k_border_partial(const double* __restrict__ q, const double* __restrict__ ds,
                                                       int64_t n_ib, int nq, int nblk, double* __restrict__ partial) {
  __shared__ double red[kB];
  const int c = blockIdx.y;
  const int64_t beg = (int64_t)blockIdx.x * kElemsPerBlock;
  const int64_t end = beg + kElemsPerBlock < n_ib ? beg + kElemsPerBlock : n_ib;
  double s = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kB) s += (ds ? ds[i] : 1.0) * q[i * nq + c];
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

// Marker side of the transposed operator.  G holds, per marker, the interpolated adjoint grid
// fields (scalar: D_d w for d < D, then w when eta > 0; Stokes: the fields dual to A11, A12, A22
// (and eta Q1, eta Q2)); the result is
//   scalar  y_i = h^-D ds_i (sum_d n_id G_i,d - eta G_i,D) + b p_i + eta ds_i pu
//   Stokes  y_ic = h^-D ds_i sum_f (d c_f / d Q_c) G_i,f + b p_ic + eta ds_i pu_c
// with c_f the per-marker spread coefficients 2 Q1 n1, Q1 n2 + Q2 n1, 2 Q2 n2, eta Q1, eta Q2.
__global__ void k_adj_combine(int stokes, int dim, int64_t n_ib, int ng, double hDinv, double eta,
                              const double* __restrict__ G, const double* __restrict__ nrm,
                              const double* __restrict__ ds, const double* __restrict__ p, double b,
                              const double* __restrict__ pu, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ib) return;
  const double* Gi = G + i * ng;
  const double w = hDinv * ds[i];
  if (!stokes) {
    double s = 0.0;
    for (int d = 0; d < dim; ++d) s += nrm[i * dim + d] * Gi[d];
    if (ng > dim) s -= eta * Gi[dim];
    double v = w * s;
    if (p) v += b * p[i];
    if (pu) v += eta * ds[i] * pu[0];
    y[i] = v;
    return;
  }
  const double n1 = nrm[2 * i], n2 = nrm[2 * i + 1];
  double s1 = 2.0 * n1 * Gi[0] + n2 * Gi[1];
  double s2 = n1 * Gi[1] + 2.0 * n2 * Gi[2];
  if (ng > 3) {
    s1 += eta * Gi[3];
    s2 += eta * Gi[4];
  }
  double v1 = w * s1, v2 = w * s2;
  if (p) {
    v1 += b * p[2 * i];
    v2 += b * p[2 * i + 1];
  }
  if (pu) {
    v1 += eta * ds[i] * pu[0];
    v2 += eta * ds[i] * pu[1];
  }
  y[2 * i] = v1;
  y[2 * i + 1] = v2;
}

// Per-marker weights of the grid fields whose kernel-derivative gathers make up dL/dX:
//   scalar  [u: -mu_i] [D_d r: -h^-D ds_i Q_i n_id] [r: eta h^-D ds_i Q_i (eta > 0)]
//   Stokes  [u_c: -mu_ic] [Z_f: h^-D ds_i c_f,i for the nf spread fields]
__global__ void k_adj_coefs(int stokes, int dim, int64_t n_ib, int nc, double hDinv, double eta,
                            const double* __restrict__ mu, const double* __restrict__ q,
                            const double* __restrict__ nrm, const double* __restrict__ ds,
                            double* __restrict__ coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ib) return;
  double* c = coef + i * nc;
  const double w = hDinv * ds[i];
  if (!stokes) {
    c[0] = -mu[i];
    for (int d = 0; d < dim; ++d) c[1 + d] = -w * q[i] * nrm[i * dim + d];
    if (nc > dim + 1) c[dim + 1] = eta * w * q[i];
    return;
  }
  const double q1 = q[2 * i], q2 = q[2 * i + 1], n1 = nrm[2 * i], n2 = nrm[2 * i + 1];
  c[0] = -mu[2 * i];
  c[1] = -mu[2 * i + 1];
  c[2] = w * 2.0 * q1 * n1;
  c[3] = w * (q1 * n2 + q2 * n1);
  c[4] = w * 2.0 * q2 * n2;
  if (nc > 5) {
    c[5] = w * eta * q1;
    c[6] = w * eta * q2;
  }
}

// One Arnoldi step's vector work.  MODE 0: d_j = V_j . w (j < k); MODE 1: w -= V h, then
// d_j = V_j . w; MODE 2: w -= V h, then d_0 = w . w.  A block handles 256 elements, one per thread
// (the thread updates its element and then reads it, so no barrier is needed between the update and
// the dots); dot products are taken eight at a time, each thread keeping eight partial products and
// the block adding them in a fixed tree.  The per-block partials are added by k_arnoldi_reduce, one
// block per dot product, in a fixed order, so the sums do not depend on scheduling.  (A last-block
// reduction inside the first kernel would need device-wide fences, which write back the per-XCD L2
// caches and cost more than the second launch.)
constexpr int kArnChunk = 256;
constexpr int kArnGroup = 8;

// Sum of p[0..nblk) by one wave: lane strides, then a butterfly.  Every wave and workgroup that
// sums the same values gets the same bits (the butterfly's pairwise sums commute), so a dot product
// reduced redundantly by each workgroup that needs it equals the copy the host receives.
__device__ __forceinline__ double wave_sum(const double* __restrict__ p, int nblk, int lane) {
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += p[b];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  return s;
}

// Arnoldi vector work on 256-element blocks.  mode 0: pout[j][b] = block b's part of V_j . w.
// mode 1 / 2: h_j = the sums of pin[j][*] (the previous mode's dots, reduced in every workgroup;
// workgroup 0 also stores them to hout), w -= V h, then mode 1 pout[j][b] = V_j . w, mode 2
// pout[0][b] = w . w; j < k <= 256.
template <int MODE>
__global__ __launch_bounds__(kB) void k_arnoldi(const double* __restrict__ V, int64_t ldv, int k, double* w,
                                                const double* __restrict__ pin, double* __restrict__ hout,
                                                int64_t n, int nblk, double* __restrict__ pout) {
  __shared__ double red[kArnGroup][kB];
  __shared__ double hs[256];
  const int64_t e = (int64_t)blockIdx.x * kArnChunk + threadIdx.x;
  const bool in = e < n;
  double we = in ? w[e] : 0.0;
  if (MODE > 0) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < k; j += kB / 64) {
      const double v = wave_sum(pin + (int64_t)j * nblk, nblk, lane);
      if (lane == 0) hs[j] = v;
    }
    __syncthreads();
    if (blockIdx.x == 0)
      for (int j = threadIdx.x; j < k; j += kB) hout[j] = hs[j];
    if (in) {
      for (int j = 0; j < k; ++j) we -= V[j * ldv + e] * hs[j];
      w[e] = we;
    }
  }
  const int nd = MODE == 2 ? 1 : k;
  for (int d0 = 0; d0 < nd; d0 += kArnGroup) {
#pragma unroll
    for (int g = 0; g < kArnGroup; ++g) {
      const int d = d0 + g;
      double p = 0.0;
      if (in && d < nd) p = (MODE == 2 ? we : V[d * ldv + e]) * we;
      red[g][threadIdx.x] = p;
    }
    __syncthreads();
    for (int st = kB / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) {
#pragma unroll
        for (int g = 0; g < kArnGroup; ++g) red[g][threadIdx.x] += red[g][threadIdx.x + st];
      }
      __syncthreads();
    }
    if (threadIdx.x < kArnGroup && d0 + threadIdx.x < nd) pout[(d0 + threadIdx.x) * nblk + blockIdx.x] = red[threadIdx.x][0];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ batched (segmented) vectors
// A batch vector is the concatenation of the problems' vectors; block b of a segmented dot covers
// [beg[b], end[b]) inside one problem's segment, and problem p owns blocks pb0[p] .. pb0[p+1]-1.
__global__ __launch_bounds__(kB) void k_bmultidot(const double* __restrict__ V, int64_t ldv, int k,
                                                  const double* __restrict__ w, const int64_t* __restrict__ beg,
                                                  const int64_t* __restrict__ end, int nblk,
                                                  double* __restrict__ partial) {
  __shared__ double red[kB];
  const int64_t b0 = beg[blockIdx.x], b1 = end[blockIdx.x];
  for (int j = 0; j < k; ++j) {
    const double* vj = V + j * ldv;
    double s = 0.0;
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kB) s += vj[e] * w[e];
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

// out[p * ostride + j] = sum of problem p's partial sums of dot j (grid: k x nprob)
__global__ void k_breduce(const double* __restrict__ partial, int nblk, const int* __restrict__ pb0, int ostride,
                          double* __restrict__ out) {
  const int j = blockIdx.x, p = blockIdx.y;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = pb0[p]; b < pb0[p + 1]; ++b) s += partial[j * nblk + b];
    out[p * ostride + j] = s;
  }
}

// w[e] -= sum_j V_j[e] H[seg(e)][j]
__global__ void k_bgemv_sub(const double* __restrict__ V, int64_t ldv, int k, const double* __restrict__ H,
                            int hs, const int* __restrict__ seg, double* __restrict__ w, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const double* hp = H + (int64_t)seg[e] * hs;
    double s = w[e];
    for (int j = 0; j < k; ++j) s -= V[j * ldv + e] * hp[j];
    w[e] = s;
  }
}

// x[e] = sum_j V_j[e] Y[seg(e)][j]
__global__ void k_blincomb(const double* __restrict__ V, int64_t ldv, int k, const double* __restrict__ Y, int ys,
                           const int* __restrict__ seg, double* __restrict__ x, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const double* yp = Y + (int64_t)seg[e] * ys;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += V[j * ldv + e] * yp[j];
    x[e] = s;
  }
}

// dst[e] = src[e] * sc[seg(e)]
__global__ void k_bscale(const double* __restrict__ src, const double* __restrict__ sc, const int* __restrict__ seg,
                         double* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e] * sc[seg[e]];
}

// ------------------------------------------------------------------ GMRES least squares
// The Givens-rotated Hessenberg matrix R, the rotations and the rotated right-hand side g of one
// GMRES solve live in device memory (layout gm_* below), so the least-squares problem is updated
// and solved on the device in double precision.  Step j's column is h1[i] + h2[i] (i <= j, the two
// Gram-Schmidt passes) and |w| below it; the rotations of the earlier steps are applied to it, the
// new rotation zeroes |w|, g is rotated, and res = |g[j+1]| / |b| is the Krylov residual estimate.
// Once res <= tol or the Arnoldi process breaks down the state is frozen: steps queued after that
// change nothing, and k stays the number of steps the solution uses.
__device__ __forceinline__ double* gm_cs(double* gs) { return gs + GM_HDR; }
__device__ __forceinline__ double* gm_sn(double* gs, int mx) { return gs + GM_HDR + mx; }
__device__ __forceinline__ double* gm_g(double* gs, int mx) { return gs + GM_HDR + 2 * mx; }
__device__ __forceinline__ double* gm_y(double* gs, int mx) { return gs + GM_HDR + 3 * mx + 1; }
__device__ __forceinline__ double* gm_R(double* gs, int mx) { return gs + GM_HDR + 4 * mx + 2; }

// Run by a whole workgroup of kB threads (the sequential rotation sweep by thread 0 on values staged
// in LDS).  bnorm2 = |b|^2 (read at step 0), nrm2 = |w|^2 of this step.
__device__ void givens_step(const double* __restrict__ h1, const double* __restrict__ h2, double nrm2,
                            double bnorm2, int j, int mx, double tol, double* gs) {
  __shared__ double col[257], c_s[256], s_s[256];
  __shared__ int frozen;
  if (threadIdx.x == 0) frozen = j > 0 && gs[GM_DONE] != 0.0;
  __syncthreads();
  if (frozen) return;
  const double* cs = gm_cs(gs);
  const double* sn = gm_sn(gs, mx);
  for (int i = threadIdx.x; i <= j; i += kB) {
    col[i] = h1[i] + h2[i];
    if (i < j) {
      c_s[i] = cs[i];
      s_s[i] = sn[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* g = gm_g(gs, mx);
    double beta;
    if (j == 0) {
      beta = sqrt(bnorm2 < 0.0 ? 0.0 : bnorm2);
      gs[GM_BETA] = beta;
      g[0] = beta;
    } else {
      beta = gs[GM_BETA];
    }
    const double hn = sqrt(nrm2 < 0.0 ? 0.0 : nrm2);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double t = c_s[i] * col[i] + s_s[i] * col[i + 1];
      col[i + 1] = -s_s[i] * col[i] + c_s[i] * col[i + 1];
      col[i] = t;
    }
    double res = 0.0;
    bool stop = true;
    if (beta > 0.0) {
      const double r = hypot(col[j], col[j + 1]);
      const double c = col[j] / r, sv = col[j + 1] / r;
      gm_cs(gs)[j] = c;
      gm_sn(gs, mx)[j] = sv;
      col[j] = r;
      g[j + 1] = -sv * g[j];
      g[j] = c * g[j];
      res = fabs(g[j + 1]) / beta;
      const bool breakdown = !(hn > 1e-300 * beta);
      stop = res <= tol || breakdown || !(res == res);
      gs[GM_K] = (double)(j + 1);
    } else {
      gs[GM_K] = 0.0;
    }
    gs[GM_RES] = res;
    gs[GM_HN] = hn;
    gs[GM_DONE] = stop ? 1.0 : 0.0;
  }
  __syncthreads();
  double* R = gm_R(gs, mx) + (int64_t)j * (mx + 1);
  for (int i = threadIdx.x; i <= j; i += kB) R[i] = col[i];
}

// The least-squares solution y = R^-1 g of the k = gs[GM_K] steps, by one workgroup: with k <= 64
// the triangle is staged in LDS once, otherwise each column is read as the substitution reaches it.
// gate: nothing unless the state's convergence flag is set (a finish queued behind a step that the
// host predicts to be the last, before it has seen that step's result).
__global__ __launch_bounds__(kB) void k_gmres_y(double* gs, int mx, int gate) {
  __shared__ double tri[64 * 64];
  __shared__ double gv[256];
  __shared__ double yv;
  if (gate && gs[GM_DONE] == 0.0) return;
  const int k = (int)gs[GM_K];
  const double* R = gm_R(gs, mx);
  const double* g = gm_g(gs, mx);
  for (int i = threadIdx.x; i < k; i += kB) gv[i] = g[i];
  const bool staged = k <= 64;
  if (staged)
    for (int e = threadIdx.x; e < k * k; e += kB) {
      const int c = e / k, i = e - c * k;
      tri[c * 64 + i] = i <= c ? R[(int64_t)c * (mx + 1) + i] : 0.0;
    }
  __syncthreads();
  double* y = gm_y(gs, mx);
  for (int c = k - 1; c >= 0; --c) {
    const double* rc = staged ? tri + c * 64 : R + (int64_t)c * (mx + 1);
    if (threadIdx.x == 0) {
      yv = gv[c] / rc[c];
      y[c] = yv;
    }
    __syncthreads();
    const double v = yv;
    for (int i = threadIdx.x; i < c; i += kB) gv[i] -= rc[i] * v;
    __syncthreads();
  }
}

// Copy n doubles into host-mapped memory, then (after a system-scope fence) the sequence tag, so a
// host that sees the tag sees the values.
// With pnorm set, src[norm_at] is first set to the sum of pnorm[0..nblk) (as k_arnoldi reduces).
__global__ __launch_bounds__(kB) void k_publish(double* src, int n, const double* __restrict__ pnorm, int nblk,
                                                int norm_at, double* dst, unsigned* tag, unsigned seq) {
  if (pnorm) {
    if (threadIdx.x < 64) {
      const double v = wave_sum(pnorm, nblk, threadIdx.x);
      if (threadIdx.x == 0) src[norm_at] = v;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += kB) dst[i] = src[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence_system();
    *reinterpret_cast<volatile unsigned*>(tag) = seq;
  }
}

// The end of an Arnoldi step in one launch: every workgroup reduces the norm partials itself (in the
// same order, so with the same bits) and scales its part of w into vdst (and vdst2) by 1/|w|, or by
// 0 where |w| is 0 or not finite; workgroup 0 also stores |w|^2 at h[norm_at], runs the step's
// least-squares update (givens_step) and copies the state's scalars (GM_PUB of them) to the host
// slot, then writes the tag.
__global__ __launch_bounds__(kB) void k_publish_scale(double* h, const double* __restrict__ pnorm, int nblk,
                                                      int norm_at, double* gs, int j, int mx, double tol, double* dst,
                                                      unsigned* tag, unsigned seq, const double* w, double* vdst,
                                                      double* vdst2, int64_t nv) {
  __shared__ double nrm2;
  if (threadIdx.x < 64) {
    const double v = wave_sum(pnorm, nblk, threadIdx.x);
    if (threadIdx.x == 0) nrm2 = v;
  }
  __syncthreads();
  const double v = nrm2;
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) h[norm_at] = v;
    givens_step(h, h + 256, v, h[GM_BNORM2_AT], j, mx, tol, gs);
    __syncthreads();
    if (threadIdx.x < GM_PUB) dst[threadIdx.x] = gs[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence_system();
      *reinterpret_cast<volatile unsigned*>(tag) = seq;
    }
  }
  const double hh = sqrt(v < 0.0 ? 0.0 : v);
  const double sc = (hh > 0.0 && hh < INFINITY) ? 1.0 / hh : 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nv; e += (int64_t)gridDim.x * blockDim.x) {
    const double x = w[e] * sc;
    vdst[e] = x;
    if (vdst2) vdst2[e] = x;
  }
}

// The Arnoldi step and its publication in one workgroup and one launch, for vectors of at most
// kB entries (the marker systems of small problems, where the four launches of the blocked path
// are mostly launch latency): thread t owns entry t and keeps it in a register; the dot products
// are taken eight at a time, a butterfly in each wave and then the four waves' sums in order
// (deterministic; the rounding differs from the blocked path's tree).
__device__ __forceinline__ void wg_sum8(double (&v)[kArnGroup], double (*lds)[kArnGroup]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int g = 0; g < kArnGroup; ++g)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[g] += __shfl_xor(v[g], off);
  if (lane == 0)
#pragma unroll
    for (int g = 0; g < kArnGroup; ++g) lds[wave][g] = v[g];
  __syncthreads();
#pragma unroll
  for (int g = 0; g < kArnGroup; ++g) v[g] = ((lds[0][g] + lds[1][g]) + lds[2][g]) + lds[3][g];
  __syncthreads();
}

__global__ __launch_bounds__(kB) void k_arnoldi_small(const double* __restrict__ V, int64_t ldv, int k, double* w,
                                                      int64_t n, double* h, int norm_at, double* gs, int mx,
                                                      double tol, double* dst, unsigned* tag, unsigned seq,
                                                      double* vdst, double* vdst2) {
  __shared__ double lds[4][kArnGroup];
  __shared__ double hs[256];
  const int e = threadIdx.x;
  const bool in = e < n;
  double we = in ? w[e] : 0.0;
  // two Gram-Schmidt passes: h[j] = V_j . w, w -= V h; h[256 + j] = V_j . w, w -= V h[256..]
  for (int pass = 0; pass < 2; ++pass) {
    for (int d0 = 0; d0 < k; d0 += kArnGroup) {
      double acc[kArnGroup];
#pragma unroll
      for (int g = 0; g < kArnGroup; ++g) acc[g] = (in && d0 + g < k) ? V[(int64_t)(d0 + g) * ldv + e] * we : 0.0;
      wg_sum8(acc, lds);
      if (threadIdx.x == 0)
#pragma unroll
        for (int g = 0; g < kArnGroup; ++g)
          if (d0 + g < k) hs[d0 + g] = acc[g];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += kB) h[256 * pass + j] = hs[j];
    if (in) {
      for (int j = 0; j < k; ++j) we -= V[(int64_t)j * ldv + e] * hs[j];
      w[e] = we;
    }
    __syncthreads();
  }
  // |w|^2, the least-squares update, the publication (values, then the tag after a system-scope
  // fence), w / |w|
  double sq[kArnGroup] = {we * we, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  wg_sum8(sq, lds);
  const double v = sq[0];
  if (threadIdx.x == 0) h[norm_at] = v;
  __syncthreads();
  givens_step(h, h + 256, v, h[GM_BNORM2_AT], k - 1, mx, tol, gs);
  __syncthreads();
  if (threadIdx.x < GM_PUB) dst[threadIdx.x] = gs[threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence_system();
    *reinterpret_cast<volatile unsigned*>(tag) = seq;
  }
  const double nr = sqrt(v < 0.0 ? 0.0 : v);
  const double sc = (nr > 0.0 && nr < INFINITY) ? 1.0 / nr : 0.0;
  if (in) {
    const double x = we * sc;
    vdst[e] = x;
    if (vdst2) vdst2[e] = x;
  }
}

// ------------------------------------------------------------------ batched GMRES on the device
// One workgroup per problem does a whole Arnoldi step of its problem: both classical Gram-Schmidt
// passes over its segment [off[p], off[p] + len[p]) of the batch vectors (dot products eight at a
// time, each a fixed tree over the workgroup), |w|^2, the least-squares update of its own state
// gs + p * gstride (givens_step), and the normalisation of w into the next basis vector and the
// apply's input xin.  A problem whose state was already frozen writes zeros there (its later
// applies run on zeros) and changes nothing else.  The step number j comes from the host.
__device__ __forceinline__ double wg_tree(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int st = kB / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kB) void k_batch_arnoldi(const double* __restrict__ V, int64_t ldv, int j,
                                                      double* __restrict__ w, const int64_t* __restrict__ off,
                                                      const int64_t* __restrict__ len, const double* __restrict__ bn2,
                                                      double* gsb, int64_t gstride, int mx, double tol,
                                                      double* __restrict__ vnext, double* __restrict__ xin) {
  __shared__ double red[kArnGroup][kB];
  __shared__ double hv[2][256];
  __shared__ int frozen;
  const int p = blockIdx.x;
  const int64_t beg = off[p], n = len[p];
  double* gs = gsb + (int64_t)p * gstride;
  if (threadIdx.x == 0) frozen = j > 0 && gs[GM_DONE] != 0.0;
  __syncthreads();
  if (frozen) {
    for (int64_t e = threadIdx.x; e < n; e += kB) {
      vnext[beg + e] = 0.0;
      if (xin) xin[beg + e] = 0.0;
    }
    return;
  }
  const int k = j + 1;
  double* wp = w + beg;
  for (int pass = 0; pass < 2; ++pass) {
    for (int d0 = 0; d0 < k; d0 += kArnGroup) {
      double acc[kArnGroup];
#pragma unroll
      for (int g = 0; g < kArnGroup; ++g) acc[g] = 0.0;
      for (int64_t e = threadIdx.x; e < n; e += kB) {
        const double we = wp[e];
#pragma unroll
        for (int g = 0; g < kArnGroup; ++g)
          if (d0 + g < k) acc[g] += V[(int64_t)(d0 + g) * ldv + beg + e] * we;
      }
#pragma unroll
      for (int g = 0; g < kArnGroup; ++g) red[g][threadIdx.x] = acc[g];
      __syncthreads();
      for (int st = kB / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
#pragma unroll
          for (int g = 0; g < kArnGroup; ++g) red[g][threadIdx.x] += red[g][threadIdx.x + st];
        }
        __syncthreads();
      }
      if (threadIdx.x < kArnGroup && d0 + threadIdx.x < k) hv[pass][d0 + threadIdx.x] = red[threadIdx.x][0];
      __syncthreads();
    }
    for (int64_t e = threadIdx.x; e < n; e += kB) {
      double we = wp[e];
      for (int i = 0; i < k; ++i) we -= V[(int64_t)i * ldv + beg + e] * hv[pass][i];
      wp[e] = we;
    }
    __syncthreads();
  }
  double sq = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += kB) sq += wp[e] * wp[e];
  const double nrm2 = wg_tree(sq, &red[0][0]);
  givens_step(hv[0], hv[1], nrm2, bn2[p], j, mx, tol, gs);
  __syncthreads();
  const double hn = sqrt(nrm2 < 0.0 ? 0.0 : nrm2);
  const double beta = gs[GM_BETA];
  const double sc = (hn > 1e-300 * beta && hn < INFINITY) ? 1.0 / hn : 0.0;
  for (int64_t e = threadIdx.x; e < n; e += kB) {
    const double x = wp[e] * sc;
    vnext[beg + e] = x;
    if (xin) xin[beg + e] = x;
  }
}

// The same step for problems of at most 1024 R unknowns with 1024 threads per problem, each thread
// keeping its R entries of w in registers: dot products eight at a time, a butterfly in each wave
// and then the sixteen waves' sums in order (deterministic; grouped differently from the 256-thread
// form above).  (Keeping the first eight basis vectors in registers as well, to read them once per
// step, needs more than the 128 registers a thread has at this workgroup size: it spilled.)
template <int R>
__global__ __launch_bounds__(1024) void k_batch_arnoldi_r(const double* __restrict__ V, int64_t ldv, int j,
                                                          double* __restrict__ w, const int64_t* __restrict__ off,
                                                          const int64_t* __restrict__ len,
                                                          const double* __restrict__ bn2, double* gsb, int64_t gstride,
                                                          int mx, double tol, double* __restrict__ vnext,
                                                          double* __restrict__ xin) {
  constexpr int NT = 1024, NW = NT / 64;
  __shared__ double part[NW][kArnGroup];
  __shared__ double hv[2][256];
  __shared__ int frozen;
  const int p = blockIdx.x;
  const int64_t beg = off[p], n = len[p];
  double* gs = gsb + (int64_t)p * gstride;
  if (threadIdx.x == 0) frozen = j > 0 && gs[GM_DONE] != 0.0;
  __syncthreads();
  if (frozen) {
    for (int64_t e = threadIdx.x; e < n; e += NT) {
      vnext[beg + e] = 0.0;
      if (xin) xin[beg + e] = 0.0;
    }
    return;
  }
  const int k = j + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* vb = V + beg;
  double we[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t e = threadIdx.x + (int64_t)r * NT;
    we[r] = e < n ? w[beg + e] : 0.0;
  }
  auto block_sum8 = [&](double (&v)[kArnGroup]) {
#pragma unroll
    for (int g = 0; g < kArnGroup; ++g)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v[g] += __shfl_xor(v[g], o);
    if (lane == 0)
#pragma unroll
      for (int g = 0; g < kArnGroup; ++g) part[wave][g] = v[g];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < kArnGroup; ++g) {
      double t = part[0][g];
      for (int q = 1; q < NW; ++q) t += part[q][g];
      v[g] = t;
    }
    __syncthreads();
  };
  for (int pass = 0; pass < 2; ++pass) {
    for (int d0 = 0; d0 < k; d0 += kArnGroup) {
      double acc[kArnGroup];
#pragma unroll
      for (int g = 0; g < kArnGroup; ++g) {
        acc[g] = 0.0;
        if (d0 + g < k)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int64_t e = threadIdx.x + (int64_t)r * NT;
            if (e < n) acc[g] += vb[(int64_t)(d0 + g) * ldv + e] * we[r];
          }
      }
      block_sum8(acc);
      if (threadIdx.x == 0)
#pragma unroll
        for (int g = 0; g < kArnGroup; ++g)
          if (d0 + g < k) hv[pass][d0 + g] = acc[g];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t e = threadIdx.x + (int64_t)r * NT;
      double x = we[r];
      if (e < n)
        for (int i = 0; i < k; ++i) x -= vb[(int64_t)i * ldv + e] * hv[pass][i];
      we[r] = e < n ? x : 0.0;
    }
  }
  double sq[kArnGroup] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < R; ++r) sq[0] += we[r] * we[r];
  block_sum8(sq);
  const double nrm2 = sq[0];
  givens_step(hv[0], hv[1], nrm2, bn2[p], j, mx, tol, gs);
  __syncthreads();
  const double hn = sqrt(nrm2 < 0.0 ? 0.0 : nrm2);
  const double beta = gs[GM_BETA];
  const double sc = (hn > 1e-300 * beta && hn < INFINITY) ? 1.0 / hn : 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t e = threadIdx.x + (int64_t)r * NT;
    if (e < n) {
      const double x = we[r] * sc;
      vnext[beg + e] = x;
      if (xin) xin[beg + e] = x;
    }
  }
}

// Problem p's segment of a batch vector to or from its own array: to_batch: base[off[p] + e] =
// ptr[p][e]; otherwise ptr[p][e] = base[off[p] + e] (one launch for every problem).
__global__ void k_seg_copy(const double* const* __restrict__ ptr, const int64_t* __restrict__ off,
                           const int64_t* __restrict__ len, double* __restrict__ base, int to_batch) {
  const int p = blockIdx.y;
  const int64_t n = len[p];
  double* seg = base + off[p];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    if (to_batch) seg[e] = ptr[p][e];
    else const_cast<double*>(ptr[p])[e] = seg[e];
  }
}

// V[0] segment of problem p = b / |b| (0 when |b| is 0 or not finite), also into xin
__global__ void k_batch_start(const double* __restrict__ b, const int64_t* __restrict__ off,
                              const int64_t* __restrict__ len, const double* __restrict__ bn2,
                              double* __restrict__ v0, double* __restrict__ xin) {
  const int p = blockIdx.x;
  const double nb = sqrt(bn2[p] < 0.0 ? 0.0 : bn2[p]);
  const double sc = (nb > 0.0 && nb < INFINITY) ? 1.0 / nb : 0.0;
  for (int64_t e = threadIdx.x; e < len[p]; e += blockDim.x) {
    const double x = b[off[p] + e] * sc;
    v0[off[p] + e] = x;
    if (xin) xin[off[p] + e] = x;
  }
}

// The first GM_PUB scalars of every problem's state to the host slot, then the tag
__global__ __launch_bounds__(kB) void k_batch_publish(const double* gsb, int64_t gstride, int np, double* dst,
                                                      unsigned* tag, unsigned seq) {
  for (int i = threadIdx.x; i < np * GM_PUB; i += kB) dst[i] = gsb[(int64_t)(i / GM_PUB) * gstride + i % GM_PUB];
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence_system();
    *reinterpret_cast<volatile unsigned*>(tag) = seq;
  }
}

// Per problem: y = R^-1 g of its GM_K steps into Y[p][0..kmax) (zeros beyond its own count)
__global__ __launch_bounds__(kB) void k_batch_y(double* gsb, int64_t gstride, int mx, int kmax, double* Y, int ys) {
  __shared__ double gv[256];
  __shared__ double yv;
  double* gs = gsb + (int64_t)blockIdx.x * gstride;
  const int k = (int)gs[GM_K];
  const double* R = gm_R(gs, mx);
  const double* g = gm_g(gs, mx);
  double* y = Y + (int64_t)blockIdx.x * ys;
  for (int i = threadIdx.x; i < k; i += kB) gv[i] = g[i];
  for (int i = k + threadIdx.x; i < kmax; i += kB) y[i] = 0.0;
  __syncthreads();
  for (int c = k - 1; c >= 0; --c) {
    const double* rc = R + (int64_t)c * (mx + 1);
    if (threadIdx.x == 0) {
      yv = gv[c] / rc[c];
      y[c] = yv;
    }
    __syncthreads();
    const double v = yv;
    for (int i = threadIdx.x; i < c; i += kB) gv[i] -= rc[i] * v;
    __syncthreads();
  }
}

inline unsigned blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

}  // namespace

void kr_publish_scale(double* h, const double* pnorm, int nblk, int norm_at, double* gs, int j, int mx, double tol,
                      double* host_dst, unsigned* host_tag, unsigned seq, const double* w, double* dst, double* dst2,
                      int64_t nv, hipStream_t st) {
  if (j < 0 || j >= mx || mx > 256) throw Error(-2, "kr_publish_scale: 0 <= j < mx <= 256");
  hipLaunchKernelGGL(k_publish_scale, dim3(blocks_for(nv)), dim3(kB), 0, st, h, pnorm, nblk, norm_at, gs, j, mx, tol,
                     host_dst, host_tag, seq, w, dst, dst2, nv);
  IBDL_LAUNCH_CHECK();
}

void kr_arnoldi_small(const double* V, int64_t ldv, int k, double* w, int64_t n, double* h, int norm_at, double* gs,
                      int mx, double tol, double* host_dst, unsigned* host_tag, unsigned seq, double* dst,
                      double* dst2, hipStream_t st) {
  if (n > kSmallN || k < 1 || k > mx || mx > 256) throw Error(-2, "kr_arnoldi_small: n <= kSmallN and 1 <= k <= mx <= 256");
  hipLaunchKernelGGL(k_arnoldi_small, dim3(1), dim3(kB), 0, st, V, ldv, k, w, n, h, norm_at, gs, mx, tol, host_dst,
                     host_tag, seq, dst, dst2);
  IBDL_LAUNCH_CHECK();
}

size_t kr_gmres_state_doubles(int mx) { return (size_t)GM_HDR + 4 * (size_t)mx + 2 + (size_t)mx * (mx + 1); }

void kr_gmres_y(double* gs, int mx, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_y, dim3(1), dim3(kB), 0, st, gs, mx, 0);
  IBDL_LAUNCH_CHECK();
}

const double* kr_gmres_ydev(double* gs, int mx) { return gs + GM_HDR + 3 * mx + 1; }

void kr_gmres_finish(double* gs, int mx, const double* V, int64_t ldv, double* x, int64_t n, bool gate,
                     hipStream_t st) {
  if (mx > 256) throw Error(-1, "kr_gmres_finish: at most 256 basis vectors");
  hipLaunchKernelGGL(k_gmres_y, dim3(1), dim3(kB), 0, st, gs, mx, gate ? 1 : 0);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_lincomb_state, dim3(blocks_for(n)), dim3(256), 0, st, V, ldv, (const double*)gs,
                     kr_gmres_ydev(gs, mx), x, n, gate ? 1 : 0);
  IBDL_LAUNCH_CHECK();
}

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
  if (k > 256) throw Error(-1, "kr_lincomb: at most 256 basis vectors");
  hipLaunchKernelGGL(k_lincomb, dim3(blocks_for(n)), dim3(256), 0, st, V, ldv, k, y, x, n);
  IBDL_LAUNCH_CHECK();
}

void kr_scale(const double* src, double s, double* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(256), 0, st, src, s, dst, n);
  IBDL_LAUNCH_CHECK();
}

void kr_scale_norm(const double* src, const double* nrm2, double floor, double* dst, double* dst2, int64_t n,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_scale_norm, dim3(blocks_for(n)), dim3(256), 0, st, src, nrm2, floor, dst, dst2, n);
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

int kr_arnoldi_nblk(int64_t n) { return (int)((n + kArnChunk - 1) / kArnChunk) > 0 ? (int)((n + kArnChunk - 1) / kArnChunk) : 1; }

void kr_arnoldi_step(const double* V, int64_t ldv, int k, double* w, int64_t n, double* partial, int nblk,
                     double* h, hipStream_t st) {
  if (k < 1 || k > 256) throw Error(-2, "Arnoldi step: 1 <= k <= 256");
  double* p0 = partial;
  double* p1 = partial + (int64_t)k * nblk;
  double* p2 = p1 + (int64_t)k * nblk;
  hipLaunchKernelGGL(k_arnoldi<0>, dim3(nblk), dim3(kB), 0, st, V, ldv, k, w, nullptr, nullptr, n, nblk, p0);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_arnoldi<1>, dim3(nblk), dim3(kB), 0, st, V, ldv, k, w, p0, h, n, nblk, p1);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_arnoldi<2>, dim3(nblk), dim3(kB), 0, st, V, ldv, k, w, p1, h + 256, n, nblk, p2);
  IBDL_LAUNCH_CHECK();
}

void kr_publish(double* src, int n, const double* pnorm, int nblk, int norm_at, double* host_dst,
                unsigned* host_tag, unsigned seq, hipStream_t st) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(kB), 0, st, src, n, pnorm, nblk, norm_at, host_dst, host_tag, seq);
  IBDL_LAUNCH_CHECK();
}

void kb_multidot(const double* V, int64_t ldv, int k, const double* w, const KrylovSegments& sg, double* partial,
                 int ostride, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_bmultidot, dim3(sg.nblk), dim3(kB), 0, st, V, ldv, k, w, sg.beg, sg.end, sg.nblk, partial);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_breduce, dim3(k, sg.nprob), dim3(64), 0, st, partial, sg.nblk, sg.pb0, ostride, out);
  IBDL_LAUNCH_CHECK();
}

void kb_gemv_sub(const double* V, int64_t ldv, int k, const double* H, int hs, const KrylovSegments& sg, double* w,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_bgemv_sub, dim3(blocks_for(sg.n)), dim3(256), 0, st, V, ldv, k, H, hs, sg.seg, w, sg.n);
  IBDL_LAUNCH_CHECK();
}

void kb_lincomb(const double* V, int64_t ldv, int k, const double* Y, int ys, const KrylovSegments& sg, double* x,
                hipStream_t st) {
  hipLaunchKernelGGL(k_blincomb, dim3(blocks_for(sg.n)), dim3(256), 0, st, V, ldv, k, Y, ys, sg.seg, x, sg.n);
  IBDL_LAUNCH_CHECK();
}

void kb_scale(const double* src, const double* sc, const KrylovSegments& sg, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_bscale, dim3(blocks_for(sg.n)), dim3(256), 0, st, src, sc, sg.seg, dst, sg.n);
  IBDL_LAUNCH_CHECK();
}

void kb_seg_copy(const double* const* ptr, const int64_t* off, const int64_t* len, int np, int64_t maxlen,
                 double* base, bool to_batch, hipStream_t st) {
  const unsigned bx = (unsigned)std::min<int64_t>((maxlen + 255) / 256, 64);
  hipLaunchKernelGGL(k_seg_copy, dim3(bx > 0 ? bx : 1, np), dim3(256), 0, st, ptr, off, len, base, to_batch ? 1 : 0);
  IBDL_LAUNCH_CHECK();
}

void kb_gmres_start(const double* b, const int64_t* off, const int64_t* len, int np, const double* bn2, double* v0,
                    double* xin, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_start, dim3(np), dim3(256), 0, st, b, off, len, bn2, v0, xin);
  IBDL_LAUNCH_CHECK();
}

void kb_arnoldi(const double* V, int64_t ldv, int j, double* w, const int64_t* off, const int64_t* len, int np,
                int64_t maxlen, const double* bn2, double* gsb, int64_t gstride, int mx, double tol, double* vnext,
                double* xin, hipStream_t st) {
  if (j < 0 || j >= mx || mx > 256) throw Error(-2, "kb_arnoldi: 0 <= j < mx <= 256");
  if (maxlen <= 1024)
    hipLaunchKernelGGL(k_batch_arnoldi_r<1>, dim3(np), dim3(1024), 0, st, V, ldv, j, w, off, len, bn2, gsb, gstride,
                       mx, tol, vnext, xin);
  else if (maxlen <= 2048)
    hipLaunchKernelGGL(k_batch_arnoldi_r<2>, dim3(np), dim3(1024), 0, st, V, ldv, j, w, off, len, bn2, gsb, gstride,
                       mx, tol, vnext, xin);
  else if (maxlen <= 4096)
    hipLaunchKernelGGL(k_batch_arnoldi_r<4>, dim3(np), dim3(1024), 0, st, V, ldv, j, w, off, len, bn2, gsb, gstride,
                       mx, tol, vnext, xin);
  else
    hipLaunchKernelGGL(k_batch_arnoldi, dim3(np), dim3(kB), 0, st, V, ldv, j, w, off, len, bn2, gsb, gstride, mx, tol,
                       vnext, xin);
  IBDL_LAUNCH_CHECK();
}

void kb_publish(const double* gsb, int64_t gstride, int np, double* host_dst, unsigned* host_tag, unsigned seq,
                hipStream_t st) {
  hipLaunchKernelGGL(k_batch_publish, dim3(1), dim3(kB), 0, st, gsb, gstride, np, host_dst, host_tag, seq);
  IBDL_LAUNCH_CHECK();
}

void kb_gmres_y(double* gsb, int64_t gstride, int np, int mx, int kmax, double* Y, int ys, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_y, dim3(np), dim3(kB), 0, st, gsb, gstride, mx, kmax, Y, ys);
  IBDL_LAUNCH_CHECK();
}

void adj_combine(int stokes, int dim, int64_t n_ib, int ng, double hDinv, double eta, const double* G,
                 const double* nrm, const double* ds, const double* p, double b, const double* pu, double* y,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_adj_combine, dim3((unsigned)((n_ib + 255) / 256)), dim3(256), 0, st, stokes, dim, n_ib, ng,
                     hDinv, eta, G, nrm, ds, p, b, pu, y);
  IBDL_LAUNCH_CHECK();
}

void adj_coefs(int stokes, int dim, int64_t n_ib, int nc, double hDinv, double eta, const double* mu,
               const double* q, const double* nrm, const double* ds, double* coef, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_coefs, dim3((unsigned)((n_ib + 255) / 256)), dim3(256), 0, st, stokes, dim, n_ib, nc,
                     hDinv, eta, mu, q, nrm, ds, coef);
  IBDL_LAUNCH_CHECK();
}

}  // namespace ibdl
