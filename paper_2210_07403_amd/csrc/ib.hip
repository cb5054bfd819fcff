// Lagrangian-Eulerian coupling on gfx950: marker setup, tile binning, spread S (and the fused
// dipole spread S~ = div S(q n) of the finite-difference discretisation), interpolation S*.
//
// Spread is owner-computes: one workgroup owns one tile of grid nodes, loads the markers whose
// 6-node window meets the tile into LDS, and every thread sums the contributions to its own
// nodes in registers.  There are no atomics on grid data, so the result is deterministic, and
// every tile (zeros included) is written exactly once with coalesced stores.
//
// Kernel windows: node indices s, s+1, ..., s+5 per axis with s = floor((X - origin)/h) - 2;
// the 4-point kernels are non-zero on the middle four, the 6-point B-spline on all six.
#include "kernels.h"

namespace ibdl {
namespace {

constexpr int kCH = 64;  // markers staged per LDS chunk

__device__ __forceinline__ double phi_eval(int kernel, double r) {
  const double a = fabs(r);
  if (kernel == KID_PESKIN4) {
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
    if (a < 2.0) return (5.0 - 2.0 * a - sqrt(fmax(-7.0 + 12.0 * a - 4.0 * a * a, 0.0))) * 0.125;
    return 0.0;
  }
  if (kernel == KID_COS4) return a < 2.0 ? 0.25 * (1.0 + cospi(0.5 * a)) : 0.0;
  // quintic B-spline, 6 points
  if (a <= 1.0) return 11.0 / 20.0 - a * a / 2.0 + a * a * a * a / 4.0 - a * a * a * a * a / 12.0;
  if (a <= 2.0)
    return 17.0 / 40.0 + 5.0 * a / 8.0 - 7.0 * a * a / 4.0 + 5.0 * a * a * a / 4.0 - 3.0 * a * a * a * a / 8.0 +
           a * a * a * a * a / 24.0;
  if (a < 3.0)
    return 81.0 / 40.0 - 27.0 * a / 8.0 + 9.0 * a * a / 4.0 - 3.0 * a * a * a / 4.0 + a * a * a * a / 8.0 -
           a * a * a * a * a / 120.0;
  return 0.0;
}

// ------------------------------------------------------------------ marker setup and binning
__device__ __forceinline__ void marker_tiles(const MarkerGeom& g, const int* s, int (&tl)[3][2], int (&nt)[3]) {
  for (int d = 0; d < 3; ++d) {
    if (d < g.dim) {
      const int t0 = s[d] / g.tile[d];
      const int t1 = ((s[d] + 5) & (g.n[d] - 1)) / g.tile[d];
      tl[d][0] = t0;
      tl[d][1] = t1;
      nt[d] = (t1 != t0) ? 2 : 1;
    } else {
      tl[d][0] = tl[d][1] = 0;
      nt[d] = 1;
    }
  }
}

__global__ void k_marker_setup(MarkerGeom g, int64_t n_ib, const double* __restrict__ X, int* __restrict__ s,
                               double* __restrict__ f, int* __restrict__ tile_count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ib) return;
  int si[3] = {0, 0, 0};
  for (int d = 0; d < g.dim; ++d) {
    const double n = (double)g.n[d];
    double xi = (X[i * g.dim + d] - g.origin[d]) / g.h;
    xi = xi - n * floor(xi / n);                 // wrap into [0, n)
    if (!(xi >= 0.0 && xi < n)) xi = 0.0;        // non-finite input: keep indices in range
    const double b = floor(xi);
    int bi = (int)b;
    if (bi >= g.n[d]) bi = g.n[d] - 1;
    f[i * 3 + d] = xi - (double)bi;
    si[d] = (bi - 2 + 2 * g.n[d]) & (g.n[d] - 1);
    s[i * 3 + d] = si[d];
  }
  for (int d = g.dim; d < 3; ++d) {
    s[i * 3 + d] = 0;
    f[i * 3 + d] = 0.0;
  }
  int tl[3][2], nt[3];
  marker_tiles(g, si, tl, nt);
  for (int a = 0; a < nt[2]; ++a)
    for (int b = 0; b < nt[1]; ++b)
      for (int c = 0; c < nt[0]; ++c) {
        const int id = (tl[2][a] * g.ntile[1] + tl[1][b]) * g.ntile[0] + tl[0][c];
        atomicAdd(&tile_count[id], 1);
      }
}

__global__ void k_fill(MarkerGeom g, int64_t n_ib, const int* __restrict__ s, const int* __restrict__ off,
                       int* __restrict__ cur, int* __restrict__ list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ib) return;
  int si[3] = {s[i * 3], s[i * 3 + 1], s[i * 3 + 2]};
  int tl[3][2], nt[3];
  marker_tiles(g, si, tl, nt);
  for (int a = 0; a < nt[2]; ++a)
    for (int b = 0; b < nt[1]; ++b)
      for (int c = 0; c < nt[0]; ++c) {
        const int id = (tl[2][a] * g.ntile[1] + tl[1][b]) * g.ntile[0] + tl[0][c];
        const int pos = off[id] + atomicAdd(&cur[id], 1);
        list[pos] = (int)i;
      }
}

// exclusive scan of cnt[0..n) into off[0..n]; one block of 1024 threads
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ cnt, int* __restrict__ off, int n) {
  __shared__ int buf[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = i < n ? cnt[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int st = 1; st < 1024; st <<= 1) {
      const int t = threadIdx.x >= st ? buf[threadIdx.x - st] : 0;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < n) off[i] = carry + buf[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) off[n] = carry;
}

// sort each tile's marker list ascending (rank sort; marker indices in a tile are unique)
__global__ __launch_bounds__(256) void k_sort_tiles(const int* __restrict__ off, const int* __restrict__ tmp,
                                                    int* __restrict__ list) {
  const int t = blockIdx.x;
  const int b = off[t], e = off[t + 1], L = e - b;
  for (int a = threadIdx.x; a < L; a += blockDim.x) {
    const int v = tmp[b + a];
    int r = 0;
    for (int k = 0; k < L; ++k) r += tmp[b + k] < v;
    list[b + r] = v;
  }
}

// ------------------------------------------------------------------ spread
template <typename T, int D>
__global__ __launch_bounds__(256) void k_spread(SpreadArgs a, T* __restrict__ out) {
  constexpr int TX = (D == 2) ? 16 : 8, TY = (D == 2) ? 16 : 8, TZ = (D == 2) ? 1 : 8;
  constexpr int PPT = (TX * TY * TZ) / 256;  // nodes per thread: 1 (2-D) or 2 (3-D)
  __shared__ int s_s[kCH][3];
  __shared__ T s_w[kCH][3][6];
  __shared__ T s_g[kCH][3][6];
  __shared__ T s_c[kCH][5];
  const MarkerGeom& g = a.g;
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int tx = tile % g.ntile[0];
  const int ty = (tile / g.ntile[0]) % g.ntile[1];
  const int tz = tile / (g.ntile[0] * g.ntile[1]);
  int jx[PPT], jy[PPT], jz[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int lp = tid + p * 256;
    jx[p] = tx * TX + lp % TX;
    jy[p] = ty * TY + (lp / TX) % TY;
    jz[p] = tz * TZ + lp / (TX * TY);
  }
  T acc[PPT][5];
#pragma unroll
  for (int p = 0; p < PPT; ++p)
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[p][c] = 0;
  const int beg = a.tile_off[tile], end = a.tile_off[tile + 1];
  const double hD = (D == 2) ? g.h * g.h : g.h * g.h * g.h;
  for (int c0 = beg; c0 < end; c0 += kCH) {
    const int cnt = (end - c0) < kCH ? (end - c0) : kCH;
    if (tid < cnt) {
      const int m = a.list[c0 + tid];
      for (int d = 0; d < 3; ++d) {
        s_s[tid][d] = a.s[m * 3 + d];
        double w[8];
        w[0] = 0.0;
        w[7] = 0.0;
        const double fr = a.f[m * 3 + d];
        for (int t = 0; t < 6; ++t) w[t + 1] = (d < D) ? phi_eval(a.kernel, (double)(t - 2) - fr) : 0.0;
        for (int t = 0; t < 6; ++t) {
          s_w[tid][d][t] = (T)w[t + 1];
          s_g[tid][d][t] = (T)((w[t + 2] - w[t]) / (2.0 * g.h));
        }
      }
      const double base = a.ds[m] / hD;
      double cf[5] = {0, 0, 0, 0, 0};
      if (a.mode == SP_PLAIN) {
        for (int c = 0; c < a.nf; ++c) cf[c] = a.q[(int64_t)m * a.nf + c] * base;
      } else if (a.mode == SP_FDDIV || a.mode == SP_SCALAR_VEC) {
        const double qm = a.q[m];
        for (int d = 0; d < D; ++d) cf[d] = qm * a.nrm[(int64_t)m * D + d] * base;
        const double mass = a.mass ? (a.eta * qm + (a.m ? a.m[m] : 0.0)) * base : 0.0;
        cf[a.mode == SP_FDDIV ? 3 : D] = mass;
      } else {  // SP_STOKES (2-D)
        const double q1 = a.q[2 * (int64_t)m], q2 = a.q[2 * (int64_t)m + 1];
        const double n1 = a.nrm[2 * (int64_t)m], n2 = a.nrm[2 * (int64_t)m + 1];
        cf[0] = 2.0 * q1 * n1 * base;
        cf[1] = (q1 * n2 + q2 * n1) * base;
        cf[2] = 2.0 * q2 * n2 * base;
        cf[3] = a.eta * q1 * base;
        cf[4] = a.eta * q2 * base;
      }
      for (int c = 0; c < 5; ++c) s_c[tid][c] = (T)cf[c];
    }
    __syncthreads();
    for (int k = 0; k < cnt; ++k) {
      const int sx = s_s[k][0], sy = s_s[k][1], sz = s_s[k][2];
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        const int ox = (jx[p] - sx) & (g.n[0] - 1);
        const int oy = (jy[p] - sy) & (g.n[1] - 1);
        const int oz = (D == 3) ? ((jz[p] - sz) & (g.n[2] - 1)) : 0;
        if (ox < 6 && oy < 6 && oz < 6) {
          const T wx = s_w[k][0][ox], wy = s_w[k][1][oy];
          const T wz = (D == 3) ? s_w[k][2][oz] : (T)1;
          if (a.mode == SP_FDDIV) {
            const T gx = s_g[k][0][ox], gy = s_g[k][1][oy];
            T v = s_c[k][0] * gx * wy * wz + s_c[k][1] * wx * gy * wz + s_c[k][3] * wx * wy * wz;
            if (D == 3) v += s_c[k][2] * wx * wy * s_g[k][2][oz];
            acc[p][0] += v;
          } else {
            const T w = wx * wy * wz;
#pragma unroll
            for (int c = 0; c < 5; ++c)
              if (c < a.nf) acc[p][c] += s_c[k][c] * w;
          }
        }
      }
    }
    __syncthreads();
  }
  const int64_t ntot = (int64_t)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    if (jx[p] < g.n[0] && jy[p] < g.n[1] && (D == 2 || jz[p] < g.n[2])) {
      const int64_t idx = ((int64_t)jz[p] * g.n[1] + jy[p]) * g.n[0] + jx[p];
      for (int c = 0; c < a.nf; ++c) out[c * ntot + idx] = acc[p][c];
    }
  }
}

// ------------------------------------------------------------------ interpolation
template <typename T, int D, int K>
__global__ __launch_bounds__(256) void k_interp(InterpArgs a, const T* __restrict__ u, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_ib) return;
  const MarkerGeom& g = a.g;
  constexpr int T0 = (K == 4) ? 1 : 0;
  T w[3][K];
  int ix[3][K];
  for (int d = 0; d < 3; ++d) {
    const double fr = a.f[i * 3 + d];
    const int s = a.s[i * 3 + d];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      w[d][t] = (d < D) ? (T)phi_eval(a.kernel, (double)(t + T0 - 2) - fr) : (T)(t == 0);
      ix[d][t] = (d < D) ? ((s + t + T0) & (g.n[d] - 1)) : 0;
    }
  }
  const int64_t ntot = (int64_t)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
  for (int c = 0; c < a.nf; ++c) {
    const T* uc = u + c * ntot;
    T acc = 0;
    constexpr int KZ = (D == 3) ? K : 1;
#pragma unroll
    for (int tz = 0; tz < KZ; ++tz) {
#pragma unroll
      for (int ty = 0; ty < K; ++ty) {
        const T wyz = w[1][ty] * (D == 3 ? w[2][tz] : (T)1);
        const int64_t row = ((int64_t)(D == 3 ? ix[2][tz] : 0) * g.n[1] + ix[1][ty]) * g.n[0];
        T rs = 0;
#pragma unroll
        for (int tx = 0; tx < K; ++tx) rs += uc[row + ix[0][tx]] * w[0][tx];
        acc += rs * wyz;
      }
    }
    double v = a.a * (double)acc;
    if (a.x) v += a.b * a.x[i * a.nf + c];
    if (a.ub) v += a.ub[c];
    out[i * a.nf + c] = v;
  }
}

// ------------------------------------------------------------------ grid elementwise
template <typename T>
__global__ void k_axpby(T* __restrict__ y, double a, const T* __restrict__ x, double b, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (T)(a * (double)x[e] + b * (double)y[e]);
}

template <typename T>
__global__ void k_add_const(T* __restrict__ y, const double* __restrict__ cdev, int ncomp, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ncomp; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (T)((double)y[e] + cdev[e / n]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_grid_partial(const T* __restrict__ x, int64_t n, int nblk,
                                                      double* __restrict__ partial) {
  __shared__ double red[256];
  const int comp = blockIdx.y;
  const T* xc = x + comp * n;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)nblk * 256) s += (double)xc[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[comp * nblk + blockIdx.x] = red[0];
}

__global__ void k_partial_final(const double* __restrict__ partial, int nblk, double scale, double* __restrict__ out) {
  const int comp = blockIdx.x;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[comp * nblk + b];
    out[comp] = s * scale;
  }
}

inline unsigned grid_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

}  // namespace

void markers_setup(const MarkerGeom& g, int64_t n_ib, const double* X, int* s, double* f, int* tile_count,
                   hipStream_t st) {
  const int64_t ntile = (int64_t)g.ntile[0] * g.ntile[1] * g.ntile[2];
  IBDL_HIP(hipMemsetAsync(tile_count, 0, sizeof(int) * ntile, st));
  if (n_ib > 0)
    hipLaunchKernelGGL(k_marker_setup, dim3((unsigned)((n_ib + 255) / 256)), dim3(256), 0, st, g, n_ib, X, s, f,
                       tile_count);
  IBDL_LAUNCH_CHECK();
}

void markers_bin(const MarkerGeom& g, int64_t n_ib, const int* s, const int* tile_count, int* tile_off,
                 int* tile_cur, int* list, int* list_tmp, hipStream_t st) {
  const int ntile = g.ntile[0] * g.ntile[1] * g.ntile[2];
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, tile_count, tile_off, ntile);
  IBDL_LAUNCH_CHECK();
  IBDL_HIP(hipMemsetAsync(tile_cur, 0, sizeof(int) * ntile, st));
  if (n_ib > 0)
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n_ib + 255) / 256)), dim3(256), 0, st, g, n_ib, s, tile_off,
                       tile_cur, list_tmp);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sort_tiles, dim3(ntile), dim3(256), 0, st, tile_off, list_tmp, list);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void spread(const SpreadArgs& a, T* out, hipStream_t st) {
  const int ntile = a.g.ntile[0] * a.g.ntile[1] * a.g.ntile[2];
  if (a.g.dim == 2)
    hipLaunchKernelGGL((k_spread<T, 2>), dim3(ntile), dim3(256), 0, st, a, out);
  else
    hipLaunchKernelGGL((k_spread<T, 3>), dim3(ntile), dim3(256), 0, st, a, out);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void interp(const InterpArgs& a, const T* u, double* out, hipStream_t st) {
  if (a.n_ib == 0) return;
  const dim3 grid((unsigned)((a.n_ib + 255) / 256));
  const bool six = a.kernel == KID_BSPLINE6;
  if (a.g.dim == 2) {
    if (six) hipLaunchKernelGGL((k_interp<T, 2, 6>), grid, dim3(256), 0, st, a, u, out);
    else hipLaunchKernelGGL((k_interp<T, 2, 4>), grid, dim3(256), 0, st, a, u, out);
  } else {
    if (six) hipLaunchKernelGGL((k_interp<T, 3, 6>), grid, dim3(256), 0, st, a, u, out);
    else hipLaunchKernelGGL((k_interp<T, 3, 4>), grid, dim3(256), 0, st, a, u, out);
  }
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void grid_axpby(T* y, double a, const T* x, double b, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_axpby<T>), dim3(grid_blocks(n)), dim3(256), 0, st, y, a, x, b, n);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void grid_add_const(T* y, const double* c_dev, int ncomp, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_add_const<T>), dim3(grid_blocks(n * ncomp)), dim3(256), 0, st, y, c_dev, ncomp, n);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void grid_sum(const T* x, int ncomp, int64_t n, double* partial, int nblk, double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_grid_partial<T>), dim3(nblk, ncomp), dim3(256), 0, st, x, n, nblk, partial);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_partial_final, dim3(ncomp), dim3(64), 0, st, partial, nblk, 1.0, out);
  IBDL_LAUNCH_CHECK();
}

#define IBDL_IB_INST(T)                                                                   \
  template void spread<T>(const SpreadArgs&, T*, hipStream_t);                            \
  template void interp<T>(const InterpArgs&, const T*, double*, hipStream_t);             \
  template void grid_axpby<T>(T*, double, const T*, double, int64_t, hipStream_t);        \
  template void grid_add_const<T>(T*, const double*, int, int64_t, hipStream_t);          \
  template void grid_sum<T>(const T*, int, int64_t, double*, int, double*, hipStream_t);
IBDL_IB_INST(float)
IBDL_IB_INST(double)

}  // namespace ibdl
