// Indicator function and near-boundary interpolation (2-D), Sec. 5.3.3 (interpolation for
// near-boundary points) and Sec. 5.3.4 (flagging interior and exterior points).
//
// The indicator's grid solve runs through the FFT pipeline (ibdl.hip); here are its last step
// (shift to 0 at the corner node, threshold at 1/2) and the kernels of the interpolation: binning
// the markers into cells, marking the nodes within m1 h of a marker, listing the marked nodes of
// Omega, and the per-node interpolation (three nearest markers by a search of the cells in rings
// around the node, one wave per node).
#include <algorithm>
#include <cmath>

#include "kernels.h"

// No contraction into fused multiply-adds anywhere in this file: node positions, distances and
// the segment parameter are rounded as in a plain evaluation, so that the discrete choices (which
// nodes are near, which markers are nearest, which segment) come out as in the oracle.
#pragma clang fp contract(off)

namespace ibdl {
namespace {

template <typename T>
__global__ void k_indicator_finish(const T* __restrict__ reg_in, int64_t n, T* __restrict__ chi,
                                   T* __restrict__ reg_out) {
  const T corner = reg_in[0];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const T v = reg_in[e] - corner;
    chi[e] = v >= (T)0.5 ? (T)1 : (T)0;
    if (reg_out) reg_out[e] = v;
  }
}

__global__ void k_set(double* __restrict__ x, double v, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    x[e] = v;
}

// squared distance, dx^2 + dy^2
__device__ __forceinline__ double dist2(double px, double py, double qx, double qy) {
  const double dx = px - qx, dy = py - qy;
  const double a = dx * dx, b = dy * dy;
  return a + b;
}

// flag every node within m1 h of marker i (unwrapped node positions; wrapped indices)
__global__ void k_near_mark(const double* __restrict__ X, int64_t n_ib, NearGeom g, double m1,
                            unsigned char* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ib) return;
  const double x = X[2 * i], y = X[2 * i + 1];
  const int R = (int)ceil(m1) + 1;
  const int ix = (int)floor((x - g.ox) / g.h), iy = (int)floor((y - g.oy) / g.h);
  const double r2 = (m1 * g.h) * (m1 * g.h);
  for (int dj = -R; dj <= R + 1; ++dj)
    for (int di = -R; di <= R + 1; ++di) {
      const int jj = iy + dj, ii = ix + di;
      const double px = g.ox + ii * g.h, py = g.oy + jj * g.h;
      if (dist2(px, py, x, y) <= r2) {
        const int wj = ((jj % g.ny) + g.ny) % g.ny, wi = ((ii % g.nx) + g.nx) % g.nx;
        flag[(int64_t)wj * g.nx + wi] = 1;
      }
    }
}

// list the flagged nodes of Omega
template <typename T>
__global__ void k_near_list(const unsigned char* __restrict__ flag, const T* __restrict__ omega, int64_t n,
                            int* __restrict__ count, int* __restrict__ list) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && flag[e] && omega[e] != (T)0) list[atomicAdd(count, 1)] = (int)e;
}

// The true distance to p of the three nearest markers, kept sorted by (distance, index).
struct Near3 {
  double d[3];
  int i[3];
  __device__ void init() {
    for (int k = 0; k < 3; ++k) {
      d[k] = INFINITY;
      i[k] = 0x7fffffff;
    }
  }
  __device__ void push(double dd, int ii) {
    if (dd > d[2] || (dd == d[2] && ii > i[2])) return;
    if (dd < d[1] || (dd == d[1] && ii < i[1])) {
      d[2] = d[1];
      i[2] = i[1];
      if (dd < d[0] || (dd == d[0] && ii < i[0])) {
        d[1] = d[0];
        i[1] = i[0];
        d[0] = dd;
        i[0] = ii;
      } else {
        d[1] = dd;
        i[1] = ii;
      }
    } else {
      d[2] = dd;
      i[2] = ii;
    }
  }
};

// closest point of the segment [x1, x2] to p: x_A = x2 + clamp(t) (x1 - x2); returns unclamped t
__device__ __forceinline__ double seg_param(double px, double py, double x1, double y1, double x2, double y2) {
  const double dx = x1 - x2, dy = y1 - y2;
  const double num = (px - x2) * dx + (py - y2) * dy;
  const double den = dx * dx + dy * dy;
  return num / den;
}

template <typename T>
__device__ double bilinear(const T* __restrict__ u, const NearGeom& g, double bx, double by) {
  const double fx = (bx - g.ox) / g.h, fy = (by - g.oy) / g.h;
  const int i0 = (int)floor(fx), j0 = (int)floor(fy);
  const double ax = fx - i0, ay = fy - j0;
  const int ia = ((i0 % g.nx) + g.nx) % g.nx, ib = (((i0 + 1) % g.nx) + g.nx) % g.nx;
  const int ja = ((j0 % g.ny) + g.ny) % g.ny, jb = (((j0 + 1) % g.ny) + g.ny) % g.ny;
  const double u00 = u[(int64_t)ja * g.nx + ia], u10 = u[(int64_t)ja * g.nx + ib];
  const double u01 = u[(int64_t)jb * g.nx + ia], u11 = u[(int64_t)jb * g.nx + ib];
  return ax * ay * u11 + ay * (1.0 - ax) * u01 + ax * (1.0 - ay) * u10 + (1.0 - ax - ay + ax * ay) * u00;
}

constexpr int kNB = 256;        // threads per block: four waves, one node per wave at a time
constexpr int kNBBlocks = 2048; // grid-stride over the listed nodes

// Markers binned by position into square cells of kCell x kCell grid nodes (cell index clamped to
// the grid, so markers outside the box land in a border cell): counts, then a cursor fill.
constexpr int kCell = 8;

__device__ __forceinline__ int cell_of(double v, double o, double w, int nc) {
  const double c = floor((v - o) / w);
  return c < 0.0 ? 0 : (c >= (double)nc ? nc - 1 : (int)c);
}

__global__ void k_cell_count(const double* __restrict__ X, int64_t n_ib, NearGeom g, int ncx, int ncy,
                             int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ib) return;
  const double w = kCell * g.h;
  atomicAdd(&cnt[cell_of(X[2 * i + 1], g.oy, w, ncy) * ncx + cell_of(X[2 * i], g.ox, w, ncx)], 1);
}

__global__ void k_cell_fill(const double* __restrict__ X, int64_t n_ib, NearGeom g, int ncx, int ncy,
                            int* __restrict__ cur, int* __restrict__ list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ib) return;
  const double w = kCell * g.h;
  list[atomicAdd(&cur[cell_of(X[2 * i + 1], g.oy, w, ncy) * ncx + cell_of(X[2 * i], g.ox, w, ncx)], 1)] = (int)i;
}

// merge the 64 lanes' lists by a butterfly of exchanges (every lane ends with the same three)
__device__ __forceinline__ void merge_wave(Near3& nr) {
  for (int off = 32; off >= 1; off >>= 1) {
    double od[3];
    int oi[3];
    for (int c = 0; c < 3; ++c) {
      od[c] = __shfl_xor(nr.d[c], off, 64);
      oi[c] = __shfl_xor(nr.i[c], off, 64);
    }
    for (int c = 0; c < 3; ++c) nr.push(od[c], oi[c]);
  }
}

// One wave per listed node.  The three nearest markers by (distance, index) are found over the
// marker cells in square rings around the node's cell: the lanes split a ring's cells, each
// keeping its own three nearest, and a butterfly merges them into lane 0's list (the other lanes
// start the next ring empty, so no marker is counted twice).  Every marker of a cell outside rings
// 0..W is more than W kCell h away along one axis, so once the third-nearest distance is at most
// that, no unvisited marker can enter the three; the order is total (indices differ), so the
// result is the three markers a sequential scan of all markers finds.
template <typename T>
__global__ __launch_bounds__(kNB) void k_near_fix(const double* __restrict__ X, const double* __restrict__ Ub,
                                                  int ubs, int64_t n_ib, NearGeom g, double m2, const int* __restrict__ count,
                                                  const int* __restrict__ list, const int* __restrict__ cell_off,
                                                  const int* __restrict__ cell_list, int ncx, int ncy,
                                                  const T* __restrict__ u, T* __restrict__ out) {
  const int n = *count;
  const int lane = threadIdx.x & 63;
  const int nwaves = gridDim.x * (kNB / 64);
  const double2* __restrict__ X2 = reinterpret_cast<const double2*>(X);
  const double cw = kCell * g.h;
  const int wmax = ncx > ncy ? ncx : ncy;
  for (int k = blockIdx.x * (kNB / 64) + (threadIdx.x >> 6); k < n; k += nwaves) {
    const int e = list[k];
    const int pi = e % g.nx, pj = e / g.nx;
    const double px = g.ox + pi * g.h, py = g.oy + pj * g.h;
    const int pcx = cell_of(px, g.ox, cw, ncx), pcy = cell_of(py, g.oy, cw, ncy);
    Near3 nr;
    nr.init();
    for (int W = 0; W <= wmax; ++W) {
      const int ncell = W == 0 ? 1 : 8 * W;   // the ring of cells at Chebyshev distance W
      for (int c = lane; c < ncell; c += 64) {
        int dx, dy;
        if (W == 0) {
          dx = dy = 0;
        } else if (c < 2 * W + 1) {            // bottom row
          dx = c - W;
          dy = -W;
        } else if (c < 4 * W + 2) {            // top row
          dx = c - (2 * W + 1) - W;
          dy = W;
        } else {                               // left and right columns without the corners
          const int r = c - (4 * W + 2);
          dx = (r & 1) ? W : -W;
          dy = -W + 1 + (r >> 1);
        }
        const int cx = pcx + dx, cy = pcy + dy;
        if (cx < 0 || cx >= ncx || cy < 0 || cy >= ncy) continue;
        const int cell = cy * ncx + cx;
        for (int q = cell_off[cell]; q < cell_off[cell + 1]; ++q) {
          const int m = cell_list[q];
          const double2 xm = X2[m];
          nr.push(dist2(px, py, xm.x, xm.y), m);
        }
      }
      merge_wave(nr);
      // a marker outside rings 0..W is more than W cw away (less a margin for the rounding of the
      // cell assignments)
      const double bound = W > 0 ? ((double)W - 1e-6) * cw : 0.0;
      if (W > 0 && nr.d[2] <= bound * bound) break;
      if (lane != 0) nr.init();
    }
    if (lane != 0) continue;
    int a = nr.i[0], b = nr.i[1];
    double t = seg_param(px, py, X[2 * a], X[2 * a + 1], X[2 * b], X[2 * b + 1]);
    if (!(t >= 0.0 && t <= 1.0) && n_ib >= 3) {   // the two of the three nearest markers farthest apart
      const int p3[3][2] = {{nr.i[0], nr.i[1]}, {nr.i[0], nr.i[2]}, {nr.i[1], nr.i[2]}};
      double best = -1.0;
      for (int q = 0; q < 3; ++q) {
        const double s = dist2(X[2 * p3[q][0]], X[2 * p3[q][0] + 1], X[2 * p3[q][1]], X[2 * p3[q][1] + 1]);
        if (s > best) {
          best = s;
          a = p3[q][0];
          b = p3[q][1];
        }
      }
      t = seg_param(px, py, X[2 * a], X[2 * a + 1], X[2 * b], X[2 * b + 1]);
    }
    const double tc = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    const double x1 = X[2 * a], y1 = X[2 * a + 1], x2 = X[2 * b], y2 = X[2 * b + 1];
    const double xa = x2 + tc * (x1 - x2), ya = y2 + tc * (y1 - y2);
    const double l12 = sqrt(dist2(x1, y1, x2, y2));
    const double uA = Ub[(int64_t)a * ubs] * sqrt(dist2(xa, ya, x2, y2)) / l12 +
                      Ub[(int64_t)b * ubs] * sqrt(dist2(xa, ya, x1, y1)) / l12;
    const double dpa = sqrt(dist2(px, py, xa, ya));
    double up = uA;
    if (dpa > 0.0) {
      const double xb = xa + (px - xa) / dpa * (m2 * g.h), yb = ya + (py - ya) / dpa * (m2 * g.h);
      const double uB = bilinear<T>(u, g, xb, yb);
      const double dab = sqrt(dist2(xb, yb, xa, ya));
      up = uA * sqrt(dist2(xb, yb, px, py)) / dab + uB * dpa / dab;
    }
    out[e] = (T)up;
  }
}

}  // namespace

template <typename T>
void indicator_finish(const T* reg_in, int64_t n, T* chi, T* reg_out, hipStream_t st) {
  const int64_t nb = (n + 255) / 256 > 4096 ? 4096 : (n + 255) / 256;
  hipLaunchKernelGGL((k_indicator_finish<T>), dim3((unsigned)nb), dim3(256), 0, st, reg_in, n, chi, reg_out);
  IBDL_LAUNCH_CHECK();
}

void fill_value(double* x, double v, int64_t n, hipStream_t st) {
  const int64_t nb = (n + 255) / 256 > 4096 ? 4096 : ((n + 255) / 256 > 0 ? (n + 255) / 256 : 1);
  hipLaunchKernelGGL(k_set, dim3((unsigned)nb), dim3(256), 0, st, x, v, n);
  IBDL_LAUNCH_CHECK();
}

int64_t near_list_cap(int64_t n_ib, double m1, int64_t npoints) {
  const int64_t R = (int64_t)std::ceil(m1) + 1;
  const int64_t box = (2 * R + 2) * (2 * R + 2);
  return std::min(npoints, n_ib * box);
}

int near_cells(const NearGeom& g, int* ncx, int* ncy) {
  *ncx = std::max(g.nx / kCell, 1);
  *ncy = std::max(g.ny / kCell, 1);
  return *ncx * *ncy;
}

void near_bin(const double* X, int64_t n_ib, const NearGeom& g, int* cell_cnt, int* cell_off, int* cell_list,
              hipStream_t st) {
  int ncx, ncy;
  const int nc = near_cells(g, &ncx, &ncy);
  IBDL_HIP(hipMemsetAsync(cell_cnt, 0, sizeof(int) * nc, st));
  if (n_ib > 0) {
    hipLaunchKernelGGL(k_cell_count, dim3((unsigned)((n_ib + 255) / 256)), dim3(256), 0, st, X, n_ib, g, ncx, ncy,
                       cell_cnt);
    IBDL_LAUNCH_CHECK();
  }
  exclusive_scan(cell_cnt, cell_off, nc, st);
  IBDL_HIP(hipMemcpyAsync(cell_cnt, cell_off, sizeof(int) * nc, hipMemcpyDeviceToDevice, st));   // fill cursors
  if (n_ib > 0) {
    hipLaunchKernelGGL(k_cell_fill, dim3((unsigned)((n_ib + 255) / 256)), dim3(256), 0, st, X, n_ib, g, ncx, ncy,
                       cell_cnt, cell_list);
    IBDL_LAUNCH_CHECK();
  }
}

template <typename T>
void near_boundary(const double* X, const double* Ub, int nc, int64_t n_ib, const NearGeom& g, double m1, double m2,
                   const T* omega, const T* u, T* out, unsigned char* flag, int* count, int* list,
                   const int* cell_off, const int* cell_list, hipStream_t st) {
  int ncx, ncy;
  near_cells(g, &ncx, &ncy);
  const int64_t n = (int64_t)g.nx * g.ny;
  IBDL_HIP(hipMemcpyAsync(out, u, sizeof(T) * n * nc, hipMemcpyDeviceToDevice, st));
  IBDL_HIP(hipMemsetAsync(flag, 0, n, st));
  IBDL_HIP(hipMemsetAsync(count, 0, sizeof(int), st));
  if (n_ib == 0) return;
  hipLaunchKernelGGL(k_near_mark, dim3((unsigned)((n_ib + 255) / 256)), dim3(256), 0, st, X, n_ib, g, m1, flag);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_near_list<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, flag, omega, n, count,
                     list);
  IBDL_LAUNCH_CHECK();
  const int64_t waves = near_list_cap(n_ib, m1, n);
  const int64_t nblk = std::min<int64_t>((waves + kNB / 64 - 1) / (kNB / 64), kNBBlocks);
  for (int c = 0; c < nc; ++c) {   // component c: boundary values Ub[i * nc + c], field c
    hipLaunchKernelGGL((k_near_fix<T>), dim3((unsigned)nblk), dim3(kNB), 0, st, X, Ub + c, nc, n_ib, g, m2, count,
                       list, cell_off, cell_list, ncx, ncy, u + c * n, out + c * n);
    IBDL_LAUNCH_CHECK();
  }
}

#define IBDL_NB_INST(T)                                                                                    \
  template void indicator_finish<T>(const T*, int64_t, T*, T*, hipStream_t);                              \
  template void near_boundary<T>(const double*, const double*, int, int64_t, const NearGeom&, double, double, \
                                 const T*, const T*, T*, unsigned char*, int*, int*, const int*, const int*,    \
                                 hipStream_t);
IBDL_NB_INST(float)
IBDL_NB_INST(double)

}  // namespace ibdl
