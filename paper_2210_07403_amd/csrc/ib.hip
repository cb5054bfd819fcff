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

// d phi / d r, the derivative of each piece in |r| times the sign of r
__device__ __forceinline__ double dphi_eval(int kernel, double r) {
  const double a = fabs(r), sg = r < 0.0 ? -1.0 : 1.0;
  double v = 0.0;
  if (kernel == KID_PESKIN4) {
    if (a <= 1.0) v = (-2.0 + (4.0 - 8.0 * a) / (2.0 * sqrt(1.0 + 4.0 * a - 4.0 * a * a))) * 0.125;
    else if (a < 2.0) v = (-2.0 - (12.0 - 8.0 * a) / (2.0 * sqrt(fmax(-7.0 + 12.0 * a - 4.0 * a * a, 1e-300)))) * 0.125;
    return sg * v;
  }
  if (kernel == KID_COS4) return a < 2.0 ? -0.125 * M_PI * sinpi(0.5 * r) : 0.0;
  if (a <= 1.0) v = -a + a * a * a - 5.0 * a * a * a * a / 12.0;
  else if (a <= 2.0) v = 5.0 / 8.0 - 7.0 * a / 2.0 + 15.0 * a * a / 4.0 - 3.0 * a * a * a / 2.0 + 5.0 * a * a * a * a / 24.0;
  else if (a < 3.0) v = -27.0 / 8.0 + 9.0 * a / 2.0 - 9.0 * a * a / 4.0 + a * a * a / 2.0 - a * a * a * a / 24.0;
  return sg * v;
}

// ------------------------------------------------------------------ marker setup and binning
// Tiles met by a marker's 6-node window along each axis: tile indices j0 .. j0 + cnt - 1 (mod ntile).
__device__ __forceinline__ void marker_tiles(const MarkerGeom& g, const int* s, int (&j0)[3], int (&cnt)[3]) {
  for (int d = 0; d < 3; ++d) {
    if (d < g.dim) {
      j0[d] = s[d] / g.tile[d];
      cnt[d] = (s[d] + 5) / g.tile[d] - j0[d] + 1;
      if (cnt[d] > g.ntile[d]) cnt[d] = g.ntile[d];
    } else {
      j0[d] = 0;
      cnt[d] = 1;
    }
  }
}

__device__ __forceinline__ int tile_id(const MarkerGeom& g, const int (&j0)[3], int a, int b, int c) {
  const int tz = (j0[2] + a) % g.ntile[2], ty = (j0[1] + b) % g.ntile[1], tx = (j0[0] + c) % g.ntile[0];
  return (tz * g.ntile[1] + ty) * g.ntile[0] + tx;
}

__global__ void k_marker_setup(MarkerGeom g, int kernel, int64_t n_ib, const double* __restrict__ X,
                               int* __restrict__ s, double* __restrict__ f, double* __restrict__ wt,
                               int* __restrict__ tile_count, const int* __restrict__ pid) {
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
  // kernel weights W[t] = phi((s + t) - X/h) on the 6-node window and centred differences
  // G[t] = (W[t+1] - W[t-1]) / 2h (W = 0 outside the window), per axis; unit weight off-dimension
  for (int d = 0; d < 3; ++d) {
    double w[8];
    w[0] = w[7] = 0.0;
    for (int t = 0; t < 6; ++t)
      w[t + 1] = d < g.dim ? phi_eval(kernel, (double)(t - 2) - f[i * 3 + d]) : (t == 2 ? 1.0 : 0.0);
    double* row = wt + (i * 3 + d) * 12;
    for (int t = 0; t < 6; ++t) {
      row[t] = w[t + 1];
      row[6 + t] = d < g.dim ? (w[t + 2] - w[t]) * (0.5 / g.h) : 0.0;
    }
  }
  int j0[3], nt[3];
  marker_tiles(g, si, j0, nt);
  const int toff = pid ? pid[i] * g.ntile[0] * g.ntile[1] * g.ntile[2] : 0;   // tiles of problem pid[i]
  for (int a = 0; a < nt[2]; ++a)
    for (int b = 0; b < nt[1]; ++b)
      for (int c = 0; c < nt[0]; ++c) atomicAdd(&tile_count[toff + tile_id(g, j0, a, b, c)], 1);
}

__global__ void k_fill(MarkerGeom g, int64_t n_ib, const int* __restrict__ s, const int* __restrict__ off,
                       int* __restrict__ cur, int* __restrict__ list, const int* __restrict__ pid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ib) return;
  int si[3] = {s[i * 3], s[i * 3 + 1], s[i * 3 + 2]};
  int j0[3], nt[3];
  marker_tiles(g, si, j0, nt);
  const int toff = pid ? pid[i] * g.ntile[0] * g.ntile[1] * g.ntile[2] : 0;
  for (int a = 0; a < nt[2]; ++a)
    for (int b = 0; b < nt[1]; ++b)
      for (int c = 0; c < nt[0]; ++c) {
        const int id = toff + tile_id(g, j0, a, b, c);
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

// per-precision weight table: (W[t], G[t]) pairs, t < 6, padded with zeros at t = 6, 7
template <typename T>
__global__ void k_wtab(const double* __restrict__ wt, int64_t n_ib, cplx<T>* __restrict__ tab) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (marker, axis, tap)
  if (e >= n_ib * 24) return;
  const int64_t r = e >> 3;
  const int t = (int)(e & 7);
  tab[e] = t < 6 ? mk<cplx<T>>((T)wt[r * 12 + t], (T)wt[r * 12 + 6 + t]) : mk<cplx<T>>((T)0, (T)0);
}

// busy tiles along x of each listed row as a bit mask: bit t >> seg_group_log2 for tile (t, strip of
// the row), t < ntx
__global__ void k_row_segments(MarkerGeom g, const int* __restrict__ tile_off, const int* __restrict__ rows,
                               int64_t nact, unsigned long long* __restrict__ seg) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nact) return;
  const int w = rows ? rows[r] : (int)r, y = w % g.n[1], z = w / g.n[1];
  // z counts planes, or problems of a batch in 2-D (tile[2] = 1 there): tiles are numbered
  // problem-major, so the strip index runs on across a batch's problems
  const int64_t strip = y / g.tile[1] + (int64_t)g.ntile[1] * (z / g.tile[2]);
  const int gs = seg_group_log2(g);
  unsigned long long m = 0;
  for (int t = 0; t < g.ntile[0]; ++t) {
    const int64_t id = strip * g.ntile[0] + t;
    if (tile_off[id + 1] > tile_off[id]) m |= 1ull << (t >> gs);
  }
  seg[r] = m;
}

// ids of the tiles with at least one candidate, in increasing order (off is the exclusive scan of
// the 0/1 flags computed by k_busy_flags)
__global__ void k_busy_flags(const int* __restrict__ cnt, int* __restrict__ flag, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = cnt[i] > 0 ? 1 : 0;
}
__global__ void k_busy_ids(const int* __restrict__ cnt, const int* __restrict__ foff, const int* __restrict__ off,
                           int4* __restrict__ busy, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && cnt[i] > 0) busy[foff[i]] = make_int4(i, off[i], off[i + 1], 0);
}

// The busy tiles in decreasing order of their candidate count (ties by tile id): the spread's
// workgroups then start with the longest tiles and end with the shortest, which evens out the
// CUs' finishing times.  Rank sort; *nptr = number of busy tiles.
// groups: the tiles (in tile-id order, i.e. in slabs) are first cut into the 8 XCD-contiguous
// ranges of xcd_chunk, and each range is ordered on its own, so that a spread reading entry
// xcd_chunk(b, n) gives each XCD one slab of neighbouring tiles, longest first; their markers'
// data then stay in that XCD's L2.
__device__ __forceinline__ int xcd_range_lo(int x, int n) {   // first index of XCD range x of [0, n)
  const int q = n / 8, r = n % 8;
  return x * q + (x < r ? x : r);
}
__global__ __launch_bounds__(256) void k_busy_order(const int4* __restrict__ in, const int* __restrict__ nptr,
                                                    int4* __restrict__ out, int groups) {
  __shared__ int sc[256];
  const int n = *nptr;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int4 v = i < n ? in[i] : make_int4(0, 0, 0, 0);
  const int c = v.z - v.y;
  int lo = 0, hi = n;
  if (groups) {
    const int q = n / 8, r = n % 8;
    const int x = i < r * (q + 1) ? i / (q + 1) : r + (q > 0 ? (i - r * (q + 1)) / q : 0);
    lo = xcd_range_lo(x, n);
    hi = xcd_range_lo(x + 1, n);
  }
  int rk = 0;
  for (int k0 = 0; k0 < n; k0 += 256) {
    __syncthreads();
    if (k0 + (int)threadIdx.x < n) {
      const int4 u = in[k0 + threadIdx.x];
      sc[threadIdx.x] = u.z - u.y;
    }
    __syncthreads();
    const int kn = n - k0 < 256 ? n - k0 : 256;
    for (int k = 0; k < kn; ++k) {
      const int ck = sc[k];
      const int kk = k0 + k;
      rk += (kk >= lo && kk < hi) && ((ck > c) || (ck == c && kk < i));
    }
  }
  if (i < n) out[lo + rk] = v;
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
// Owner-computes spread with the candidate list of a tile split over the 4 waves of a workgroup:
// wave w accumulates candidates w, w+4, w+8, ... of the (sorted) list in registers, and the four
// partial sums are added in wave order at the end, so the result is deterministic.  The loader
// thread of each candidate evaluates the kernel weights W and the centred-difference weights G
// at the tile's own node positions (zero outside the marker's window), so the accumulation loop
// is branch-free and reads a handful of packed LDS vectors per candidate.
constexpr int kT3X = 16, kT3Y = 4, kT3Z = 8;   // 3-D tile; lane (x, y) owns a z-column of 8
constexpr int kT2X = 16, kT2Y = 16;            // 2-D tile; lane (x, y-group) owns 4 consecutive y

template <typename T> struct Pack4;
template <> struct Pack4<float> { using type = float4; };
template <> struct Pack4<double> { using type = double4; };

// per-marker coefficients of the spread fields (times ds / h^D)
__device__ __forceinline__ void spread_coefs(const SpreadArgs& a, int m, int D, double base, double* cf) {
  for (int c = 0; c < 8; ++c) cf[c] = 0.0;
  if (a.mode == SP_PLAIN) {
    for (int c = 0; c < 5; ++c)
      if (c < a.nf) cf[c] = a.q[(int64_t)m * a.nf + c] * base;
  } else if (a.mode == SP_STOKES) {
    const double q1 = a.q[2 * (int64_t)m], q2 = a.q[2 * (int64_t)m + 1];
    const double n1 = a.nrm[2 * (int64_t)m], n2 = a.nrm[2 * (int64_t)m + 1];
    cf[0] = 2.0 * q1 * n1 * base;
    cf[1] = (q1 * n2 + q2 * n1) * base;
    cf[2] = 2.0 * q2 * n2 * base;
    cf[3] = a.eta * q1 * base;
    cf[4] = a.eta * q2 * base;
  } else {  // SP_FDDIV: c_d = q n_d, mass in slot 3; SP_SCALAR_VEC: c_d = q n_d, mass in slot D
    const double qm = a.q[m];
    for (int d = 0; d < 3; ++d)
      if (d < D) cf[d] = qm * a.nrm[(int64_t)m * D + d] * base;
    const double mass = a.mass ? (a.eta * qm + (a.m ? a.m[m] : 0.0)) * base : 0.0;
    cf[a.mode == SP_FDDIV ? 3 : D] = mass;
  }
}

// coefficient c of marker m: the value spread_coefs leaves in cf[c] (3-D modes)
__device__ __forceinline__ double spread_coef(const SpreadArgs& a, int m, int D, double base, int c) {
  if (a.mode == SP_PLAIN) return c < a.nf ? a.q[(int64_t)m * a.nf + c] * base : 0.0;
  const double qm = a.q[m];
  if (c < D) return qm * a.nrm[(int64_t)m * D + c] * base;
  if (c == (a.mode == SP_FDDIV ? 3 : D)) return a.mass ? (a.eta * qm + (a.m ? a.m[m] : 0.0)) * base : 0.0;
  return 0.0;
}


// Lanes used per wave for candidates in one pass (LDS budget: 32 KiB / 48 KiB per block).
template <typename T> constexpr int spread_lanes() { return sizeof(T) == 4 ? 64 : 32; }

// broadcast a lane's value to the whole wave (scalar register), any 32/64-bit type
template <typename T> __device__ __forceinline__ T bcast(T v, int lane) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
  } else {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __builtin_bit_cast(T, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
  }
}

// ------------------------------------------------------------------ 3-D spread on the matrix cores
// A tile's spread is a sum of rank-1 tensor products, i.e. a matrix product
//   out[(y,z), x] = sum_k P[(y,z), k] Q[k, x],   k = (candidate, term),
// with Q a kernel row along x and P the matching (y,z) factor.  Finite-difference dipole field:
//   term 0: P = c_x W_y W_z,                          Q = G_x
//   term 1: P = c_y G_y W_z + c_z W_y G_z + c_m W_y W_z,  Q = W_x
// other modes (field c): P = cf_c W_y W_z, Q = W_x.  The 16 x 4 x 8 tile is two 16 x 16 blocks of
// (y,z) rows against 16 x columns; v_mfma_{f32,f64}_16x16x4 adds four k per instruction.  Operand
// layout (both precisions): lane l supplies P[l % 16][l / 16] and Q[l / 16][l % 16]; result row
// 4 (l / 16) + v (f32) or l / 16 + 4 v (f64), column l % 16.  The four waves take K-steps round
// robin and their partial tiles are added in wave order, so the result is deterministic.
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

constexpr int kSpreadWaves = 4, kSpreadCands = 64;   // launch shape of the 3-D spread
// NW waves per tile (64 NW threads) share the K-steps; SC candidates are staged per pass, four
// lanes each

template <typename T, int NF, bool FD, int NW, int SC>
__global__ __launch_bounds__(64 * NW) void k_spread3m(SpreadArgs a, const cplx<T>* __restrict__ wtab,
                                                      T* __restrict__ out) {
  using T2 = cplx<T>;
  using M = Mfma<T>;
  constexpr int kSC = SC, NTH = 64 * NW;
  constexpr int PER = (kSC * 4 + NTH - 1) / NTH;     // staging items (candidate, quarter) per thread
  constexpr int NC = FD ? 4 : NF;                    // coefficients per candidate
  constexpr int STAGE = kSC * 24 * (int)sizeof(T2) + kSC * NC * (int)sizeof(T) + kSC * 4 * (int)sizeof(int);
  constexpr int RED = NW * 512 * (int)sizeof(T);     // one field's wave partials
  __shared__ __align__(16) unsigned char smem[STAGE > RED ? STAGE : RED];
  T2(*s_w)[24] = reinterpret_cast<T2(*)[24]>(smem);                       // marker weight rows
  T(*s_c)[NC] = reinterpret_cast<T(*)[NC]>(smem + kSC * 24 * sizeof(T2));  // coefficients
  int(*s_o)[4] = reinterpret_cast<int(*)[4]>(smem + kSC * 24 * sizeof(T2) + kSC * NC * sizeof(T));
  const MarkerGeom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int4 bt = a.busy[a.xcd ? xcd_chunk((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x];
  const int tile = bt.x;
  const int ntl = g.ntile[0] * g.ntile[1] * g.ntile[2];
  const int prob = tile / ntl, tl = tile - prob * ntl;
  const int tx = tl % g.ntile[0];
  const int ty = (tl / g.ntile[0]) % g.ntile[1];
  const int tz = tl / (g.ntile[0] * g.ntile[1]);
  const int x0 = tx * kT3X, y0 = ty * kT3Y, z0 = tz * kT3Z;
  const double hD = g.h * g.h * g.h;
  const int mx = g.n[0] - 1, my = g.n[1] - 1, mz = g.n[2] - 1;
  typename M::v4 acc[NF][2];
#pragma unroll
  for (int c = 0; c < NF; ++c) acc[c][0] = acc[c][1] = typename M::v4{0, 0, 0, 0};
  const int beg = bt.y, end = bt.z;
  constexpr int NT = FD ? 2 : 1, CPS = 4 / NT;       // terms per candidate, candidates per K-step
  const int kk = lane >> 4, i16 = lane & 15;
  const int yy = i16 & 3, zz = i16 >> 2;
  // staging: four lanes per candidate (lane quarter p loads window offset p < 3, forms the field
  // coefficients p, p + 4, ... and loads entries 6p .. 6p + 5 of the weight row), all loads of a
  // pass issued at once;
  // the next pass's marker ids are fetched while the current pass accumulates
  int m_next[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int scand = (tid + p * NTH) >> 2;
    m_next[p] = (scand < kSC && scand < end - beg) ? a.list[beg + scand] : -1;
  }
  for (int c0 = beg; c0 < end; c0 += kSC) {
    const int cnt = end - c0 < kSC ? end - c0 : kSC;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int it = tid + p * NTH, scand = it >> 2, part = it & 3;
      if (scand >= kSC) break;
      const int m = m_next[p];
      const bool live = m >= 0;
      const int mm = live ? m : 0;   // padding candidates read marker 0 and store zeros
      const T2* wrow = wtab + (int64_t)mm * 24 + 6 * part;
      T2 w6[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) w6[i] = wrow[i];
      const int o = a.s[mm * 3 + (part < 3 ? part : 0)];
      const double base = a.raw ? 1.0 : a.ds[mm] / hD;
      T cv[(NC + 3) / 4];
#pragma unroll
      for (int j = 0; j < (NC + 3) / 4; ++j)
        cv[j] = (part + 4 * j < NC) ? (T)spread_coef(a, mm, 3, base, part + 4 * j) : (T)0;
      m_next[p] = (c0 + kSC + scand < end) ? a.list[c0 + kSC + scand] : -1;
#pragma unroll
      for (int i = 0; i < 6; ++i) s_w[scand][6 * part + i] = live ? w6[i] : mk<T2>((T)0, (T)0);
      if (part < 3) s_o[scand][part] = live ? o : 6;
#pragma unroll
      for (int j = 0; j < (NC + 3) / 4; ++j)
        if (part + 4 * j < NC) s_c[scand][part + 4 * j] = live ? cv[j] : (T)0;
    }
    __syncthreads();
    const int nsteps = (cnt + CPS - 1) / CPS;
    for (int st = wave; st < nsteps; st += NW) {
      const int cand = st * CPS + kk / NT;
      // tile node -> window tap (6 and 7 hold zeros)
      const int tx_ = min((x0 + i16 - s_o[cand][0]) & mx, 6);
      const int ty_ = min((y0 + yy - s_o[cand][1]) & my, 6);
      const int tza = min((z0 + zz - s_o[cand][2]) & mz, 6);
      const int tzb = min((z0 + zz + 4 - s_o[cand][2]) & mz, 6);
      const T2 xv = s_w[cand][tx_], yv = s_w[cand][8 + ty_];
      const T2 za = s_w[cand][16 + tza], zb = s_w[cand][16 + tzb];
      if constexpr (FD) {
        const bool t0 = (kk & 1) == 0;
        const T cx = s_c[cand][0], cy = s_c[cand][1], cz = s_c[cand][2], cm = s_c[cand][3];
        const T q = t0 ? xv.y : xv.x;
        const T pyz = cy * yv.y + cm * yv.x, wy = yv.x;
        const T pa = t0 ? cx * wy * za.x : pyz * za.x + cz * wy * za.y;
        const T pb = t0 ? cx * wy * zb.x : pyz * zb.x + cz * wy * zb.y;
        acc[0][0] = M::mma(pa, q, acc[0][0]);
        acc[0][1] = M::mma(pb, q, acc[0][1]);
      } else {
        const T q = xv.x, wa = yv.x * za.x, wb = yv.x * zb.x;
#pragma unroll
        for (int c = 0; c < NF; ++c) {
          if (c < a.nf) {
            const T cf = s_c[cand][c];
            acc[c][0] = M::mma(cf * wa, q, acc[c][0]);
            acc[c][1] = M::mma(cf * wb, q, acc[c][1]);
          }
        }
      }
    }
    __syncthreads();
  }
  // fixed-order sum of the waves' partial tiles, field by field
  T* red = reinterpret_cast<T*>(smem);   // [wave][block][v][lane]
  const int64_t ntot = (int64_t)g.n[0] * g.n[1] * g.n[2];
  out += (int64_t)prob * a.nf * ntot;
#pragma unroll
  for (int c = 0; c < NF; ++c) {
    if (c >= a.nf) break;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[((wave * 2 + b) * 4 + v) * 64 + lane] = acc[c][b][v];
    __syncthreads();
    for (int o = tid; o < 512; o += NTH) {
      const int b = o >> 8, v = (o >> 6) & 3, l = o & 63;
      T val = red[(b * 4 + v) * 64 + l];
#pragma unroll
      for (int w = 1; w < NW; ++w) val += red[((w * 2 + b) * 4 + v) * 64 + l];
      const int i = M::row(l, v);          // (y, z) row within the block
      const int x = l & 15, y = i & 3, z = (i >> 2) + 4 * b;
      out[c * ntot + ((int64_t)(z0 + z) * g.n[1] + (y0 + y)) * g.n[0] + x0 + x] = val;
    }
    __syncthreads();
  }
}

// The finite-difference dipole field (one output field) with the candidates' weights resolved at
// the tile's own nodes once per pass.  Each candidate's record holds G_x and W_x at the 16 x columns
// (the Q operand of terms 0 and 1) and the (W, G) pairs of its 4 y rows and 8 z planes, zero outside
// its window; the four staging lanes of a candidate fill seven of these 28 positions each, reading
// the taps the window offsets in lofs select.  A K-step then takes its operands' factors from the
// record directly: term 0 P = (c_x W_y) W_z, term 1 P = (c_y G_y + c_m W_y) W_z + (c_z W_y) G_z.
// Same products and accumulation order as k_spread3m.
template <typename T, int NW, int SC>
__global__ __launch_bounds__(64 * NW, 8) void k_spread3f(SpreadArgs a, const cplx<T>* __restrict__ wtab,
                                                      T* __restrict__ out) {
  using T2 = cplx<T>;
  using M = Mfma<T>;
  constexpr int NTH = 64 * NW;
  constexpr int PER = (SC * 4 + NTH - 1) / NTH;      // staging items (candidate, quarter) per thread
  constexpr int RS = 56;                             // record: G_x[16], W_x[16], y (W, G)[4], z (W, G)[8]
  constexpr int STAGE = SC * (RS + 4) * (int)sizeof(T);
  constexpr int RED = NW * 512 * (int)sizeof(T);
  __shared__ __align__(16) unsigned char smem[STAGE > RED ? STAGE : RED];
  T* s_r = reinterpret_cast<T*>(smem);
  T(*s_c)[4] = reinterpret_cast<T(*)[4]>(smem + SC * RS * sizeof(T));   // c_x, c_y, c_z, c_m
  const MarkerGeom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int4 bt = a.busy[a.xcd ? xcd_chunk((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x];
  const int tile = bt.x;
  const int ntl = g.ntile[0] * g.ntile[1] * g.ntile[2];
  const int prob = tile / ntl, tl = tile - prob * ntl;
  const int tx = tl % g.ntile[0];
  const int ty = (tl / g.ntile[0]) % g.ntile[1];
  const int tz = tl / (g.ntile[0] * g.ntile[1]);
  const int x0 = tx * kT3X, y0 = ty * kT3Y, z0 = tz * kT3Z;
  const double hD = g.h * g.h * g.h;
  const int mx = g.n[0] - 1, my = g.n[1] - 1, mz = g.n[2] - 1;
  typename M::v4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  const int beg = bt.y, end = bt.z;
  const int i16 = lane & 15, yy = i16 & 3, zz = i16 >> 2;
  const bool t0 = ((lane >> 4) & 1) == 0;            // term of this lane's k column
  const int qoff = (t0 ? 0 : 16) + i16;
  int m_next[PER], o_next[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int scand = (tid + p * NTH) >> 2;
    const bool in = scand < SC && scand < end - beg;
    m_next[p] = in ? a.list[beg + scand] : -1;
    o_next[p] = in ? a.lofs[beg + scand] : 0;
  }
  for (int c0 = beg; c0 < end; c0 += SC) {
    const int cnt = end - c0 < SC ? end - c0 : SC;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int it = tid + p * NTH, scand = it >> 2, part = it & 3;
      if (scand >= SC) break;
      const int m = m_next[p], d = o_next[p];
      const bool live = m >= 0;
      const int mm = live ? m : 0;   // padding candidates read marker 0 and store zeros
      // lane quarter p resolves x columns p, p + 4, p + 8, p + 12, y row p and z planes p, p + 4; the
      // weight row is read at 32-bit byte offsets from the launch-uniform table
      const unsigned wrow = (unsigned)mm * 24u * (unsigned)sizeof(T2);
      const int dx = d & 1023, dy = (d >> 10) & 1023, dz = (d >> 20) & 1023;
      unsigned slot[7];
#pragma unroll
      for (int i = 0; i < 4; ++i) slot[i] = (unsigned)((part + 4 * i - dx) & mx);
      slot[4] = (unsigned)((part - dy) & my);
      slot[5] = (unsigned)((part - dz) & mz);
      slot[6] = (unsigned)((part + 4 - dz) & mz);
      T2 e[7];
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        const unsigned base = i < 4 ? 0u : (i == 4 ? 8u : 16u);
        const unsigned sl = base + (slot[i] < 6u ? slot[i] : 6u);   // taps 6 and 7 of a row are zero
        e[i] = *reinterpret_cast<const T2*>(reinterpret_cast<const char*>(wtab) + (wrow + sl * (unsigned)sizeof(T2)));
      }
      const T cv = (T)spread_coef(a, mm, 3, a.raw ? 1.0 : a.ds[mm] / hD, part);
      const bool more = c0 + SC + scand < end;
      m_next[p] = more ? a.list[c0 + SC + scand] : -1;
      o_next[p] = more ? a.lofs[c0 + SC + scand] : 0;
      T* r = s_r + scand * RS;
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        const T w = live ? e[i].x : (T)0, gd = live ? e[i].y : (T)0;
        if (i < 4) {            // x column: G_x (term 0), W_x (term 1)
          r[part + 4 * i] = gd;
          r[16 + part + 4 * i] = w;
        } else {                // y row / z plane: (W, G)
          const int o = i == 4 ? 32 + 2 * part : (i == 5 ? 40 + 2 * part : 48 + 2 * part);
          r[o] = w;
          r[o + 1] = gd;
        }
      }
      s_c[scand][part] = live ? cv : (T)0;
    }
    __syncthreads();
    const int nsteps = (cnt + 1) >> 1;
    for (int st = wave; st < nsteps; st += NW) {
      const int cand = 2 * st + (lane >> 5);
      const T* r = s_r + cand * RS;
      const T q = r[qoff];
      const T2 yv = *reinterpret_cast<const T2*>(r + 32 + 2 * yy);
      const T2 za = *reinterpret_cast<const T2*>(r + 40 + 2 * zz);
      const T2 zb = *reinterpret_cast<const T2*>(r + 48 + 2 * zz);
      const T cx = s_c[cand][0], cy = s_c[cand][1], cz = s_c[cand][2], cm = s_c[cand][3];
      const T u = t0 ? cx * yv.x : cy * yv.y + cm * yv.x;
      const T v = t0 ? (T)0 : cz * yv.x;
      acc0 = M::mma(u * za.x + v * za.y, q, acc0);
      acc1 = M::mma(u * zb.x + v * zb.y, q, acc1);
    }
    __syncthreads();
  }
  // fixed-order sum of the waves' partial tiles
  T* red = reinterpret_cast<T*>(smem);   // [wave][block][v][lane]
  const int64_t ntot = (int64_t)g.n[0] * g.n[1] * g.n[2];
  out += (int64_t)prob * ntot;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    red[((wave * 2 + 0) * 4 + v) * 64 + lane] = acc0[v];
    red[((wave * 2 + 1) * 4 + v) * 64 + lane] = acc1[v];
  }
  __syncthreads();
  for (int o = tid; o < 512; o += NTH) {
    const int b = o >> 8, v = (o >> 6) & 3, l = o & 63;
    T val = red[(b * 4 + v) * 64 + l];
#pragma unroll
    for (int w = 1; w < NW; ++w) val += red[((w * 2 + b) * 4 + v) * 64 + l];
    const int i = M::row(l, v);
    const int x = l & 15, y = i & 3, z = (i >> 2) + 4 * b;
    out[((int64_t)(z0 + z) * g.n[1] + (y0 + y)) * g.n[0] + x0 + x] = val;
  }
}

// 2-D: a tile of TX x TY nodes (TX TY = 256, TY = 4 (64 / TX) rows); lane (x, y-group) owns
// y = 4 yg + j' (j' < 4); the owning lane of a candidate writes its x row and its tile-aligned y
// column (TY pairs) to LDS; coefficients and the x window start are broadcast.  s_x and s_y are the
// caller's LDS: [4][LW][8] and [4][LW][TY] (T, T) pairs.
template <typename T, int NF, int TX>
__device__ __forceinline__ void spread2_tile(const SpreadArgs& a, const cplx<T>* __restrict__ wtab, T* __restrict__ out,
                                             const int4 bt, cplx<T> (*s_x)[spread_lanes<T>()][8], cplx<T>* s_yraw) {
  using T2 = cplx<T>;
  constexpr int LW = spread_lanes<T>();
  constexpr int TY = 256 / TX;
  static_assert(TX * TY == 256 && TX >= 4 && TX <= 64, "2-D tile of 256 nodes, 64 lanes of 4 rows");
  auto s_y = reinterpret_cast<T2 (*)[LW][TY]>(s_yraw);
  const MarkerGeom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tile = bt.x;
  const int ntl = g.ntile[0] * g.ntile[1];
  const int prob = tile / ntl, tl = tile - prob * ntl;
  const int tx = tl % g.ntile[0];
  const int ty = tl / g.ntile[0];
  const int x0 = tx * TX, y0 = ty * TY;
  const int lx = lane % TX, yg = lane / TX;
  const int mx = g.n[0] - 1, my = g.n[1] - 1;
  const bool fddiv = NF == 1 && a.mode == SP_FDDIV;
  T acc[4][NF];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int c = 0; c < NF; ++c) acc[j][c] = 0;
  const int beg = bt.y, end = bt.z;
  const double hD = g.h * g.h;
  for (int c0 = beg; c0 < end; c0 += 4 * LW) {
    const int left = end - c0 - wave;
    const int cnt = left <= 0 ? 0 : ((left + 3) / 4 < LW ? (left + 3) / 4 : LW);
    int sx = 0;
    T cf[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) cf[c] = 0;
    if (lane < cnt) {
      const int m = a.list[c0 + 4 * lane + wave];
      const T2* row = wtab + (int64_t)m * 24;
#pragma unroll
      for (int t = 0; t < 8; ++t) s_x[wave][lane][t] = row[t];
      sx = a.s[m * 3 + 0];
      const int sy = a.s[m * 3 + 1];
#pragma unroll
      for (int y = 0; y < TY; ++y) s_y[wave][lane][y] = row[8 + min((y0 + y - sy) & my, 6)];
      double c8[8];
      spread_coefs(a, m, 2, a.raw ? 1.0 : a.ds[m] / hD, c8);
#pragma unroll
      for (int c = 0; c < 5; ++c) cf[c] = (T)c8[c];
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const int bx = bcast(sx, j);
      const T2 xv = s_x[wave][j][min((x0 + lx - bx) & mx, 6)];
      T2 yv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) yv[q] = s_y[wave][j][4 * yg + q];
      if (fddiv) {
        // v = c_x G_x W_y + c_y W_x G_y + c_mass W_x W_y
        const T ax = bcast(cf[0], j) * xv.y + bcast(cf[3], j) * xv.x, ay = bcast(cf[1], j) * xv.x;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q][0] += ax * yv[q].x + ay * yv[q].y;
      } else {
#pragma unroll
        for (int c = 0; c < NF; ++c) {
          if (c < a.nf) {
            const T cx = bcast(cf[c], j) * xv.x;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q][c] += cx * yv[q].x;
          }
        }
      }
    }
    __syncthreads();
  }
  T* red = reinterpret_cast<T*>(s_yraw);   // needs 4 * 4 * 64 values: [4][LW][TY] pairs hold them
  const int64_t ntot = (int64_t)g.n[0] * g.n[1];
  out += (int64_t)prob * a.nf * ntot;
#pragma unroll
  for (int c = 0; c < NF; ++c) {
    if (c >= a.nf) break;
#pragma unroll
    for (int q = 0; q < 4; ++q) red[(wave * 4 + q) * 64 + lane] = acc[q][c];
    __syncthreads();
    {
      const int o = tid;                // 256 tile nodes, one per thread
      const int q = o >> 6, l = o & 63; // l: (x, y-group), q: y within the group
      const T v = ((red[(0 * 4 + q) * 64 + l] + red[(1 * 4 + q) * 64 + l]) + red[(2 * 4 + q) * 64 + l]) +
                  red[(3 * 4 + q) * 64 + l];
      const int x = l % TX, y = 4 * (l / TX) + q;
      out[c * ntot + (int64_t)(y0 + y) * g.n[0] + x0 + x] = v;
    }
    __syncthreads();
  }
}

template <typename T, int NF>
__global__ __launch_bounds__(256) void k_spread2(SpreadArgs a, const cplx<T>* __restrict__ wtab, T* __restrict__ out) {
  constexpr int LW = spread_lanes<T>();
  __shared__ cplx<T> s_x[4][LW][8];
  __shared__ cplx<T> s_y[4 * LW * kT2Y];
  spread2_tile<T, NF, kT2X>(a, wtab, out, a.busy[blockIdx.x], s_x, s_y);
}

// The spread of several grid groups (a batch) in one persistent launch over a single work list,
// items[k] = (group, busy-tile index), ordered by decreasing candidate count across all groups:
// workgroup b takes items b, b + G, b + 2 G, ... (G workgroups), so the longest tiles go first and
// every workgroup ends with short ones.  (A shared atomic counter was measured slower: 4,500 tiles
// serialise on one address.)  Each group has its own arguments, weight table, output fields and
// tile width (16, 32 or 64 nodes along x); its densities are qbase + qoff.
template <typename T>
__global__ __launch_bounds__(256) void k_spread2_queue(const SpreadGroup* __restrict__ gd, const int2* __restrict__ items,
                                                       int nitems, const double* __restrict__ qbase) {
  constexpr int LW = spread_lanes<T>();
  __shared__ cplx<T> s_x[4][LW][8];
  __shared__ cplx<T> s_y[4 * LW * 16];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 gi = items[it];
    const int gsel = __builtin_amdgcn_readfirstlane(gi.x);
    SpreadArgs a = gd[gsel].a;
    a.q = qbase + gd[gsel].qoff;
    const int4 bt = a.busy[gi.y];
    const cplx<T>* wt = reinterpret_cast<const cplx<T>*>(gd[gsel].wtab);
    T* out = reinterpret_cast<T*>(gd[gsel].out);
    const int tw = gd[gsel].tx;
    if (tw == 32) spread2_tile<T, 1, 32>(a, wt, out, bt, s_x, s_y);
    else if (tw == 64) spread2_tile<T, 1, 64>(a, wt, out, bt, s_x, s_y);
    else spread2_tile<T, 1, 16>(a, wt, out, bt, s_x, s_y);
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
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double* row = a.wt + (i * 3 + d) * 12;
    const int s = a.s[i * 3 + d];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      w[d][t] = (d < D) ? (T)row[t + T0] : (T)(t == 0);
      ix[d][t] = (d < D) ? ((s + t + T0) & (g.n[d] - 1)) : 0;
    }
  }
  const int64_t ntot = (int64_t)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
  if (a.pid) u += (int64_t)a.pid[i] * a.nf * ntot;
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

// 4-point kernels: a group of RL = 4^(D-1) lanes per marker, lane r of the group sums the 4 x-taps of
// stencil row r; the row sums are reduced across the group by a fixed butterfly (deterministic).
template <typename T, int D>
__global__ __launch_bounds__(256) void k_interp4(InterpArgs a, const cplx<T>* __restrict__ wtab, const T* __restrict__ u,
                                                 double* __restrict__ out) {
  constexpr int RL = (D == 3) ? 16 : 4;
  // XCD-contiguous marker ranges: markers close in index share grid lines, so they share an L2
  const int64_t gid = (int64_t)xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t i = gid / RL;
  const int r = (int)(gid % RL);
  const bool valid = i < a.n_ib;
  const int64_t im = valid ? i : 0;
  const MarkerGeom& g = a.g;
  const cplx<T>* row = wtab + im * 24;       // axis d taps at row[d*8 + t], t = 1..4 non-zero
  const int sx = a.s[im * 3 + 0], sy = a.s[im * 3 + 1], sz = a.s[im * 3 + 2];
  const int ty = r & 3, tz = r >> 2;         // stencil row (y tap, z tap)
  const T wyz = row[8 + 1 + ty].x * (D == 3 ? row[16 + 1 + tz].x : (T)1);
  const int64_t base = ((int64_t)(D == 3 ? ((sz + 1 + tz) & (g.n[2] - 1)) : 0) * g.n[1] +
                        ((sy + 1 + ty) & (g.n[1] - 1))) * g.n[0];
  int ix[4];
  T wx[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    ix[t] = (sx + 1 + t) & (g.n[0] - 1);
    wx[t] = row[1 + t].x;
  }
  const int64_t ntot = (int64_t)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
  if (a.pid) u += (int64_t)a.pid[im] * a.nf * ntot;
  for (int c = 0; c < a.nf; ++c) {
    const T* uc = u + c * ntot + base;
    T v = ((uc[ix[0]] * wx[0] + uc[ix[1]] * wx[1]) + uc[ix[2]] * wx[2] + uc[ix[3]] * wx[3]) * wyz;
#pragma unroll
    for (int off = 1; off < RL; off <<= 1) v += __shfl_xor(v, off, RL);
    if (valid && r == 0) {
      double o = a.a * (double)v;
      if (a.x) o += a.b * a.x[i * a.nf + c];
      if (a.ub) o += a.ub[c];
      out[i * a.nf + c] = o;
    }
  }
}

// The interpolation (4-point kernels, 2-D) of several grid groups in one launch: marker i of the
// concatenation belongs to the group g with m0[g] <= i < m0[g + 1] (gd[g].m0); it reads that group's
// fields and weight table and writes out[i] = a S*u + b x[i] (one field per marker).
template <typename T>
__global__ __launch_bounds__(256) void k_interp4_groups(const InterpGroup* __restrict__ gd, int ng, int64_t ntot_m,
                                                        const double* __restrict__ xbase, double* __restrict__ out) {
  constexpr int RL = 4;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = gid / RL;
  const int r = (int)(gid % RL);
  const bool valid = i < ntot_m;
  const int64_t ic = valid ? i : 0;
  int gsel = 0;
  while (gsel + 1 < ng && ic >= gd[gsel + 1].m0) ++gsel;
  const InterpGroup& G = gd[gsel];
  const MarkerGeom& g = G.a.g;
  const int64_t im = ic - G.m0;
  const cplx<T>* row = reinterpret_cast<const cplx<T>*>(G.wtab) + im * 24;
  const int sx = G.a.s[im * 3 + 0], sy = G.a.s[im * 3 + 1];
  const int ty = r & 3;
  const T wyz = row[8 + 1 + ty].x;
  const int64_t base = (int64_t)((sy + 1 + ty) & (g.n[1] - 1)) * g.n[0];
  int ix[4];
  T wx[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    ix[t] = (sx + 1 + t) & (g.n[0] - 1);
    wx[t] = row[1 + t].x;
  }
  const int64_t ntot = (int64_t)g.n[0] * g.n[1];
  const T* uc = reinterpret_cast<const T*>(G.u) + (int64_t)G.a.pid[im] * ntot + base;
  T v = ((uc[ix[0]] * wx[0] + uc[ix[1]] * wx[1]) + uc[ix[2]] * wx[2] + uc[ix[3]] * wx[3]) * wyz;
#pragma unroll
  for (int off = 1; off < RL; off <<= 1) v += __shfl_xor(v, off, RL);
  if (valid && r == 0) {
    double o = G.a.a * (double)v;
    if (xbase) o += G.a.b * xbase[i];
    out[i] = o;
  }
}

// Transpose of the fused FD divergence spread (SP_FDDIV), for the scalar transposed operator with
// centred differences.  Per marker, over the 6-node window (G_d spans all 6 taps, W the inner 4),
//   v_i = sum_y w(y) [sum_d n_id G_d(y) prod_{e != d} W_e(y) + eta prod_e W_e(y)]
// and, since Phi D_d = -(the G_d-weighted interpolation) when D_d is the centred difference,
//   y_i = -h^-D ds_i v_i + b p_i + eta ds_i pu        (p = a.x, b = a.b; pu: the ubar entries or null)
// which equals h^-D ds_i (sum_d n_id Phi D_d w - eta Phi w) + b p_i + eta ds_i pu.
// 3-D: 32 lanes per marker, one per (y, z) stencil row of the 6 x 6 window less its 4 corners
// (W_y and W_z both vanish there); 2-D: 8 lanes, the first 6 one per y row.  Each lane reads the 6
// x taps of its row against A G_x + B W_x; the row sums are reduced by a fixed butterfly.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_interp_div(InterpArgs a, const cplx<T>* __restrict__ wtab,
                                                    const T* __restrict__ u, const double* __restrict__ nrm,
                                                    const double* __restrict__ ds, double eta, double hDinv,
                                                    const double* __restrict__ pu, double* __restrict__ y) {
  constexpr int RL = (D == 3) ? 32 : 8;
  const int64_t gid = (int64_t)xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t i = gid / RL;
  const int r = (int)(gid % RL);
  const bool valid = i < a.n_ib;
  const int64_t im = valid ? i : 0;
  const MarkerGeom& g = a.g;
  const cplx<T>* row = wtab + im * 24;       // axis d taps at row[d*8 + t], t < 6
  int ty = r, tz = 0;
  if (D == 3) {
    const int k = r + 1 + (r >= 4 ? 1 : 0) + (r >= 28 ? 1 : 0);   // skips k = 0, 5, 30, 35
    ty = k % 6;
    tz = k / 6;
  }
  const bool live = D == 3 || r < 6;
  const cplx<T> py = row[8 + (live ? ty : 0)];
  const cplx<T> pz = D == 3 ? row[16 + tz] : mk<cplx<T>>((T)1, (T)0);
  const T n0 = (T)nrm[im * D], n1 = (T)nrm[im * D + 1], n2 = D == 3 ? (T)nrm[im * D + 2] : (T)0;
  const T A = n0 * py.x * pz.x;
  const T B = n1 * py.y * pz.x + n2 * py.x * pz.y + (T)eta * py.x * pz.x;
  const int sx = a.s[im * 3 + 0], sy = a.s[im * 3 + 1], sz = a.s[im * 3 + 2];
  const int64_t base = ((int64_t)(D == 3 ? ((sz + tz) & (g.n[2] - 1)) : 0) * g.n[1] + ((sy + ty) & (g.n[1] - 1))) *
                       g.n[0];
  T v = 0;
  if (live) {
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const cplx<T> px = row[t];
      v += u[base + ((sx + t) & (g.n[0] - 1))] * (A * px.y + B * px.x);
    }
  }
#pragma unroll
  for (int off = 1; off < RL; off <<= 1) v += __shfl_xor(v, off, RL);
  if (valid && r == 0) {
    double o = -hDinv * ds[i] * (double)v;
    if (a.x) o += a.b * a.x[i];
    if (pu) o += eta * ds[i] * pu[0];
    y[i] = o;
  }
}

// ------------------------------------------------------------------ active rows
// Rows y of plane z that a marker's 6-node window meets: [s_y, s_y + 5] for z in [s_z, s_z + 5]
// (mod n); a window that wraps around y marks the whole plane.
__global__ void k_rows_init(int* __restrict__ lo, int* __restrict__ hi, int nplanes, int ny) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z < nplanes) {
    lo[z] = ny;
    hi[z] = -1;
  }
}

// per-block limits in LDS first (many markers share a plane), then one global update per touched plane
__global__ __launch_bounds__(256) void k_rows_mark(MarkerGeom g, int64_t n_ib, const int* __restrict__ s,
                                                   int* __restrict__ lo, int* __restrict__ hi) {
  extern __shared__ int sm[];
  const int ny = g.n[1];
  const int nz = g.dim == 3 ? g.n[2] : 1;
  int* slo = sm;
  int* shi = sm + nz;
  for (int z = threadIdx.x; z < nz; z += blockDim.x) {
    slo[z] = ny;
    shi[z] = -1;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_ib) {
    const int sy = s[i * 3 + 1];
    const int ylo = sy + 5 < ny ? sy : 0;
    const int yhi = sy + 5 < ny ? sy + 5 : ny - 1;
    const int nw = g.dim == 3 ? 6 : 1;
    for (int t = 0; t < nw; ++t) {
      const int z = g.dim == 3 ? (s[i * 3 + 2] + t) & (nz - 1) : 0;
      atomicMin(&slo[z], ylo);
      atomicMax(&shi[z], yhi);
    }
  }
  __syncthreads();
  for (int z = threadIdx.x; z < nz; z += blockDim.x) {
    if (shi[z] >= 0) {
      atomicMin(&lo[z], slo[z]);
      atomicMax(&hi[z], shi[z]);
    }
  }
}

// per-plane row counts, the (lo, hi) pairs used by the y-pass masks, and then the row list
__global__ void k_rows_count(const int* __restrict__ lo, const int* __restrict__ hi, int nplanes,
                             int* __restrict__ cnt, int2* __restrict__ lim) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nplanes) return;
  const bool any = hi[z] >= lo[z];
  cnt[z] = any ? hi[z] - lo[z] + 1 : 0;
  lim[z] = any ? make_int2(lo[z], hi[z]) : make_int2(1, 0);
}

__global__ void k_rows_list(const int* __restrict__ lo, const int* __restrict__ cnt, const int* __restrict__ off,
                            int nplanes, int ny, int* __restrict__ rows) {
  const int z = blockIdx.x;
  if (z >= nplanes) return;
  for (int k = threadIdx.x; k < cnt[z]; k += blockDim.x) rows[off[z] + k] = z * ny + lo[z] + k;
}


// ------------------------------------------------------------------ kernel-derivative gather
// One thread per marker over its K^D window (K = 4: taps 1..4 of the 6-node window; K = 6: all),
// in double: out[i][e] = sum_x F_i(x) (-phi'(r_e)/h) prod_{d != e} phi(r_d), r_d = (x_d - X_id)/h.
template <typename T, int D, int K>
__global__ __launch_bounds__(256) void k_gather_dx(GatherArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_ib) return;
  const MarkerGeom& g = a.g;
  constexpr int T0 = (K == 4) ? 1 : 0;
  double w[3][K], dw[3][K];
  int ix[3][K];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int s = a.s[i * 3 + d];
    const double fr = a.f[i * 3 + d];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const double r = (double)(t + T0 - 2) - fr;
      w[d][t] = d < D ? phi_eval(a.kernel, r) : (t == 0 ? 1.0 : 0.0);
      dw[d][t] = d < D ? -dphi_eval(a.kernel, r) / g.h : 0.0;
      ix[d][t] = d < D ? ((s + t + T0) & (g.n[d] - 1)) : 0;
    }
  }
  double cf[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) cf[k] = k < a.nfield ? a.coef[i * a.nfield + k] : 0.0;
  double acc[3] = {0.0, 0.0, 0.0};
  constexpr int KZ = (D == 3) ? K : 1;
  for (int tz = 0; tz < KZ; ++tz) {
    for (int ty = 0; ty < K; ++ty) {
      const int64_t row = ((int64_t)(D == 3 ? ix[2][tz] : 0) * g.n[1] + ix[1][ty]) * g.n[0];
      const double wz = D == 3 ? w[2][tz] : 1.0, dwz = D == 3 ? dw[2][tz] : 0.0;
      for (int tx = 0; tx < K; ++tx) {
        const int64_t idx = row + ix[0][tx];
        double F = 0.0;
        for (int k = 0; k < a.nfield; ++k) F += cf[k] * (double)static_cast<const T*>(a.field[k])[idx];
        acc[0] += F * dw[0][tx] * w[1][ty] * wz;
        acc[1] += F * w[0][tx] * dw[1][ty] * wz;
        if (D == 3) acc[2] += F * w[0][tx] * w[1][ty] * dwz;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < D; ++e) a.out[i * D + e] = acc[e];
}

// ------------------------------------------------------------------ grid elementwise
template <typename T>
__global__ void k_axpby(T* __restrict__ y, double a, const T* __restrict__ x, double b, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (T)(a * (double)x[e] + b * (double)y[e]);
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ x, D* __restrict__ y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (D)x[e];
}

template <typename T>
__global__ void k_fill(T* __restrict__ y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (T)0;
}

// flag |= 1 when x holds a NaN or an infinity
template <typename T>
__global__ void k_nonfinite(const T* __restrict__ x, int64_t n, unsigned* __restrict__ flag) {
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    bad = bad || !isfinite(x[e]);
  if (bad) atomicOr(flag, 1u);
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

void markers_setup(const MarkerGeom& g, int kernel, int64_t n_ib, const double* X, int* s, double* f, double* wt,
                   int* tile_count, hipStream_t st, const int* pid, int nprob) {
  const int64_t ntile = (int64_t)g.ntile[0] * g.ntile[1] * g.ntile[2] * nprob;
  IBDL_HIP(hipMemsetAsync(tile_count, 0, sizeof(int) * ntile, st));
  if (n_ib > 0)
    hipLaunchKernelGGL(k_marker_setup, dim3((unsigned)((n_ib + 255) / 256)), dim3(256), 0, st, g, kernel, n_ib, X,
                       s, f, wt, tile_count, pid);
  IBDL_LAUNCH_CHECK();
}

// one workgroup per busy tile: the window starts of its candidates relative to the tile's first node
__global__ __launch_bounds__(256) void k_list_offsets(MarkerGeom g, const int4* __restrict__ busy,
                                                      const int* __restrict__ list, const int* __restrict__ s,
                                                      int* __restrict__ lofs) {
  const int4 bt = busy[blockIdx.x];
  const int tl = bt.x % (g.ntile[0] * g.ntile[1] * g.ntile[2]);
  const int o0 = (tl % g.ntile[0]) * g.tile[0];
  const int o1 = ((tl / g.ntile[0]) % g.ntile[1]) * g.tile[1];
  const int o2 = (tl / (g.ntile[0] * g.ntile[1])) * g.tile[2];
  for (int i = bt.y + (int)threadIdx.x; i < bt.z; i += (int)blockDim.x) {
    const int m = list[i];
    const int d0 = (s[3 * m] - o0) & (g.n[0] - 1), d1 = (s[3 * m + 1] - o1) & (g.n[1] - 1);
    const int d2 = (s[3 * m + 2] - o2) & (g.n[2] - 1);
    lofs[i] = d0 | (d1 << 10) | (d2 << 20);
  }
}

void markers_list_offsets(const MarkerGeom& g, const int4* busy, int nbusy, const int* list, const int* s, int* lofs,
                          hipStream_t st) {
  if (g.dim != 3) throw Error(-1, "list offsets: 3-D grids only");
  if (g.n[0] > 1024 || g.n[1] > 1024 || g.n[2] > 1024) throw Error(-1, "list offsets: axes of at most 1024 nodes");
  if (nbusy <= 0) return;
  hipLaunchKernelGGL(k_list_offsets, dim3((unsigned)nbusy), dim3(256), 0, st, g, busy, list, s, lofs);
  IBDL_LAUNCH_CHECK();
}

void markers_bin(const MarkerGeom& g, int64_t n_ib, const int* s, const int* tile_count, int* tile_off,
                 int* tile_cur, int* list, int* list_tmp, int4* busy, int4* busy_tmp, int* busy_off, hipStream_t st,
                 const int* pid, int nprob, int xcd_groups) {
  const int ntile = g.ntile[0] * g.ntile[1] * g.ntile[2] * nprob;
  hipLaunchKernelGGL(k_busy_flags, dim3((ntile + 255) / 256), dim3(256), 0, st, tile_count, tile_cur, ntile);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, tile_cur, busy_off, ntile);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, tile_count, tile_off, ntile);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_busy_ids, dim3((ntile + 255) / 256), dim3(256), 0, st, tile_count, busy_off, tile_off,
                     busy_tmp, ntile);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_busy_order, dim3((ntile + 255) / 256), dim3(256), 0, st, busy_tmp, busy_off + ntile, busy,
                     xcd_groups);
  IBDL_LAUNCH_CHECK();
  IBDL_HIP(hipMemsetAsync(tile_cur, 0, sizeof(int) * ntile, st));
  if (n_ib > 0)
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n_ib + 255) / 256)), dim3(256), 0, st, g, n_ib, s, tile_off,
                       tile_cur, list_tmp, pid);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sort_tiles, dim3(ntile), dim3(256), 0, st, tile_off, list_tmp, list);
  IBDL_LAUNCH_CHECK();
}

void exclusive_scan(const int* cnt, int* off, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, cnt, off, n);
  IBDL_LAUNCH_CHECK();
}

void markers_row_segments(const MarkerGeom& g, const int* tile_off, const int* rows, int64_t nact,
                          unsigned long long* seg, hipStream_t st) {
  if (nact <= 0) return;
  hipLaunchKernelGGL(k_row_segments, dim3((unsigned)((nact + 255) / 256)), dim3(256), 0, st, g, tile_off, rows, nact,
                     seg);
  IBDL_LAUNCH_CHECK();
}

void markers_rows(const MarkerGeom& g, int64_t n_ib, const int* s, int* lo, int* hi, int* cnt, int* off, int2* lim,
                  int* rows, hipStream_t st) {
  const int nplanes = g.dim == 3 ? g.n[2] : 1;
  hipLaunchKernelGGL(k_rows_init, dim3((nplanes + 255) / 256), dim3(256), 0, st, lo, hi, nplanes, g.n[1]);
  IBDL_LAUNCH_CHECK();
  if (n_ib > 0)
    hipLaunchKernelGGL(k_rows_mark, dim3((unsigned)((n_ib + 255) / 256)), dim3(256), sizeof(int) * 2 * nplanes, st,
                       g, n_ib, s, lo, hi);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_rows_count, dim3((nplanes + 255) / 256), dim3(256), 0, st, lo, hi, nplanes, cnt, lim);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, cnt, off, nplanes);
  IBDL_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_rows_list, dim3(nplanes), dim3(256), 0, st, lo, cnt, off, nplanes, g.n[1], rows);
  IBDL_LAUNCH_CHECK();
}


template <typename T>
void grid_fill_zero(T* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_blocks(n)), dim3(256), 0, st, y, n);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void nonfinite_flag(const T* x, int64_t n, unsigned* flag, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_nonfinite<T>), dim3(grid_blocks(n)), dim3(256), 0, st, x, n, flag);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void spread(const SpreadArgs& a, const cplx<T>* wtab, T* out, hipStream_t st) {
  // nodes outside the non-empty tiles are not written: the caller clears the fields first
  if (a.nbusy == 0) return;
  const bool one = a.nf == 1;
  if (a.g.dim == 2) {
    if (one) hipLaunchKernelGGL((k_spread2<T, 1>), dim3(a.nbusy), dim3(256), 0, st, a, wtab, out);
    else hipLaunchKernelGGL((k_spread2<T, 5>), dim3(a.nbusy), dim3(256), 0, st, a, wtab, out);
  } else {
    if (a.mode == SP_STOKES) throw Error(-1, "3-D spread: the Stokes mode is two-dimensional");
    constexpr int NW = kSpreadWaves, SC = kSpreadCands;
    if (one && a.mode == SP_FDDIV && a.lofs)
      hipLaunchKernelGGL((k_spread3f<T, NW, SC>), dim3(a.nbusy), dim3(64 * NW), 0, st, a, wtab, out);
    else if (one && a.mode == SP_FDDIV)
      hipLaunchKernelGGL((k_spread3m<T, 1, true, NW, SC>), dim3(a.nbusy), dim3(64 * NW), 0, st, a, wtab, out);
    else if (one)
      hipLaunchKernelGGL((k_spread3m<T, 1, false, NW, SC>), dim3(a.nbusy), dim3(64 * NW), 0, st, a, wtab, out);
    else
      hipLaunchKernelGGL((k_spread3m<T, 5, false, NW, SC>), dim3(a.nbusy), dim3(64 * NW), 0, st, a, wtab, out);
  }
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void spread2_queue(const SpreadGroup* gd, const int2* items, int nitems, const double* qbase, int nblocks,
                   hipStream_t st) {
  if (nitems <= 0) return;
  const int nb = nblocks > 0 ? (nblocks < nitems ? nblocks : nitems) : nitems;
  hipLaunchKernelGGL((k_spread2_queue<T>), dim3((unsigned)nb), dim3(256), 0, st, gd, items, nitems, qbase);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void interp4_groups(const InterpGroup* gd, int ng, int64_t ntot_m, const double* xbase, double* out, hipStream_t st) {
  if (ntot_m <= 0) return;
  const int64_t lanes = ntot_m * 4;
  hipLaunchKernelGGL((k_interp4_groups<T>), dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st, gd, ng, ntot_m,
                     xbase, out);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void weight_table(const double* wt, int64_t n_ib, cplx<T>* tab, hipStream_t st) {
  const int64_t n = n_ib * 24;
  if (n > 0) hipLaunchKernelGGL((k_wtab<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, wt, n_ib, tab);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void interp(const InterpArgs& a, const cplx<T>* wtab, const T* u, double* out, hipStream_t st) {
  if (a.n_ib == 0) return;
  const bool six = a.kernel == KID_BSPLINE6;
  if (six) {
    const dim3 grid((unsigned)((a.n_ib + 255) / 256));
    if (a.g.dim == 2) hipLaunchKernelGGL((k_interp<T, 2, 6>), grid, dim3(256), 0, st, a, u, out);
    else hipLaunchKernelGGL((k_interp<T, 3, 6>), grid, dim3(256), 0, st, a, u, out);
  } else {
    const int64_t lanes = a.n_ib * (a.g.dim == 3 ? 16 : 4);
    const dim3 grid((unsigned)((lanes + 255) / 256));
    if (a.g.dim == 2) hipLaunchKernelGGL((k_interp4<T, 2>), grid, dim3(256), 0, st, a, wtab, u, out);
    else hipLaunchKernelGGL((k_interp4<T, 3>), grid, dim3(256), 0, st, a, wtab, u, out);
  }
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void interp_div(const InterpArgs& a, const cplx<T>* wtab, const T* u, const double* nrm, const double* ds, double eta,
                double hDinv, const double* pu, double* y, hipStream_t st) {
  if (a.n_ib == 0) return;
  if (a.kernel == KID_BSPLINE6) throw Error(-2, "interp_div: 4-point kernels only");
  const int64_t lanes = a.n_ib * (a.g.dim == 3 ? 32 : 8);
  const dim3 grid((unsigned)((lanes + 255) / 256));
  if (a.g.dim == 2)
    hipLaunchKernelGGL((k_interp_div<T, 2>), grid, dim3(256), 0, st, a, wtab, u, nrm, ds, eta, hDinv, pu, y);
  else hipLaunchKernelGGL((k_interp_div<T, 3>), grid, dim3(256), 0, st, a, wtab, u, nrm, ds, eta, hDinv, pu, y);
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void gather_dx(const GatherArgs& a, hipStream_t st) {
  if (a.n_ib == 0) return;
  if (a.nfield < 1 || a.nfield > 8) throw Error(-1, "gather_dx: 1..8 fields");
  const dim3 grid((unsigned)((a.n_ib + 255) / 256));
  const bool six = a.kernel == KID_BSPLINE6;
  if (a.g.dim == 2) {
    if (six) hipLaunchKernelGGL((k_gather_dx<T, 2, 6>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_gather_dx<T, 2, 4>), grid, dim3(256), 0, st, a);
  } else {
    if (six) hipLaunchKernelGGL((k_gather_dx<T, 3, 6>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_gather_dx<T, 3, 4>), grid, dim3(256), 0, st, a);
  }
  IBDL_LAUNCH_CHECK();
}

void grid_widen(const float* x, double* y, int64_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_blocks(n)), dim3(256), 0, st, x, y, n);
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
  template void spread<T>(const SpreadArgs&, const cplx<T>*, T*, hipStream_t);            \
  template void weight_table<T>(const double*, int64_t, cplx<T>*, hipStream_t);           \
  template void grid_fill_zero<T>(T*, int64_t, hipStream_t);                              \
  template void nonfinite_flag<T>(const T*, int64_t, unsigned*, hipStream_t);             \
  template void interp<T>(const InterpArgs&, const cplx<T>*, const T*, double*, hipStream_t); \
  template void interp_div<T>(const InterpArgs&, const cplx<T>*, const T*, const double*, const double*, double, \
                              double, const double*, double*, hipStream_t);                \
  template void grid_axpby<T>(T*, double, const T*, double, int64_t, hipStream_t);        \
  template void gather_dx<T>(const GatherArgs&, hipStream_t);                             \
  template void grid_add_const<T>(T*, const double*, int, int64_t, hipStream_t);          \
  template void grid_sum<T>(const T*, int, int64_t, double*, int, double*, hipStream_t);  \
  template void spread2_queue<T>(const SpreadGroup*, const int2*, int, const double*, int, hipStream_t); \
  template void interp4_groups<T>(const InterpGroup*, int, int64_t, const double*, double*, hipStream_t);
IBDL_IB_INST(float)
IBDL_IB_INST(double)

}  // namespace ibdl
