// Periodic-grid FFT passes for gfx950 (wave64), hand-written Stockham autosort.
//
// A line of N points is owned by T = N / RMAX threads; thread i holds elements i + s*T
// (s < RMAX) in registers.  Each radix-R stage does R-point DFTs in registers; stages
// exchange through LDS; the first stage reads global memory and the last stage leaves the
// natural-order result in the same register pattern, so a forward and an inverse transform
// chain without an LDS round trip (used by the fused last-axis pass).
//
// Passes:  x axis  real <-> half spectrum, by an N/2-point complex FFT of (x_2n + i x_2n+1)
//                  and the standard even/odd split; rows are staged in LDS with coalesced
//                  cooperative loads and stores.
//          strided in-place C2C along y (3-D middle axis), tiles of W adjacent lines so each
//                  row of the tile is one contiguous segment.
//          fused   last axis: forward FFT of every input field, Fourier multiplier
//                  (screened Poisson / Poisson / Brinkman-Stokes, see mult_coef), inverse FFT of
//                  the output fields, in one kernel: the spectra never go back to HBM.
#include "kernels.h"

namespace ibdl {
namespace {

constexpr int kBlock = 256;
constexpr int kLdsBytes = 65536;
// The single-field line passes (strided, and the fused scalar pass) take up to 512 threads and
// 96 KiB of LDS per workgroup (gfx950 gives a workgroup up to 160 KiB): a tile of 32 lines of 256
// float points, 256-byte segments per row.  The multi-field passes keep 256 threads, which leaves
// their lines the registers they need.
constexpr int kLineBlock = 512;
constexpr int kLineLds = 98304;

// Stockham plan of a length-N line: RMAX elements per thread (the radix of every stage but the last),
// T = N / RMAX threads per line
constexpr int plan_rmax(int N) { return (N <= 16) ? N : ((N == 32 || N == 64 || N == 512) ? 8 : 16); }
template <int N, int RMX = plan_rmax(N)> struct Plan {
  static constexpr int RMAX = RMX;
  static constexpr int T = N / RMAX;
  static constexpr int LR = ilog2c(RMAX);
  static constexpr int NFULL = ilog2c(N) / LR;
  static constexpr int REM = N >> (NFULL * LR);
  static constexpr int NST = NFULL + (REM > 1 ? 1 : 0);
  static constexpr int radix(int s) { return s < NFULL ? RMAX : REM; }
  static constexpr int pw(int s) { return 1 << (s * LR); }
};

__host__ __device__ constexpr double c16(int m) {
  return m == 0 ? 1.0 : m == 1 ? 0.92387953251128675613 : m == 2 ? 0.70710678118654752440
       : m == 3 ? 0.38268343236508977173 : m == 4 ? 0.0 : m == 5 ? -0.38268343236508977173
       : m == 6 ? -0.70710678118654752440 : -0.92387953251128675613;
}
__host__ __device__ constexpr double s16(int m) {
  return m == 0 ? 0.0 : m == 1 ? 0.38268343236508977173 : m == 2 ? 0.70710678118654752440
       : m == 3 ? 0.92387953251128675613 : m == 4 ? 1.0 : m == 5 ? 0.92387953251128675613
       : m == 6 ? 0.70710678118654752440 : 0.38268343236508977173;
}

// In-register DFT of size R (2, 4, 8, 16), natural order in and out.
template <int R, bool INV, typename C>
__device__ __forceinline__ void dft(C* x) {
  using T = decltype(C::x);
  if constexpr (R == 2) {
    C a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 4) {
    C s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
    C s13 = cadd(x[1], x[3]), d13 = mul_mi<INV>(csub(x[1], x[3]));
    x[0] = cadd(s02, s13);
    x[2] = csub(s02, s13);
    x[1] = cadd(d02, d13);
    x[3] = csub(d02, d13);
  } else {
    constexpr int H = R / 2;
    C e[H], o[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      e[j] = x[2 * j];
      o[j] = x[2 * j + 1];
    }
    dft<H, INV>(e);
    dft<H, INV>(o);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int m = k * (16 / R);
      C t;
      if (k == 0) {
        t = o[k];
      } else if (4 * k == R) {
        t = mul_mi<INV>(o[k]);
      } else {
        C w = mk<C>((T)c16(m), (T)(INV ? s16(m) : -s16(m)));
        t = cmul(o[k], w);
      }
      x[k] = cadd(e[k], t);
      x[k + H] = csub(e[k], t);
    }
  }
}

// BATCH (a table in global memory): all twiddles of the stage are loaded before the first is used,
// so that their loads are in flight together rather than one latency each; a table staged in LDS
// is read as it is used.
template <int N, int S, bool INV, bool BATCH, int RMX, typename C>
__device__ __forceinline__ void stage_compute(C* v, int i, const C* __restrict__ tw, int tws) {
  using P = Plan<N, RMX>;
  constexpr int R = P::radix(S), PP = P::pw(S), NB = P::RMAX / R, TT = P::T;
  if constexpr (PP > 1) {
    C w[NB][R];
#pragma unroll
    for (int m = 0; m < NB; ++m) {
      const int k = (i + m * TT) & (PP - 1);
#pragma unroll
      for (int j = 1; j < R; ++j) w[m][j] = tw[(j * k * (N / (PP * R))) * tws];
    }
    if constexpr (BATCH) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
      for (int j = 1; j < R; ++j) {
        if (INV) w[m][j].y = -w[m][j].y;
        v[m + j * NB] = cmul(v[m + j * NB], w[m][j]);
      }
  }
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    C x[R];
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = v[m + j * NB];
    dft<R, INV>(x);
#pragma unroll
    for (int j = 0; j < R; ++j) v[m + j * NB] = x[j];
  }
}

// LDS slot of line element e: e * es, or, for a contiguous line (es = 1) with PAD > 0, e plus one
// pad slot every 2^PAD elements, so that a stage's strided stores do not fall into the same banks
template <int PAD> __device__ __forceinline__ int lslot(int e, int es) { return PAD ? e + (e >> PAD) : e * es; }

template <int N, int S, int RMX, int PAD = 0, typename C>
__device__ __forceinline__ void stage_store(const C* v, int i, C* lds, int es) {
  using P = Plan<N, RMX>;
  constexpr int R = P::radix(S), PP = P::pw(S), NB = P::RMAX / R, TT = P::T;
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    const int b = i + m * TT;
    const int k = b & (PP - 1);
#pragma unroll
    for (int j = 0; j < R; ++j) lds[lslot<PAD>((b - k) * R + k + j * PP, es)] = v[m + j * NB];
  }
}

template <int N, int RMX, int PAD = 0, typename C>
__device__ __forceinline__ void line_load(C* v, int i, const C* lds, int es) {
#pragma unroll
  for (int s = 0; s < RMX; ++s) v[s] = lds[lslot<PAD>(i + s * Plan<N, RMX>::T, es)];
}

// Global loads / stores of a line's register elements i + s*T: element o0 + (i + s*T) * es of the
// launch-uniform array base.  Addresses are base plus a 32-bit byte offset (the launchers check
// that no launch spans 4 GiB), i.e. a scalar base and one 32-bit register per access.  One
// validity branch per line; the row mask is uniform across the launch, so its test is a scalar
// branch around the masked form.
template <typename C> __device__ __forceinline__ const C& at(const C* base, unsigned byte) {
  return *reinterpret_cast<const C*>(reinterpret_cast<const char*>(base) + (size_t)byte);
}
template <typename C> __device__ __forceinline__ C& at(C* base, unsigned byte) {
  return *reinterpret_cast<C*>(reinterpret_cast<char*>(base) + (size_t)byte);
}

template <int N, int RMX, typename C>
__device__ __forceinline__ void line_gload(C* v, const C* __restrict__ base, unsigned o0, unsigned es, int i,
                                           bool valid, const RowMask& m) {
  constexpr int RM = RMX, TT = Plan<N, RMX>::T;
  if (!valid) {
#pragma unroll
    for (int s = 0; s < RM; ++s) v[s] = mk<C>(0, 0);
    return;
  }
  const unsigned b0 = (o0 + (unsigned)i * es) * (unsigned)sizeof(C), step = TT * es * (unsigned)sizeof(C);
  if (m.load) {
#pragma unroll
    for (int s = 0; s < RM; ++s) {
      const int y = i + s * TT;
      v[s] = (y >= m.lo && y <= m.hi) ? at(base, b0 + s * step) : mk<C>(0, 0);
    }
  } else {
#pragma unroll
    for (int s = 0; s < RM; ++s) v[s] = at(base, b0 + s * step);
  }
}

template <int N, int RMX, typename C>
__device__ __forceinline__ void line_gstore(const C* v, C* __restrict__ base, unsigned o0, unsigned es, int i,
                                            bool valid, const RowMask& m) {
  constexpr int RM = RMX, TT = Plan<N, RMX>::T;
  if (!valid) return;
  const unsigned b0 = (o0 + (unsigned)i * es) * (unsigned)sizeof(C), step = TT * es * (unsigned)sizeof(C);
  if (m.store) {
#pragma unroll
    for (int s = 0; s < RM; ++s) {
      const int y = i + s * TT;
      if (y >= m.lo && y <= m.hi) at(base, b0 + s * step) = v[s];
    }
  } else {
#pragma unroll
    for (int s = 0; s < RM; ++s) at(base, b0 + s * step) = v[s];
  }
}

// 1/x: the hardware reciprocal in single precision (about one ulp, well inside what the float
// path resolves), an exact division in double
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Full line transform on registers v (pattern i + s*T).  All threads of the block must call it
// (it contains block barriers when N needs more than one stage).  lds: this line's exchange
// buffer with element stride es; the caller must not rely on its contents afterwards.
template <int N, bool INV, bool BATCH = false, int RMX = plan_rmax(N), int PAD = 0, int S = 0, typename C>
__device__ __forceinline__ void fft_line(C* v, int i, C* lds, int es, const C* __restrict__ tw, int tws) {
  if constexpr (S < Plan<N, RMX>::NST) {
    stage_compute<N, S, INV, BATCH, RMX>(v, i, tw, tws);
    if constexpr (S + 1 < Plan<N, RMX>::NST) {
      __syncthreads();
      stage_store<N, S, RMX, PAD>(v, i, lds, es);
      __syncthreads();
      line_load<N, RMX, PAD>(v, i, lds, es);
    }
    fft_line<N, INV, BATCH, RMX, PAD, S + 1>(v, i, lds, es, tw, tws);
  }
}

// copy n twiddles tw[e * tws] into LDS at dst; the first read follows a block barrier
template <typename C>
__device__ __forceinline__ const C* stage_table(C* dst, const C* __restrict__ tw, int n, int tid, int nthr,
                                                int tws = 1) {
  for (int e = tid; e < n; e += nthr) dst[e] = tw[e * tws];
  return dst;
}

constexpr int pow2floor(int v) { return v >= 2 ? 2 * pow2floor(v / 2) : 1; }

// Rows per block of the x-axis passes (rows of M = nx / 2 complex points).  Up to M = 1024: as many
// rows as fit 256 threads and 64 KiB of LDS beside the twiddle table.  Longer rows (M = 2048, 4096:
// 4096 and 8192 points along x) take one row per block and M / 8 threads, and read the twiddle table
// from global memory (it stays in L2), which leaves the row alone in LDS (up to 72 KiB) and two or
// more blocks per CU.
constexpr int kMaxRow = 4096;
constexpr int xrmax(int M) { return plan_rmax(M) < 8 ? plan_rmax(M) : 8; }   // elements per thread, x passes
template <typename TR, int M> struct RowCfg {
  static constexpr int RMX = xrmax(M);
  static constexpr int T = Plan<M, RMX>::T;
  static constexpr int BLK = T > kBlock ? T : kBlock;   // launch bound
  static constexpr bool TWL = M <= 1024;                 // twiddle table staged in LDS
  static constexpr int SZ = (int)sizeof(cplx<TR>);
  static constexpr int PAD = 3;      // line exchanges pad one slot every 8 elements
  static constexpr int LS = M + (M >> PAD) + 1;  // LDS row stride (complex elements)
  static constexpr int R0 = BLK / T;
  static constexpr int RL = TWL ? pow2floor((kLdsBytes - 2 * M * SZ) / (LS * SZ)) : 1;
  static constexpr int RPB = (R0 < RL ? R0 : RL) > 0 ? (R0 < RL ? R0 : RL) : 1;
  static constexpr int NT = RPB * T;  // threads per block
  static constexpr int LDSB = (RPB * LS + (TWL ? 2 * M : 0)) * SZ;
  static_assert(TWL ? LDSB <= kLdsBytes : LDSB <= 163840, "x pass: LDS over budget");
};

// ------------------------------------------------------------------ x axis, forward R2C
// TI: element type of the input rows (float rows widened on load for a double transform)
template <typename T, int M, typename TI = T>
__global__ __launch_bounds__((RowCfg<T, M>::BLK)) void k_x_r2c(const TI* __restrict__ in, cplx<T>* __restrict__ out,
                                                  int64_t nrows, const cplx<T>* __restrict__ twg, int RPB,
                                                  RowList rl, int64_t pitch) {
  using C = cplx<T>;
  using RC = RowCfg<T, M>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int tid = threadIdx.x;
  const int NT = RPB * RC::T;
  const C* tw = RC::TWL ? stage_table(lds + RPB * RC::LS, twg, 2 * M, tid, NT) : twg;
  const int64_t row0 = (int64_t)blockIdx.x * RPB;
  const int nvalid = (int)((nrows - row0) < RPB ? (nrows - row0) : RPB);
  __shared__ int64_t rbase[kBlock];   // row index of each block row (active-row list or contiguous)
  __shared__ unsigned long long rseg[kBlock];   // busy x-segments of each block row
  __shared__ int64_t rsub[kBlock];              // forcing row to subtract, or -1
  for (int r = tid; r < RPB; r += NT) {
    rbase[r] = r < nvalid ? rl.row(row0 + r) : 0;
    rseg[r] = r < nvalid ? rl.segmask(row0 + r) : 0ull;
    rsub[r] = r < nvalid ? rl.sub_row(row0 + r) : -1;
  }
  __syncthreads();
  const cplx<TI>* src = reinterpret_cast<const cplx<TI>*>(in);
  const C* sub = static_cast<const C*>(rl.sub);
  // every load of a thread is issued before the first LDS write (RPB * M values, M / T per thread)
  constexpr int K = M / RC::T;
  C ld[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int e = tid + j * NT, r = e / M, c = e - r * M;
    ld[j] = mk<C>(0, 0);
    if ((rseg[r] >> (c >> rl.seg_log2)) & 1ull) {
      const cplx<TI> x = src[rbase[r] * M + c];
      ld[j] = mk<C>((T)x.x, (T)x.y);
    }
    if (rsub[r] >= 0) {
      const C f = sub[rsub[r] * M + c];
      ld[j] = mk<C>(ld[j].x - f.x, ld[j].y - f.y);
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int e = tid + j * NT, r = e / M, c = e - r * M;
    lds[r * RC::LS + c] = ld[j];
  }
  __syncthreads();
  const int row = tid / RC::T, i = tid - row * RC::T;
  C v[RC::RMX];
  if (row < RPB) line_load<M, RC::RMX>(v, i, lds + row * RC::LS, 1);
  fft_line<M, false, !RC::TWL, RC::RMX, RC::PAD>(v, i, lds + (row < RPB ? row : 0) * RC::LS, 1, tw, 2);
  __syncthreads();
  if (row < RPB) {
#pragma unroll
    for (int s = 0; s < RC::RMX; ++s) lds[row * RC::LS + i + s * RC::T] = v[s];
  }
  __syncthreads();
  constexpr int KO = (M + 1 + RC::T - 1) / RC::T;   // M + 1 outputs per row
  C wk_[KO];
#pragma unroll
  for (int j = 0; j < KO; ++j) wk_[j] = tw[(tid + j * NT) % (M + 1)];   // twiddles first, loads together
#pragma unroll
  for (int j = 0; j < KO; ++j) {
    const int e = tid + j * NT;
    if (e < nvalid * (M + 1)) {
      const int r = e / (M + 1), k = e - r * (M + 1);
      const C zk = lds[r * RC::LS + (k == M ? 0 : k)];
      const C zm = lds[r * RC::LS + (k == 0 ? 0 : M - k)];
      const C E = mk<C>((zk.x + zm.x) * (T)0.5, (zk.y - zm.y) * (T)0.5);
      const C O = mk<C>((zk.y + zm.y) * (T)0.5, -(zk.x - zm.x) * (T)0.5);
      out[rbase[r] * pitch + k] = cadd(E, cmul(wk_[j], O));
    }
  }
}

// ------------------------------------------------------------------ x axis, inverse C2R
template <typename T, int M>
__global__ __launch_bounds__((RowCfg<T, M>::BLK)) void k_x_c2r(const cplx<T>* __restrict__ in, T* __restrict__ out,
                                                  int64_t nrows, const cplx<T>* __restrict__ twg, int RPB,
                                                  RowList rl, int64_t pitch) {
  using C = cplx<T>;
  using RC = RowCfg<T, M>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int tid = threadIdx.x;
  const int NT = RPB * RC::T;
  const C* tw = RC::TWL ? stage_table(lds + RPB * RC::LS, twg, 2 * M, tid, NT) : twg;
  const int64_t row0 = (int64_t)blockIdx.x * RPB;
  const int nvalid = (int)((nrows - row0) < RPB ? (nrows - row0) : RPB);
  __shared__ int64_t rbase[kBlock];
  for (int r = tid; r < RPB; r += NT) rbase[r] = r < nvalid ? rl.row(row0 + r) : 0;
  __syncthreads();
  // every load of a thread is issued before the first LDS write
  constexpr int KI = (M + 1 + RC::T - 1) / RC::T;
  C ld[KI];
#pragma unroll
  for (int j = 0; j < KI; ++j) {
    const int e = tid + j * NT, r = e / (M + 1), k = e - r * (M + 1);
    ld[j] = mk<C>(0, 0);
    if (e < RPB * (M + 1) && r < nvalid) ld[j] = in[rbase[r] * pitch + k];
  }
#pragma unroll
  for (int j = 0; j < KI; ++j) {
    const int e = tid + j * NT, r = e / (M + 1), k = e - r * (M + 1);
    if (e < RPB * (M + 1)) lds[r * RC::LS + k] = ld[j];
  }
  __syncthreads();
  // Z'_k = (X_k + conj X_{M-k}) + i conj(W^k) (X_k - conj X_{M-k}); each thread owns a pair (k, M-k)
  constexpr int HP = M / 2 + 1, KP = (HP + RC::T - 1) / RC::T;
  C wk_[KP], wm_[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) {   // twiddles first: their loads are issued together
    const int k = (tid + j * NT) % HP;
    wk_[j] = cconj(tw[k]);
    wm_[j] = cconj(tw[M - k]);
  }
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int e = tid + j * NT;
    if (e < nvalid * HP) {
      const int r = e / HP, k = e - r * HP;
      C* rowp = lds + r * RC::LS;
      const C a = rowp[k], b = rowp[M - k];
      const C wk = wk_[j], wm = wm_[j];
      const C za = cadd(mk<C>(a.x + b.x, a.y - b.y), cmul(mk<C>(-wk.y, wk.x), mk<C>(a.x - b.x, a.y + b.y)));
      rowp[k] = za;
      if (k != 0 && 2 * k != M) {
        const C zb = cadd(mk<C>(b.x + a.x, b.y - a.y), cmul(mk<C>(-wm.y, wm.x), mk<C>(b.x - a.x, b.y + a.y)));
        rowp[M - k] = zb;
      }
    }
  }
  __syncthreads();
  const int row = tid / RC::T, i = tid - row * RC::T;
  C v[RC::RMX];
  if (row < RPB) line_load<M, RC::RMX>(v, i, lds + row * RC::LS, 1);
  fft_line<M, true, !RC::TWL, RC::RMX, RC::PAD>(v, i, lds + (row < RPB ? row : 0) * RC::LS, 1, tw, 2);
  __syncthreads();
  if (row < RPB) {
#pragma unroll
    for (int s = 0; s < RC::RMX; ++s) lds[row * RC::LS + i + s * RC::T] = v[s];
  }
  __syncthreads();
  C* dst = reinterpret_cast<C*>(out);
#pragma unroll
  for (int j = 0; j < M / RC::T; ++j) {
    const int e = tid + j * NT;
    if (e < nvalid * M) {
      const int r = e / M, c = e - r * M;
      dst[rbase[r] * M + c] = lds[r * RC::LS + c];
    }
  }
}

// tile width (lines per block) for strided and fused passes
// elements per thread of the strided and fused passes: at most 8 in double precision up to N = 256,
// whose 16-element lines need more registers than leave room for a second wave per SIMD (longer
// lines keep 16, or their tiles would narrow below 64-byte segments)
template <typename T> constexpr int rmax_t(int N) {
  return sizeof(T) == 8 && N <= 256 && plan_rmax(N) > 8 ? 8 : plan_rmax(N);
}
// Elements per thread of the general fused last-axis passes: those that keep two accumulators or
// two input spectra per element (Stokes, the transposed Stokes pass) and the 1024-point double
// ones hold 8 instead of 16, and 4 for double two-accumulator lines of 512 points or more, which
// keeps them clear of register spills and raises occupancy (the single-field pass k_fused1 keeps
// the default).
template <typename T> constexpr int fused_rmax(int N, int nacc) {
  return (sizeof(T) == 8 && nacc >= 2 && N >= 512) ? 4   // double, two accumulators, long lines
         : (plan_rmax(N) > 8 && (nacc >= 2 || (sizeof(T) == 8 && N >= 1024)) ? 8 : rmax_t<T>(N));
}
template <typename T, int N, int RX = rmax_t<T>(N), int BLK = kBlock, int LDS = kLdsBytes> struct TileCfg {
  static constexpr int RMX = RX;
  static constexpr int T_ = Plan<N, RMX>::T;
  static constexpr int W0 = BLK / T_;
  static constexpr int WL = LDS / (N * (int)sizeof(cplx<T>));
  // lines per tile: a power of two (the kernels split a thread index into line and element by it)
  static constexpr int W = pow2floor((W0 < WL ? W0 : WL) > 0 ? (W0 < WL ? W0 : WL) : 1);
  static constexpr int NT = W * T_;  // threads per block
  // twiddles staged in LDS when the table fits beside the widest tile (all but 1024 in double)
  static constexpr bool TWL = (W * N + N) * (int)sizeof(cplx<T>) <= LDS;
};
// the single-field passes' tile configuration
template <typename T, int N, int RX = rmax_t<T>(N)> using LineCfg = TileCfg<T, N, RX, kLineBlock, kLineLds>;
// Radix plans of the single-field line passes: plan 0 holds rmax_t elements per thread, plan 1 half
// as many (twice the threads per line, one more radix stage) where that leaves at least 4 and a line
// fits a workgroup; the launch-shape timing picks one per pass.
template <typename T> constexpr int plan_rx(int N, int plan) {
  return plan == 1 && rmax_t<T>(N) >= 8 && N / (rmax_t<T>(N) / 2) <= kLineBlock ? rmax_t<T>(N) / 2 : rmax_t<T>(N);
}

// Tile of this workgroup in the strided and last-axis passes.  A tile of W lines reads and writes
// W adjacent elements of each row; when they fill less than a 128-byte cache line the line is
// shared with the neighbouring tiles, which are then kept on one XCD so that it is fetched into one
// L2 once rather than into several.
template <typename C> __device__ __forceinline__ unsigned tile_of_block(int W) {
  return W * (int)sizeof(C) < 128 ? (unsigned)xcd_chunk((int)blockIdx.x, (int)gridDim.x) : blockIdx.x;
}

// Lines of the last-axis passes come in rows of `inner`: x modes 0 .. vinner - 1, then pitch
// padding.  With tiles of W consecutive lines, a row's last tile holds its last x mode (the Nyquist
// one) beside W - 1 padding lines: at 256 points along x, one tile in nine.  Where W divides
// vinner - 1 (both powers of two) the tiles are assigned instead as LineMap on = 1 describes, so that
// no tile holds padding; the tiles of last modes read W rows' lines (1 / (vinner - 1) of the data,
// but one cache line per element and row) and come first, so that they do not finish last.  (The
// strided passes keep the plain assignment: there the gathered last-mode tiles cost more than the
// padding lines did.)
inline LineMap line_map(int64_t nlines, int64_t inner, int64_t vinner, int W, int64_t* nblocks) {
  LineMap m;
  const int64_t lead = vinner - 1;
  const auto pow2 = [](int64_t v) { return v > 0 && (v & (v - 1)) == 0; };
  if (inner > vinner && W >= 1 && pow2(W) && lead >= W && lead % W == 0 && pow2(lead / W) && nlines % inner == 0 &&
      nlines / inner <= (int64_t)UINT32_MAX / 2) {
    m.on = 1;
    m.lw = __builtin_ctzll((unsigned long long)W);
    m.lm = __builtin_ctzll((unsigned long long)(lead / W));
    m.rows = (unsigned)(nlines / inner);
    m.nlast = (unsigned)(((int64_t)m.rows + W - 1) / W);
    *nblocks = (int64_t)m.nlast + (int64_t)m.rows * (lead / W);
  } else {
    *nblocks = (nlines + W - 1) / W;
  }
  return m;
}

// row lq and x mode li of column c of tile t; false for padding and for lines past the last row
__device__ __forceinline__ bool tile_lines(const LineMap& m, unsigned t, int c, int W, unsigned inner,
                                           unsigned vinner, int64_t nlines, unsigned& lq, unsigned& li) {
  if (m.on) {
    if (t < m.nlast) {   // last x modes: strided rows, slower per tile, so dispatched first
      lq = (t << m.lw) + (unsigned)c;
      li = vinner - 1;
      return lq < m.rows;
    }
    t -= m.nlast;
    lq = t >> m.lm;
    li = ((t & ((1u << m.lm) - 1u)) << m.lw) + (unsigned)c;
    return true;
  }
  const unsigned l = t * (unsigned)W + (unsigned)c;
  lq = l / inner;
  li = l - lq * inner;
  return l < nlines && li < vinner;
}

// ------------------------------------------------------------------ strided in-place C2C
template <typename T, int N, bool INV, int RX = rmax_t<T>(N)>
__global__ __launch_bounds__(kLineBlock) void k_strided(cplx<T>* __restrict__ data, int64_t nlines, int64_t inner,
                                                        int64_t outer, int64_t es, const cplx<T>* __restrict__ twg,
                                                        int W, RowMask rm, int64_t vinner) {
  using C = cplx<T>;
  using TC = LineCfg<T, N, RX>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int tid = threadIdx.x;
  const C* tw = TC::TWL ? stage_table(lds + N * W, twg, N, tid, W * TC::T_) : twg;
  const int c = tid & (W - 1), i = tid / W;
  const unsigned l = tile_of_block<C>(W) * (unsigned)W + c;
  const unsigned lq = l / (unsigned)inner, li = l - lq * (unsigned)inner;
  const bool valid = l < nlines && li < vinner;
  const unsigned lp = rm.phys_plane(lq);
  const unsigned base = valid ? lp * (unsigned)outer + li : 0u;
  const RowMask pm = rm.plane(valid ? lp : 0);   // rows of this line's plane that matter
  C v[TC::RMX];
  line_gload<N, TC::RMX>(v, data, base, (unsigned)es, i, valid, pm);
  fft_line<N, INV, !TC::TWL, TC::RMX>(v, i, lds + c, W, tw, 1);
  line_gstore<N, TC::RMX>(v, data, base, (unsigned)es, i, valid, pm);
}

// ------------------------------------------------------------------ Fourier multiplier
// Coefficient of input field kind fk for output component o at one mode.
//   scalar:  u^ = alpha*sc * (sum_f c_f F^_f) / (c2*sigma - c0),  c_f = i k~_d (FK_D*) or 1 (FK_MASS);
//            zero where c2*sigma - c0 = 0 (mean-zero inverse).
//   Stokes:  u^ = alpha*sc * [ i k~ s^/ell + (1/lam) P^ (G^ + mu v^) ],  ell = -sigma,
//            lam = c2*ell + c0, P^ = I - k~ k~^T / ell (I at ell = 0), s = (A11 + A22)/2,
//            v_i = sum_j i k~_j A_ij; 1/ell and 1/lam read as 0 where they vanish.
//   pressure (mode 3, Stokes fields, one output; the G fields hold eta S Q - g~):
//            p^ = alpha*sc * [ -i k~_j G^_j + mu k~_i k~_j A^_ij + (c2 sigma - c0) s^ ] / ell.
template <typename T>
__device__ __forceinline__ cplx<T> mult_coef(const MultDesc& md, int fk, int o, T sig, const T* kt) {
  using C = cplx<T>;
  if (!md.stokes) {
    const T den = (T)md.c2 * sig - (T)md.c0;
    const T g = den == (T)0 ? (T)0 : (T)(md.alpha * md.sc) * recip(den);
    if (fk == FK_MASS) return mk<C>(g, 0);
    return mk<C>(0, g * kt[fk]);
  }
  const T ell = -sig;
  const T il = ell == (T)0 ? (T)0 : recip(ell);
  const T lam = (T)md.c2 * ell + (T)md.c0;
  const T is = lam == (T)0 ? (T)0 : recip(lam);
  const T ko = kt[o];
  const T P0 = (o == 0 ? (T)1 : (T)0) - ko * kt[0] * il;
  const T P1 = (o == 1 ? (T)1 : (T)0) - ko * kt[1] * il;
  const T mu = (T)md.mu, a = (T)(md.alpha * md.sc);
  if (md.mode == 3) {   // pressure (2-D): [i k~.(g^ - f^) + (c2 sigma - c0) s^] / ell
    const T lamh = (T)0.5 * ((T)md.c2 * sig - (T)md.c0);
    switch (fk) {
      case FK_A11: return mk<C>(a * il * (mu * kt[0] * kt[0] + lamh), 0);
      case FK_A12: return mk<C>(a * il * ((T)2 * mu * kt[0] * kt[1]), 0);
      case FK_A22: return mk<C>(a * il * (mu * kt[1] * kt[1] + lamh), 0);
      case FK_G1: return mk<C>(0, -a * il * kt[0]);
      default: return mk<C>(0, -a * il * kt[1]);
    }
  }
  switch (fk) {
    case FK_A11: return mk<C>(0, a * ((T)0.5 * ko * il + mu * is * P0 * kt[0]));
    case FK_A12: return mk<C>(0, a * (mu * is * (P0 * kt[1] + P1 * kt[0])));
    case FK_A22: return mk<C>(0, a * ((T)0.5 * ko * il + mu * is * P1 * kt[1]));
    case FK_G1: return mk<C>(a * is * P0, 0);
    default: return mk<C>(a * is * P1, 0);
  }
}

// The Stokes coefficient of mult_coef with 1/ell and 1/lam of the mode given (2-D: k~ = (k0, k1)).
template <typename T>
__device__ __forceinline__ cplx<T> stokes_coef(const MultDesc& md, int fk, int o, T sig, T k0, T k1, T il, T is) {
  using C = cplx<T>;
  const T ko = o == 0 ? k0 : k1;
  const T P0 = (o == 0 ? (T)1 : (T)0) - ko * k0 * il;
  const T P1 = (o == 1 ? (T)1 : (T)0) - ko * k1 * il;
  const T mu = (T)md.mu, a = (T)(md.alpha * md.sc);
  if (md.mode == 3) {
    const T lamh = (T)0.5 * ((T)md.c2 * sig - (T)md.c0);
    switch (fk) {
      case FK_A11: return mk<C>(a * il * (mu * k0 * k0 + lamh), 0);
      case FK_A12: return mk<C>(a * il * ((T)2 * mu * k0 * k1), 0);
      case FK_A22: return mk<C>(a * il * (mu * k1 * k1 + lamh), 0);
      case FK_G1: return mk<C>(0, -a * il * k0);
      default: return mk<C>(0, -a * il * k1);
    }
  }
  switch (fk) {
    case FK_A11: return mk<C>(0, a * ((T)0.5 * ko * il + mu * is * P0 * k0));
    case FK_A12: return mk<C>(0, a * (mu * is * (P0 * k1 + P1 * k0)));
    case FK_A22: return mk<C>(0, a * ((T)0.5 * ko * il + mu * is * P1 * k1));
    case FK_G1: return mk<C>(a * is * P0, 0);
    default: return mk<C>(a * is * P1, 0);
  }
}

// Where a line of the last-axis passes lives and which modes it holds.  3-D: line l of the (jy, jx)
// plane, elements strided by P, element e is mode e; 2-D: line jx, elements strided by P = nxp.
// SPLIT (2-D lines of a four-step y transform, md.split = N1, see fft_fused_last): line
// (jx, k1 = l / nxp) holds the y modes k1 + N1 e, stored from row k1 N with stride nxp, and takes the
// twiddles w_n^(e k1) between the two factors' transforms.
template <int N, bool SPLIT> struct LineGeo {
  unsigned base, es;   // first element, element stride
  int k1, ms;
  __device__ __forceinline__ LineGeo(const MultDesc& md, int l, int64_t P, int jx, int jy2) {
    if constexpr (SPLIT) {
      base = (unsigned)(jy2 * N * md.nxp + jx);
      es = (unsigned)md.nxp;
      k1 = jy2;
      ms = md.split;
    } else {
      base = (unsigned)l;
      es = (unsigned)P;
      k1 = 0;
      ms = 1;
    }
  }
  __device__ __forceinline__ int mode(int e) const {   // mode index along the line of element e
    if constexpr (SPLIT) return k1 + ms * e;
    else return e;
  }
  __device__ __forceinline__ int tws() const { return SPLIT ? ms : 1; }   // twiddle stride of the N-point transforms
};

// the four-step twiddles w_n^(e k1) (conjugated for the inverse) on a line's register elements
template <int RM, int TT, typename C>
__device__ __forceinline__ void split_twiddle(C* v, int i, int k1, const C* __restrict__ twn, bool inv) {
  C w[RM];
#pragma unroll
  for (int s = 0; s < RM; ++s) w[s] = twn[(i + s * TT) * k1];
#pragma unroll
  for (int s = 0; s < RM; ++s) v[s] = cmul(v[s], inv ? cconj(w[s]) : w[s]);
}

template <typename T, int N, int NO, bool STOKES, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_fused(cplx<T>* __restrict__ data, int64_t P, MultDesc md,
                                                  const cplx<T>* __restrict__ twg, int W, int64_t bstride, RowMask rm) {
  using C = cplx<T>;
  using TC = TileCfg<T, N, fused_rmax<T>(N, NO)>;
  constexpr int RM = TC::RMX, TT = TC::T_;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  data += (int64_t)blockIdx.y * bstride;   // problem of a batch
  const int tid = threadIdx.x;
  const int tws = SPLIT ? md.split : 1;
  const C* tw = TC::TWL ? stage_table(lds + N * W, twg, N, tid, W * TC::T_, tws) : twg;
  const int ltws = TC::TWL ? 1 : tws;
  const int c = tid & (W - 1), i = tid / W;
  unsigned lq_, li_;   // row and x mode of this thread's line; padding lines are skipped
  const bool valid = tile_lines(md.map, tile_of_block<C>(W), c, W, (unsigned)md.nxp, (unsigned)md.nxh, P, lq_, li_);
  const int l = (int)(lq_ * (unsigned)md.nxp + li_);
  const int64_t FS = P * N;
  // mode indices of this line: 2-D l = jx (+ nxp k1 with a split), e = jy; 3-D l = jy*nxh + jx, e = jz
  const int jx = (int)(valid ? li_ : 0u);
  const int jy2 = (int)(valid ? lq_ : 0u);
  const bool d3 = md.dim == 3;
  const LineGeo<N, SPLIT> lg(md, l, P, jx, jy2);
  const T* sgl = static_cast<const T*>(md.sig[d3 ? 2 : 1]);   // symbols along the line
  const T* ktl_ = static_cast<const T*>(md.kt[d3 ? 2 : 1]);
  T sig_l = static_cast<const T*>(md.sig[0])[jx];
  T ktl[3];
  ktl[0] = static_cast<const T*>(md.kt[0])[jx];
  ktl[1] = 0;
  ktl[2] = 0;
  if (d3) {
    sig_l += static_cast<const T*>(md.sig[1])[jy2];
    ktl[1] = static_cast<const T*>(md.kt[1])[jy2];
  }
  const int la = d3 ? 2 : 1;   // index of the line axis among the derivative components
  C acc[NO][RM];
#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int s = 0; s < RM; ++s) acc[o][s] = mk<C>(0, 0);
  T gfac[RM];   // scalar: multiplier alpha*sc / (c2 sigma - c0); Stokes (2-D): 1/ell
  T glam[STOKES ? RM : 1];   // Stokes: 1/lam
  if constexpr (!STOKES) {
#pragma unroll
    for (int s = 0; s < RM; ++s) {
      const T den = (T)md.c2 * (sig_l + sgl[lg.mode(i + s * TT)]) - (T)md.c0;
      gfac[s] = den == (T)0 ? (T)0 : (T)(md.alpha * md.sc) * recip(den);
    }
  } else {
#pragma unroll
    for (int s = 0; s < RM; ++s) {
      const T ell = -(sig_l + sgl[lg.mode(i + s * TT)]);
      gfac[s] = ell == (T)0 ? (T)0 : recip(ell);
      const T lam = (T)md.c2 * ell + (T)md.c0;
      glam[s] = lam == (T)0 ? (T)0 : recip(lam);
    }
  }

  for (int f = 0; f < md.nc; ++f) {
    C v[RM];
    line_gload<N, RM>(v, data, (unsigned)(f * FS + lg.base), lg.es, i, valid, rm);
    if constexpr (SPLIT) split_twiddle<RM, TT>(v, i, lg.k1, twg, false);
    fft_line<N, false, !TC::TWL, RM>(v, i, lds + c, W, tw, ltws);
    const int fk = md.fk[f];
    if constexpr (!STOKES) {
      if (fk == FK_MASS) {
#pragma unroll
        for (int s = 0; s < RM; ++s) acc[0][s] = cadd(acc[0][s], cscale(v[s], gfac[s]));
      } else if (fk == la) {   // derivative along the line axis: k~ varies per element
#pragma unroll
        for (int s = 0; s < RM; ++s) acc[0][s] = cadd(acc[0][s], mul_ir(v[s], gfac[s] * ktl_[lg.mode(i + s * TT)]));
      } else {                 // derivative across lines: k~ is constant on the line
        const T kc = ktl[fk];
#pragma unroll
        for (int s = 0; s < RM; ++s) acc[0][s] = cadd(acc[0][s], mul_ir(v[s], gfac[s] * kc));
      }
    } else {
#pragma unroll
      for (int s = 0; s < RM; ++s) {   // Stokes is two-dimensional: k~ = (k~ across lines, k~ along)
        const int e = lg.mode(i + s * TT);
        const T sig = sig_l + sgl[e];
#pragma unroll
        for (int o = 0; o < NO; ++o)
          acc[o][s] = cadd(acc[o][s], cmul(stokes_coef<T>(md, fk, o, sig, ktl[0], ktl_[e], gfac[s], glam[s]), v[s]));
      }
    }
  }
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    fft_line<N, true, !TC::TWL, RM>(acc[o], i, lds + c, W, tw, ltws);
    if constexpr (SPLIT) split_twiddle<RM, TT>(acc[o], i, lg.k1, twg, true);
    line_gstore<N, RM>(acc[o], data, (unsigned)(o * FS + lg.base), lg.es, i, valid, rm);
  }
}

// The Stokes pass of 2-D problems with up to five input fields, the transforms of all fields taken
// together: each radix stage works on every field's registers before one pair of barriers and one
// LDS exchange (a buffer per field), and the two outputs' inverse transforms likewise.  A line
// then waits for the latency of two transforms instead of nc + 2 in sequence (k_fused<.., STOKES>).
// The double-precision 1024-point lines (one line of 256 threads per workgroup, half a thousand
// lines per problem) stay bound by the L2 requests of their 16-byte row accesses.  Twiddles are
// read from global memory (L2).
constexpr int kStokesFields = 5;
constexpr int kStokesLds = 81920;   // two workgroups per CU
template <typename T, int N> struct StokesCfg {
  static constexpr int RMX = fused_rmax<T>(N, 2);
  static constexpr int T_ = Plan<N, RMX>::T;
  static constexpr int W0 = kBlock / T_;
  static constexpr int WL = kStokesLds / (kStokesFields * N * (int)sizeof(cplx<T>));
  static constexpr int W = pow2floor((W0 < WL ? W0 : WL) > 0 ? (W0 < WL ? W0 : WL) : 1);
  static constexpr int NT = W * T_;
};

template <int N, bool INV, int NF, int RMX, int S = 0, typename C>
__device__ __forceinline__ void fft_lines_multi(C (&v)[NF][RMX], int nf, int i, C* lds, int es, int fstride,
                                                const C* __restrict__ tw, int tws) {
  if constexpr (S < Plan<N, RMX>::NST) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
      if (f < nf) stage_compute<N, S, INV, true, RMX>(v[f], i, tw, tws);
    if constexpr (S + 1 < Plan<N, RMX>::NST) {
      __syncthreads();
#pragma unroll
      for (int f = 0; f < NF; ++f)
        if (f < nf) stage_store<N, S, RMX>(v[f], i, lds + f * fstride, es);
      __syncthreads();
#pragma unroll
      for (int f = 0; f < NF; ++f)
        if (f < nf) line_load<N, RMX>(v[f], i, lds + f * fstride, es);
    }
    fft_lines_multi<N, INV, NF, RMX, S + 1>(v, nf, i, lds, es, fstride, tw, tws);
  }
}

template <typename T, int N, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_fused_stokes2(cplx<T>* __restrict__ data, int64_t P, MultDesc md,
                                                          const cplx<T>* __restrict__ twg, int W, int64_t bstride,
                                                          RowMask rm) {
  using C = cplx<T>;
  using SC = StokesCfg<T, N>;
  constexpr int RM = SC::RMX, TT = SC::T_, NF = kStokesFields;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  data += (int64_t)blockIdx.y * bstride;   // problem of a batch
  const int tid = threadIdx.x;
  const int tws = SPLIT ? md.split : 1;
  const int c = tid & (W - 1), i = tid / W;
  unsigned lq_, li_;   // row and x mode of this thread's line; padding lines are skipped
  const bool valid = tile_lines(md.map, tile_of_block<C>(W), c, W, (unsigned)md.nxp, (unsigned)md.nxh, P, lq_, li_);
  const int l = (int)(lq_ * (unsigned)md.nxp + li_);
  const int64_t FS = P * N;
  const int jx = (int)(valid ? li_ : 0u);
  const int jy2 = (int)(valid ? lq_ : 0u);
  const LineGeo<N, SPLIT> lg(md, l, P, jx, jy2);
  const T* sgl = static_cast<const T*>(md.sig[1]);
  const T* ktl_ = static_cast<const T*>(md.kt[1]);
  const T sig_l = static_cast<const T*>(md.sig[0])[jx];
  const T kx = static_cast<const T*>(md.kt[0])[jx];
  const int nc = md.nc;
  C v[NF][RM];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    if (f < nc) {
      line_gload<N, RM>(v[f], data, (unsigned)(f * FS + lg.base), lg.es, i, valid, rm);
      if constexpr (SPLIT) split_twiddle<RM, TT>(v[f], i, lg.k1, twg, false);
    } else {
#pragma unroll
      for (int s = 0; s < RM; ++s) v[f][s] = mk<C>(0, 0);
    }
  }
  fft_lines_multi<N, false, NF, RM>(v, nc, i, lds + c, W, N * W, twg, tws);
  C acc[2][RM];
#pragma unroll
  for (int s = 0; s < RM; ++s) {
    const int e = lg.mode(i + s * TT);
    const T sig = sig_l + sgl[e];
    const T ke = ktl_[e];
    const T ell = -sig;
    const T il = ell == (T)0 ? (T)0 : recip(ell);
    const T lam = (T)md.c2 * ell + (T)md.c0;
    const T is = lam == (T)0 ? (T)0 : recip(lam);
    acc[0][s] = mk<C>(0, 0);
    acc[1][s] = mk<C>(0, 0);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (f < nc) {
        acc[0][s] = cadd(acc[0][s], cmul(stokes_coef<T>(md, md.fk[f], 0, sig, kx, ke, il, is), v[f][s]));
        acc[1][s] = cadd(acc[1][s], cmul(stokes_coef<T>(md, md.fk[f], 1, sig, kx, ke, il, is), v[f][s]));
      }
    }
  }
  fft_lines_multi<N, true, 2, RM>(acc, 2, i, lds + c, W, N * W, twg, tws);
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    if constexpr (SPLIT) split_twiddle<RM, TT>(acc[o], i, lg.k1, twg, true);
    line_gstore<N, RM>(acc[o], data, (unsigned)(o * FS + lg.base), lg.es, i, valid, rm);
  }
}

// Single scalar field (the finite-difference operator and the scalar grid solve): forward FFT,
// multiply by the real factor alpha*sc / (c2 sigma - c0) in registers, inverse FFT.
template <typename T, int N, bool SPLIT, int RX = rmax_t<T>(N)>
__global__ __launch_bounds__(kLineBlock) void k_fused1(cplx<T>* __restrict__ data, int64_t P, MultDesc md,
                                                       const cplx<T>* __restrict__ twg, int W, int64_t bstride,
                                                       RowMask rm) {
  using C = cplx<T>;
  using TC = LineCfg<T, N, RX>;   // one field, one real factor: no spills at 16 elements per thread
  constexpr int RM = TC::RMX, TT = TC::T_;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  data += (int64_t)blockIdx.y * bstride;   // problem of a batch
  const int tid = threadIdx.x;
  const int tws = SPLIT ? md.split : 1;
  const C* tw = TC::TWL ? stage_table(lds + N * W, twg, N, tid, W * TC::T_, tws) : twg;
  const int ltws = TC::TWL ? 1 : tws;
  const int c = tid & (W - 1), i = tid / W;
  unsigned lq_, li_;   // row and x mode of this thread's line; padding lines are skipped
  const bool valid = tile_lines(md.map, tile_of_block<C>(W), c, W, (unsigned)md.nxp, (unsigned)md.nxh, P, lq_, li_);
  const int l = (int)(lq_ * (unsigned)md.nxp + li_);
  const int jx = (int)(valid ? li_ : 0u);
  const int jy2 = (int)(valid ? lq_ : 0u);
  const bool d3 = md.dim == 3;
  const LineGeo<N, SPLIT> lg(md, l, P, jx, jy2);
  const T* sgl = static_cast<const T*>(md.sig[d3 ? 2 : 1]);
  T sig_l = static_cast<const T*>(md.sig[0])[jx];
  if (d3) sig_l += static_cast<const T*>(md.sig[1])[jy2];
  C v[RM];
  line_gload<N, RM>(v, data, lg.base, lg.es, i, valid, rm);
  if constexpr (SPLIT) split_twiddle<RM, TT>(v, i, lg.k1, twg, false);
  fft_line<N, false, !TC::TWL, RM>(v, i, lds + c, W, tw, ltws);
  const T num = (T)(md.alpha * md.sc), c2 = (T)md.c2, c0 = (T)md.c0;
#pragma unroll
  for (int s = 0; s < RM; ++s) {
    const T den = c2 * (sig_l + sgl[lg.mode(i + s * TT)]) - c0;
    v[s] = cscale(v[s], den == (T)0 ? (T)0 : num * recip(den));
  }
  fft_line<N, true, !TC::TWL, RM>(v, i, lds + c, W, tw, ltws);
  if constexpr (SPLIT) split_twiddle<RM, TT>(v, i, lg.k1, twg, true);
  line_gstore<N, RM>(v, data, lg.base, lg.es, i, valid, rm);
}

// Transposed / multi-output pass: the NI input spectra stay in registers after their forward
// FFTs and the no outputs are formed, inverse transformed and stored one at a time (inputs are
// all read before the first store, and each workgroup owns its lines in every field).
template <typename T, int N, int NI, int MODE, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_fused_adj(cplx<T>* __restrict__ data, int64_t P, int no, MultDesc md,
                                                      const cplx<T>* __restrict__ twg, int W, int64_t bstride, RowMask rm) {
  using C = cplx<T>;
  using TC = TileCfg<T, N, fused_rmax<T>(N, NI)>;
  constexpr int RM = TC::RMX, TT = TC::T_;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  data += (int64_t)blockIdx.y * bstride;   // problem of a batch
  const int tid = threadIdx.x;
  const int tws = SPLIT ? md.split : 1;
  const C* tw = TC::TWL ? stage_table(lds + N * W, twg, N, tid, W * TC::T_, tws) : twg;
  const int ltws = TC::TWL ? 1 : tws;
  const int c = tid & (W - 1), i = tid / W;
  unsigned lq_, li_;   // row and x mode of this thread's line; padding lines are skipped
  const bool valid = tile_lines(md.map, tile_of_block<C>(W), c, W, (unsigned)md.nxp, (unsigned)md.nxh, P, lq_, li_);
  const int l = (int)(lq_ * (unsigned)md.nxp + li_);
  const int64_t FS = P * N;
  const int jx = (int)(valid ? li_ : 0u);
  const int jy2 = (int)(valid ? lq_ : 0u);
  const bool d3 = md.dim == 3;
  const LineGeo<N, SPLIT> lg(md, l, P, jx, jy2);
  const T* sgl = static_cast<const T*>(md.sig[d3 ? 2 : 1]);
  const T* ktl_ = static_cast<const T*>(md.kt[d3 ? 2 : 1]);
  T sig_l = static_cast<const T*>(md.sig[0])[jx];
  T ktl[3];
  ktl[0] = static_cast<const T*>(md.kt[0])[jx];
  ktl[1] = 0;
  ktl[2] = 0;
  if (d3) {
    sig_l += static_cast<const T*>(md.sig[1])[jy2];
    ktl[1] = static_cast<const T*>(md.kt[1])[jy2];
  }
  const int la = d3 ? 2 : 1;
  C v[NI][RM];
#pragma unroll
  for (int f = 0; f < NI; ++f) {
    line_gload<N, RM>(v[f], data, (unsigned)(f * FS + lg.base), lg.es, i, valid, rm);
    if constexpr (SPLIT) split_twiddle<RM, TT>(v[f], i, lg.k1, twg, false);
    fft_line<N, false, !TC::TWL, RM>(v[f], i, lds + c, W, tw, ltws);
  }
  for (int o = 0; o < no; ++o) {
    C acc[RM];
#pragma unroll
    for (int s = 0; s < RM; ++s) {
      const int e = lg.mode(i + s * TT);
      T kt[3] = {ktl[0], ktl[1], ktl[2]};
      kt[la] = ktl_[e];
      const T sig = sig_l + sgl[e];
      if constexpr (MODE == 1) {
        const T den = (T)md.c2 * sig - (T)md.c0;
        const T g = den == (T)0 ? (T)0 : (T)(md.alpha * md.sc) * recip(den);
        const T ko = o == 0 ? kt[0] : (o == 1 ? kt[1] : kt[2]);
        acc[s] = o < md.dim ? mul_ir(v[0][s], g * ko) : cscale(v[0][s], g);
      } else {
        acc[s] = mk<C>(0, 0);
#pragma unroll
        for (int f = 0; f < NI; ++f) acc[s] = cadd(acc[s], cmul(cconj(mult_coef<T>(md, md.fk[o], f, sig, kt)), v[f][s]));
      }
    }
    fft_line<N, true, !TC::TWL, RM>(acc, i, lds + c, W, tw, ltws);
    if constexpr (SPLIT) split_twiddle<RM, TT>(acc, i, lg.k1, twg, true);
    line_gstore<N, RM>(acc, data, (unsigned)(o * FS + lg.base), lg.es, i, valid, rm);
  }
}

// ------------------------------------------------------------------ dispatch helpers
template <typename F> void dispatch_n(int n, F&& f) {
  switch (n) {
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    case 256: f(std::integral_constant<int, 256>{}); break;
    case 512: f(std::integral_constant<int, 512>{}); break;
    case 1024: f(std::integral_constant<int, 1024>{}); break;
    default: throw Error(-2, "unsupported FFT length " + std::to_string(n));
  }
}
// x-pass rows: M = nx / 2 up to kMaxRow
template <typename F> void dispatch_row(int m, F&& f) {
  switch (m) {
    case 2048: f(std::integral_constant<int, 2048>{}); break;
    case 4096: f(std::integral_constant<int, 4096>{}); break;
    default: dispatch_n(m, f);
  }
}

// Lines longer than kMaxLine (2-D y axis of 2048 to 8192 points) run as a four-step transform
// n = kSplit * (n / kSplit): see fft_fused_last.
constexpr int kMaxLine = 1024;
constexpr int kSplit = 8;

}  // namespace

int fft_supported(int n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }

template <typename T>
int fft_x_rpb_max(int nx) {
  int r = 0;
  dispatch_row(nx / 2, [&](auto Mc) { r = RowCfg<T, decltype(Mc)::value>::RPB; });
  return r;
}

template <typename T>
int fft_line_w_max(int n, int plan) {
  int r = 0;
  dispatch_n(n > kMaxLine ? n / kSplit : n, [&](auto Nc) {
    constexpr int N = decltype(Nc)::value;
    r = plan == 1 ? LineCfg<T, N, plan_rx<T>(N, 1)>::W : LineCfg<T, N>::W;
  });
  return r;
}

template <typename T>
int fft_line_plans(int n) {
  int r = 1;
  dispatch_n(n > kMaxLine ? n / kSplit : n, [&](auto Nc) {
    constexpr int N = decltype(Nc)::value;
    r = plan_rx<T>(N, 1) != plan_rx<T>(N, 0) ? 2 : 1;
  });
  return r;
}

namespace {
int pick(int want, int max) {
  if (want <= 0 || want > max) return max;
  int v = 1;
  while (2 * v <= want) v *= 2;
  return v;
}
}  // namespace

namespace {
template <typename T, typename TI>
void x_r2c_launch(const TI* in, cplx<T>* out, int nx, int64_t nrows, const cplx<T>* tw_x, hipStream_t s, int rpb,
                  const RowList& rl, int64_t pitch) {
  if (pitch <= 0) pitch = nx / 2 + 1;
  dispatch_row(nx / 2, [&](auto Mc) {
    constexpr int M = decltype(Mc)::value;
    using RC = RowCfg<T, M>;
    const int R = pick(rpb, RC::RPB);
    const int64_t nb = (nrows + R - 1) / R;
    const size_t lds = sizeof(cplx<T>) * (R * RC::LS + (RC::TWL ? 2 * M : 0));
    if (nb > 0)
      hipLaunchKernelGGL((k_x_r2c<T, M, TI>), dim3((unsigned)nb), dim3(R * RC::T), lds, s, in, out, nrows, tw_x, R, rl,
                         pitch);
  });
  IBDL_LAUNCH_CHECK();
}
}  // namespace

template <typename T>
void fft_x_r2c(const T* in, cplx<T>* out, int nx, int64_t nrows, const cplx<T>* tw_x, hipStream_t s, int rpb,
               const RowList& rl, int64_t pitch) {
  x_r2c_launch<T, T>(in, out, nx, nrows, tw_x, s, rpb, rl, pitch);
}

void fft_x_r2c_widen(const float* in, cplx<double>* out, int nx, int64_t nrows, const cplx<double>* tw_x,
                     hipStream_t s, int rpb, const RowList& rl, int64_t pitch) {
  x_r2c_launch<double, float>(in, out, nx, nrows, tw_x, s, rpb, rl, pitch);
}

template <typename T>
void fft_x_c2r(const cplx<T>* in, T* out, int nx, int64_t nrows, const cplx<T>* tw_x, hipStream_t s, int rpb,
               const RowList& rl, int64_t pitch) {
  if (pitch <= 0) pitch = nx / 2 + 1;
  dispatch_row(nx / 2, [&](auto Mc) {
    constexpr int M = decltype(Mc)::value;
    using RC = RowCfg<T, M>;
    const int R = pick(rpb, RC::RPB);
    const int64_t nb = (nrows + R - 1) / R;
    const size_t lds = sizeof(cplx<T>) * (R * RC::LS + (RC::TWL ? 2 * M : 0));
    if (nb > 0)
      hipLaunchKernelGGL((k_x_c2r<T, M>), dim3((unsigned)nb), dim3(R * RC::T), lds, s, in, out, nrows, tw_x, R, rl,
                         pitch);
  });
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void fft_strided(cplx<T>* data, int n, int64_t nlines, int64_t inner, int64_t outer, int64_t es, bool inverse,
                 const cplx<T>* tw, hipStream_t s, int w, const RowMask& rm, int64_t vinner, int plan) {
  if (vinner <= 0) vinner = inner;
  if (nlines <= 0) return;
  int64_t lastp = (nlines - 1) / inner;   // last plane touched
  if (rm.pspan > 0) lastp = (lastp / rm.pspan) * rm.nplanes + rm.p0 + rm.pspan - 1;
  const int64_t span = lastp * outer + (inner - 1) + (int64_t)(n - 1) * es + 1;
  if (span * (int64_t)sizeof(cplx<T>) > (int64_t)UINT32_MAX || nlines > INT32_MAX)
    throw Error(-2, "strided FFT pass: one launch may not span 4 GiB");
  dispatch_n(n, [&](auto Nc) {
    constexpr int N = decltype(Nc)::value;
    auto launch = [&](auto rxc) {
      constexpr int RX = decltype(rxc)::value;
      using TC = LineCfg<T, N, RX>;
      const int W = pick(w, TC::W);
      const int64_t nb = (nlines + W - 1) / W;
      const size_t lds = sizeof(cplx<T>) * (N * W + (TC::TWL ? N : 0));
      const dim3 blk(W * TC::T_);
      if (inverse)
        hipLaunchKernelGGL((k_strided<T, N, true, RX>), dim3((unsigned)nb), blk, lds, s, data, nlines, inner, outer,
                           es, tw, W, rm, vinner);
      else
        hipLaunchKernelGGL((k_strided<T, N, false, RX>), dim3((unsigned)nb), blk, lds, s, data, nlines, inner, outer,
                           es, tw, W, rm, vinner);
    };
    if (plan == 1 && plan_rx<T>(N, 1) != plan_rx<T>(N, 0))
      launch(std::integral_constant<int, plan_rx<T>(N, 1)>{});
    else
      launch(std::integral_constant<int, plan_rx<T>(N, 0)>{});
  });
  IBDL_LAUNCH_CHECK();
}

template <typename T>
void fft_fused_last(cplx<T>* data, int n, int64_t P, int no, const MultDesc& md, const cplx<T>* tw, hipStream_t s,
                    int batch, int64_t bstride, int w, const RowMask& rm, int plan) {
  if (batch < 1) return;
  if (n > kMaxLine) {
    // Four-step transform of the 2-D y lines, n = N1 N2 (N1 = kSplit): with y = j1 N2 + j2 and mode
    // k = k1 + N1 k2, the n-point DFT is an N1-point DFT over j1 for each j2 (a strided pass whose
    // result k1 stays at row k1 N2 + j2), the twiddles w_n^(j2 k1), and an N2-point DFT over j2 for
    // each k1, which leaves mode k1 + N1 k2 at row k1 N2 + k2.  The fused pass runs on those N2-point
    // lines (twiddles, transform, multiplier at the modes they hold, inverse, conjugate twiddles) and
    // an inverse N1-point pass per output field restores natural order.  Row masks do not carry over
    // to the split lines: the caller provides dense fields (every row valid) and takes every row back.
    if (md.dim != 2 || batch != 1 || n % kSplit != 0 || n / kSplit > kMaxLine)
      throw Error(-2, "fused FFT pass: lines over 1024 points are supported for single 2-D problems up to 8192");
    const int N2 = n / kSplit;
    const int64_t FS = P * n;
    const int64_t nin = std::max(md.nc, 1);
    for (int64_t f = 0; f < nin; ++f)
      fft_strided<T>(data + f * FS, kSplit, P * N2, P, P, (int64_t)N2 * P, false, tw, s, 0, RowMask(), md.nxh);
    MultDesc m2 = md;
    m2.split = kSplit;
    fft_fused_last<T>(data, N2, P * kSplit, no, m2, tw, s, 1, 0, w, RowMask(), plan);
    for (int o = 0; o < no; ++o)
      fft_strided<T>(data + o * FS, kSplit, P * N2, P, P, (int64_t)N2 * P, true, tw, s, 0, RowMask(), md.nxh);
    return;
  }
  const int64_t nf = std::max<int64_t>(std::max(md.nc, no), 1);
  if (nf * P * n * (int64_t)sizeof(cplx<T>) > (int64_t)UINT32_MAX || P > INT32_MAX)
    throw Error(-2, "fused FFT pass: one problem's fields may not span 4 GiB");
  dispatch_n(n, [&](auto Nc) {
    constexpr int N = decltype(Nc)::value;
    // launch shape of a kernel whose tile configuration is TC: lines per block, grid, LDS
    MultDesc mdl = md;   // with the tile map of the chosen width
    auto tiles = [&](int W) {
      int64_t nb = 0;
      mdl.map = line_map(P, md.nxp, md.nxh, W, &nb);
      return dim3((unsigned)nb, (unsigned)batch);
    };
    auto shape = [&](auto tc, int& W, dim3& grid, dim3& blk, size_t& lds) {
      using TC = decltype(tc);
      W = pick(w, TC::W);
      grid = tiles(W);
      blk = dim3(W * TC::T_);
      lds = sizeof(cplx<T>) * (N * W + (TC::TWL ? N : 0));
    };
    auto run = [&](auto splitc) {
      constexpr bool SP = decltype(splitc)::value;
      int W = 0;
      dim3 grid, blk;
      size_t lds = 0;
      const MultDesc& md = mdl;
      if (md.mode == 1 && md.nc == 1 && no >= 1 && no <= md.dim + 1) {
        shape(TileCfg<T, N, fused_rmax<T>(N, 1)>{}, W, grid, blk, lds);
        hipLaunchKernelGGL((k_fused_adj<T, N, 1, 1, SP>), grid, blk, lds, s, data, P, no, md, tw, W, bstride, rm);
      } else if (md.mode == 2 && md.stokes && md.nc == 2 && no >= 1 && no <= 5) {
        shape(TileCfg<T, N, fused_rmax<T>(N, 2)>{}, W, grid, blk, lds);
        hipLaunchKernelGGL((k_fused_adj<T, N, 2, 2, SP>), grid, blk, lds, s, data, P, no, md, tw, W, bstride, rm);
      } else if (md.mode == 3 && md.stokes && md.dim == 2 && no == 1) {
        shape(TileCfg<T, N, fused_rmax<T>(N, 1)>{}, W, grid, blk, lds);
        hipLaunchKernelGGL((k_fused<T, N, 1, true, SP>), grid, blk, lds, s, data, P, md, tw, W, bstride, rm);
      } else if (md.mode != 0) {
        throw Error(-2, "fused pass: unsupported transposed multiplier");
      } else if (!md.stokes && no == 1 && md.nc == 1 && md.fk[0] == FK_MASS) {
        if (plan == 1 && plan_rx<T>(N, 1) != plan_rx<T>(N, 0)) {
          constexpr int RX = plan_rx<T>(N, 1);
          shape(LineCfg<T, N, RX>{}, W, grid, blk, lds);
          hipLaunchKernelGGL((k_fused1<T, N, SP, RX>), grid, blk, lds, s, data, P, md, tw, W, bstride, rm);
        } else {
          shape(LineCfg<T, N>{}, W, grid, blk, lds);
          hipLaunchKernelGGL((k_fused1<T, N, SP>), grid, blk, lds, s, data, P, md, tw, W, bstride, rm);
        }
      } else if (!md.stokes && no == 1) {
        shape(TileCfg<T, N, fused_rmax<T>(N, 1)>{}, W, grid, blk, lds);
        hipLaunchKernelGGL((k_fused<T, N, 1, false, SP>), grid, blk, lds, s, data, P, md, tw, W, bstride, rm);
      } else if (md.stokes && no == 2 && md.dim == 2 && md.nc <= kStokesFields) {
        using SC = StokesCfg<T, N>;
        W = pick(w, SC::W);
        grid = tiles(W);
        blk = dim3(W * SC::T_);
        lds = sizeof(cplx<T>) * (size_t)kStokesFields * N * W;
        hipLaunchKernelGGL((k_fused_stokes2<T, N, SP>), grid, blk, lds, s, data, P, md, tw, W, bstride, rm);
      } else if (md.stokes && no == 2) {
        shape(TileCfg<T, N, fused_rmax<T>(N, 2)>{}, W, grid, blk, lds);
        hipLaunchKernelGGL((k_fused<T, N, 2, true, SP>), grid, blk, lds, s, data, P, md, tw, W, bstride, rm);
      } else {
        throw Error(-2, "fused pass: unsupported multiplier / output count");
      }
    };
    if (md.split > 1) {
      // the factor lines of 2048- to 8192-point y axes
      if constexpr (N >= kMaxLine * 2 / kSplit) {
        if (md.dim != 2 || batch != 1) throw Error(-2, "fused pass: four-step lines are single 2-D problems");
        run(std::true_type{});
      } else {
        throw Error(-2, "fused pass: four-step lines of " + std::to_string(N) + " points are not built");
      }
    } else {
      run(std::false_type{});
    }
  });
  IBDL_LAUNCH_CHECK();
}

#define IBDL_FFT_INST(T)                                                                                   \
  template void fft_x_r2c<T>(const T*, cplx<T>*, int, int64_t, const cplx<T>*, hipStream_t, int,         \
                             const RowList&, int64_t);                                                     \
  template void fft_x_c2r<T>(const cplx<T>*, T*, int, int64_t, const cplx<T>*, hipStream_t, int,         \
                             const RowList&, int64_t);                                                     \
  template void fft_strided<T>(cplx<T>*, int, int64_t, int64_t, int64_t, int64_t, bool, const cplx<T>*,   \
                               hipStream_t, int, const RowMask&, int64_t, int);                            \
  template void fft_fused_last<T>(cplx<T>*, int, int64_t, int, const MultDesc&, const cplx<T>*, hipStream_t, \
                                  int, int64_t, int, const RowMask&, int);                                 \
  template int fft_x_rpb_max<T>(int);                                                                      \
  template int fft_line_w_max<T>(int, int);                                                                \
  template int fft_line_plans<T>(int);
IBDL_FFT_INST(float)
IBDL_FFT_INST(double)

}  // namespace ibdl
