// Host-side launchers of the HIP kernels (implemented in fft.hip, ib.hip, krylov.hip).
#pragma once

#include "common.h"

namespace ibdl {

// ------------------------------------------------------------------ Fourier multiplier
// Field kinds of the inputs of the fused last-axis pass.
enum FieldKind {
  FK_DX = 0, FK_DY = 1, FK_DZ = 2,   // scalar: contributes i k~_d F^ (spectral divergence)
  FK_MASS = 3,                       // scalar: contributes F^
  FK_A11 = 4, FK_A12 = 5, FK_A22 = 6,  // Stokes dipole tensor components
  FK_G1 = 7, FK_G2 = 8               // Stokes single-layer / forcing components
};

// Rows (x-lines, index z * ny + y within a field) that carry data.  A spread field is zero outside
// the rows its markers' windows meet, and the interpolation reads only those rows, so the x passes
// can run over a list of them and the y passes can skip the loads / stores of the others.
// A spread also writes every node of each tile that a marker window meets (its busy tiles) and
// nothing else, so with seg set the forward x pass reads only the busy x-segments of a row and takes
// the others as zero: seg[r] has bit t set when x-segment t (2^seg_log2 complex values, one tile
// wide) of listed row r is in a busy tile.  The fields need no clearing then.
// With sub set, the forward x pass reads (field f, row w) minus sub[(f - sub_f0) * rpf + w] for the
// nsub fields from sub_f0 on (a dense forcing of the grid type, [nsub][rows per field][nx]).
struct RowList {
  const int* rows = nullptr;   // active rows of one field, increasing (NULL: every row)
  int64_t nact = 0;            // active rows per field
  int64_t rpf = 0;             // rows per field
  const unsigned long long* seg = nullptr;   // busy x-segments per listed row, or per row without a
  int seg_log2 = 3;                          // list (NULL: read everything)
  const void* sub = nullptr;
  int sub_f0 = 0, nsub = 0;
  __device__ int64_t row(int64_t r) const { return rows ? (int64_t)rows[r % nact] + (r / nact) * rpf : r; }
  __device__ unsigned long long segmask(int64_t r) const {
    return seg ? seg[rows ? r % nact : r % rpf] : ~0ull;
  }
  __device__ int64_t sub_row(int64_t r) const {   // row of sub to subtract from listed row r, or -1
    if (!sub) return -1;
    const int64_t f = rows ? r / nact : r / rpf;
    const int64_t w = rows ? (int64_t)rows[r % nact] : r % rpf;
    return (f >= sub_f0 && f < sub_f0 + nsub) ? (f - sub_f0) * rpf + w : -1;
  }
};
struct RowMask {
  const int2* lim = nullptr;   // per plane z: rows y in [lim.x, lim.y] matter (NULL: all)
  int nplanes = 1;
  int load = 0;                // read only those rows (others are zero)
  int store = 0;               // write only those rows
  int lo = 0, hi = 1 << 30;    // limits of the current plane (2-D: set by the host; else plane())
  // strided passes: when pspan > 0 the launch covers only planes p0 .. p0 + pspan - 1 of each field;
  // logical plane j is physical plane (j / pspan) * nplanes + p0 + j % pspan
  int p0 = 0, pspan = 0;
  __device__ unsigned phys_plane(unsigned j) const {
    if (pspan <= 0) return j;
    const unsigned f = j / (unsigned)pspan;
    return f * (unsigned)nplanes + (unsigned)p0 + (j - f * (unsigned)pspan);
  }
  __device__ RowMask plane(int64_t line_plane) const {
    RowMask m = *this;
    if (lim) {
      const int2 v = lim[line_plane % nplanes];
      m.lo = v.x;
      m.hi = v.y;
    }
    return m;
  }
  __device__ bool keep(int y) const { return !load || (y >= lo && y <= hi); }
  __device__ bool keep_out(int y) const { return !store || (y >= lo && y <= hi); }
};

// Assignment of tiles of W lines to the lines of a last-axis pass (set by fft_fused_last):
// on = 0, tile t holds lines t W .. t W + W - 1; on = 1, the first nlast tiles hold the last x mode
// of W consecutive rows (rows in all) and the others W consecutive x modes below the last of one row
// (2^lm tiles per row, W = 2^lw)
struct LineMap {
  int on = 0, lw = 0, lm = 0;
  unsigned nlast = 0, rows = 0;
};

struct MultDesc {
  int mode;         // 0: forward multiplier; 1: scalar gradient outputs; 2: transposed Stokes;
                    // 3: Stokes pressure
  int dim;          // 2 or 3
  int nxh;          // nx/2 + 1 modes along x
  int nxp;          // row pitch of the half spectrum (>= nxh; lines with x index >= nxh are padding)
  int stokes;       // 0: scalar multiplier, 1: Stokes multiplier
  int nc;           // input fields
  int fk[8];        // kind of each input field
  double sc;        // overall scale (1 / number of grid points)
  double c0, c2;    // symbol of -L is c2 * ell(k) + c0 with ell = -sigma (scalar: L = c2 Delta - c0)
  double mu;        // Stokes viscosity in the dipole term
  double alpha;     // overall sign / factor
  const void* sig[3];  // per-axis Laplacian symbol components (grid type)
  const void* kt[3];   // per-axis derivative symbols k~ (grid type)
  int split;           // 2-D lines of a four-step y transform: N1 > 1 (set by fft_fused_last); 0 or 1: none
  LineMap map;         // tiles -> lines (set by fft_fused_last)
};

// Tunable launch shapes: rpb = rows per block of the x passes, w = lines per block of the strided
// and fused passes (powers of two; 0 or anything above the maximum means the maximum that fits
// 256 threads and 64 KiB of LDS).
template <typename T> int fft_x_rpb_max(int nx);
template <typename T> int fft_line_w_max(int n, int plan = 0);
// radix plans of the single-field line passes of length n (1 or 2; plan 1 halves the elements per thread)
template <typename T> int fft_line_plans(int n);
// x passes over nrows rows (with a row list: nrows = active rows per field x fields)
// pitch: spectrum row pitch in complex values (0: nx/2 + 1)
template <typename T>
void fft_x_r2c(const T* in, cplx<T>* out, int nx, int64_t nrows, const cplx<T>* tw_x, hipStream_t s, int rpb = 0,
               const RowList& rl = RowList(), int64_t pitch = 0);
// the double forward x pass reading float rows (widened on load)
void fft_x_r2c_widen(const float* in, cplx<double>* out, int nx, int64_t nrows, const cplx<double>* tw_x,
                     hipStream_t s, int rpb = 0, const RowList& rl = RowList(), int64_t pitch = 0);
template <typename T>
void fft_x_c2r(const cplx<T>* in, T* out, int nx, int64_t nrows, const cplx<T>* tw_x, hipStream_t s, int rpb = 0,
               const RowList& rl = RowList(), int64_t pitch = 0);
// in-place strided C2C pass: line l starts at (l / inner) * outer + (l % inner), element stride es;
// lines with l % inner >= vinner are padding and skipped (vinner 0: none)
template <typename T>
void fft_strided(cplx<T>* data, int n, int64_t nlines, int64_t inner, int64_t outer, int64_t es,
                 bool inverse, const cplx<T>* tw, hipStream_t s, int w = 0, const RowMask& rm = RowMask(),
                 int64_t vinner = 0, int plan = 0);
// in-place fused pass along the last axis (length n, plane size P): forward FFT of the nc input
// fields, multiplier, inverse FFT of the no output fields (written to fields 0..no-1).
// mode 1 (one scalar input F): outputs i k~_o g F^ for o < dim, then g F^, g = alpha sc/(c2 sigma - c0);
// mode 2 (two Stokes components): output o = sum_c conj(m(fk[o], c)) F^_c, the transpose of the
// forward Stokes multiplier m(kind, component).
// batch problems with the same multiplier: problem b's fields start bstride elements after b-1's.
// 2-D lines of 2048 to 8192 points (one problem) run as a four-step transform in three passes; their
// fields must be valid on every row (rm is not applied) and every output row is written.
// plan: radix plan of the single-field scalar pass (fft_line_plans); the other passes keep theirs.
template <typename T>
void fft_fused_last(cplx<T>* data, int n, int64_t P, int no, const MultDesc& md, const cplx<T>* tw,
                    hipStream_t s, int batch = 1, int64_t bstride = 0, int w = 0,
                    const RowMask& rm = RowMask(), int plan = 0);
int fft_supported(int n);

// ------------------------------------------------------------------ markers, spread, interp
enum KernelId { KID_PESKIN4 = 0, KID_COS4 = 1, KID_BSPLINE6 = 2 };

struct MarkerGeom {
  int dim;
  int n[3];            // grid points per axis
  double origin[3];
  double h;
  int tile[3];         // tile edge per axis (2-D: 16 x 16; 3-D: 16 x 4 x 8)
  int ntile[3];        // tiles per axis
};
// log2 of the x-tiles per bit of the busy-segment masks (RowList::seg): 0 up to 64 tiles along x;
// wider 2-D grids group 2, 4, ... tiles per bit, since a mask has 64 bits
__host__ __device__ inline int seg_group_log2(const MarkerGeom& g) {
  int s = 0;
  while ((g.ntile[0] >> s) > 64) ++s;
  return s;
}

// marker setup: window start s[i][3] (wrapped), fractional offset f[i][3], weight table
// wt[i][3][12] (kernel weights W[0..5] and centred differences G[0..5] on the window), tile counts
// Batches: pid[i] is marker i's problem and tiles are numbered problem-major (nprob * ntile).
void markers_setup(const MarkerGeom& g, int kernel, int64_t n_ib, const double* X, int* s, double* f,
                   double* wt, int* tile_count, hipStream_t st, const int* pid = nullptr, int nprob = 1);
// bin markers by tile (sorted candidate lists) and list the non-empty tiles: busy[0..nbusy) with
// nbusy = busy_off[ntile], each (tile id, tile_off[tile], tile_off[tile + 1], 0), in decreasing
// order of candidate count (ties by tile id); busy_tmp: scratch of the same size
void markers_bin(const MarkerGeom& g, int64_t n_ib, const int* s, const int* tile_count,
                 int* tile_off, int* tile_cur, int* list, int* list_tmp, int4* busy, int4* busy_tmp, int* busy_off,
                 hipStream_t st, const int* pid = nullptr, int nprob = 1, int xcd_groups = 0);


// 3-D: the window starts of every listed candidate relative to its tile's first node, one int per
// list entry: bits 10a .. 10a + 9 hold (s_a - tile origin_a) mod n_a for axis a (n_a <= 1024)
void markers_list_offsets(const MarkerGeom& g, const int4* busy, int nbusy, const int* list, const int* s, int* lofs,
                          hipStream_t st);

// Active rows of the markers' windows: lo/hi [planes] (scratch), cnt/off [planes + 1] (scratch),
// lim [planes] = (lo, hi) per plane, rows = the row list (up to ny * planes entries), increasing;
// the count is off[planes].  planes = nz in 3-D, 1 in 2-D.
void markers_rows(const MarkerGeom& g, int64_t n_ib, const int* s, int* lo, int* hi, int* cnt, int* off, int2* lim,
                  int* rows, hipStream_t st);
// seg[r] = bit mask of the busy tiles along x that listed row r (rows[r], r < nact; row r itself
// when rows is NULL) passes through, 2^seg_group_log2(g) tiles per bit
void markers_row_segments(const MarkerGeom& g, const int* tile_off, const int* rows, int64_t nact,
                          unsigned long long* seg, hipStream_t st);

enum SpreadMode {
  SP_PLAIN = 0,     // nf fields: coef_c = f[i][c] ds_i h^-D
  SP_FDDIV = 1,     // 1 field: FD divergence of S(q n) + (eta q + m) S-term, fused in the stencil
  SP_SCALAR_VEC = 2,// dim (+1) fields: q n_d ds h^-D (and (eta q + m) ds h^-D)
  SP_STOKES = 3     // 3 or 5 fields: A11, A12, A22 (and eta Q1, eta Q2), times ds h^-D
};

struct SpreadArgs {
  MarkerGeom g;
  int kernel;
  int mode;
  int nf;             // output fields
  int mass;           // SP_FDDIV / SP_SCALAR_VEC: include the mass term
  int raw;            // SP_PLAIN: coef_c = f[i][c] (no ds_i h^-D): the transpose of S*
  double eta;
  const int* tile_off;
  const int* list;
  const int4* busy;   // non-empty tiles: (tile id, list begin, list end, 0)
  int nbusy;
  int xcd;            // busy is ordered in XCD ranges (markers_bin xcd_groups): workgroup b takes
                      // entry xcd_chunk(b, nbusy) (3-D spread)
  const int* lofs;    // 3-D: window starts of the list entries relative to their tiles
                      // (markers_list_offsets), or NULL
  const int* s;
  const double* f;
  const double* wt;   // per-marker weight table [n_ib][3][12]
  const double* q;    // densities [n_ib][nq] (or generic values [n_ib][nf] for SP_PLAIN)
  const double* m;    // optional extra mass values [n_ib] (Neumann V_b), may be null
  const double* nrm;  // [n_ib][dim]
  const double* ds;   // [n_ib]
};
// Spread over the non-empty tiles only: nodes of empty tiles are left untouched, so the caller
// clears the nf output fields first (grid_fill_zero).  A batch tile id p * ntile + t writes problem
// p's fields at out + p * nf * (grid points).  wtab: per-precision weight table
// [n_ib][3][8] of (W, G) pairs (weight_table).
template <typename T> void grid_fill_zero(T* y, int64_t n, hipStream_t st);
// *flag |= 1 when x[0..n) holds a NaN or an infinity (flag cleared by the caller)
template <typename T> void nonfinite_flag(const T* x, int64_t n, unsigned* flag, hipStream_t st);
template <typename T> void spread(const SpreadArgs& a, const cplx<T>* wtab, T* out, hipStream_t st);
template <typename T> void weight_table(const double* wt, int64_t n_ib, cplx<T>* tab, hipStream_t st);
// One grid group of a batch for the single-launch spread: its arguments (q is replaced by
// qbase + qoff at run time), weight table, output fields (of the grid type) and 2-D tile width.
struct SpreadGroup {
  SpreadArgs a;
  const void* wtab;
  void* out;
  int64_t qoff;
  int tx;
};
// The FD divergence spread (one field, 2-D, 4-point kernels) of several groups in one persistent
// launch of nblocks workgroups (0: one per item) over the work list items[k] = (group, busy-tile
// index), workgroup b taking items b, b + nblocks, ...
template <typename T>
void spread2_queue(const SpreadGroup* gd, const int2* items, int nitems, const double* qbase, int nblocks,
                   hipStream_t st);

struct InterpArgs {
  MarkerGeom g;
  int kernel;
  int nf;
  int64_t n_ib;
  const int* s;
  const double* f;
  const double* wt;    // per-marker weight table [n_ib][3][12]
  double a;            // out = a * S*u + b * x + ub
  double b;
  const double* x;     // [n_ib][nf] or null
  const double* ub;    // [nf] or null
  const int* pid;      // batch: marker i reads fields at u + pid[i] * nf * (grid points); or null
};
template <typename T> void interp(const InterpArgs& a, const cplx<T>* wtab, const T* u, double* out, hipStream_t st);
// One grid group of a batch for the single-launch interpolation: arguments (a.pid set), weight table,
// fields, and the index m0 of its first marker in the concatenation.
struct InterpGroup {
  InterpArgs a;
  const void* wtab;
  const void* u;
  int64_t m0;
};
// out[i] = a S*u + b x[i] for the ntot_m markers of ng groups (2-D, 4-point kernels, one field),
// x = xbase (may be null); gd: device array of ng groups in marker order.
template <typename T>
void interp4_groups(const InterpGroup* gd, int ng, int64_t ntot_m, const double* xbase, double* out, hipStream_t st);
// Transpose of the SP_FDDIV spread (4-point kernels): y_i = -h^-D ds_i sum_y w(y) [sum_d n_id G_d W W
// + eta W W W] + b p_i + eta ds_i pu, with p = a.x and b = a.b (p, pu may be null); one field w.
template <typename T>
void interp_div(const InterpArgs& a, const cplx<T>* wtab, const T* u, const double* nrm, const double* ds, double eta,
                double hDinv, const double* pu, double* y, hipStream_t st);

// Kernel-derivative gather: out[i][e] = sum_x F_i(x) d/dX_ie prod_d phi((x_d - X_id)/h), with
// F_i(x) = sum_k coef[i][k] field_k(x) (field_k of the grid type; at most 8 fields).
struct GatherArgs {
  MarkerGeom g;
  int kernel;
  int64_t n_ib;
  const int* s;
  const double* f;
  int nfield;
  const void* field[8];
  const double* coef;   // [n_ib][nfield]
  double* out;          // [n_ib][dim]
};
template <typename T> void gather_dx(const GatherArgs& a, hipStream_t st);

// ------------------------------------------------------------------ grid elementwise
template <typename T> void grid_axpby(T* y, double a, const T* x, double b, int64_t n, hipStream_t st);
void grid_widen(const float* x, double* y, int64_t n, hipStream_t st);   // y = (double) x
template <typename T> void grid_add_const(T* y, const double* c_dev, int ncomp, int64_t n, hipStream_t st);
template <typename T> void grid_sum(const T* x, int ncomp, int64_t n, double* partial, int nblk, double* out,
                                    hipStream_t st);

// ------------------------------------------------------------------ Krylov vectors (double)
void kr_multidot(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* partial,
                 int nblk, double* out, hipStream_t st);
void kr_gemv_sub(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t n, hipStream_t st);
void kr_lincomb(const double* V, int64_t ldv, int k, const double* y, double* x, int64_t n, hipStream_t st);
void kr_scale(const double* src, double s, double* dst, int64_t n, hipStream_t st);
// dst (and dst2 unless NULL) = src / sqrt(max(*nrm2, 0)) with the norm read on the device; zero
// when the norm is not above floor or not finite
void kr_scale_norm(const double* src, const double* nrm2, double floor, double* dst, double* dst2, int64_t n,
                   hipStream_t st);
void kr_axpby(double* y, double a, const double* x, double b, int64_t n, hipStream_t st);
void kr_border(const double* q, const double* ds, int64_t n_ib, int nq, double eta, double* out,
               double* partial, int nblk, hipStream_t st);
void kr_add(double* dst, const double* a, const double* b, int n, hipStream_t st);
int kr_nblk(int64_t n);
// One Arnoldi step's vector work, classical Gram-Schmidt twice on w against V_0..V_{k-1}
// (three launches; each reduces the previous one's block partial sums itself, in a fixed order):
// h[j] = V_j . w, w -= V h; h[256 + j] = V_j . w, w -= V h[256..]; the block partial sums of w . w
// are left at partial + 2 k nblk (reduced by kr_publish).  partial: (2 k + 1) * nblk doubles with
// nblk = kr_arnoldi_nblk(n); k <= 256.
void kr_arnoldi_step(const double* V, int64_t ldv, int k, double* w, int64_t n, double* partial, int nblk,
                     double* h, hipStream_t st);
int kr_arnoldi_nblk(int64_t n);
// Copy src[0..n) to host_dst, with src[norm_at] first set to the sum of pnorm[0..nblk) unless pnorm
// is NULL.  host_dst / host_tag: device addresses of host-mapped, coherent pinned memory; the tag is
// written last, after a system-scope fence
void kr_publish(double* src, int n, const double* pnorm, int nblk, int norm_at, double* host_dst,
                unsigned* host_tag, unsigned seq, hipStream_t st);
// GMRES least-squares state in device memory (kr_gmres_state_doubles(mx) doubles for at most mx
// steps): scalars GM_BETA (|b|), GM_RES (Krylov residual estimate / |b|), GM_K (steps the solution
// uses), GM_DONE (1 once res <= tol or the process broke down: later steps leave the state alone),
// GM_HN (|w| of the last step), then the rotations, the rotated right-hand side, the solution y and
// the rotated Hessenberg columns.  The first GM_PUB scalars are what a step publishes to the host.
enum { GM_BETA = 0, GM_RES = 1, GM_K = 2, GM_DONE = 3, GM_HN = 4, GM_PUB = 5, GM_HDR = 16 };
// the Arnoldi scratch h holds the first Gram-Schmidt pass at [0, 256), the second at [256, 512),
// |w|^2 at 512 and |b|^2 at GM_BNORM2_AT
constexpr int GM_BNORM2_AT = 520;
size_t kr_gmres_state_doubles(int mx);
// End of Arnoldi step j (w orthogonalised by kr_arnoldi_step, its norm partials at pnorm): h[norm_at]
// = |w|^2, the least-squares update of step j in gs (tolerance tol, at most mx <= 256 steps), the
// state's first GM_PUB scalars copied to the host slot, the tag; and, in the same launch, dst (and
// dst2 if set) = w / |w| over nv entries (0 where the norm is 0 or not finite), every workgroup
// reducing the partials itself in the same order.
void kr_publish_scale(double* h, const double* pnorm, int nblk, int norm_at, double* gs, int j, int mx, double tol,
                      double* host_dst, unsigned* host_tag, unsigned seq, const double* w, double* dst, double* dst2,
                      int64_t nv, hipStream_t st);
// kr_arnoldi_step and kr_publish_scale in one workgroup and one launch for n <= kSmallN (step k - 1,
// k basis vectors); deterministic, its sums group the entries differently from the blocked path
constexpr int kSmallN = 256;
void kr_arnoldi_small(const double* V, int64_t ldv, int k, double* w, int64_t n, double* h, int norm_at, double* gs,
                      int mx, double tol, double* host_dst, unsigned* host_tag, unsigned seq, double* dst,
                      double* dst2, hipStream_t st);
// y = R^-1 g of the state's GM_K steps, in device memory at kr_gmres_ydev(gs, mx)
void kr_gmres_y(double* gs, int mx, hipStream_t st);
const double* kr_gmres_ydev(double* gs, int mx);
// y = R^-1 g and x = V y over the state's GM_K steps; gate: only if the state's convergence flag is
// set when the kernels run (queued behind a step predicted to be the last)
void kr_gmres_finish(double* gs, int mx, const double* V, int64_t ldv, double* x, int64_t n, bool gate,
                     hipStream_t st);

// ------------------------------------------------------------------ batched Krylov vectors
// Concatenated per-problem vectors of total length n: seg[e] is element e's problem; dot-product
// block b covers [beg[b], end[b]) of one problem, whose blocks are pb0[p] .. pb0[p+1]-1.
struct KrylovSegments {
  int nprob = 0;
  int64_t n = 0;
  int nblk = 0;
  const int* seg = nullptr;
  const int64_t* beg = nullptr;
  const int64_t* end = nullptr;
  const int* pb0 = nullptr;
};
// out[p * ostride + j] = <V_j, w> over problem p's segment, j < k
void kb_multidot(const double* V, int64_t ldv, int k, const double* w, const KrylovSegments& sg, double* partial,
                 int ostride, double* out, hipStream_t st);
void kb_gemv_sub(const double* V, int64_t ldv, int k, const double* H, int hs, const KrylovSegments& sg, double* w,
                 hipStream_t st);
void kb_lincomb(const double* V, int64_t ldv, int k, const double* Y, int ys, const KrylovSegments& sg, double* x,
                hipStream_t st);
void kb_scale(const double* src, const double* sc, const KrylovSegments& sg, double* dst, hipStream_t st);
// Batched GMRES on the device, one workgroup per problem; off[p], len[p] (device) locate problem p's
// segment of the batch vectors, bn2[p] = |b_p|^2, gsb + p * gstride its least-squares state
// (kr_gmres_state_doubles(mx) doubles each).
// Copy every problem's own array ptr[p] (device array of np device pointers) into its segment of a
// batch vector (to_batch) or back, in one launch; maxlen: the largest len[p].
void kb_seg_copy(const double* const* ptr, const int64_t* off, const int64_t* len, int np, int64_t maxlen,
                 double* base, bool to_batch, hipStream_t st);
// V[0] (and xin) = b / |b| per problem.
void kb_gmres_start(const double* b, const int64_t* off, const int64_t* len, int np, const double* bn2, double* v0,
                    double* xin, hipStream_t st);
// Arnoldi step j of every problem (w = A V_j): CGS2, |w|, the least-squares update, then vnext (and
// xin) = w / |w|; problems already converged write zeros and keep their state.
// maxlen: the largest len[p] (problems of at most 4096 unknowns keep w in registers).
void kb_arnoldi(const double* V, int64_t ldv, int j, double* w, const int64_t* off, const int64_t* len, int np,
                int64_t maxlen, const double* bn2, double* gsb, int64_t gstride, int mx, double tol, double* vnext,
                double* xin, hipStream_t st);
// every problem's first GM_PUB state scalars to the host slot ([np][GM_PUB]), then the tag
void kb_publish(const double* gsb, int64_t gstride, int np, double* host_dst, unsigned* host_tag, unsigned seq,
                hipStream_t st);
// Y[p][0..kmax) = the least-squares solution of problem p (zeros beyond its step count)
void kb_gmres_y(double* gsb, int64_t gstride, int np, int mx, int kmax, double* Y, int ys, hipStream_t st);

// ------------------------------------------------------------------ near-boundary tools (2-D)
struct NearGeom {
  int nx, ny;       // grid points per axis
  double ox, oy;    // origin
  double h;
};
// chi = (reg_in - reg_in[0] >= 1/2), reg_out (unless NULL) = reg_in - reg_in[0]; n values
template <typename T>
void indicator_finish(const T* reg_in, int64_t n, T* chi, T* reg_out, hipStream_t st);
void fill_value(double* x, double v, int64_t n, hipStream_t st);
// capacity of the node list near_boundary needs
int64_t near_list_cap(int64_t n_ib, double m1, int64_t npoints);
// out = u ([nc][ny][nx]), then every node with omega != 0 within m1 h of a marker X[i] (2-D,
// [n_ib][2]) gets the near-boundary interpolation of each component c (boundary values
// Ub[i * nc + c], second point m2 h inside).  Scratch: flag [nx * ny] bytes, count [1], list
// [near_list_cap].
template <typename T>
void near_boundary(const double* X, const double* Ub, int nc, int64_t n_ib, const NearGeom& g, double m1, double m2,
                   const T* omega, const T* u, T* out, unsigned char* flag, int* count, int* list,
                   const int* cell_off, const int* cell_list, hipStream_t st);
// Marker cells of the near-boundary search (squares of 8 x 8 nodes): their number (and ncx, ncy),
// and the binning of the n_ib markers X: cell_cnt [cells] scratch, cell_off [cells + 1], cell_list
// [n_ib] (marker ids by cell).
int near_cells(const NearGeom& g, int* ncx, int* ncy);
void near_bin(const double* X, int64_t n_ib, const NearGeom& g, int* cell_cnt, int* cell_off, int* cell_list,
              hipStream_t st);
// off[0..n] = exclusive scan of cnt[0..n) (one workgroup)
void exclusive_scan(const int* cnt, int* off, int n, hipStream_t st);

// ------------------------------------------------------------------ MINRES (device recurrences)
// State slots of the double-buffered scalar recurrence (MR_NSTATE doubles per copy).
enum { MR_BETA = 0, MR_C1, MR_S1, MR_C2, MR_S2, MR_ETA, MR_BETA1, MR_DONE, MR_ITERS, MR_ALPHA, MR_TOL, MR_NSTATE };
int mr_nblk(int64_t n);
// beta1 = |b|_wt; v = b / beta1; vprev = w1 = w2 = x = 0; state initialised.  partial: mr_nblk(n).
void mr_start(const double* b, const double* wt, int64_t n, double tol, double* v, double* vprev, double* w1,
              double* w2, double* x, double* partial, double* state, hipStream_t st);
// One iteration after p = A v: reads state `in`, writes state `out` (another copy); hist[k-1] =
// the recurrence residual / beta1.  partial: 2 mr_nblk(n) doubles.
void mr_iteration(double* v, double* vprev, double* p, double* w1, double* w2, double* x, const double* wt,
                  int64_t n, double* partial, const double* in, double* out, double* hist, int64_t hist_cap,
                  hipStream_t st);

// ------------------------------------------------------------------ force and line integrals (2-D)
// out[3] = (B_x, B_y, L) of the completed density Q [n_ib][2]: B = -eta sum ds Q, L = -eta sum ds X x Q
void net_force(const double* X, const double* Q, const double* ds, int64_t n_ib, double eta, double* out,
               hipStream_t st);
// out[0] = h * sum_k u[k * stride], k < n
template <typename T>
void line_sum(const T* u, int64_t stride, int64_t n, double h, double* out, hipStream_t st);

// ------------------------------------------------------------------ adjoint, marker side
// y = h^-D ds (.) (combination of the interpolated adjoint fields G [n_ib][ng]) + b p + eta ds pu
void adj_combine(int stokes, int dim, int64_t n_ib, int ng, double hDinv, double eta, const double* G,
                 const double* nrm, const double* ds, const double* p, double b, const double* pu, double* y,
                 hipStream_t st);
// per-marker weights coef [n_ib][nc] of the fields gathered with kernel derivatives for dL/dX
void adj_coefs(int stokes, int dim, int64_t n_ib, int nc, double hDinv, double eta, const double* mu,
               const double* q, const double* nrm, const double* ds, double* coef, hipStream_t st);

}  // namespace ibdl
