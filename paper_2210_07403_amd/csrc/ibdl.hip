// Host runtime and C ABI: handle lifecycle, per-precision grid workspaces, the IBDL operator
// pipelines (spread -> FFT passes with the fused multiplier -> interpolation), right-hand sides,
// grid recovery and the device-resident GMRES.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <memory>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/ibdl.h"
#include "kernels.h"
#include "ns.h"
#include "tables.h"
#include "tune.h"

using namespace ibdl;

namespace {

constexpr int kSlot = 1024;   // doubles per host-mapped Arnoldi slot (h1, h2 and the norm)
constexpr int kYOff = 2 * kSlot + 128;   // host-mapped doubles before the GMRES solution y
constexpr int kYSlot = 256;

template <typename T> struct GridWork {
  cplx<T>* tw[3] = {nullptr, nullptr, nullptr};
  T* sig[3] = {nullptr, nullptr, nullptr};
  T* kt[3] = {nullptr, nullptr, nullptr};
  T* real = nullptr;
  cplx<T>* spec = nullptr;
  cplx<T>* wtab = nullptr;   // marker weight table in this precision
  int nfields = 0;
  LaunchShape shape;         // launch shapes of the operator apply's FFT passes (measured)
  bool tuned = false;
};

std::string g_create_error;

}  // namespace

namespace ibdl {
// the message ibdl_last_error(NULL) returns: the last failed ibdl_create or handle-free call
void set_global_error(const std::string& msg) { g_create_error = msg; }
}  // namespace ibdl

struct ibdl_s {
  ibdl_config_t cfg{};
  int dim = 2;
  int n[3] = {1, 1, 1};
  double h = 0;
  int64_t ntot = 0, nxh = 0, nxp = 0, nspec = 0;   // nxp: half-spectrum row pitch (128-byte rows)
  int64_t n_ib = 0;
  int nq = 1;
  bool has_ubar = false;
  int64_t n_aug = 0;
  // Single-layer method (IBSL): the density spreads with weight 1 and no dipole (normals held at
  // zero), no identity term, border rows sum_i (ds_i / mean ds) F_i; solved with MINRES.
  bool sl = false;
  double sl_border = 0.0;       // 1 / mean(ds)
  double* mr = nullptr;         // MINRES vectors vprev, w1, w2 [3][n_aug]
  double* mr_state = nullptr;   // two copies of the scalar recurrence state (32 doubles)
  double* mr_wt = nullptr;      // inner-product weights [n_aug]
  double* mr_hist = nullptr;
  int64_t mr_hist_cap = 0;
  void* ns_scratch = nullptr;   // Navier-Stokes step: forcing and raw velocity, [4][grid] of the grid type
  hipStream_t st = nullptr;
  hipStream_t aux = nullptr;    // second stream: the double-precision residual beside the recovery
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double *X = nullptr, *nrm = nullptr, *ds = nullptr;
  int* s = nullptr;
  double* f = nullptr;
  double* wt = nullptr;   // per-marker kernel weight table [n_ib][3][12]
  int *tile_count = nullptr, *tile_off = nullptr, *tile_cur = nullptr, *list = nullptr, *list_tmp = nullptr;
  int* lofs = nullptr;   // 3-D: window starts of the list entries relative to their tiles
  int4* busy = nullptr;
  int4* busy_tmp = nullptr;
  int* busy_off = nullptr;
  int nbusy = 0;
  unsigned long long* seg = nullptr;       // busy x-segments of each active row (RowList::seg)
  unsigned long long* seg_all = nullptr;   // busy x-segments of every row of a field
  // active rows (rows of the markers' windows): list for the x passes, per-plane limits for y
  int *row_lo = nullptr, *row_hi = nullptr, *row_cnt = nullptr, *row_off = nullptr, *rows = nullptr;
  int2* row_lim = nullptr;
  int64_t nact = 0;
  int64_t seg_read = 0;       // (active row, busy x-segment) pairs the apply's forward x pass reads
  int lim2d[2] = {0, -1};     // 2-D: the one plane's limits, on the host
  int zlim[2] = {0, -1};      // 3-D: first and last z plane holding an active row, on the host
  bool check = false;         // IBDL_CHECK=1 at creation: device arrays scanned for NaN / Inf
  unsigned* chk = nullptr;    // the scan's flag
  MarkerGeom geom{};
  std::unique_ptr<GridWork<float>> w32;
  std::unique_ptr<GridWork<double>> w64;
  double* V = nullptr;
  int vcap = 0;
  double* gm = nullptr;       // GMRES least-squares state on the device (kr_gmres_state_doubles)
  int gmcap = 0;
  double* small = nullptr;    // 1024 doubles of small device scratch
  double* partial = nullptr;  // partial sums
  int pcap = 0;
  double* vb = nullptr;       // right-hand side
  double* vr = nullptr;       // residual scratch
  double* hostbuf = nullptr;  // pinned host scratch (1024 doubles)
  // host-mapped coherent memory for the per-iteration Arnoldi values: the GPU writes them and a
  // sequence tag, the host polls the tag (no copy-engine transfer, no stream-sync wake-up)
  // host-mapped Arnoldi values: two slots of kSlot doubles, then one 64-byte tag per slot, then
  // the least-squares solution y of the last GMRES call (kYSlot doubles, read by the device)
  double* hmap = nullptr;
  double* hmap_dev = nullptr;
  volatile unsigned* htag = nullptr;
  unsigned* htag_dev = nullptr;
  unsigned seq = 0;
  // the working-precision operator apply (and its transpose) captured in HIP graphs, replayed from
  // the fixed vectors gx -> gy inside GMRES (rebuilt when the markers change)
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  double *gx = nullptr, *gy = nullptr;
  bool use_graph = true;
  void drop_graphs() {
    for (int k = 0; k < 2; ++k) {
      if (gexec[k]) (void)hipGraphExecDestroy(gexec[k]);
      if (graph[k]) (void)hipGraphDestroy(graph[k]);
      gexec[k] = nullptr;
      graph[k] = nullptr;
    }
  }
  double* ones = nullptr;     // indicator: the unit density [n_ib]
  unsigned char* nb_flag = nullptr;   // near-boundary scratch: node flags [grid]
  int* nb_count = nullptr;            // near-boundary scratch: listed nodes [1]
  int* nb_list = nullptr;             // near-boundary scratch: node list
  int64_t nb_cap = 0;
  int *nb_cell_cnt = nullptr, *nb_cell_off = nullptr, *nb_cell_list = nullptr;   // marker cells
  bool nb_cells_ready = false;
  double* g64 = nullptr;      // refinement: the forcing widened to double ([nq][grid])
  double* vx = nullptr;       // refinement: correction of one round [n_aug]
  double* adj_m = nullptr;    // adjoint: interpolated fields / gather weights [n_ib][8]
  double* adj_mu = nullptr;   // adjoint solution [n_aug]
  std::vector<void*> allocs;
  std::string err;
  // optional per-stage timing with HIP events on the handle's stream
  bool timing = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> evpool;
  double stage_ms[16] = {0};
  int64_t stage_n[16] = {0};
  hipEvent_t take_event() {
    if (evpool.empty()) {
      hipEvent_t e;
      IBDL_HIP(hipEventCreate(&e));
      return e;
    }
    hipEvent_t e = evpool.back();
    evpool.pop_back();
    return e;
  }
  void collect() {
    for (auto& p : pending) {
      float ms = 0;
      IBDL_HIP(hipEventSynchronize(p.second.second));
      IBDL_HIP(hipEventElapsedTime(&ms, p.second.first, p.second.second));
      stage_ms[p.first] += ms;
      stage_n[p.first] += 1;
      evpool.push_back(p.second.first);
      evpool.push_back(p.second.second);
    }
    pending.clear();
  }

  void dfree(void* p) {
    if (!p) return;
    for (size_t k = 0; k < allocs.size(); ++k)
      if (allocs[k] == p) {
        if (st) IBDL_HIP(hipStreamSynchronize(st));
        IBDL_HIP(hipFree(p));
        allocs.erase(allocs.begin() + (long)k);
        return;
      }
  }
  template <typename T> void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 16;
    IBDL_HIP(hipMalloc(&p, bytes));
    allocs.push_back(p);
    return p;
  }
  ~ibdl_s() {
    if (!allocs.empty()) {
      if (st) (void)hipStreamSynchronize(st);
      else (void)hipDeviceSynchronize();
    }
    for (void* p : allocs) (void)hipFree(p);
    drop_graphs();
    if (hostbuf) (void)hipHostFree(hostbuf);
    if (hmap) (void)hipHostFree(hmap);
    for (auto& p : pending) {
      (void)hipEventDestroy(p.second.first);
      (void)hipEventDestroy(p.second.second);
    }
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    if (aux) (void)hipStreamSynchronize(aux);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (aux) (void)hipStreamDestroy(aux);
  }
  bool mixed() const { return cfg.precision == IBDL_MIXED; }
  bool stokes() const { return cfg.pde == IBDL_PDE_STOKES; }
  bool neumann() const { return cfg.bc == IBDL_BC_NEUMANN; }
  bool fd() const { return cfg.disc == IBDL_DISC_FD2; }
  // identity term of the operator: Q/2 (Dirichlet), -U/2 (Neumann), none for the single layer
  double half() const { return sl ? 0.0 : (neumann() ? -0.5 : 0.5); }
  // border rows: eta sum ds Q (completed double layer), sum (ds / mean ds) F (single layer)
  double border_w() const { return sl ? sl_border : cfg.eta; }
  double kappa() const { return cfg.pde == IBDL_PDE_POISSON ? 0.0 : cfg.kappa; }
  // grid fields needed at once (real and spectral)
  int fields_needed() const {
    if (stokes()) return 5;
    if (fd()) return 1;
    return dim + 1;
  }
  template <typename T> GridWork<T>& work();
};

template <> GridWork<float>& ibdl_s::work<float>() {
  if (!w32) w32.reset(new GridWork<float>());
  return *w32;
}
template <> GridWork<double>& ibdl_s::work<double>() {
  if (!w64) w64.reset(new GridWork<double>());
  return *w64;
}

namespace {

// Stage ids reported by ibdl_get_timing.
enum Stage { ST_SPREAD = 0, ST_FFT_X_FWD = 1, ST_FFT_Y_FWD = 2, ST_FUSED = 3, ST_FFT_Y_INV = 4, ST_FFT_X_INV = 5,
             ST_INTERP = 6, ST_KRYLOV = 7, ST_FILL = 8, ST_COUNT = 9 };

struct StageTimer {
  ibdl_s* h;
  int id;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(ibdl_s* h_, int id_) : h(h_), id(id_) {
    if (h->timing) {
      a = h->take_event();
      b = h->take_event();
      IBDL_HIP(hipEventRecord(a, h->st));
    }
  }
  ~StageTimer() {
    if (a) {
      (void)hipEventRecord(b, h->st);
      h->pending.push_back({id, {a, b}});
    }
  }
};

template <typename T> GridWork<T>& ensure_work(ibdl_s* h) {
  GridWork<T>& W = h->work<T>();
  if (W.real) return W;
  const int nf = h->fields_needed();
  W.nfields = nf;
  W.real = (T*)h->dalloc<T>(sizeof(T) * h->ntot * nf);
  W.spec = (cplx<T>*)h->dalloc<T>(sizeof(cplx<T>) * h->nspec * nf);
  W.wtab = (cplx<T>*)h->dalloc<T>(sizeof(cplx<T>) * h->n_ib * 24);
  weight_table<T>(h->wt, h->n_ib, W.wtab, h->st);
  GridTables<T> G = make_grid_tables<T>(h->dim, h->n, h->cfg.L, h->h, h->fd(),
                                        [&](size_t bytes) { return h->dalloc<T>(bytes); });
  for (int d = 0; d < 3; ++d) {
    W.tw[d] = G.tw[d];
    W.sig[d] = G.sig[d];
    W.kt[d] = G.kt[d];
  }
  return W;
}

template <typename T> GridWork<T>& ensure_fields(ibdl_s* h, int nf) {
  GridWork<T>& W = ensure_work<T>(h);
  if (W.nfields >= nf) return W;
  h->dfree(W.real);
  h->dfree(W.spec);
  W.real = (T*)h->dalloc<T>(sizeof(T) * h->ntot * nf);
  W.spec = (cplx<T>*)h->dalloc<T>(sizeof(cplx<T>) * h->nspec * nf);
  W.nfields = nf;
  return W;
}

template <typename T> MultDesc base_desc(ibdl_s* h, GridWork<T>& W) {
  MultDesc md{};
  md.dim = h->dim;
  md.nxh = (int)h->nxh;
  md.nxp = (int)h->nxp;
  md.sc = 1.0 / (double)h->ntot;
  md.mu = h->cfg.mu;
  for (int d = 0; d < 3; ++d) {
    md.sig[d] = d < h->dim ? W.sig[d] : W.sig[0];
    md.kt[d] = d < h->dim ? W.kt[d] : W.kt[0];
  }
  if (h->stokes()) {
    md.stokes = 1;
    md.c2 = h->cfg.mu;
    md.c0 = h->cfg.kappa * h->cfg.kappa;
  } else {
    md.stokes = 0;
    md.c2 = 1.0;
    md.c0 = h->kappa() * h->kappa();
  }
  return md;
}

// real fields src[0..nin) -> spectra -> fused multiplier -> real fields dst[0..nout).
// Row modes: ROWS_DENSE every row; ROWS_SPARSE src is zero outside the active rows and only the
// active rows of dst are needed (the operator apply), so the x passes run over the row list and the
// y passes mask the other rows; ROWS_OUT a dense src whose result is needed on the active rows only
// (a right-hand side that is interpolated next).
enum RowsMode { ROWS_DENSE = 0, ROWS_SPARSE = 1, ROWS_OUT = 2 };

// srcf: float input fields for a double pipeline (widened as the forward x pass reads them; src unused)
template <typename T>
void pipeline(ibdl_s* h, GridWork<T>& W, const T* src, int nin, T* dst, int nout, const MultDesc& md,
              int rows = ROWS_DENSE, bool busy_only = false, const T* sub = nullptr, int sub_f0 = 0, int nsub = 0,
              const float* srcf = nullptr) {
  const int64_t rows_per_field = h->ntot / h->n[0];
  // 2-D grids of more than 1024 points along y: the last-axis pass is a four-step transform that
  // reads and writes every row, so the forward x pass covers every row (those the markers do not
  // reach come out zero without being read) and the y row limits are not applied
  const bool split = h->dim == 2 && h->n[1] > 1024;
  const bool sin = rows == ROWS_SPARSE && !split, sout = rows != ROWS_DENSE;
  RowList rl_in, rl_out;
  RowMask fwd, inv, fused;
  rl_in.rpf = rows_per_field;
  if (busy_only) {   // src holds a spread's output: only its busy tiles were written
    rl_in.seg = sin ? h->seg : h->seg_all;
    rl_in.seg_log2 = __builtin_ctz((unsigned)h->geom.tile[0] / 2) + seg_group_log2(h->geom);
  }
  rl_in.sub = sub;   // minus a dense forcing on fields sub_f0 .. sub_f0 + nsub - 1
  rl_in.sub_f0 = sub_f0;
  rl_in.nsub = nsub;
  if (sout) {
    rl_out.rows = h->rows;
    rl_out.nact = h->nact;
    rl_out.rpf = rows_per_field;
    if (sin) {
      rl_in.rows = h->rows;
      rl_in.nact = h->nact;
    }
    if (h->dim == 3) {
      // only the planes with active rows matter on the way out (the inverse y pass and the
      // last-axis stores), and on the way in when the input is zero elsewhere
      fwd.lim = inv.lim = h->row_lim;
      fwd.nplanes = inv.nplanes = h->n[2];
      fwd.load = sin ? 1 : 0;
      inv.store = 1;
      inv.p0 = h->zlim[0];
      inv.pspan = std::max(0, h->zlim[1] - h->zlim[0] + 1);
      if (sin) {
        fwd.p0 = inv.p0;
        fwd.pspan = inv.pspan;
      }
      fused.load = sin ? 1 : 0;
      fused.store = 1;
      fused.lo = h->zlim[0];
      fused.hi = h->zlim[1];
    } else if (!split) {
      fused.load = sin ? 1 : 0;
      fused.store = 1;
      fused.lo = h->lim2d[0];
      fused.hi = h->lim2d[1];
    }
  }
  const bool tuned = rows == ROWS_SPARSE;   // the measured shapes are those of the apply
  const int64_t rin = sin ? h->nact * nin : rows_per_field * nin;
  const int64_t rout = sout ? h->nact * nout : rows_per_field * nout;
  {
    StageTimer t(h, ST_FFT_X_FWD);
    if constexpr (std::is_same<T, double>::value) {
      if (srcf) fft_x_r2c_widen(srcf, W.spec, h->n[0], rin, W.tw[0], h->st, tuned ? W.shape.rpb : 0, rl_in, h->nxp);
      else fft_x_r2c<T>(src, W.spec, h->n[0], rin, W.tw[0], h->st, tuned ? W.shape.rpb : 0, rl_in, h->nxp);
    } else {
      if (srcf) throw Error(IBDL_ERR_UNSUPPORTED, "float input fields are for the double pipeline");
      fft_x_r2c<T>(src, W.spec, h->n[0], rin, W.tw[0], h->st, tuned ? W.shape.rpb : 0, rl_in, h->nxp);
    }
  }
  if (h->dim == 3) {
    StageTimer t(h, ST_FFT_Y_FWD);
    fft_strided<T>(W.spec, h->n[1], (int64_t)nin * (fwd.pspan ? fwd.pspan : h->n[2]) * h->nxp, h->nxp,
                   h->nxp * h->n[1], h->nxp, false, W.tw[1], h->st, tuned ? W.shape.wy : 0, fwd, h->nxh,
                   tuned ? W.shape.py : 0);
  }
  const int last = h->dim - 1;
  const int64_t P = h->nspec / h->n[last];
  {
    StageTimer t(h, ST_FUSED);
    fft_fused_last<T>(W.spec, h->n[last], P, nout, md, W.tw[last], h->st, 1, 0, tuned ? W.shape.wz : 0, fused,
                      tuned ? W.shape.pz : 0);
  }
  if (h->dim == 3 && !(sout && inv.pspan == 0)) {
    StageTimer t(h, ST_FFT_Y_INV);
    fft_strided<T>(W.spec, h->n[1], (int64_t)nout * (inv.pspan ? inv.pspan : h->n[2]) * h->nxp, h->nxp,
                   h->nxp * h->n[1], h->nxp, true, W.tw[1], h->st, tuned ? W.shape.wy : 0, inv, h->nxh,
                   tuned ? W.shape.py : 0);
  }
  {
    StageTimer t(h, ST_FFT_X_INV);
    fft_x_c2r<T>(W.spec, dst, h->n[0], rout, W.tw[0], h->st, tuned ? W.shape.rpb : 0, rl_out, h->nxp);
  }
}


SpreadArgs spread_args(ibdl_s* h, int mode, int nf, const double* q) {
  SpreadArgs a{};
  a.g = h->geom;
  a.kernel = h->cfg.kernel;
  a.mode = mode;
  a.nf = nf;
  a.eta = h->cfg.eta;
  a.tile_off = h->tile_off;
  a.list = h->list;
  a.busy = h->busy;
  a.nbusy = h->nbusy;
  a.xcd = h->dim == 3 ? 1 : 0;
  // the tile-aligned FD spread addresses weight rows by 32-bit byte offsets
  a.lofs = h->n_ib * 24 * (int64_t)sizeof(cplx<double>) <= (int64_t)UINT32_MAX ? h->lofs : nullptr;
  a.s = h->s;
  a.f = h->f;
  a.wt = h->wt;
  a.q = q;
  a.nrm = h->nrm;
  a.ds = h->ds;
  return a;
}

// the spread with this precision's tables and coefficient scratch.  Where a busy-segment bit covers
// several x-tiles (2-D grids over 1024 points wide) the idle tiles of a busy segment are read too, so
// the output fields are cleared first.
template <typename T> void spread_w(ibdl_s* h, SpreadArgs a, GridWork<T>& W, T* out) {
  if (seg_group_log2(h->geom) > 0) grid_fill_zero<T>(out, (int64_t)a.nf * h->ntot, h->st);
  spread<T>(a, W.wtab, out, h->st);
}

InterpArgs interp_args(ibdl_s* h, int nf, double a, double b, const double* x, const double* ub) {
  InterpArgs ia{};
  ia.g = h->geom;
  ia.kernel = h->cfg.kernel;
  ia.nf = nf;
  ia.n_ib = h->n_ib;
  ia.s = h->s;
  ia.f = h->f;
  ia.wt = h->wt;
  ia.a = a;
  ia.b = b;
  ia.x = x;
  ia.ub = ub;
  return ia;
}

void ensure_partial(ibdl_s* h, int need) {
  if (h->pcap >= need) return;
  h->partial = (double*)h->dalloc<double>(sizeof(double) * need);
  h->pcap = need;
}

// The spread fields and Fourier multiplier of the density-to-grid map: Stokes A11, A12, A22 (and
// eta Q1, eta Q2 or the forcing); FD scalar one fused divergence field (plus the mass term);
// spectral scalar the D components of q n (plus the mass field).
struct DensityPlan {
  int mode = SP_FDDIV;
  int nf = 1;       // spread fields = multiplier inputs
  int nout = 1;
  MultDesc md{};
};

template <typename T> DensityPlan density_plan(ibdl_s* h, GridWork<T>& W, bool mass) {
  DensityPlan p;
  p.md = base_desc<T>(h, W);
  MultDesc& md = p.md;
  if (h->stokes()) {
    p.mode = SP_STOKES;
    p.nf = mass ? 5 : 3;
    p.nout = 2;
    const int kinds[5] = {FK_A11, FK_A12, FK_A22, FK_G1, FK_G2};
    for (int i = 0; i < p.nf; ++i) md.fk[i] = kinds[i];
    md.alpha = 1.0;
  } else if (h->fd()) {
    p.mode = SP_FDDIV;
    p.nf = 1;
    md.fk[0] = FK_MASS;
    md.alpha = -1.0;
  } else {
    p.mode = SP_SCALAR_VEC;
    p.nf = h->dim + (mass ? 1 : 0);
    for (int d = 0; d < h->dim; ++d) md.fk[d] = FK_DX + d;
    if (mass) md.fk[h->dim] = FK_MASS;
    md.alpha = -1.0;
  }
  md.nc = p.nf;
  return p;
}

// Density q (device, [n_ib][nq]) -> grid field u[q] induced by it (plus optional mass values m and
// forcing g as in the grid recovery), written to dst (nq fields).
template <typename T>
void density_to_grid(ibdl_s* h, const double* q, const double* m, const T* g, T* dst, bool sparse = false) {
  GridWork<T>& W = ensure_work<T>(h);
  const bool mass = h->cfg.eta > 0 || m != nullptr || g != nullptr;
  const DensityPlan pl = density_plan<T>(h, W, mass);
  SpreadArgs a = spread_args(h, pl.mode, pl.nf, q);
  // FD: the mass term of the fused field carries eta q and m; a forcing is subtracted afterwards
  a.mass = pl.mode == SP_FDDIV ? ((h->cfg.eta > 0 || m != nullptr) ? 1 : 0) : (mass ? 1 : 0);
  a.m = m;
  // The x pass reads the spread's busy tiles only (nothing to clear) and subtracts the forcing g
  // from its field(s) as it loads them.
  {
    StageTimer t(h, ST_SPREAD);
    spread_w<T>(h, a, W, W.real);
  }
  const int sub_f0 = pl.mode == SP_STOKES ? 3 : (pl.mode == SP_FDDIV ? 0 : h->dim);
  pipeline<T>(h, W, W.real, pl.nf, dst, pl.nout, pl.md, sparse ? ROWS_SPARSE : ROWS_DENSE, true, g, sub_f0,
              g ? (pl.mode == SP_STOKES ? 2 : 1) : 0);
}

// Launch shapes of the apply's FFT passes by measurement on the handle's own arrays: rows per
// block of the x passes; lines per block and radix plan of the y passes and of the fused pass.
// Widths run from the largest that fits down to an eighth of it.
template <typename T> void tune_apply(ibdl_s* h, GridWork<T>& W) {
  const DensityPlan pl = density_plan<T>(h, W, h->cfg.eta > 0);
  const TuneKey key{0, h->dim, h->n[0], h->n[1], h->n[2], (int)sizeof(T), pl.nf, pow2_bucket(h->nact)};
  if (tune_get(key, &W.shape)) return;
  grid_fill_zero<T>(W.real, h->ntot * W.nfields, h->st);
  grid_fill_zero<T>(reinterpret_cast<T*>(W.spec), h->nspec * 2 * W.nfields, h->st);
  const int64_t rpf = h->ntot / h->n[0];
  RowList rl;
  rl.rows = h->rows;
  rl.nact = h->nact;
  rl.rpf = rpf;
  RowMask fwd, inv, fused;
  if (h->dim == 3) {
    fwd.lim = inv.lim = h->row_lim;
    fwd.nplanes = inv.nplanes = h->n[2];
    fwd.load = 1;
    inv.store = 1;
    fwd.p0 = inv.p0 = h->zlim[0];
    fwd.pspan = inv.pspan = std::max(0, h->zlim[1] - h->zlim[0] + 1);
    fused.load = fused.store = 1;
    fused.lo = h->zlim[0];
    fused.hi = h->zlim[1];
  } else {
    fused.load = fused.store = 1;
    fused.lo = h->lim2d[0];
    fused.hi = h->lim2d[1];
  }
  hipEvent_t e0, e1;
  IBDL_HIP(hipEventCreate(&e0));
  IBDL_HIP(hipEventCreate(&e1));
  // Candidates (radix plan, width) from the widest down to an eighth of it for each plan, timed in
  // three interleaved rounds of one warm-up and eight timed runs each; a candidate's time is its best
  // round (the rounds absorb clock and neighbour noise, which at 10-30 us per pass is of the size of
  // the differences).  A later candidate (narrower, or the second plan) must be clearly faster: on
  // ties the wider one moves fewer bytes (full 128-byte lines).
  using Cand = std::pair<int, int>;
  auto widths = [](int plan, int wmax, std::vector<Cand>& out) {
    for (int w = wmax; w >= 1 && w * 8 >= wmax; w /= 2) out.push_back(Cand(plan, w));
  };
  auto best_of = [&](const std::vector<Cand>& cand, auto&& run) {
    std::vector<float> tmin(cand.size(), 1e30f);
    for (int round = 0; round < 3; ++round)
      for (size_t c = 0; c < cand.size(); ++c) {
        run(cand[c].first, cand[c].second);
        IBDL_HIP(hipEventRecord(e0, h->st));
        for (int k = 0; k < 8; ++k) run(cand[c].first, cand[c].second);
        IBDL_HIP(hipEventRecord(e1, h->st));
        IBDL_HIP(hipEventSynchronize(e1));
        float ms = 0;
        IBDL_HIP(hipEventElapsedTime(&ms, e0, e1));
        tmin[c] = std::min(tmin[c], ms);
      }
    Cand best = cand[0];
    float best_ms = tmin[0];
    for (size_t c = 1; c < cand.size(); ++c)
      if (tmin[c] < 0.97f * best_ms) {
        best_ms = tmin[c];
        best = cand[c];
      }
    return best;
  };
  LaunchShape sh;
  {
    std::vector<Cand> cand;
    widths(0, fft_x_rpb_max<T>(h->n[0]), cand);
    sh.rpb = best_of(cand, [&](int, int r) {
      fft_x_r2c<T>(W.real, W.spec, h->n[0], h->nact * pl.nf, W.tw[0], h->st, r, rl, h->nxp);
      fft_x_c2r<T>(W.spec, W.real, h->n[0], h->nact * pl.nout, W.tw[0], h->st, r, rl, h->nxp);
    }).second;
  }
  if (h->dim == 3) {
    std::vector<Cand> cand;
    for (int p = 0; p < fft_line_plans<T>(h->n[1]); ++p) widths(p, fft_line_w_max<T>(h->n[1], p), cand);
    const Cand c = best_of(cand, [&](int p, int w) {
      fft_strided<T>(W.spec, h->n[1], (int64_t)pl.nf * fwd.pspan * h->nxp, h->nxp, h->nxp * h->n[1], h->nxp, false,
                     W.tw[1], h->st, w, fwd, h->nxh, p);
      fft_strided<T>(W.spec, h->n[1], (int64_t)pl.nout * inv.pspan * h->nxp, h->nxp, h->nxp * h->n[1], h->nxp, true,
                     W.tw[1], h->st, w, inv, h->nxh, p);
    });
    sh.py = c.first;
    sh.wy = c.second;
  }
  const int last = h->dim - 1;
  {
    // the second radix plan exists for the single-field scalar pass only
    const bool single = !pl.md.stokes && pl.nout == 1 && pl.md.nc == 1 && pl.md.fk[0] == FK_MASS;
    std::vector<Cand> cand;
    for (int p = 0; p < (single ? fft_line_plans<T>(h->n[last]) : 1); ++p)
      widths(p, fft_line_w_max<T>(h->n[last], p), cand);
    const Cand c = best_of(cand, [&](int p, int w) {
      fft_fused_last<T>(W.spec, h->n[last], h->nspec / h->n[last], pl.nout, pl.md, W.tw[last], h->st, 1, 0, w, fused,
                        p);
    });
    sh.pz = c.first;
    sh.wz = c.second;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  W.shape = sh;
  tune_put(key, sh);
}

// y = A q
template <typename T> void apply_t(ibdl_s* h, const double* q, double* y) {
  GridWork<T>& W = ensure_work<T>(h);
  if (!W.tuned) {
    tune_apply<T>(h, W);
    W.tuned = true;
  }
  density_to_grid<T>(h, q, nullptr, nullptr, W.real, true);
  const double* ub = h->has_ubar ? q + h->n_ib * h->nq : nullptr;
  InterpArgs ia = interp_args(h, h->nq, 1.0, h->half(), q, ub);
  {
    StageTimer t(h, ST_INTERP);
    interp<T>(ia, W.wtab, W.real, y, h->st);
  }
  if (h->has_ubar) {
    const int nblk = kr_nblk(h->n_ib);
    ensure_partial(h, nblk * h->nq);
    kr_border(q, h->ds, h->n_ib, h->nq, h->border_w(), y + h->n_ib * h->nq, h->partial, nblk, h->st);
  }
}

// u = L^-1 rhs (scalar) or L^-1 P rhs (Stokes); rhsf: the right-hand side as float fields instead
template <typename T> void grid_solve_t(ibdl_s* h, const T* rhs, T* u, int rows = ROWS_DENSE,
                                        const float* rhsf = nullptr) {
  GridWork<T>& W = ensure_work<T>(h);
  MultDesc md = base_desc<T>(h, W);
  if (h->stokes()) {
    md.nc = 2;
    md.fk[0] = FK_G1;
    md.fk[1] = FK_G2;
    md.alpha = -1.0;
    pipeline<T>(h, W, rhs, 2, u, 2, md, rows, false, nullptr, 0, 0, rhsf);
  } else {
    md.nc = 1;
    md.fk[0] = FK_MASS;
    md.alpha = 1.0;
    pipeline<T>(h, W, rhs, 1, u, 1, md, rows, false, nullptr, 0, 0, rhsf);
  }
}

// gf: the forcing as float fields (a mixed handle's, for the double right-hand side of the
// refinement; g is then unused); the Dirichlet solve widens it as it reads it
template <typename T> void rhs_t(ibdl_s* h, const double* data, const T* g, double* b, const float* gf = nullptr) {
  GridWork<T>& W = ensure_work<T>(h);
  const int64_t nb = h->n_ib * h->nq;
  if (gf && h->neumann()) throw Error(IBDL_ERR_UNSUPPORTED, "float forcing for the double Neumann right-hand side");
  if (gf) {
    grid_solve_t<T>(h, nullptr, W.real, ROWS_OUT, gf);
    InterpArgs ia = interp_args(h, h->nq, -1.0, 1.0, data, nullptr);
    interp<T>(ia, W.wtab, W.real, b, h->st);
  } else if (h->neumann()) {
    SpreadArgs a = spread_args(h, SP_PLAIN, 1, data);
    grid_fill_zero<T>(W.real, h->ntot, h->st);
    spread_w<T>(h, a, W, W.real);
    if (g) grid_axpby<T>(W.real, -1.0, g, 1.0, h->ntot, h->st);
    grid_solve_t<T>(h, W.real, W.real, ROWS_OUT);   // only the rows the interpolation reads
    InterpArgs ia = interp_args(h, 1, 1.0, 0.0, nullptr, nullptr);
    interp<T>(ia, W.wtab, W.real, b, h->st);
  } else if (g) {
    grid_solve_t<T>(h, g, W.real, ROWS_OUT);
    InterpArgs ia = interp_args(h, h->nq, -1.0, 1.0, data, nullptr);
    interp<T>(ia, W.wtab, W.real, b, h->st);
  } else {
    IBDL_HIP(hipMemcpyAsync(b, data, sizeof(double) * nb, hipMemcpyDeviceToDevice, h->st));
  }
  if (h->has_ubar) {
    if (g || gf) {
      const int nblk = 256;
      ensure_partial(h, nblk * h->nq);
      if (gf) grid_sum<float>(gf, h->nq, h->ntot, h->partial, nblk, b + nb, h->st);
      else grid_sum<T>(g, h->nq, h->ntot, h->partial, nblk, b + nb, h->st);
      const double hD = pow(h->h, (double)h->dim) * (h->sl ? h->sl_border : 1.0);
      kr_scale(b + nb, hD, b + nb, h->nq, h->st);
    } else {
      IBDL_HIP(hipMemsetAsync(b + nb, 0, sizeof(double) * h->nq, h->st));
    }
  }
}

template <typename T> void recover_t(ibdl_s* h, const double* q, const double* data, const T* g, T* u) {
  density_to_grid<T>(h, q, h->neumann() ? data : nullptr, g, u);
  if (h->has_ubar) grid_add_const<T>(u, q + h->n_ib * h->nq, h->nq, h->ntot, h->st);
}

// ------------------------------------------------------------------ transposed operator
// The operator is A = [[J/2 + Phi K, ubar columns], [border rows]] with Phi the interpolation
// matrix (S* = Phi), K the density-to-grid map u[Q] (scalar: -L^-1 (S~ + eta S); Stokes: the
// Sec. 6.3.2 map) and J = +-I.  Its transpose needs K^T, which is, per marker, h^-D ds_i times the
// derivative of the spread coefficients applied to Phi (transposed multiplier) of a grid field:
//   scalar:  K^T v = h^-D ds (.) (sum_d n_d Phi D_d L^-1 v - eta Phi L^-1 v)   (D_d^T = -D_d)
//   Stokes:  K^T v = h^-D ds (.) sum_f (d c_f / d Q) Phi T_f^T v
// adj_grid applies the grid part to the nq fields at src and leaves its nout fields at dst.
int adj_nout(ibdl_s* h) {
  if (h->stokes()) return h->cfg.eta > 0 ? 5 : 3;
  return h->dim + (h->cfg.eta > 0 ? 1 : 0);
}

// rows: ROWS_SPARSE for the transposed apply (spread input), ROWS_OUT for a dense input whose
// adjoint fields are only interpolated at the markers next (their active rows)
template <typename T> void adj_grid(ibdl_s* h, GridWork<T>& W, const T* src, T* dst, int rows, bool busy_only = false) {
  MultDesc md = base_desc<T>(h, W);
  const int nout = adj_nout(h);
  md.alpha = 1.0;
  if (h->stokes()) {
    md.mode = 2;
    md.nc = 2;
    const int kinds[5] = {FK_A11, FK_A12, FK_A22, FK_G1, FK_G2};
    for (int o = 0; o < nout; ++o) md.fk[o] = kinds[o];
  } else {
    md.mode = 1;
    md.nc = 1;
    md.fk[0] = FK_MASS;
  }
  pipeline<T>(h, W, src, md.nc, dst, nout, md, rows, busy_only);
}

// FD scalar: the transposed operator is taken as the exact transpose of the forward's fused
// divergence spread, so the grid part forms the one field w = L^-1 v (instead of D_d w and w) and
// the marker side is the dual-weight interpolation interp_div.
bool adj_folded(ibdl_s* h) { return !h->stokes() && h->fd() && h->cfg.kernel != IBDL_K_BSPLINE6; }

template <typename T> void adj_solve(ibdl_s* h, GridWork<T>& W, const T* src, T* dst, int rows, bool busy_only) {
  MultDesc md = base_desc<T>(h, W);
  md.nc = 1;
  md.fk[0] = FK_MASS;
  md.alpha = 1.0;
  pipeline<T>(h, W, src, 1, dst, 1, md, rows, busy_only);
}

template <typename T> void adj_markers_div(ibdl_s* h, GridWork<T>& W, const double* p, double b, const double* pu,
                                           double* y) {
  InterpArgs ia = interp_args(h, 1, 1.0, b, p, nullptr);
  StageTimer t(h, ST_INTERP);
  interp_div<T>(ia, W.wtab, W.real, h->nrm, h->ds, h->cfg.eta, 1.0 / pow(h->h, (double)h->dim), pu, y, h->st);
}

void ensure_adj(ibdl_s* h) {
  if (h->adj_m) return;
  h->adj_m = (double*)h->dalloc<double>(sizeof(double) * h->n_ib * 8);
  h->adj_mu = (double*)h->dalloc<double>(sizeof(double) * h->n_aug);
}

// interpolate the nout adjoint fields at W.real and combine them per marker into y (+ b p, ubar terms)
template <typename T> void adj_markers(ibdl_s* h, GridWork<T>& W, const double* p, double b, const double* pu,
                                       double* y) {
  const int nout = adj_nout(h);
  InterpArgs ia = interp_args(h, nout, 1.0, 0.0, nullptr, nullptr);
  {
    StageTimer t(h, ST_INTERP);
    interp<T>(ia, W.wtab, W.real, h->adj_m, h->st);
  }
  const double hDinv = 1.0 / pow(h->h, (double)h->dim);
  adj_combine(h->stokes() ? 1 : 0, h->dim, h->n_ib, nout, hDinv, h->cfg.eta, h->adj_m, h->nrm, h->ds, p, b, pu, y,
              h->st);
}

// y = A^T p
template <typename T> void apply_adj_t(ibdl_s* h, const double* p, double* y) {
  const bool fold = adj_folded(h);
  GridWork<T>& W = ensure_fields<T>(h, fold ? h->nq : std::max(adj_nout(h), h->nq));
  ensure_adj(h);
  SpreadArgs a = spread_args(h, SP_PLAIN, h->nq, p);
  a.raw = 1;
  {
    StageTimer t(h, ST_SPREAD);
    spread_w<T>(h, a, W, W.real);
  }
  const double half = h->neumann() ? -0.5 : 0.5;
  const double* pu = h->has_ubar ? p + h->n_ib * h->nq : nullptr;
  if (fold) {
    adj_solve<T>(h, W, W.real, W.real, ROWS_SPARSE, true);
    adj_markers_div<T>(h, W, p, half, pu, y);
  } else {
    adj_grid<T>(h, W, W.real, W.real, ROWS_SPARSE, true);
    adj_markers<T>(h, W, p, half, pu, y);
  }
  if (h->has_ubar) {
    const int nblk = kr_nblk(h->n_ib);
    ensure_partial(h, nblk * h->nq);
    kr_border(p, nullptr, h->n_ib, h->nq, 1.0, y + h->n_ib * h->nq, h->partial, nblk, h->st);
  }
}

// right-hand side of the adjoint system: the gradient of <psi, u> with respect to q
template <typename T> void adj_rhs_t(ibdl_s* h, const T* psi, double* g) {
  const bool fold = adj_folded(h);
  GridWork<T>& W = ensure_fields<T>(h, fold ? h->nq : std::max(adj_nout(h), h->nq));
  ensure_adj(h);
  IBDL_HIP(hipMemcpyAsync(W.real, psi, sizeof(T) * h->ntot * h->nq, hipMemcpyDeviceToDevice, h->st));
  if (fold) {
    adj_solve<T>(h, W, W.real, W.real, ROWS_OUT, false);
    adj_markers_div<T>(h, W, nullptr, 0.0, nullptr, g);
  } else {
    adj_grid<T>(h, W, W.real, W.real, ROWS_OUT);
    adj_markers<T>(h, W, nullptr, 0.0, nullptr, g);
  }
  if (h->has_ubar) {
    const int nblk = 256;
    ensure_partial(h, nblk * h->nq);
    grid_sum<T>(psi, h->nq, h->ntot, h->partial, nblk, g + h->n_ib * h->nq, h->st);
  }
}

// dL/dX from the adjoint solution mu, the forward density q and grid solution u:
//   dL/dX_ie = -sum_c mu_ic (Phi'_e u_c)_i + sum_k coef_ik (Phi'_e R_k)_i
// with R the adjoint fields of r = L^-1 (Phi^T mu - psi) (scalar: D_d r and r) or of
// r = psi - Phi^T mu (Stokes: T_f^T r), and Phi'_e the derivative of the interpolation weights.
template <typename T> void grad_X_t(ibdl_s* h, const double* q, const T* u, const T* psi, double* dX) {
  GridWork<T>& W = ensure_fields<T>(h, std::max(adj_nout(h), h->nq));
  ensure_adj(h);
  SpreadArgs a = spread_args(h, SP_PLAIN, h->nq, h->adj_mu);
  a.raw = 1;
  grid_fill_zero<T>(W.real, h->ntot * h->nq, h->st);
  spread_w<T>(h, a, W, W.real);
  if (h->stokes()) grid_axpby<T>(W.real, 1.0, psi, -1.0, h->ntot * h->nq, h->st);
  else grid_axpby<T>(W.real, -1.0, psi, 1.0, h->ntot, h->st);
  adj_grid<T>(h, W, W.real, W.real, ROWS_OUT);
  const int nout = adj_nout(h);
  const int nc = h->nq + nout;
  const double hDinv = 1.0 / pow(h->h, (double)h->dim);
  adj_coefs(h->stokes() ? 1 : 0, h->dim, h->n_ib, nc, hDinv, h->cfg.eta, h->adj_mu, q, h->nrm, h->ds, h->adj_m,
            h->st);
  GatherArgs ga{};
  ga.g = h->geom;
  ga.kernel = h->cfg.kernel;
  ga.n_ib = h->n_ib;
  ga.s = h->s;
  ga.f = h->f;
  ga.nfield = nc;
  for (int c = 0; c < h->nq; ++c) ga.field[c] = u + c * h->ntot;
  for (int k = 0; k < nout; ++k) ga.field[h->nq + k] = W.real + k * h->ntot;
  ga.coef = h->adj_m;
  ga.out = dX;
  gather_dx<T>(ga, h->st);
}

void apply_any(ibdl_s* h, const double* q, double* y, bool force64, bool trans = false) {
  if (trans) {
    if (h->mixed() && !force64) apply_adj_t<float>(h, q, y);
    else apply_adj_t<double>(h, q, y);
    return;
  }
  if (h->mixed() && !force64) apply_t<float>(h, q, y);
  else apply_t<double>(h, q, y);
}

double host_norm(ibdl_s* h, const double* v, int64_t n) {
  const int nblk = kr_nblk(n);
  ensure_partial(h, nblk);
  kr_multidot(v, n, 1, v, n, h->partial, nblk, h->small, h->st);
  IBDL_HIP(hipMemcpyAsync(h->hostbuf, h->small, sizeof(double), hipMemcpyDeviceToHost, h->st));
  IBDL_HIP(hipStreamSynchronize(h->st));
  return sqrt(h->hostbuf[0]);
}

// Wait for a publication: poll its tag for up to 2 ms (an iteration's GPU work is well below that),
// then fall back to a stream synchronisation, after which the tag must be there.
const volatile double* wait_published(ibdl_s* h, int slot, unsigned seq) {
  volatile unsigned* tag = h->htag + 16 * slot;
  const auto t0 = std::chrono::steady_clock::now();
  while (*tag != seq) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
      IBDL_HIP(hipStreamSynchronize(h->st));
      if (*tag != seq) throw Error(IBDL_ERR_HIP, "Arnoldi values did not reach the host");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return h->hmap + slot * kSlot;
}

// GMRES applies the working-precision operator (transposed with trans) by replaying a HIP graph
// captured from direct launches, reading gx and writing gy.  Captures it on first use; returns
// false when applies are launched directly instead (stage timing on, or graphs disabled).
bool ensure_graph(ibdl_s* h, bool trans) {
  if (h->timing || !h->use_graph) return false;
  const int64_t n = h->n_aug;
  const int k = trans ? 1 : 0;
  if (h->gexec[k]) return true;
  if (!h->gx) {
    h->gx = (double*)h->dalloc<double>(sizeof(double) * n);
    h->gy = (double*)h->dalloc<double>(sizeof(double) * n);
  }
  // a direct run first allocates every workspace and measures the launch shapes
  IBDL_HIP(hipMemsetAsync(h->gx, 0, sizeof(double) * n, h->st));
  apply_any(h, h->gx, h->gy, false, trans);
  IBDL_HIP(hipStreamSynchronize(h->st));
  hipStream_t main = h->st;
  h->st = h->aux;
  IBDL_HIP(hipStreamBeginCapture(h->aux, hipStreamCaptureModeThreadLocal));
  try {
    apply_any(h, h->gx, h->gy, false, trans);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(h->aux, &g);
    if (g) (void)hipGraphDestroy(g);
    h->st = main;
    throw;
  }
  h->st = main;
  IBDL_HIP(hipStreamEndCapture(h->aux, &h->graph[k]));
  IBDL_HIP(hipGraphInstantiate(&h->gexec[k], h->graph[k], nullptr, nullptr, 0));
  return true;
}

// GMRES, x0 = 0, no restart; classical Gram-Schmidt twice, the Givens rotations and the
// least-squares solution on the device, in double precision.  The device runs ahead of the host:
// step j + 1 (normalise w_j into V[j+1] with the norm the device computed, apply, orthogonalise,
// update the least-squares state, publish its residual) is queued before the host waits for step
// j's residual.  The state freezes at the step that converges, so a step queued after it changes
// nothing but V[j+2] and scratch.
int gmres(ibdl_s* h, const double* b, double tol, int maxit, double* x, ibdl_info_t* info, int* iters,
          double* relres, bool trans = false, double* beta_out = nullptr, double stop_beta = -1.0) {
  const int64_t n = h->n_aug;
  if (beta_out) *beta_out = 0.0;
  if (maxit > 200) throw Error(IBDL_ERR_ARG, "maxit must be at most 200");
  if (h->vcap < maxit + 1) {
    h->V = (double*)h->dalloc<double>(sizeof(double) * n * (maxit + 1));
    h->vcap = maxit + 1;
  }
  if (h->gmcap < maxit) {
    h->gm = (double*)h->dalloc<double>(sizeof(double) * kr_gmres_state_doubles(maxit));
    h->gmcap = maxit;
  }
  const int mx = h->gmcap;
  const int nblk = kr_nblk(n);
  const int anblk = kr_arnoldi_nblk(n);
  ensure_partial(h, std::max(nblk * (maxit + 2), anblk * (2 * maxit + 3)));
  *iters = 0;
  *relres = 0.0;
  const bool graph = ensure_graph(h, trans);
  double* gin = graph ? h->gx : nullptr;
  // |b|^2 (small[GM_BNORM2_AT]) and V[0] = b / |b| (also the graph's input) on the device, so that
  // step 0 is queued without a host round trip; step 0's least-squares update takes |b| from there
  kr_multidot(b, n, 1, b, n, h->partial, nblk, h->small + GM_BNORM2_AT, h->st);
  kr_scale_norm(b, h->small + GM_BNORM2_AT, 0.0, h->V, gin, n, h->st);
  unsigned seq[2] = {0, 0};
  // queue Arnoldi step j (V[j] is in place, and in gx for the graph): apply, orthogonalise, update
  // the least-squares state, publish it and, in the same launch, normalise w into V[j+1] (and gx)
  auto step = [&](int j) {
    double* w;
    if (graph) {
      IBDL_HIP(hipGraphLaunch(h->gexec[trans ? 1 : 0], h->st));
      w = h->gy;
    } else {
      w = h->V + (int64_t)(j + 1) * n;
      apply_any(h, h->V + (int64_t)j * n, w, false, trans);
    }
    const int slot = j & 1;
    seq[slot] = ++h->seq;
    if (n <= kSmallN) {   // one workgroup holds the vectors: the whole step in one launch
      kr_arnoldi_small(h->V, n, j + 1, w, n, h->small, 512, h->gm, mx, tol, h->hmap_dev + slot * kSlot,
                       h->htag_dev + 16 * slot, seq[slot], h->V + (int64_t)(j + 1) * n, gin, h->st);
      return;
    }
    kr_arnoldi_step(h->V, n, j + 1, w, n, h->partial, anblk, h->small, h->st);
    kr_publish_scale(h->small, h->partial + (int64_t)2 * (j + 1) * anblk, anblk, 512, h->gm, j, mx, tol,
                     h->hmap_dev + slot * kSlot, h->htag_dev + 16 * slot, seq[slot], w, h->V + (int64_t)(j + 1) * n,
                     gin, n, h->st);
  };
  step(0);
  int k = 0;
  double res = 1.0;
  int gated = -1;                       // step behind which a gated finish is queued
  int done_at = -1;                     // step whose result carried the convergence flag
  std::vector<double> rs(maxit, 1.0);   // residual estimates of the steps the host has seen
  for (int j = 0; j < maxit; ++j) {
    // Step j + 1 is queued ahead unless step j is predicted to converge: the residual ratio of the
    // last two steps, applied once more, brings it to tol.  A step queued after convergence would
    // delay whatever follows on the stream by a whole apply.  Behind a step predicted to be the
    // last, the solution y and x = V y are queued at once, gated on the device's convergence flag,
    // so that they follow the step without waiting for the host; if the step does not converge
    // they do nothing and the next step follows them.
    bool ahead = j + 1 < maxit && !(j == 0 && stop_beta > 0.0);
    if (ahead && j >= 2) {
      ahead = rs[j - 1] * (rs[j - 1] / rs[j - 2]) > tol;
      if (!ahead) {
        kr_gmres_finish(h->gm, mx, h->V, n, x, n, true, h->st);
        gated = j;
      }
    }
    if (ahead) step(j + 1);
    const volatile double* hv = wait_published(h, j & 1, seq[j & 1]);
    const double beta = hv[GM_BETA], hn = hv[GM_HN];
    if (j == 0 && beta_out) *beta_out = beta;
    // |b| already small enough for the caller: no solve (x is left alone)
    if (j == 0 && stop_beta > 0.0 && beta <= stop_beta) {
      *iters = 0;
      *relres = 0.0;
      return IBDL_OK;
    }
    if (j == 0 && !(beta > 0.0)) {   // b = 0: x = 0 (behind the queued steps, which ran on zeros)
      if (!std::isfinite(beta)) throw Error(IBDL_ERR_NONFINITE, "right-hand side is not finite");
      IBDL_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, h->st));
      IBDL_HIP(hipStreamSynchronize(h->st));
      return IBDL_OK;
    }
    if (!std::isfinite(hn) || !std::isfinite((double)hv[GM_RES]))
      throw Error(IBDL_ERR_NONFINITE, "non-finite value in the Arnoldi process");
    res = hv[GM_RES];
    rs[j] = res;
    k = (int)hv[GM_K];
    if (info && info->history && j < info->history_cap) info->history[j] = res;
    if (hv[GM_DONE] != 0.0) {
      done_at = j;
      break;
    }
    if (!ahead && j + 1 < maxit) step(j + 1);
  }
  // y = R^-1 g on the device, then x = V y; both are left to the stream, so the caller's next work
  // queues behind them (already queued when the converged step had a gated finish behind it)
  if (!(done_at >= 0 && done_at == gated)) kr_gmres_finish(h->gm, mx, h->V, n, x, n, false, h->st);
  *iters = k;
  *relres = res;
  return res <= tol ? IBDL_OK : IBDL_NOT_CONVERGED;
}

// MINRES for the single layer method, x0 = 0 (the device recurrences of minres.hip).  The
// iterations are queued in groups of 16 between looks at the device state: the state's done flag
// freezes x at the first iteration that meets tol, so the later iterations of a group cost their
// applies but change nothing.
int minres(ibdl_s* h, const double* b, double tol, int maxit, double* x, ibdl_info_t* info, int* iters,
           double* relres) {
  const int64_t n = h->n_aug;
  if (!h->mr) {
    h->mr = (double*)h->dalloc<double>(sizeof(double) * 3 * n);
    h->mr_state = (double*)h->dalloc<double>(sizeof(double) * 32);
  }
  if (h->mr_hist_cap < maxit) {
    if (h->mr_hist) h->dfree(h->mr_hist);
    h->mr_hist = (double*)h->dalloc<double>(sizeof(double) * maxit);
    h->mr_hist_cap = maxit;
  }
  ensure_partial(h, 2 * mr_nblk(n));
  const bool graph = ensure_graph(h, false);
  if (!h->gx) {
    h->gx = (double*)h->dalloc<double>(sizeof(double) * n);
    h->gy = (double*)h->dalloc<double>(sizeof(double) * n);
  }
  double *vprev = h->mr, *w1 = h->mr + n, *w2 = h->mr + 2 * n;
  double* st[2] = {h->mr_state, h->mr_state + 16};
  mr_start(b, h->mr_wt, n, tol, h->gx, vprev, w1, w2, x, h->partial, st[0], h->st);
  double* hs = h->hostbuf + 900;   // host copy of the state
  int k = 0;
  bool done = false;
  while (k < maxit && !done) {
    const int group = std::min(16, maxit - k);
    for (int i = 0; i < group; ++i, ++k) {
      if (graph) IBDL_HIP(hipGraphLaunch(h->gexec[0], h->st));
      else apply_any(h, h->gx, h->gy, false);
      mr_iteration(h->gx, vprev, h->gy, w1, w2, x, h->mr_wt, n, h->partial, st[k & 1], st[(k + 1) & 1], h->mr_hist,
                   h->mr_hist_cap, h->st);
    }
    IBDL_HIP(hipMemcpyAsync(hs, st[k & 1], sizeof(double) * MR_NSTATE, hipMemcpyDeviceToHost, h->st));
    IBDL_HIP(hipStreamSynchronize(h->st));
    if (!std::isfinite(hs[MR_ETA])) throw Error(IBDL_ERR_NONFINITE, "non-finite value in the Lanczos process");
    done = hs[MR_DONE] != 0.0;
  }
  const int it = (int)hs[MR_ITERS];
  const double beta1 = hs[MR_BETA1];
  const double res = beta1 > 0.0 ? fabs(hs[MR_ETA]) / beta1 : 0.0;
  if (info && info->history && it > 0) {
    const int nh = std::min(it, info->history_cap);
    if (nh > 0) {
      IBDL_HIP(hipMemcpyAsync(info->history, h->mr_hist, sizeof(double) * nh, hipMemcpyDeviceToHost, h->st));
      IBDL_HIP(hipStreamSynchronize(h->st));
    }
  }
  *iters = it;
  *relres = res;
  return done ? IBDL_OK : IBDL_NOT_CONVERGED;
}

// Gradients of a loss of the recovered grid solution (dL/du = psi) with respect to the marker
// positions and the boundary data, by the adjoint method: A^T mu = (du/dq)^T psi, dL/ddata = mu.
template <typename T>
int backward_t(ibdl_s* h, const double* q, const T* u, const T* psi, double tol, int maxit, double* dX,
               double* ddata, ibdl_info_t* info) {
  ensure_adj(h);
  adj_rhs_t<T>(h, psi, h->vb);
  int iters = 0;
  double relres = 0.0;
  const int status = gmres(h, h->vb, tol, maxit, h->adj_mu, info, &iters, &relres, true);
  apply_any(h, h->adj_mu, h->vr, true, true);
  kr_axpby(h->vr, 1.0, h->vb, -1.0, h->n_aug, h->st);
  const double rn = host_norm(h, h->vr, h->n_aug);
  const double bn = host_norm(h, h->vb, h->n_aug);
  if (ddata)
    IBDL_HIP(hipMemcpyAsync(ddata, h->adj_mu, sizeof(double) * h->n_ib * h->nq, hipMemcpyDeviceToDevice, h->st));
  if (dX) grad_X_t<T>(h, q, u, psi, dX);
  IBDL_HIP(hipStreamSynchronize(h->st));
  if (info) {
    info->iters = iters;
    info->status = status;
    info->krylov_relres = relres;
    info->true_relres_fp64 = (bn > 0 || std::isnan(bn)) ? rn / bn : 0.0;
  }
  return status;
}

// grid points per axis: powers of two from 16 to 1024, and in 2-D up to 8192 (lines over 1024
// points run as four-step transforms)
bool pow2_in_range(int64_t v, int dim) { return v >= 16 && v <= (dim == 2 ? 8192 : 1024) && (v & (v - 1)) == 0; }

void validate(const ibdl_config_t* c, int64_t n_ib) {
  if (!c) throw Error(IBDL_ERR_ARG, "cfg is NULL");
  if (c->dim != 2 && c->dim != 3) throw Error(IBDL_ERR_ARG, "dim must be 2 or 3");
  if (n_ib < 1 || n_ib > (int64_t)1 << 30) throw Error(IBDL_ERR_ARG, "n_ib out of range");
  double h0 = 0;
  for (int d = 0; d < c->dim; ++d) {
    if (!pow2_in_range(c->n[d], c->dim))
      throw Error(IBDL_ERR_UNSUPPORTED, "grid size must be a power of two in [16, 1024] (in 2-D up to 8192)");
    if (!(c->L[d] > 0) || !std::isfinite(c->L[d]) || !std::isfinite(c->origin[d]))
      throw Error(IBDL_ERR_ARG, "box lengths must be positive and finite");
    const double hd = c->L[d] / (double)c->n[d];
    if (d == 0) h0 = hd;
    else if (fabs(hd - h0) > 1e-12 * h0) throw Error(IBDL_ERR_ARG, "grid spacing must be equal on every axis");
  }
  if (c->pde < 0 || c->pde > 2) throw Error(IBDL_ERR_ARG, "unknown pde");
  if (!(c->kappa >= 0) || !std::isfinite(c->kappa)) throw Error(IBDL_ERR_ARG, "kappa must be finite and >= 0");
  if (c->pde == IBDL_PDE_SCREENED && !(c->kappa > 0))
    throw Error(IBDL_ERR_ARG, "screened Poisson needs kappa > 0 (use IBDL_PDE_POISSON)");
  if (c->pde == IBDL_PDE_STOKES && (!(c->mu > 0) || !std::isfinite(c->mu))) throw Error(IBDL_ERR_ARG, "mu must be > 0");
  if (c->pde == IBDL_PDE_STOKES && c->dim != 2) throw Error(IBDL_ERR_UNSUPPORTED, "Stokes is implemented in 2-D");
  if (c->bc != IBDL_BC_DIRICHLET && c->bc != IBDL_BC_NEUMANN) throw Error(IBDL_ERR_ARG, "unknown bc");
  if (!(c->eta >= 0) || !std::isfinite(c->eta)) throw Error(IBDL_ERR_ARG, "eta must be finite and >= 0");
  if (c->bc == IBDL_BC_NEUMANN && (c->pde == IBDL_PDE_STOKES || c->eta != 0))
    throw Error(IBDL_ERR_UNSUPPORTED, "Neumann is implemented for the plain scalar operator");
  if (c->kernel < 0 || c->kernel > 2) throw Error(IBDL_ERR_ARG, "unknown kernel");
  if (c->disc != IBDL_DISC_FD2 && c->disc != IBDL_DISC_SPECTRAL) throw Error(IBDL_ERR_ARG, "unknown disc");
  if (c->kernel == IBDL_K_BSPLINE6 && c->disc == IBDL_DISC_FD2 && c->pde != IBDL_PDE_STOKES)
    throw Error(IBDL_ERR_UNSUPPORTED, "the B-spline kernel needs the spectral discretisation for scalar problems");
  if (c->kernel == IBDL_K_BSPLINE6 && c->pde == IBDL_PDE_STOKES && c->disc == IBDL_DISC_FD2)
    throw Error(IBDL_ERR_UNSUPPORTED, "finite-difference Stokes with the B-spline kernel is not implemented");
  if (c->precision != IBDL_FP64 && c->precision != IBDL_MIXED) throw Error(IBDL_ERR_ARG, "unknown precision");
  if (c->method != IBDL_METHOD_DL && c->method != IBDL_METHOD_SL) throw Error(IBDL_ERR_ARG, "unknown method");
  if (c->method == IBDL_METHOD_SL && c->dim != 2)
    throw Error(IBDL_ERR_UNSUPPORTED, "the single layer method is implemented in 2-D");
  if (c->method == IBDL_METHOD_SL && (c->bc != IBDL_BC_DIRICHLET || c->eta != 0))
    throw Error(IBDL_ERR_UNSUPPORTED, "the single layer method takes Dirichlet data and no completion (eta = 0)");
}

// Single layer: normals held at zero (no dipole), 1 / mean(ds) for the border rows, and the MINRES
// inner-product weights ds_i / mean(ds) per marker entry, 1 per u_bar entry.
void sl_markers(ibdl_s* h) {
  IBDL_HIP(hipMemsetAsync(h->nrm, 0, sizeof(double) * h->n_ib * h->dim, h->st));
  std::vector<double> ds(h->n_ib);
  IBDL_HIP(hipMemcpyAsync(ds.data(), h->ds, sizeof(double) * h->n_ib, hipMemcpyDeviceToHost, h->st));
  IBDL_HIP(hipStreamSynchronize(h->st));
  double sum = 0.0;
  for (double v : ds) sum += v;
  if (!(sum > 0) || !std::isfinite(sum)) throw Error(IBDL_ERR_ARG, "the spacings ds must have a positive finite sum");
  const double mean = sum / (double)h->n_ib;
  h->sl_border = 1.0 / mean;
  std::vector<double> wt(h->n_aug, 1.0);
  for (int64_t i = 0; i < h->n_ib; ++i)
    for (int c = 0; c < h->nq; ++c) wt[i * h->nq + c] = ds[i] / mean;
  if (!h->mr_wt) h->mr_wt = (double*)h->dalloc<double>(sizeof(double) * h->n_aug);
  IBDL_HIP(hipMemcpyAsync(h->mr_wt, wt.data(), sizeof(double) * h->n_aug, hipMemcpyHostToDevice, h->st));
  IBDL_HIP(hipStreamSynchronize(h->st));
}

void build_markers(ibdl_s* h) {
  h->drop_graphs();
  h->nb_cells_ready = false;
  markers_setup(h->geom, h->cfg.kernel, h->n_ib, h->X, h->s, h->f, h->wt, h->tile_count, h->st);
  markers_bin(h->geom, h->n_ib, h->s, h->tile_count, h->tile_off, h->tile_cur, h->list, h->list_tmp, h->busy,
              h->busy_tmp, h->busy_off, h->st, nullptr, 1, h->dim == 3 ? 1 : 0);
  markers_rows(h->geom, h->n_ib, h->s, h->row_lo, h->row_hi, h->row_cnt, h->row_off, h->row_lim, h->rows, h->st);
  const int ntile = h->geom.ntile[0] * h->geom.ntile[1] * h->geom.ntile[2];
  const int nplanes = h->dim == 3 ? h->n[2] : 1;
  int nb = 0, na = 0;
  std::vector<int2> lim(nplanes);
  IBDL_HIP(hipMemcpyAsync(&nb, h->busy_off + ntile, sizeof(int), hipMemcpyDeviceToHost, h->st));
  IBDL_HIP(hipMemcpyAsync(&na, h->row_off + nplanes, sizeof(int), hipMemcpyDeviceToHost, h->st));
  IBDL_HIP(hipMemcpyAsync(lim.data(), h->row_lim, sizeof(int2) * nplanes, hipMemcpyDeviceToHost, h->st));
  IBDL_HIP(hipStreamSynchronize(h->st));
  h->nbusy = nb;
  h->nact = na;
  if (h->lofs) markers_list_offsets(h->geom, h->busy, nb, h->list, h->s, h->lofs, h->st);
  h->lim2d[0] = lim[0].x;
  h->lim2d[1] = lim[0].y;
  // the planes with active rows; planes between them without any are inside the range (a window
  // wrapping the periodic boundary in z makes it the whole axis)
  h->zlim[0] = nplanes;
  h->zlim[1] = -1;
  for (int z = 0; z < nplanes; ++z)
    if (lim[z].x <= lim[z].y) {
      h->zlim[0] = std::min(h->zlim[0], z);
      h->zlim[1] = std::max(h->zlim[1], z);
    }
  {   // busy x-segments of the active rows; their count is reported by ibdl_spread_tiles
    markers_row_segments(h->geom, h->tile_off, h->rows, na, h->seg, h->st);
    markers_row_segments(h->geom, h->tile_off, nullptr, (int64_t)h->n[1] * (h->dim == 3 ? h->n[2] : 1), h->seg_all,
                         h->st);
    std::vector<unsigned long long> seg(na);
    if (na > 0)
      IBDL_HIP(hipMemcpyAsync(seg.data(), h->seg, sizeof(unsigned long long) * na, hipMemcpyDeviceToHost, h->st));
    IBDL_HIP(hipStreamSynchronize(h->st));
    int64_t cnt = 0;
    for (unsigned long long m : seg) cnt += __builtin_popcountll(m);
    h->seg_read = cnt;
  }
  if (h->w32 && h->w32->wtab) weight_table<float>(h->wt, h->n_ib, h->w32->wtab, h->st);
  if (h->w64 && h->w64->wtab) weight_table<double>(h->wt, h->n_ib, h->w64->wtab, h->st);
}

// IBDL_CHECK=1: the arrays a call takes and returns are scanned on the device for NaN and
// infinities; one hit makes the call return IBDL_ERR_NONFINITE.  Each scan waits for the stream.
template <typename T> void check_finite(ibdl_s* h, const T* p, int64_t n, const char* what) {
  if (!h->check || !p || n <= 0) return;
  IBDL_HIP(hipMemsetAsync(h->chk, 0, sizeof(unsigned), h->st));
  nonfinite_flag<T>(p, n, h->chk, h->st);
  unsigned v = 0;
  IBDL_HIP(hipMemcpyAsync(&v, h->chk, sizeof(unsigned), hipMemcpyDeviceToHost, h->st));
  IBDL_HIP(hipStreamSynchronize(h->st));
  if (v) throw Error(IBDL_ERR_NONFINITE, std::string(what) + " holds a non-finite value");
}
// a grid array of nf fields in the handle's grid type
void check_grid(ibdl_s* h, const void* p, int nf, const char* what) {
  if (h->mixed()) check_finite<float>(h, (const float*)p, h->ntot * nf, what);
  else check_finite<double>(h, (const double*)p, h->ntot * nf, what);
}
void check_markers(ibdl_s* h) {
  check_finite<double>(h, h->X, h->n_ib * h->dim, "X");
  if (!h->sl) check_finite<double>(h, h->nrm, h->n_ib * h->dim, "nrm");
  check_finite<double>(h, h->ds, h->n_ib, "ds");
}

template <typename F> ibdl_status_t guarded(ibdl_s* h, F&& fn) {
  if (!h) return IBDL_ERR_ARG;
  try {
    return (ibdl_status_t)fn();
  } catch (const Error& e) {
    h->err = e.what();
    return (ibdl_status_t)e.code;
  } catch (const std::exception& e) {
    h->err = e.what();
    return IBDL_ERR_HIP;
  }
}

}  // namespace

// ------------------------------------------------------------------ near-boundary tools (2-D)
// Indicator of the interior of the markers' curve(s): Delta chi = -S~ 1 (mean zero), shifted to
// 0 at the corner node, thresholded at 1/2 (Sec. 5.3.4).
template <typename T> void indicator_t(ibdl_s* h, T* chi, T* reg) {
  const int nf = h->fd() ? 1 : h->dim;
  GridWork<T>& W = ensure_fields<T>(h, nf);
  if (!h->ones) h->ones = (double*)h->dalloc<double>(sizeof(double) * h->n_ib);
  fill_value(h->ones, 1.0, h->n_ib, h->st);
  SpreadArgs a = spread_args(h, h->fd() ? SP_FDDIV : SP_SCALAR_VEC, nf, h->ones);
  a.mass = 0;
  spread_w<T>(h, a, W, W.real);
  MultDesc md = base_desc<T>(h, W);
  md.mode = 0;
  md.stokes = 0;
  md.c2 = 1.0;
  md.c0 = 0.0;
  md.alpha = -1.0;
  md.nc = nf;
  if (h->fd()) md.fk[0] = FK_MASS;
  else
    for (int d = 0; d < h->dim; ++d) md.fk[d] = FK_DX + d;
  pipeline<T>(h, W, W.real, nf, W.real, 1, md, ROWS_DENSE, true);
  indicator_finish<T>(W.real, h->ntot, chi, reg, h->st);
}

// Near-boundary interpolation (Sec. 5.3.3) of u into out on the nodes of omega.
template <typename T>
void near_boundary_t(ibdl_s* h, const double* Ub, const T* omega, const T* u, double m1, double m2, T* out) {
  const int64_t cap = near_list_cap(h->n_ib, m1, h->ntot);
  if (!h->nb_flag) {
    h->nb_flag = (unsigned char*)h->dalloc<double>((size_t)h->ntot);
    h->nb_count = (int*)h->dalloc<int>(sizeof(int));
  }
  if (h->nb_cap < cap) {
    if (h->nb_list) h->dfree(h->nb_list);
    h->nb_list = (int*)h->dalloc<int>(sizeof(int) * cap);
    h->nb_cap = cap;
  }
  NearGeom g;
  g.nx = h->n[0];
  g.ny = h->n[1];
  g.ox = h->geom.origin[0];
  g.oy = h->geom.origin[1];
  g.h = h->h;
  if (!h->nb_cells_ready) {   // marker cells of the nearest-marker search, once per marker set
    int ncx, ncy;
    const int nc = near_cells(g, &ncx, &ncy);
    if (!h->nb_cell_off) {
      h->nb_cell_cnt = (int*)h->dalloc<int>(sizeof(int) * nc);
      h->nb_cell_off = (int*)h->dalloc<int>(sizeof(int) * (nc + 1));
      h->nb_cell_list = (int*)h->dalloc<int>(sizeof(int) * h->n_ib);
    }
    near_bin(h->X, h->n_ib, g, h->nb_cell_cnt, h->nb_cell_off, h->nb_cell_list, h->st);
    h->nb_cells_ready = true;
  }
  near_boundary<T>(h->X, Ub, h->nq, h->n_ib, g, m1, m2, omega, u, out, h->nb_flag, h->nb_count, h->nb_list,
                   h->nb_cell_off, h->nb_cell_list, h->st);
}

// (u . grad) u of a 2-D velocity field: the four spectral (or centred-difference) derivatives by
// two gradient passes of the FFT pipeline (symbol i k~, no inverse), then the products.
template <typename T> void advection_t(ibdl_s* h, const T* u, T* out) {
  GridWork<T>& W = ensure_fields<T>(h, 4);
  MultDesc md = base_desc<T>(h, W);
  md.mode = 1;
  md.stokes = 0;
  md.c2 = 0.0;
  md.c0 = -1.0;   // multiplier alpha sc / (c2 sigma - c0) = sc: a plain derivative
  md.alpha = 1.0;
  md.nc = 1;
  md.fk[0] = FK_MASS;
  for (int c = 0; c < 2; ++c) pipeline<T>(h, W, u + c * h->ntot, 1, W.real + 2 * c * h->ntot, 2, md, ROWS_DENSE);
  ns_advect_combine<T>(u, W.real, h->ntot, out, h->st);
}

// Mean-zero pressure of the Brinkman / Stokes grid solution with density q and forcing g: the
// spread fields of the apply (the single-layer fields carry eta S Q - g~) through the pressure
// multiplier.
template <typename T> void pressure_t(ibdl_s* h, const double* q, const T* g, T* p) {
  GridWork<T>& W = ensure_work<T>(h);
  const bool mass = h->cfg.eta > 0 || g != nullptr;
  DensityPlan pl = density_plan<T>(h, W, mass);
  SpreadArgs a = spread_args(h, pl.mode, pl.nf, q);
  a.mass = mass ? 1 : 0;
  a.m = nullptr;
  spread_w<T>(h, a, W, W.real);
  MultDesc md = pl.md;
  md.mode = 3;
  md.alpha = 1.0;
  pipeline<T>(h, W, W.real, pl.nf, p, 1, md, ROWS_DENSE, true, g, 3, g ? 2 : 0);
}

// Control-volume force (Sec. 6.5) of u with time derivative ut and pressure p over a grid box.
template <typename T>
void cv_force_t(ibdl_s* h, const T* u, const T* uprev, double dt, const T* p, const T* omega, double rho,
                const int* box, double* out) {
  GridWork<T>& W = ensure_fields<T>(h, 4);
  MultDesc md = base_desc<T>(h, W);
  md.mode = 1;
  md.stokes = 0;
  md.c2 = 0.0;
  md.c0 = -1.0;
  md.alpha = 1.0;
  md.nc = 1;
  md.fk[0] = FK_MASS;
  for (int c = 0; c < 2; ++c) pipeline<T>(h, W, u + c * h->ntot, 1, W.real + 2 * c * h->ntot, 2, md, ROWS_DENSE);
  cv_force<T>(u, uprev, dt, p, omega, W.real, h->n[0], h->n[1], box, h->h, rho, h->cfg.mu, out, h->st);
}

// One step of the Navier-Stokes IMEX scheme (Sec. 6.5).  On entry u = u^n, u_prev = u^{n-1},
// n = N(u^n), n_prev = N(u^{n-1}); on return u = u^{n+1} (recovered, near-boundary interpolated,
// strip reset), u_prev = u^n, n = N(u^{n+1}), n_prev = N(u^n), q = the density.
template <typename T>
int ns_step_t(ibdl_s* h, const ibdl_ns_params_t& p, const double* Ub, const T* omega, T* u_prev, T* u, T* n_prev,
              T* n, double* q, T* g_out, ibdl_info_t* info) {
  const int64_t nn = 2 * h->ntot;
  if (!h->ns_scratch) h->ns_scratch = h->dalloc<T>(sizeof(T) * 2 * nn);
  T* g = static_cast<T*>(h->ns_scratch);
  T* raw = g + nn;
  ns_forcing<T>(u, u_prev, n, n_prev, p.rho, p.dt, nn, g, h->st);
  if (g_out) IBDL_HIP(hipMemcpyAsync(g_out, g, sizeof(T) * nn, hipMemcpyDeviceToDevice, h->st));
  IBDL_HIP(hipMemcpyAsync(u_prev, u, sizeof(T) * nn, hipMemcpyDeviceToDevice, h->st));
  IBDL_HIP(hipMemcpyAsync(n_prev, n, sizeof(T) * nn, hipMemcpyDeviceToDevice, h->st));
  rhs_t<T>(h, Ub, g, h->vb);
  int iters = 0;
  double relres = 0.0;
  const int status = gmres(h, h->vb, p.tol, p.maxit, q, info, &iters, &relres);
  recover_t<T>(h, q, Ub, g, raw);
  if (p.m1 > 0) near_boundary_t<T>(h, Ub, omega, raw, p.m1, p.m2, u);
  else IBDL_HIP(hipMemcpyAsync(u, raw, sizeof(T) * nn, hipMemcpyDeviceToDevice, h->st));
  ns_strip<T>(u, h->n[0], h->n[1], p.strip, p.u_inf, h->st);
  advection_t<T>(h, u, n);
  if (info) {
    info->iters = iters;
    info->status = status;
    info->krylov_relres = relres;
    info->true_relres_fp64 = -1.0;   // not computed in a time step
  }
  return status;
}

extern "C" {

ibdl_status_t ibdl_create(const ibdl_config_t* cfg, int64_t n_ib, const double* X, const double* nrm,
                          const double* ds, ibdl_t* out) {
  if (!out) {
    g_create_error = "out is NULL";
    return IBDL_ERR_ARG;
  }
  *out = nullptr;
  std::unique_ptr<ibdl_s> h(new ibdl_s());
  try {
    validate(cfg, n_ib);
    if (!X || !ds || (!nrm && cfg->method != IBDL_METHOD_SL))
      throw Error(IBDL_ERR_ARG, "marker arrays must be non-NULL device pointers");
    h->cfg = *cfg;
    h->sl = cfg->method == IBDL_METHOD_SL;
    if (h->sl) h->cfg.eta = 1.0;   // the single layer spreads the density with weight 1
    h->st = (hipStream_t)cfg->stream;
    h->dim = cfg->dim;
    for (int d = 0; d < 3; ++d) h->n[d] = d < h->dim ? (int)cfg->n[d] : 1;
    h->h = cfg->L[0] / (double)cfg->n[0];
    h->ntot = (int64_t)h->n[0] * h->n[1] * h->n[2];
    // Krylov solvers replay the apply from a graph on small grids, where an apply is shorter than
    // the host's launches; on large grids the host queues a step ahead anyway and direct launches
    // avoid the idle gap after each graph (measured 1.7 % faster at 256^3, 3 % at 1024^2)
    h->use_graph = h->ntot < ((int64_t)1 << 20);
    h->nxh = h->n[0] / 2 + 1;
    h->nxp = (h->nxh + 15) / 16 * 16;
    h->nspec = h->nxp * h->n[1] * h->n[2];
    h->n_ib = n_ib;
    h->nq = h->stokes() ? h->dim : 1;
    h->has_ubar = h->cfg.eta > 0 && h->kappa() == 0.0;
    h->n_aug = n_ib * h->nq + (h->has_ubar ? h->nq : 0);
    MarkerGeom& g = h->geom;
    g.dim = h->dim;
    g.h = h->h;
    for (int d = 0; d < 3; ++d) {
      g.n[d] = h->n[d];
      g.origin[d] = d < h->dim ? cfg->origin[d] : 0.0;
      const int t3[3] = {16, 4, 8};
      g.tile[d] = d < h->dim ? (h->dim == 2 ? 16 : t3[d]) : 1;
      g.ntile[d] = g.n[d] / g.tile[d];
    }
    const int64_t ntile = (int64_t)g.ntile[0] * g.ntile[1] * g.ntile[2];
    const int64_t maxlist = n_ib * (h->dim == 2 ? 4 : 12);   // tiles one 6-node window can meet
    h->X = (double*)h->dalloc<double>(sizeof(double) * n_ib * h->dim);
    h->nrm = (double*)h->dalloc<double>(sizeof(double) * n_ib * h->dim);
    h->ds = (double*)h->dalloc<double>(sizeof(double) * n_ib);
    h->s = (int*)h->dalloc<int>(sizeof(int) * n_ib * 3);
    h->f = (double*)h->dalloc<double>(sizeof(double) * n_ib * 3);
    h->wt = (double*)h->dalloc<double>(sizeof(double) * n_ib * 36);
    h->tile_count = (int*)h->dalloc<int>(sizeof(int) * ntile);
    h->tile_off = (int*)h->dalloc<int>(sizeof(int) * (ntile + 1));
    h->tile_cur = (int*)h->dalloc<int>(sizeof(int) * ntile);
    h->busy = (int4*)h->dalloc<int4>(sizeof(int4) * ntile);
    h->busy_tmp = (int4*)h->dalloc<int4>(sizeof(int4) * ntile);
    h->busy_off = (int*)h->dalloc<int>(sizeof(int) * (ntile + 1));
    h->list = (int*)h->dalloc<int>(sizeof(int) * maxlist);
    h->list_tmp = (int*)h->dalloc<int>(sizeof(int) * maxlist);
    if (h->dim == 3) h->lofs = (int*)h->dalloc<int>(sizeof(int) * maxlist);
    const int nplanes = h->dim == 3 ? h->n[2] : 1;
    h->row_lo = (int*)h->dalloc<int>(sizeof(int) * nplanes);
    h->row_hi = (int*)h->dalloc<int>(sizeof(int) * nplanes);
    h->row_cnt = (int*)h->dalloc<int>(sizeof(int) * (nplanes + 1));
    h->row_off = (int*)h->dalloc<int>(sizeof(int) * (nplanes + 1));
    h->row_lim = (int2*)h->dalloc<int>(sizeof(int2) * nplanes);
    h->rows = (int*)h->dalloc<int>(sizeof(int) * (int64_t)h->n[1] * nplanes);
    h->seg = (unsigned long long*)h->dalloc<unsigned long long>(sizeof(unsigned long long) * (int64_t)h->n[1] * nplanes);
    h->seg_all =
        (unsigned long long*)h->dalloc<unsigned long long>(sizeof(unsigned long long) * (int64_t)h->n[1] * nplanes);
    h->small = (double*)h->dalloc<double>(sizeof(double) * 1024);
    h->vb = (double*)h->dalloc<double>(sizeof(double) * h->n_aug);
    h->vr = (double*)h->dalloc<double>(sizeof(double) * h->n_aug);
    IBDL_HIP(hipHostMalloc((void**)&h->hostbuf, sizeof(double) * 1024, hipHostMallocDefault));
    IBDL_HIP(hipHostMalloc((void**)&h->hmap, sizeof(double) * (kYOff + kYSlot),
                           hipHostMallocMapped | hipHostMallocCoherent));
    IBDL_HIP(hipHostGetDevicePointer((void**)&h->hmap_dev, h->hmap, 0));
    h->htag = reinterpret_cast<volatile unsigned*>(h->hmap + 2 * kSlot);
    h->htag_dev = reinterpret_cast<unsigned*>(h->hmap_dev + 2 * kSlot);
    h->htag[0] = 0;
    h->htag[16] = 0;
    IBDL_HIP(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
    IBDL_HIP(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    IBDL_HIP(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    IBDL_HIP(hipMemcpyAsync(h->X, X, sizeof(double) * n_ib * h->dim, hipMemcpyDeviceToDevice, h->st));
    if (!h->sl) IBDL_HIP(hipMemcpyAsync(h->nrm, nrm, sizeof(double) * n_ib * h->dim, hipMemcpyDeviceToDevice, h->st));
    IBDL_HIP(hipMemcpyAsync(h->ds, ds, sizeof(double) * n_ib, hipMemcpyDeviceToDevice, h->st));
    {
      const char* e = getenv("IBDL_CHECK");
      h->check = e && strcmp(e, "1") == 0;
      if (h->check) h->chk = (unsigned*)h->dalloc<unsigned>(sizeof(unsigned));
    }
    check_markers(h.get());
    if (h->sl) sl_markers(h.get());
    build_markers(h.get());
    if (h->mixed()) ensure_work<float>(h.get());
    else ensure_work<double>(h.get());
  } catch (const Error& e) {
    g_create_error = e.what();
    return (ibdl_status_t)e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return IBDL_ERR_HIP;
  }
  *out = h.release();
  return IBDL_OK;
}

ibdl_status_t ibdl_set_markers(ibdl_t h, const double* X, const double* nrm, const double* ds) {
  return guarded(h, [&]() {
    if (!X || !ds || (!nrm && !h->sl)) throw Error(IBDL_ERR_ARG, "marker arrays must be non-NULL");
    IBDL_HIP(hipMemcpyAsync(h->X, X, sizeof(double) * h->n_ib * h->dim, hipMemcpyDeviceToDevice, h->st));
    if (!h->sl) IBDL_HIP(hipMemcpyAsync(h->nrm, nrm, sizeof(double) * h->n_ib * h->dim, hipMemcpyDeviceToDevice, h->st));
    IBDL_HIP(hipMemcpyAsync(h->ds, ds, sizeof(double) * h->n_ib, hipMemcpyDeviceToDevice, h->st));
    check_markers(h);
    if (h->sl) sl_markers(h);
    build_markers(h);
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_destroy(ibdl_t h) {
  if (!h) return IBDL_ERR_ARG;
  delete h;
  return IBDL_OK;
}

ibdl_status_t ibdl_spread(ibdl_t h, const double* f, int32_t nc, void* grid) {
  return guarded(h, [&]() {
    if (!f || !grid) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (nc < 1 || nc > 5) throw Error(IBDL_ERR_ARG, "nc must be in [1, 5]");
    SpreadArgs a = spread_args(h, SP_PLAIN, nc, f);
    if (h->mixed()) {
      grid_fill_zero<float>((float*)grid, h->ntot * nc, h->st);
      spread_w<float>(h, a, ensure_work<float>(h), (float*)grid);
    } else {
      grid_fill_zero<double>((double*)grid, h->ntot * nc, h->st);
      spread_w<double>(h, a, ensure_work<double>(h), (double*)grid);
    }
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_indicator(ibdl_t h, void* chi, void* regularized) {
  return guarded(h, [&]() {
    if (!chi) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (h->dim != 2) throw Error(IBDL_ERR_UNSUPPORTED, "the indicator function is two-dimensional");
    if (h->sl) throw Error(IBDL_ERR_UNSUPPORTED, "the indicator function needs the normals of a double layer handle");
    if (h->mixed()) indicator_t<float>(h, (float*)chi, (float*)regularized);
    else indicator_t<double>(h, (double*)chi, (double*)regularized);
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_near_boundary(ibdl_t h, const double* Ub, const void* omega, const void* u, double m1, double m2,
                                 void* out) {
  return guarded(h, [&]() {
    if (!Ub || !omega || !u || !out) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (out == u) throw Error(IBDL_ERR_ARG, "out must not alias u");
    if (h->dim != 2) throw Error(IBDL_ERR_UNSUPPORTED, "the near-boundary interpolation is two-dimensional");
    if (!(m1 >= 1.0 && m2 > m1 && m2 <= 64.0)) throw Error(IBDL_ERR_ARG, "need 1 <= m1 < m2 <= 64");
    if (h->n_ib < 2) throw Error(IBDL_ERR_ARG, "the interpolation needs at least two markers");
    if (h->mixed())
      near_boundary_t<float>(h, Ub, (const float*)omega, (const float*)u, m1, m2, (float*)out);
    else
      near_boundary_t<double>(h, Ub, (const double*)omega, (const double*)u, m1, m2, (double*)out);
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_advection(ibdl_t h, const void* u, void* out) {
  return guarded(h, [&]() {
    if (!u || !out) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (u == out) throw Error(IBDL_ERR_ARG, "out must not alias u");
    if (h->dim != 2 || !h->stokes()) throw Error(IBDL_ERR_UNSUPPORTED, "the nonlinear term is for 2-D Stokes handles");
    if (h->mixed()) advection_t<float>(h, (const float*)u, (float*)out);
    else advection_t<double>(h, (const double*)u, (double*)out);
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_ns_step(ibdl_t h, const ibdl_ns_params_t* p, const double* Ub, const void* omega, void* u_prev,
                           void* u, void* n_prev, void* n, double* q, void* g_out, ibdl_info_t* info) {
  return guarded(h, [&]() {
    if (!p || !Ub || !u_prev || !u || !n_prev || !n || !q) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (h->dim != 2 || !h->stokes()) throw Error(IBDL_ERR_UNSUPPORTED, "the Navier-Stokes step is for 2-D Stokes handles");
    if (h->sl) throw Error(IBDL_ERR_UNSUPPORTED, "the Navier-Stokes step uses the double layer method");
    if (!(p->rho > 0) || !(p->dt > 0) || !std::isfinite(p->rho) || !std::isfinite(p->dt))
      throw Error(IBDL_ERR_ARG, "rho and dt must be positive and finite");
    const double k2 = 1.5 * p->rho / p->dt;
    if (fabs(h->cfg.kappa * h->cfg.kappa - k2) > 1e-10 * k2)
      throw Error(IBDL_ERR_ARG, "the handle's kappa^2 must equal 3 rho / (2 dt)");
    if (p->m1 != 0 && !(p->m1 >= 1.0 && p->m2 > p->m1 && p->m2 <= 64.0))
      throw Error(IBDL_ERR_ARG, "need m1 = 0 or 1 <= m1 < m2 <= 64");
    if (p->m1 != 0 && !omega) throw Error(IBDL_ERR_ARG, "omega is needed for the near-boundary interpolation");
    if (p->strip < 0 || p->strip > h->n[0]) throw Error(IBDL_ERR_ARG, "strip width out of range");
    if (!std::isfinite(p->u_inf) || !(p->tol >= 0)) throw Error(IBDL_ERR_ARG, "u_inf and tol must be finite");
    if (p->maxit < 1 || p->maxit > 200) throw Error(IBDL_ERR_ARG, "maxit must be in [1, 200]");
    const void* ptrs[5] = {u_prev, u, n_prev, n, g_out};
    for (int a = 0; a < 5; ++a)
      for (int b = a + 1; b < 5; ++b)
        if (ptrs[a] && ptrs[a] == ptrs[b]) throw Error(IBDL_ERR_ARG, "u_prev, u, n_prev, n and g_out must be distinct");
    if (h->mixed())
      return ns_step_t<float>(h, *p, Ub, (const float*)omega, (float*)u_prev, (float*)u, (float*)n_prev, (float*)n, q,
                              (float*)g_out, info);
    return ns_step_t<double>(h, *p, Ub, (const double*)omega, (double*)u_prev, (double*)u, (double*)n_prev,
                             (double*)n, q, (double*)g_out, info);
  });
}

ibdl_status_t ibdl_pressure(ibdl_t h, const double* q, const void* g_grid, void* p) {
  return guarded(h, [&]() {
    if (!q || !p) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (h->dim != 2 || !h->stokes()) throw Error(IBDL_ERR_UNSUPPORTED, "the pressure is for 2-D Stokes handles");
    if (h->mixed()) pressure_t<float>(h, q, (const float*)g_grid, (float*)p);
    else pressure_t<double>(h, q, (const double*)g_grid, (double*)p);
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_cv_force(ibdl_t h, const void* u, const void* u_prev, double dt, const void* p, const void* omega,
                            double rho, const int32_t* box, double* out) {
  return guarded(h, [&]() {
    if (!u || !p || !omega || !box || !out) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (u_prev && !(dt > 0 && std::isfinite(dt))) throw Error(IBDL_ERR_ARG, "dt must be positive and finite");
    if (h->dim != 2 || !h->stokes()) throw Error(IBDL_ERR_UNSUPPORTED, "the control-volume force is for 2-D Stokes handles");
    if (!(box[0] >= 0 && box[0] < box[1] && box[1] < h->n[0] && box[2] >= 0 && box[2] < box[3] && box[3] < h->n[1]))
      throw Error(IBDL_ERR_ARG, "box must satisfy 0 <= i0 < i1 < nx and 0 <= j0 < j1 < ny");
    if (!std::isfinite(rho)) throw Error(IBDL_ERR_ARG, "rho must be finite");
    const int b[4] = {box[0], box[1], box[2], box[3]};
    if (h->mixed())
      cv_force_t<float>(h, (const float*)u, (const float*)u_prev, dt, (const float*)p, (const float*)omega, rho, b,
                        out);
    else
      cv_force_t<double>(h, (const double*)u, (const double*)u_prev, dt, (const double*)p, (const double*)omega, rho,
                         b, out);
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_net_force(ibdl_t h, const double* q, double* out) {
  return guarded(h, [&]() {
    if (!q || !out) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (h->dim != 2 || !h->stokes()) throw Error(IBDL_ERR_UNSUPPORTED, "the net force is for 2-D Stokes handles");
    net_force(h->X, q, h->ds, h->n_ib, h->cfg.eta, out, h->st);
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_line_integral(ibdl_t h, const void* u, int32_t comp, int32_t axis, int64_t index, double* out) {
  return guarded(h, [&]() {
    if (!u || !out) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (h->dim != 2) throw Error(IBDL_ERR_UNSUPPORTED, "line integrals are for 2-D handles");
    if (comp < 0 || comp >= h->nq) throw Error(IBDL_ERR_ARG, "comp out of range");
    if (axis != 0 && axis != 1) throw Error(IBDL_ERR_ARG, "axis must be 0 or 1");
    if (index < 0 || index >= h->n[axis]) throw Error(IBDL_ERR_ARG, "index out of range");
    const int64_t nx = h->n[0], ny = h->n[1];
    const int64_t first = (int64_t)comp * h->ntot + (axis == 0 ? index : index * nx);
    const int64_t stride = axis == 0 ? nx : 1, len = axis == 0 ? ny : nx;
    if (h->mixed()) line_sum<float>((const float*)u + first, stride, len, h->h, out, h->st);
    else line_sum<double>((const double*)u + first, stride, len, h->h, out, h->st);
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_near_widths(ibdl_t h, double* m1, double* m2) {
  return guarded(h, [&]() {
    if (h->dim != 2) throw Error(IBDL_ERR_UNSUPPORTED, "the near-boundary interpolation is two-dimensional");
    const double w1 = h->fd() ? 6.0 : std::max(2.0 * (log2((double)h->n[0]) - 4.0), 2.0);
    if (m1) *m1 = w1;
    if (m2) *m2 = w1 + 2.0;
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_interp(ibdl_t h, const void* grid, int32_t nc, double* f) {
  return guarded(h, [&]() {
    if (!f || !grid) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (nc < 1 || nc > 5) throw Error(IBDL_ERR_ARG, "nc must be in [1, 5]");
    InterpArgs ia = interp_args(h, nc, 1.0, 0.0, nullptr, nullptr);
    if (h->mixed()) interp<float>(ia, ensure_work<float>(h).wtab, (const float*)grid, f, h->st);
    else interp<double>(ia, ensure_work<double>(h).wtab, (const double*)grid, f, h->st);
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_grid_solve(ibdl_t h, const void* rhs, void* u) {
  return guarded(h, [&]() {
    if (!rhs || !u) throw Error(IBDL_ERR_ARG, "NULL pointer");
    check_grid(h, rhs, h->nq, "rhs");
    if (h->mixed()) grid_solve_t<float>(h, (const float*)rhs, (float*)u);
    else grid_solve_t<double>(h, (const double*)rhs, (double*)u);
    check_grid(h, u, h->nq, "u");
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_apply(ibdl_t h, const double* q, double* y) {
  return guarded(h, [&]() {
    if (!q || !y) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (q == y) throw Error(IBDL_ERR_ARG, "q and y must not alias");
    check_finite<double>(h, q, h->n_aug, "q");
    apply_any(h, q, y, false);
    check_finite<double>(h, y, h->n_aug, "y");
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_solve(ibdl_t h, const double* data, const void* g_grid, double tol, int32_t maxit, double* q,
                         void* u_grid, ibdl_info_t* info) {
  return guarded(h, [&]() {
    if (!data || !q) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (!(tol >= 0) || !std::isfinite(tol)) throw Error(IBDL_ERR_ARG, "tol must be finite and >= 0");
    if (maxit < 1 || maxit > (h->sl ? 1000000 : 200))
      throw Error(IBDL_ERR_ARG, h->sl ? "maxit must be in [1, 1000000]" : "maxit must be in [1, 200]");
    check_finite<double>(h, data, h->n_ib * h->nq, "data");
    if (g_grid) check_grid(h, g_grid, h->nq, "g");
    if (h->mixed()) rhs_t<float>(h, data, (const float*)g_grid, h->vb);
    else rhs_t<double>(h, data, (const double*)g_grid, h->vb);
    int iters = 0;
    double relres = 0;
    const int status = h->sl ? minres(h, h->vb, tol, maxit, q, info, &iters, &relres)
                             : gmres(h, h->vb, tol, maxit, q, info, &iters, &relres);
    // True residual ||b - A q|| / ||b|| with a double-precision apply, queued on the handle's
    // stream right behind the solution.  On a mixed handle it uses the double work arrays and the
    // recovery the float ones, so the (shorter) recovery runs beside it on the second stream.
    const bool overlap = h->mixed() && u_grid;
    hipStream_t main = h->st;
    if (overlap) {
      IBDL_HIP(hipEventRecord(h->ev_fork, main));
      IBDL_HIP(hipStreamWaitEvent(h->aux, h->ev_fork, 0));
    }
    apply_any(h, q, h->vr, true);
    kr_axpby(h->vr, 1.0, h->vb, -1.0, h->n_aug, h->st);
    const int nblk = kr_nblk(h->n_aug);
    ensure_partial(h, nblk);
    kr_multidot(h->vr, h->n_aug, 1, h->vr, h->n_aug, h->partial, nblk, h->small + 600, h->st);
    kr_multidot(h->vb, h->n_aug, 1, h->vb, h->n_aug, h->partial, nblk, h->small + 601, h->st);
    IBDL_HIP(hipMemcpyAsync(h->hostbuf + 600, h->small + 600, 2 * sizeof(double), hipMemcpyDeviceToHost, h->st));
    if (u_grid) {
      if (overlap) h->st = h->aux;
      try {
        if (h->mixed()) recover_t<float>(h, q, data, (const float*)g_grid, (float*)u_grid);
        else recover_t<double>(h, q, data, (const double*)g_grid, (double*)u_grid);
      } catch (...) {
        h->st = main;
        throw;
      }
      h->st = main;
    }
    if (overlap) {
      IBDL_HIP(hipEventRecord(h->ev_join, h->aux));
      IBDL_HIP(hipStreamWaitEvent(main, h->ev_join, 0));
    }
    IBDL_HIP(hipStreamSynchronize(main));
    const double rn = sqrt(std::max(h->hostbuf[600], 0.0)), bn = sqrt(std::max(h->hostbuf[601], 0.0));
    if (info) {
      info->iters = iters;
      info->status = status;
      info->krylov_relres = relres;
      info->true_relres_fp64 = (bn > 0 || std::isnan(bn)) ? rn / bn : 0.0;
    }
    check_finite<double>(h, q, h->n_aug, "q");
    if (u_grid) check_grid(h, u_grid, h->nq, "u");
    return status;
  });
}

ibdl_status_t ibdl_backward(ibdl_t h, const double* q, const void* u_grid, const void* dL_du, double tol,
                            int32_t maxit, double* dL_dX, double* dL_ddata, ibdl_info_t* info) {
  return guarded(h, [&]() {
    if (!q || !u_grid || !dL_du) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (!(tol >= 0) || !std::isfinite(tol)) throw Error(IBDL_ERR_ARG, "tol must be finite and >= 0");
    if (maxit < 1 || maxit > 200) throw Error(IBDL_ERR_ARG, "maxit must be in [1, 200]");
    if (h->neumann()) throw Error(IBDL_ERR_UNSUPPORTED, "the adjoint is implemented for Dirichlet problems");
    if (h->sl) throw Error(IBDL_ERR_UNSUPPORTED, "the adjoint is implemented for the double layer method");
    check_finite<double>(h, q, h->n_aug, "q");
    check_grid(h, u_grid, h->nq, "u");
    check_grid(h, dL_du, h->nq, "dL_du");
    const int st = h->mixed()
                       ? backward_t<float>(h, q, (const float*)u_grid, (const float*)dL_du, tol, maxit, dL_dX, dL_ddata, info)
                       : backward_t<double>(h, q, (const double*)u_grid, (const double*)dL_du, tol, maxit, dL_dX, dL_ddata,
                                            info);
    check_finite<double>(h, dL_dX, h->n_ib * h->dim, "dL_dX");
    check_finite<double>(h, dL_ddata, h->n_ib * h->nq, "dL_ddata");
    return st;
  });
}

ibdl_status_t ibdl_apply_transpose(ibdl_t h, const double* p, double* y) {
  return guarded(h, [&]() {
    if (!p || !y) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (p == y) throw Error(IBDL_ERR_ARG, "p and y must not alias");
    if (h->sl) throw Error(IBDL_ERR_UNSUPPORTED, "the transposed operator is implemented for the double layer method");
    check_finite<double>(h, p, h->n_aug, "p");
    apply_any(h, p, y, false, true);
    check_finite<double>(h, y, h->n_aug, "y");
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_solve_refined(ibdl_t h, const double* data, const void* g_grid, double tol, int32_t maxit,
                                 double inner_tol, int32_t max_rounds, double* q, void* u_grid, ibdl_info_t* info) {
  return guarded(h, [&]() {
    if (!data || !q) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (!(tol >= 0) || !std::isfinite(tol)) throw Error(IBDL_ERR_ARG, "tol must be finite and >= 0");
    if (!(inner_tol > 0 && inner_tol < 1)) throw Error(IBDL_ERR_ARG, "inner_tol must be in (0, 1)");
    if (maxit < 1 || maxit > 200) throw Error(IBDL_ERR_ARG, "maxit must be in [1, 200]");
    if (max_rounds < 1 || max_rounds > 50) throw Error(IBDL_ERR_ARG, "max_rounds must be in [1, 50]");
    if (h->sl) throw Error(IBDL_ERR_UNSUPPORTED, "refinement is implemented for the double layer method");
    check_finite<double>(h, data, h->n_ib * h->nq, "data");
    if (g_grid) check_grid(h, g_grid, h->nq, "g");
    const int64_t n = h->n_aug;
    // right-hand side in double: the float forcing of a mixed handle is widened as the Dirichlet
    // solve reads it (a Neumann forcing is widened first)
    if (g_grid && h->mixed() && !h->neumann()) {
      rhs_t<double>(h, data, nullptr, h->vb, (const float*)g_grid);
    } else if (g_grid && h->mixed()) {
      if (!h->g64) h->g64 = (double*)h->dalloc<double>(sizeof(double) * h->ntot * h->nq);
      grid_widen((const float*)g_grid, h->g64, h->ntot * h->nq, h->st);
      rhs_t<double>(h, data, h->g64, h->vb);
    } else {
      rhs_t<double>(h, data, (const double*)g_grid, h->vb);
    }
    if (!h->vx) h->vx = (double*)h->dalloc<double>(sizeof(double) * n);
    const int nblk = kr_nblk(n);
    ensure_partial(h, nblk);
    // Round 0 solves A q = b directly into q (x0 = 0); round k > 0 adds the correction A d = r.
    // GMRES reports |b| with its first step.  After each round the double-precision residual
    // r = b - A q is formed on the device.  When the round's own Krylov residual predicts that r
    // meets tol, the host reads |r| at once (and the float recovery of q runs beside that residual
    // on the second stream); otherwise the next round starts without waiting, and its first step
    // reports |r|: if that already meets tol, the round stops there and q stays as it is.
    int total = 0, status = IBDL_NOT_CONVERGED;
    double rn = 0.0, bn = 0.0, krylov = 0.0, rprev = 0.0;
    bool recovered = false, known = false;
    hipStream_t main = h->st;
    for (int round = 0; round < max_rounds; ++round) {
      int it = 0;
      double rr = 0.0, beta = 0.0;
      gmres(h, round == 0 ? h->vb : h->vr, inner_tol, maxit, round == 0 ? q : h->vx, nullptr, &it, &rr, false, &beta,
            round == 0 || known ? -1.0 : tol * bn);
      if (round == 0) {
        bn = beta;
        if (!(bn > 0)) {   // b = 0: q = 0 (GMRES wrote it)
          rn = 0.0;
          status = IBDL_OK;
          break;
        }
        rprev = bn;
      } else {
        if (!known) {      // |r| of the previous round, from this round's first step
          rn = beta;
          if (!std::isfinite(rn)) throw Error(IBDL_ERR_NONFINITE, "non-finite residual in refinement");
          if (it == 0) {
            status = IBDL_OK;
            break;
          }
          rprev = rn;
        }
        kr_axpby(q, 1.0, h->vx, 1.0, n, h->st);
      }
      total += it;
      krylov = rr;
      recovered = false;
      // predicted |r|: the round's Krylov reduction of its right-hand side, but not below the float
      // operator's rounding (about 1e-7 of that right-hand side on a mixed handle)
      const double floor = h->mixed() ? 1e-7 : 1e-15;
      const bool last = std::max(rr, floor) * rprev <= tol * bn;
      const bool spec = last && u_grid && h->mixed();
      if (spec) {
        IBDL_HIP(hipEventRecord(h->ev_fork, main));
        IBDL_HIP(hipStreamWaitEvent(h->aux, h->ev_fork, 0));
      }
      apply_any(h, q, h->vr, true);
      kr_axpby(h->vr, 1.0, h->vb, -1.0, n, h->st);   // r = b - A q
      known = last;
      if (!last) continue;
      kr_multidot(h->vr, n, 1, h->vr, n, h->partial, nblk, h->small + 600, h->st);
      IBDL_HIP(hipMemcpyAsync(h->hostbuf + 600, h->small + 600, sizeof(double), hipMemcpyDeviceToHost, h->st));
      if (spec) {
        h->st = h->aux;
        try {
          recover_t<float>(h, q, data, (const float*)g_grid, (float*)u_grid);
        } catch (...) {
          h->st = main;
          throw;
        }
        h->st = main;
        IBDL_HIP(hipEventRecord(h->ev_join, h->aux));
        IBDL_HIP(hipStreamWaitEvent(main, h->ev_join, 0));
        recovered = true;
      }
      IBDL_HIP(hipStreamSynchronize(main));
      rn = sqrt(std::max(h->hostbuf[600], 0.0));
      if (!std::isfinite(rn)) throw Error(IBDL_ERR_NONFINITE, "non-finite residual in refinement");
      rprev = rn;
      if (rn <= tol * bn) {
        status = IBDL_OK;
        break;
      }
    }
    if (status != IBDL_OK && !known) {   // out of rounds with the last residual unread
      kr_multidot(h->vr, n, 1, h->vr, n, h->partial, nblk, h->small + 600, h->st);
      IBDL_HIP(hipMemcpyAsync(h->hostbuf + 600, h->small + 600, sizeof(double), hipMemcpyDeviceToHost, h->st));
      IBDL_HIP(hipStreamSynchronize(h->st));
      rn = sqrt(std::max(h->hostbuf[600], 0.0));
      if (rn <= tol * bn) status = IBDL_OK;
    }
    if (u_grid && !recovered) {
      if (h->mixed()) recover_t<float>(h, q, data, (const float*)g_grid, (float*)u_grid);
      else recover_t<double>(h, q, data, (const double*)g_grid, (double*)u_grid);
    }
    IBDL_HIP(hipStreamSynchronize(h->st));
    if (info) {
      info->iters = total;
      info->status = status;
      info->krylov_relres = krylov;
      info->true_relres_fp64 = (bn > 0 || std::isnan(bn)) ? rn / bn : 0.0;
    }
    check_finite<double>(h, q, n, "q");
    if (u_grid) check_grid(h, u_grid, h->nq, "u");
    return status;
  });
}

ibdl_status_t ibdl_set_graph(ibdl_t h, int32_t enable) {
  return guarded(h, [&]() {
    IBDL_HIP(hipStreamSynchronize(h->st));
    h->use_graph = enable != 0;
    if (!h->use_graph) h->drop_graphs();
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_set_timing(ibdl_t h, int32_t enable) {
  return guarded(h, [&]() {
    h->collect();
    h->timing = enable != 0;
    for (int i = 0; i < 16; ++i) {
      h->stage_ms[i] = 0;
      h->stage_n[i] = 0;
    }
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_get_timing(ibdl_t h, double* ms, int64_t* count, int32_t cap) {
  return guarded(h, [&]() {
    if (!ms || !count || cap < 1) throw Error(IBDL_ERR_ARG, "NULL pointer or cap < 1");
    h->collect();
    for (int i = 0; i < cap && i < ST_COUNT; ++i) {
      ms[i] = h->stage_ms[i];
      count[i] = h->stage_n[i];
    }
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_query(ibdl_t h, int64_t* n_aug, int64_t* grid_points, int32_t* nq) {
  if (!h) return IBDL_ERR_ARG;
  if (n_aug) *n_aug = h->n_aug;
  if (grid_points) *grid_points = h->ntot;
  if (nq) *nq = h->nq;
  return IBDL_OK;
}

ibdl_status_t ibdl_active_rows(ibdl_t h, int64_t* nact, int64_t* rows_total) {
  if (!h) return IBDL_ERR_ARG;
  if (nact) *nact = h->nact;
  if (rows_total) *rows_total = h->ntot / h->n[0];
  return IBDL_OK;
}

ibdl_status_t ibdl_active_span(ibdl_t h, int32_t* first, int32_t* last) {
  if (!h) return IBDL_ERR_ARG;
  int a = h->dim == 3 ? h->zlim[0] : h->lim2d[0], b = h->dim == 3 ? h->zlim[1] : h->lim2d[1];
  if (h->dim == 2 && h->n[1] > 1024) {
    a = 0;
    b = h->n[1] - 1;
  }
  if (first) *first = a;
  if (last) *last = b;
  return IBDL_OK;
}

ibdl_status_t ibdl_spread_tiles(ibdl_t h, int64_t* nbusy, int64_t* segments_read, int32_t* tile) {
  if (!h) return IBDL_ERR_ARG;
  if (nbusy) *nbusy = h->nbusy;
  if (segments_read) *segments_read = h->seg_read;
  if (tile)
    for (int d = 0; d < 3; ++d) tile[d] = h->geom.tile[d];
  return IBDL_OK;
}

ibdl_status_t ibdl_launch_shape(ibdl_t h, int32_t* rows_per_block, int32_t* lines_y, int32_t* lines_last) {
  if (!h) return IBDL_ERR_ARG;
  LaunchShape sh;
  if (h->mixed() && h->w32) sh = h->w32->shape;
  else if (!h->mixed() && h->w64) sh = h->w64->shape;
  if (rows_per_block) *rows_per_block = sh.rpb;
  if (lines_y) *lines_y = sh.wy;
  if (lines_last) *lines_last = sh.wz;
  return IBDL_OK;
}

const char* ibdl_last_error(ibdl_t h) { return h ? h->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
