// Batched IBDL solves: many independent scalar Dirichlet problems (Sec. 5.3.2) advanced together.
//
// Problems on the same grid (sizes, box, origin, kappa) form a group.  A group is one
// block-diagonal problem: its markers are concatenated (marker i belongs to problem pid[i]),
// tiles are numbered problem-major, and its grid fields are stored problem after problem, so
// one launch of each stage (zero fill, spread, x pass, fused last-axis pass, x pass,
// interpolation) serves every problem of the group.  The Krylov vectors of all problems are
// concatenated; GMRES runs per problem (its own Hessenberg matrix and Givens rotations) with
// segmented reductions, one host synchronisation per iteration for the whole batch.  The
// batched operator apply is captured once in a HIP graph and replayed every iteration.  The
// launch shapes of the FFT passes (rows per block, lines per block) are picked per group by
// timing the candidates on the group's own arrays, and remembered per (dim, grid, precision,
// problem-count bucket) for the life of the process.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ibdl.h"
#include "kernels.h"
#include "tables.h"
#include "tune.h"

using namespace ibdl;

namespace {

std::string g_batch_create_error;

using Tuned = LaunchShape;

template <typename T> struct GroupWork {
  GridTables<T> tab;
  T* real = nullptr;          // [problem][grid]
  cplx<T>* spec = nullptr;    // [problem][half spectrum]
  cplx<T>* wtab = nullptr;    // weight table in this precision
  Tuned tune;
  bool ready = false;
};

struct Group {
  int n[3] = {1, 1, 1};
  double L[3] = {1, 1, 1};
  double origin[3] = {0, 0, 0};
  double kappa = 0;
  std::vector<int> probs;     // batch indices, in group order
  MarkerGeom geom{};
  int64_t ntot = 0, nxh = 0, nspec = 0;
  int64_t nib = 0;            // markers of the group
  int64_t aoff = 0;           // offset of the group's first unknown in batch vectors
  double *X = nullptr, *nrm = nullptr, *ds = nullptr, *f = nullptr, *wt = nullptr;
  int *s = nullptr, *pid = nullptr;
  int *tile_count = nullptr, *tile_off = nullptr, *tile_cur = nullptr, *list = nullptr, *list_tmp = nullptr;
  int4* busy = nullptr;
  int4* busy_tmp = nullptr;
  int* busy_off = nullptr;
  int nbusy = 0;
  GroupWork<float> w32;
  GroupWork<double> w64;
  template <typename T> GroupWork<T>& work();
};
template <> GroupWork<float>& Group::work<float>() { return w32; }
template <> GroupWork<double>& Group::work<double>() { return w64; }

}  // namespace

struct ibdl_batch_s {
  int nprob = 0, dim = 2, kernel = 0, precision = 0, pde = 0;
  hipStream_t ust = nullptr;    // the caller's stream
  hipStream_t st = nullptr;     // the batch's own stream (capturable)
  hipEvent_t ev = nullptr;
  std::vector<Group> groups;
  std::vector<int64_t> nib, aoff;
  std::vector<int> grp;
  int64_t N = 0;                // unknowns of the whole batch
  KrylovSegments sg;
  int ld = 0;                   // leading dimension of the per-problem small tables (maxit + 2)
  double* V = nullptr;
  int vcap = 0;
  double *vb = nullptr, *vr = nullptr, *xin = nullptr, *yout = nullptr, *xsol = nullptr;
  double* partial = nullptr;
  int pcap = 0;
  double* dsmall = nullptr;     // device: h1, h2 [nprob][ld], hn, sc [nprob], Y [nprob][ld]
  double* hsmall = nullptr;     // pinned host mirror
  int scap = 0;
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int gprec = -1;               // precision of the captured graph (0 float, 1 double)
  std::vector<void*> allocs;
  std::string err;

  void* dalloc(size_t bytes) {
    void* p = nullptr;
    IBDL_HIP(hipMalloc(&p, bytes ? bytes : 16));
    allocs.push_back(p);
    return p;
  }
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    gprec = -1;
  }
  ~ibdl_batch_s() {
    if (st) (void)hipStreamSynchronize(st);
    drop_graph();
    for (void* p : allocs) (void)hipFree(p);
    if (hsmall) (void)hipHostFree(hsmall);
    if (ev) (void)hipEventDestroy(ev);
    if (st) (void)hipStreamDestroy(st);
  }
  bool mixed() const { return precision == IBDL_MIXED; }
};

namespace {

template <typename T> MultDesc group_desc(const Group& G, const GroupWork<T>& W, int dim) {
  MultDesc md{};
  md.mode = 0;
  md.dim = dim;
  md.nxh = (int)G.nxh;
  md.nxp = (int)G.nxh;
  md.stokes = 0;
  md.nc = 1;
  md.fk[0] = FK_MASS;
  md.sc = 1.0 / (double)G.ntot;
  md.c0 = G.kappa * G.kappa;
  md.c2 = 1.0;
  md.mu = 1.0;
  md.alpha = -1.0;
  for (int d = 0; d < 3; ++d) {
    md.sig[d] = d < dim ? W.tab.sig[d] : W.tab.sig[0];
    md.kt[d] = d < dim ? W.tab.kt[d] : W.tab.kt[0];
  }
  return md;
}

// the group's spread field -> -L^-1 (field), all problems of the group at once
template <typename T> void group_pipeline(ibdl_batch_s* B, Group& G, GroupWork<T>& W, const Tuned& tn) {
  const int np = (int)G.probs.size();
  const int64_t rows = (int64_t)np * (G.ntot / G.n[0]);
  const MultDesc md = group_desc<T>(G, W, B->dim);
  fft_x_r2c<T>(W.real, W.spec, G.n[0], rows, W.tab.tw[0], B->st, tn.rpb);
  if (B->dim == 3)
    fft_strided<T>(W.spec, G.n[1], (int64_t)np * G.n[2] * G.nxh, G.nxh, G.nxh * G.n[1], G.nxh, false, W.tab.tw[1],
                   B->st);
  const int last = B->dim - 1;
  fft_fused_last<T>(W.spec, G.n[last], G.nspec / G.n[last], 1, md, W.tab.tw[last], B->st, np, G.nspec, tn.wz);
  if (B->dim == 3)
    fft_strided<T>(W.spec, G.n[1], (int64_t)np * G.n[2] * G.nxh, G.nxh, G.nxh * G.n[1], G.nxh, true, W.tab.tw[1],
                   B->st);
  fft_x_c2r<T>(W.spec, W.real, G.n[0], rows, W.tab.tw[0], B->st, tn.rpb);
}

// the group's density q (its slice of a batch vector) -> grid fields u[q] = -L^-1 S~ q per problem
template <typename T> void group_density_to_grid(ibdl_batch_s* B, Group& G, GroupWork<T>& W, const double* q) {
  const int np = (int)G.probs.size();
  grid_fill_zero<T>(W.real, (int64_t)np * G.ntot, B->st);
  SpreadArgs a{};
  a.g = G.geom;
  a.kernel = B->kernel;
  a.mode = SP_FDDIV;
  a.nf = 1;
  a.mass = 0;
  a.eta = 0.0;
  a.tile_off = G.tile_off;
  a.list = G.list;
  a.busy = G.busy;
  a.nbusy = G.nbusy;
  a.s = G.s;
  a.f = G.f;
  a.wt = G.wt;
  a.q = q;
  a.nrm = G.nrm;
  a.ds = G.ds;
  spread<T>(a, W.wtab, W.real, B->st);
  group_pipeline<T>(B, G, W, W.tune);
}

template <typename T> void tune_group(ibdl_batch_s* B, Group& G, GroupWork<T>& W);

template <typename T> GroupWork<T>& group_work(ibdl_batch_s* B, Group& G) {
  GroupWork<T>& W = G.work<T>();
  if (W.ready) return W;
  const int np = (int)G.probs.size();
  W.tab = make_grid_tables<T>(B->dim, G.n, G.L, G.geom.h, true, [&](size_t bytes) { return B->dalloc(bytes); });
  W.real = (T*)B->dalloc(sizeof(T) * G.ntot * np);
  W.spec = (cplx<T>*)B->dalloc(sizeof(cplx<T>) * G.nspec * np);
  W.wtab = (cplx<T>*)B->dalloc(sizeof(cplx<T>) * G.nib * 24);
  weight_table<T>(G.wt, G.nib, W.wtab, B->st);
  grid_fill_zero<T>(W.real, G.ntot * np, B->st);
  W.ready = true;
  tune_group<T>(B, G, W);
  return W;
}

// Launch shapes by measurement: every (rows per block, lines per block) pair from the maximum
// down to an eighth of it, two warm-up and five timed runs of the group's FFT passes each; a
// narrower pair is taken only when it is at least 3% faster.
template <typename T> void tune_group(ibdl_batch_s* B, Group& G, GroupWork<T>& W) {
  const int np = (int)G.probs.size();
  const TuneKey key{1, B->dim, G.n[0], G.n[1], G.n[2], (int)sizeof(T), 1, pow2_bucket(np)};
  if (tune_get(key, &W.tune)) return;
  const int rmax = fft_x_rpb_max<T>(G.n[0]);
  const int wmax = fft_line_w_max<T>(G.n[B->dim - 1]);
  hipEvent_t e0, e1;
  IBDL_HIP(hipEventCreate(&e0));
  IBDL_HIP(hipEventCreate(&e1));
  Tuned best;
  float best_ms = 1e30f;
  for (int r = rmax; r >= 1 && r * 8 >= rmax; r /= 2)
    for (int w = wmax; w >= 1 && w * 8 >= wmax; w /= 2) {
      Tuned c;
      c.rpb = r;
      c.wz = w;
      for (int k = 0; k < 2; ++k) group_pipeline<T>(B, G, W, c);
      IBDL_HIP(hipEventRecord(e0, B->st));
      for (int k = 0; k < 5; ++k) group_pipeline<T>(B, G, W, c);
      IBDL_HIP(hipEventRecord(e1, B->st));
      IBDL_HIP(hipEventSynchronize(e1));
      float ms = 0;
      IBDL_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < 0.97f * best_ms) {   // narrower shapes must be clearly faster
        best_ms = ms;
        best = c;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  W.tune = best;
  tune_put(key, best);
}

// y = A x for every problem of the batch (Dirichlet: y = S* u[x] + x/2)
template <typename T> void batch_apply(ibdl_batch_s* B, const double* x, double* y) {
  for (Group& G : B->groups) {
    GroupWork<T>& W = group_work<T>(B, G);
    group_density_to_grid<T>(B, G, W, x + G.aoff);
    InterpArgs ia{};
    ia.g = G.geom;
    ia.kernel = B->kernel;
    ia.nf = 1;
    ia.n_ib = G.nib;
    ia.s = G.s;
    ia.f = G.f;
    ia.wt = G.wt;
    ia.a = 1.0;
    ia.b = 0.5;
    ia.x = x + G.aoff;
    ia.ub = nullptr;
    ia.pid = G.pid;
    interp<T>(ia, W.wtab, W.real, y + G.aoff, B->st);
  }
}

void apply_any(ibdl_batch_s* B, const double* x, double* y, bool force64) {
  if (B->mixed() && !force64) batch_apply<float>(B, x, y);
  else batch_apply<double>(B, x, y);
}

// Capture the batched apply xin -> yout (working precision) in a graph, after one eager run that
// allocates every workspace and tunes the launch shapes.
void ensure_graph(ibdl_batch_s* B) {
  const int prec = B->mixed() ? 0 : 1;
  if (B->gexec && B->gprec == prec) return;
  B->drop_graph();
  apply_any(B, B->xin, B->yout, false);
  IBDL_HIP(hipStreamSynchronize(B->st));
  IBDL_HIP(hipStreamBeginCapture(B->st, hipStreamCaptureModeThreadLocal));
  try {
    apply_any(B, B->xin, B->yout, false);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(B->st, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  IBDL_HIP(hipStreamEndCapture(B->st, &B->graph));
  IBDL_HIP(hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
  B->gprec = prec;
}

// yout = A src
void apply_step(ibdl_batch_s* B, const double* src) {
  if (B->use_graph) {
    ensure_graph(B);
    IBDL_HIP(hipMemcpyAsync(B->xin, src, sizeof(double) * B->N, hipMemcpyDeviceToDevice, B->st));
    IBDL_HIP(hipGraphLaunch(B->gexec, B->st));
  } else {
    apply_any(B, src, B->yout, false);
  }
}

void ensure_krylov(ibdl_batch_s* B, int maxit) {
  if (B->vcap < maxit + 1) {
    B->V = (double*)B->dalloc(sizeof(double) * B->N * (maxit + 1));
    B->vcap = maxit + 1;
  }
  const int ld = maxit + 2;
  const int need = B->nprob * (3 * ld + 2);
  if (B->scap < need || B->ld != ld) {
    B->dsmall = (double*)B->dalloc(sizeof(double) * need);
    if (B->hsmall) (void)hipHostFree(B->hsmall);
    B->hsmall = nullptr;
    IBDL_HIP(hipHostMalloc((void**)&B->hsmall, sizeof(double) * need, hipHostMallocDefault));
    B->scap = need;
    B->ld = ld;
  }
  const int pneed = B->sg.nblk * (maxit + 2);
  if (B->pcap < pneed) {
    B->partial = (double*)B->dalloc(sizeof(double) * pneed);
    B->pcap = pneed;
  }
}

// per-problem 2-norms of a batch vector (synchronises)
std::vector<double> seg_norms(ibdl_batch_s* B, const double* v) {
  double* hn = B->dsmall + 2 * B->nprob * B->ld;
  kb_multidot(v, B->N, 1, v, B->sg, B->partial, 1, hn, B->st);
  IBDL_HIP(hipMemcpyAsync(B->hsmall, hn, sizeof(double) * B->nprob, hipMemcpyDeviceToHost, B->st));
  IBDL_HIP(hipStreamSynchronize(B->st));
  std::vector<double> r(B->nprob);
  for (int p = 0; p < B->nprob; ++p) r[p] = sqrt(std::max(B->hsmall[p], 0.0));
  return r;
}

// GMRES per problem (x0 = 0, no restart, CGS2, Givens on the host), all problems in lock step.
void batch_gmres(ibdl_batch_s* B, double tol, int maxit, double* x, std::vector<int>& iters,
                 std::vector<double>& relres, std::vector<int>& status, ibdl_info_t* infos) {
  const int np = B->nprob, ld = B->ld;
  const int64_t n = B->N;
  double* h1 = B->dsmall;
  double* h2 = B->dsmall + np * ld;
  double* hn = B->dsmall + 2 * np * ld;
  double* sc = hn + np;
  double* Yd = sc + np;
  double* H1 = B->hsmall;
  double* H2 = B->hsmall + np * ld;
  double* HN = B->hsmall + 2 * np * ld;
  double* SC = HN + np;
  double* YH = SC + np;
  const std::vector<double> beta = seg_norms(B, B->vb);
  std::vector<std::vector<double>> H(np), cs(np), sn(np), gv(np);
  std::vector<char> active(np, 1);
  iters.assign(np, 0);
  relres.assign(np, 0.0);
  status.assign(np, IBDL_OK);
  for (int p = 0; p < np; ++p) {
    if (!std::isfinite(beta[p])) throw Error(IBDL_ERR_NONFINITE, "right-hand side is not finite");
    H[p].assign((size_t)(maxit + 1) * maxit, 0.0);
    cs[p].assign(maxit, 0.0);
    sn[p].assign(maxit, 0.0);
    gv[p].assign(maxit + 1, 0.0);
    gv[p][0] = beta[p];
    SC[p] = beta[p] > 0 ? 1.0 / beta[p] : 0.0;
    if (!(beta[p] > 0)) active[p] = 0;
    relres[p] = beta[p] > 0 ? 1.0 : 0.0;
  }
  IBDL_HIP(hipMemcpyAsync(sc, SC, sizeof(double) * np, hipMemcpyHostToDevice, B->st));
  kb_scale(B->vb, sc, B->sg, B->V, B->st);
  for (int j = 0; j < maxit; ++j) {
    if (std::none_of(active.begin(), active.end(), [](char a) { return a != 0; })) break;
    apply_step(B, B->V + (int64_t)j * n);
    double* w = B->yout;
    kb_multidot(B->V, n, j + 1, w, B->sg, B->partial, ld, h1, B->st);
    kb_gemv_sub(B->V, n, j + 1, h1, ld, B->sg, w, B->st);
    kb_multidot(B->V, n, j + 1, w, B->sg, B->partial, ld, h2, B->st);
    kb_gemv_sub(B->V, n, j + 1, h2, ld, B->sg, w, B->st);
    kb_multidot(w, n, 1, w, B->sg, B->partial, 1, hn, B->st);
    IBDL_HIP(hipMemcpyAsync(B->hsmall, B->dsmall, sizeof(double) * (2 * np * ld + np), hipMemcpyDeviceToHost,
                            B->st));
    IBDL_HIP(hipStreamSynchronize(B->st));
    for (int p = 0; p < np; ++p) {
      SC[p] = 0.0;
      if (!active[p]) continue;
      double* Hj = &H[p][(size_t)j * (maxit + 1)];
      for (int i = 0; i <= j; ++i) Hj[i] = H1[p * ld + i] + H2[p * ld + i];
      const double hnext = sqrt(std::max(HN[p], 0.0));
      if (!std::isfinite(hnext)) throw Error(IBDL_ERR_NONFINITE, "non-finite value in the Arnoldi process");
      Hj[j + 1] = hnext;
      const bool breakdown = !(hnext > 1e-300 * beta[p]);
      SC[p] = breakdown ? 0.0 : 1.0 / hnext;
      for (int i = 0; i < j; ++i) {
        const double t = cs[p][i] * Hj[i] + sn[p][i] * Hj[i + 1];
        Hj[i + 1] = -sn[p][i] * Hj[i] + cs[p][i] * Hj[i + 1];
        Hj[i] = t;
      }
      const double r = hypot(Hj[j], Hj[j + 1]);
      cs[p][j] = Hj[j] / r;
      sn[p][j] = Hj[j + 1] / r;
      Hj[j] = r;
      Hj[j + 1] = 0.0;
      gv[p][j + 1] = -sn[p][j] * gv[p][j];
      gv[p][j] = cs[p][j] * gv[p][j];
      iters[p] = j + 1;
      relres[p] = fabs(gv[p][j + 1]) / beta[p];
      if (infos && infos[p].history && j < infos[p].history_cap) infos[p].history[j] = relres[p];
      if (relres[p] <= tol || breakdown) active[p] = 0;
    }
    IBDL_HIP(hipMemcpyAsync(sc, SC, sizeof(double) * np, hipMemcpyHostToDevice, B->st));
    kb_scale(w, sc, B->sg, B->V + (int64_t)(j + 1) * n, B->st);
  }
  int kmax = 0;
  for (int p = 0; p < np; ++p) {
    const int k = iters[p];
    kmax = std::max(kmax, k);
    for (int i = 0; i < ld; ++i) YH[p * ld + i] = 0.0;
    for (int i = k - 1; i >= 0; --i) {
      double s = gv[p][i];
      for (int c = i + 1; c < k; ++c) s -= H[p][(size_t)c * (maxit + 1) + i] * YH[p * ld + c];
      YH[p * ld + i] = s / H[p][(size_t)i * (maxit + 1) + i];
    }
    status[p] = (beta[p] > 0 && relres[p] > tol) ? IBDL_NOT_CONVERGED : IBDL_OK;
  }
  IBDL_HIP(hipMemcpyAsync(Yd, YH, sizeof(double) * np * ld, hipMemcpyHostToDevice, B->st));
  kb_lincomb(B->V, n, std::max(kmax, 1), Yd, ld, B->sg, x, B->st);
  IBDL_HIP(hipStreamSynchronize(B->st));
}

template <typename T> void batch_recover(ibdl_batch_s* B, const double* q, void* const* u) {
  for (Group& G : B->groups) {
    GroupWork<T>& W = group_work<T>(B, G);
    group_density_to_grid<T>(B, G, W, q + G.aoff);
    for (size_t k = 0; k < G.probs.size(); ++k) {
      void* dst = u[G.probs[k]];
      if (dst)
        IBDL_HIP(hipMemcpyAsync(dst, W.real + (int64_t)k * G.ntot, sizeof(T) * G.ntot, hipMemcpyDeviceToDevice,
                                B->st));
    }
  }
}

bool pow2_ok(int64_t v) { return v >= 16 && v <= 1024 && (v & (v - 1)) == 0; }

void validate_batch(int32_t nprob, const ibdl_config_t* cfgs, const int64_t* n_ib) {
  if (nprob < 1 || nprob > 4096) throw Error(IBDL_ERR_ARG, "nprob must be in [1, 4096]");
  if (!cfgs || !n_ib) throw Error(IBDL_ERR_ARG, "NULL configuration arrays");
  const ibdl_config_t& c0 = cfgs[0];
  for (int p = 0; p < nprob; ++p) {
    const ibdl_config_t& c = cfgs[p];
    if (c.dim != c0.dim || c.precision != c0.precision || c.kernel != c0.kernel)
      throw Error(IBDL_ERR_ARG, "all problems of a batch share dim, precision and kernel");
    if (c.dim != 2 && c.dim != 3) throw Error(IBDL_ERR_ARG, "dim must be 2 or 3");
    if (c.pde != IBDL_PDE_SCREENED && c.pde != IBDL_PDE_POISSON)
      throw Error(IBDL_ERR_UNSUPPORTED, "batches hold scalar problems (screened Poisson or Poisson)");
    if (c.pde == IBDL_PDE_SCREENED && !(c.kappa > 0 && std::isfinite(c.kappa)))
      throw Error(IBDL_ERR_ARG, "screened Poisson needs a finite kappa > 0");
    if (c.bc != IBDL_BC_DIRICHLET || c.eta != 0.0)
      throw Error(IBDL_ERR_UNSUPPORTED, "batches hold plain Dirichlet problems (bc Dirichlet, eta = 0)");
    if (c.method != IBDL_METHOD_DL) throw Error(IBDL_ERR_UNSUPPORTED, "batches hold double layer problems");
    if (c.disc != IBDL_DISC_FD2) throw Error(IBDL_ERR_UNSUPPORTED, "batches use the finite-difference symbols");
    if (c.kernel != IBDL_K_PESKIN4 && c.kernel != IBDL_K_COS4)
      throw Error(IBDL_ERR_UNSUPPORTED, "batches use a 4-point kernel");
    if (c.precision != IBDL_FP64 && c.precision != IBDL_MIXED) throw Error(IBDL_ERR_ARG, "unknown precision");
    double h0 = 0;
    for (int d = 0; d < c.dim; ++d) {
      if (!pow2_ok(c.n[d])) throw Error(IBDL_ERR_UNSUPPORTED, "grid size must be a power of two in [16, 1024]");
      if (!(c.L[d] > 0) || !std::isfinite(c.L[d]) || !std::isfinite(c.origin[d]))
        throw Error(IBDL_ERR_ARG, "box lengths must be positive and finite");
      const double hd = c.L[d] / (double)c.n[d];
      if (d == 0) h0 = hd;
      else if (fabs(hd - h0) > 1e-12 * h0) throw Error(IBDL_ERR_ARG, "grid spacing must be equal on every axis");
    }
    if (n_ib[p] < 1 || n_ib[p] > ((int64_t)1 << 28)) throw Error(IBDL_ERR_ARG, "n_ib out of range");
  }
}

template <typename F> ibdl_status_t guarded(ibdl_batch_s* B, F&& fn) {
  if (!B) return IBDL_ERR_ARG;
  try {
    return (ibdl_status_t)fn();
  } catch (const Error& e) {
    B->err = e.what();
    return (ibdl_status_t)e.code;
  } catch (const std::exception& e) {
    B->err = e.what();
    return IBDL_ERR_HIP;
  }
}

}  // namespace

extern "C" {

ibdl_status_t ibdl_batch_create(int32_t nprob, const ibdl_config_t* cfgs, const int64_t* n_ib, const double* const* X,
                                const double* const* nrm, const double* const* ds, ibdl_batch_t* out) {
  if (!out) {
    g_batch_create_error = "out is NULL";
    return IBDL_ERR_ARG;
  }
  *out = nullptr;
  std::unique_ptr<ibdl_batch_s> B(new ibdl_batch_s());
  try {
    validate_batch(nprob, cfgs, n_ib);
    if (!X || !nrm || !ds) throw Error(IBDL_ERR_ARG, "marker pointer arrays must be non-NULL");
    for (int p = 0; p < nprob; ++p)
      if (!X[p] || !nrm[p] || !ds[p]) throw Error(IBDL_ERR_ARG, "marker arrays must be non-NULL device pointers");
    B->nprob = nprob;
    B->dim = cfgs[0].dim;
    B->kernel = cfgs[0].kernel;
    B->precision = cfgs[0].precision;
    B->ust = (hipStream_t)cfgs[0].stream;
    IBDL_HIP(hipStreamCreateWithFlags(&B->st, hipStreamNonBlocking));
    IBDL_HIP(hipEventCreateWithFlags(&B->ev, hipEventDisableTiming));
    IBDL_HIP(hipEventRecord(B->ev, B->ust));
    IBDL_HIP(hipStreamWaitEvent(B->st, B->ev, 0));
    const int dim = B->dim;
    // group the problems by grid
    B->grp.assign(nprob, -1);
    for (int p = 0; p < nprob; ++p) {
      const ibdl_config_t& c = cfgs[p];
      const double kap = c.pde == IBDL_PDE_POISSON ? 0.0 : c.kappa;
      int gi = -1;
      for (size_t k = 0; k < B->groups.size() && gi < 0; ++k) {
        const Group& G = B->groups[k];
        bool same = G.kappa == kap;
        for (int d = 0; d < dim; ++d)
          same = same && G.n[d] == (int)c.n[d] && G.L[d] == c.L[d] && G.origin[d] == c.origin[d];
        if (same) gi = (int)k;
      }
      if (gi < 0) {
        Group G;
        for (int d = 0; d < dim; ++d) {
          G.n[d] = (int)c.n[d];
          G.L[d] = c.L[d];
          G.origin[d] = c.origin[d];
        }
        G.kappa = kap;
        B->groups.push_back(G);
        gi = (int)B->groups.size() - 1;
      }
      B->groups[gi].probs.push_back(p);
      B->grp[p] = gi;
    }
    // unknowns: group after group, problems in group order
    B->nib.assign(n_ib, n_ib + nprob);
    B->aoff.assign(nprob, 0);
    int64_t off = 0;
    for (Group& G : B->groups) {
      G.aoff = off;
      G.nib = 0;
      for (int p : G.probs) {
        B->aoff[p] = off;
        off += n_ib[p];
        G.nib += n_ib[p];
      }
    }
    B->N = off;
    // markers, stencils and tile bins per group
    for (Group& G : B->groups) {
      const int np = (int)G.probs.size();
      MarkerGeom& g = G.geom;
      g.dim = dim;
      g.h = G.L[0] / (double)G.n[0];
      for (int d = 0; d < 3; ++d) {
        g.n[d] = d < dim ? G.n[d] : 1;
        g.origin[d] = d < dim ? G.origin[d] : 0.0;
        const int t3[3] = {16, 4, 8};
        g.tile[d] = d < dim ? (dim == 2 ? 16 : t3[d]) : 1;
        g.ntile[d] = g.n[d] / g.tile[d];
        G.n[d] = g.n[d];
      }
      G.ntot = (int64_t)G.n[0] * G.n[1] * G.n[2];
      G.nxh = G.n[0] / 2 + 1;
      G.nspec = G.nxh * G.n[1] * G.n[2];
      const int64_t ntile = (int64_t)g.ntile[0] * g.ntile[1] * g.ntile[2] * np;
      const int64_t maxlist = G.nib * (dim == 2 ? 4 : 12);
      G.X = (double*)B->dalloc(sizeof(double) * G.nib * dim);
      G.nrm = (double*)B->dalloc(sizeof(double) * G.nib * dim);
      G.ds = (double*)B->dalloc(sizeof(double) * G.nib);
      G.s = (int*)B->dalloc(sizeof(int) * G.nib * 3);
      G.f = (double*)B->dalloc(sizeof(double) * G.nib * 3);
      G.wt = (double*)B->dalloc(sizeof(double) * G.nib * 36);
      G.pid = (int*)B->dalloc(sizeof(int) * G.nib);
      G.tile_count = (int*)B->dalloc(sizeof(int) * ntile);
      G.tile_off = (int*)B->dalloc(sizeof(int) * (ntile + 1));
      G.tile_cur = (int*)B->dalloc(sizeof(int) * ntile);
      G.busy = (int4*)B->dalloc(sizeof(int4) * ntile);
      G.busy_tmp = (int4*)B->dalloc(sizeof(int4) * ntile);
      G.busy_off = (int*)B->dalloc(sizeof(int) * (ntile + 1));
      G.list = (int*)B->dalloc(sizeof(int) * maxlist);
      G.list_tmp = (int*)B->dalloc(sizeof(int) * maxlist);
      std::vector<int> pid(G.nib);
      int64_t m = 0;
      for (int k = 0; k < np; ++k) {
        const int p = G.probs[k];
        IBDL_HIP(hipMemcpyAsync(G.X + m * dim, X[p], sizeof(double) * n_ib[p] * dim, hipMemcpyDeviceToDevice, B->st));
        IBDL_HIP(hipMemcpyAsync(G.nrm + m * dim, nrm[p], sizeof(double) * n_ib[p] * dim, hipMemcpyDeviceToDevice,
                                B->st));
        IBDL_HIP(hipMemcpyAsync(G.ds + m, ds[p], sizeof(double) * n_ib[p], hipMemcpyDeviceToDevice, B->st));
        for (int64_t i = 0; i < n_ib[p]; ++i) pid[m + i] = k;
        m += n_ib[p];
      }
      IBDL_HIP(hipMemcpyAsync(G.pid, pid.data(), sizeof(int) * G.nib, hipMemcpyHostToDevice, B->st));
      markers_setup(g, B->kernel, G.nib, G.X, G.s, G.f, G.wt, G.tile_count, B->st, G.pid, np);
      markers_bin(g, G.nib, G.s, G.tile_count, G.tile_off, G.tile_cur, G.list, G.list_tmp, G.busy, G.busy_tmp,
                  G.busy_off, B->st, G.pid, np);
      int nb = 0;
      IBDL_HIP(hipMemcpyAsync(&nb, G.busy_off + ntile, sizeof(int), hipMemcpyDeviceToHost, B->st));
      IBDL_HIP(hipStreamSynchronize(B->st));
      G.nbusy = nb;
    }
    // Krylov segments: one dot-product block per 2048 unknowns of a problem
    {
      std::vector<int> seg(B->N), pb0(nprob + 1, 0);
      std::vector<int64_t> beg, end;
      std::vector<int> order;
      for (Group& G : B->groups)
        for (int p : G.probs) order.push_back(p);
      std::vector<int> first(nprob, 0), count(nprob, 0);
      for (int p : order) {
        for (int64_t e = 0; e < n_ib[p]; ++e) seg[B->aoff[p] + e] = p;
        first[p] = (int)beg.size();
        for (int64_t b = 0; b < n_ib[p]; b += 2048) {
          beg.push_back(B->aoff[p] + b);
          end.push_back(B->aoff[p] + std::min<int64_t>(b + 2048, n_ib[p]));
        }
        count[p] = (int)beg.size() - first[p];
      }
      // pb0 is indexed by problem: problem p owns blocks first[p] .. first[p] + count[p] - 1, and
      // k_breduce reads pb0[p] .. pb0[p+1]; lay the blocks out in problem order to match
      std::vector<int64_t> beg2, end2;
      for (int p = 0; p < nprob; ++p) {
        pb0[p] = (int)beg2.size();
        for (int b = 0; b < count[p]; ++b) {
          beg2.push_back(beg[first[p] + b]);
          end2.push_back(end[first[p] + b]);
        }
      }
      pb0[nprob] = (int)beg2.size();
      int* dseg = (int*)B->dalloc(sizeof(int) * B->N);
      int64_t* dbeg = (int64_t*)B->dalloc(sizeof(int64_t) * beg2.size());
      int64_t* dend = (int64_t*)B->dalloc(sizeof(int64_t) * end2.size());
      int* dpb0 = (int*)B->dalloc(sizeof(int) * (nprob + 1));
      IBDL_HIP(hipMemcpy(dseg, seg.data(), sizeof(int) * B->N, hipMemcpyHostToDevice));
      IBDL_HIP(hipMemcpy(dbeg, beg2.data(), sizeof(int64_t) * beg2.size(), hipMemcpyHostToDevice));
      IBDL_HIP(hipMemcpy(dend, end2.data(), sizeof(int64_t) * end2.size(), hipMemcpyHostToDevice));
      IBDL_HIP(hipMemcpy(dpb0, pb0.data(), sizeof(int) * (nprob + 1), hipMemcpyHostToDevice));
      B->sg.nprob = nprob;
      B->sg.n = B->N;
      B->sg.nblk = (int)beg2.size();
      B->sg.seg = dseg;
      B->sg.beg = dbeg;
      B->sg.end = dend;
      B->sg.pb0 = dpb0;
    }
    B->vb = (double*)B->dalloc(sizeof(double) * B->N);
    B->vr = (double*)B->dalloc(sizeof(double) * B->N);
    B->xin = (double*)B->dalloc(sizeof(double) * B->N);
    B->yout = (double*)B->dalloc(sizeof(double) * B->N);
    B->xsol = (double*)B->dalloc(sizeof(double) * B->N);
    IBDL_HIP(hipMemsetAsync(B->xin, 0, sizeof(double) * B->N, B->st));
    for (Group& G : B->groups) {
      if (B->mixed()) group_work<float>(B.get(), G);
      else group_work<double>(B.get(), G);
    }
    IBDL_HIP(hipStreamSynchronize(B->st));
  } catch (const Error& e) {
    g_batch_create_error = e.what();
    return (ibdl_status_t)e.code;
  } catch (const std::exception& e) {
    g_batch_create_error = e.what();
    return IBDL_ERR_HIP;
  }
  *out = B.release();
  return IBDL_OK;
}

ibdl_status_t ibdl_batch_destroy(ibdl_batch_t b) {
  if (!b) return IBDL_ERR_ARG;
  delete b;
  return IBDL_OK;
}

ibdl_status_t ibdl_batch_apply(ibdl_batch_t b, const double* const* q, double* const* y) {
  return guarded(b, [&]() {
    if (!q || !y) throw Error(IBDL_ERR_ARG, "NULL pointer array");
    IBDL_HIP(hipEventRecord(b->ev, b->ust));
    IBDL_HIP(hipStreamWaitEvent(b->st, b->ev, 0));
    for (int p = 0; p < b->nprob; ++p) {
      if (!q[p] || !y[p]) throw Error(IBDL_ERR_ARG, "NULL vector");
      IBDL_HIP(hipMemcpyAsync(b->vb + b->aoff[p], q[p], sizeof(double) * b->nib[p], hipMemcpyDeviceToDevice, b->st));
    }
    apply_step(b, b->vb);
    for (int p = 0; p < b->nprob; ++p)
      IBDL_HIP(hipMemcpyAsync(y[p], b->yout + b->aoff[p], sizeof(double) * b->nib[p], hipMemcpyDeviceToDevice, b->st));
    IBDL_HIP(hipStreamSynchronize(b->st));
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_batch_solve(ibdl_batch_t b, const double* const* data, double tol, int32_t maxit,
                               double* const* q, void* const* u, ibdl_info_t* infos) {
  return guarded(b, [&]() {
    if (!data || !q) throw Error(IBDL_ERR_ARG, "NULL pointer array");
    if (!(tol >= 0) || !std::isfinite(tol)) throw Error(IBDL_ERR_ARG, "tol must be finite and >= 0");
    if (maxit < 1 || maxit > 200) throw Error(IBDL_ERR_ARG, "maxit must be in [1, 200]");
    for (int p = 0; p < b->nprob; ++p)
      if (!data[p] || !q[p]) throw Error(IBDL_ERR_ARG, "NULL data or q pointer");
    IBDL_HIP(hipEventRecord(b->ev, b->ust));
    IBDL_HIP(hipStreamWaitEvent(b->st, b->ev, 0));
    ensure_krylov(b, maxit);
    for (int p = 0; p < b->nprob; ++p)
      IBDL_HIP(hipMemcpyAsync(b->vb + b->aoff[p], data[p], sizeof(double) * b->nib[p], hipMemcpyDeviceToDevice,
                              b->st));
    std::vector<int> iters, status;
    std::vector<double> relres;
    batch_gmres(b, tol, maxit, b->xsol, iters, relres, status, infos);
    // true residuals with a double-precision apply
    apply_any(b, b->xsol, b->vr, true);
    kr_axpby(b->vr, 1.0, b->vb, -1.0, b->N, b->st);
    const std::vector<double> rn = seg_norms(b, b->vr);
    const std::vector<double> bn = seg_norms(b, b->vb);
    for (int p = 0; p < b->nprob; ++p)
      IBDL_HIP(hipMemcpyAsync(q[p], b->xsol + b->aoff[p], sizeof(double) * b->nib[p], hipMemcpyDeviceToDevice,
                              b->st));
    if (u) {
      if (b->mixed()) batch_recover<float>(b, b->xsol, u);
      else batch_recover<double>(b, b->xsol, u);
    }
    IBDL_HIP(hipStreamSynchronize(b->st));
    int worst = IBDL_OK;
    for (int p = 0; p < b->nprob; ++p) {
      if (status[p] != IBDL_OK) worst = status[p];
      if (infos) {
        infos[p].iters = iters[p];
        infos[p].status = status[p];
        infos[p].krylov_relres = relres[p];
        infos[p].true_relres_fp64 = bn[p] > 0 ? rn[p] / bn[p] : 0.0;
      }
    }
    return worst;
  });
}

ibdl_status_t ibdl_batch_set_graph(ibdl_batch_t b, int32_t enable) {
  return guarded(b, [&]() {
    IBDL_HIP(hipStreamSynchronize(b->st));
    b->use_graph = enable != 0;
    if (!b->use_graph) b->drop_graph();
    return IBDL_OK;
  });
}

ibdl_status_t ibdl_batch_query(ibdl_batch_t b, int32_t group, int32_t* ngroups, int32_t* nprob_in_group,
                               int32_t* n, int32_t* rows_per_block, int32_t* lines_per_block) {
  return guarded(b, [&]() {
    if (ngroups) *ngroups = (int32_t)b->groups.size();
    if (group < 0) return IBDL_OK;
    if (group >= (int)b->groups.size()) throw Error(IBDL_ERR_ARG, "group out of range");
    Group& G = b->groups[group];
    const Tuned& t = b->mixed() ? G.w32.tune : G.w64.tune;
    if (nprob_in_group) *nprob_in_group = (int32_t)G.probs.size();
    if (n)
      for (int d = 0; d < 3; ++d) n[d] = G.n[d];
    if (rows_per_block) *rows_per_block = t.rpb;
    if (lines_per_block) *lines_per_block = t.wz;
    return IBDL_OK;
  });
}

const char* ibdl_batch_last_error(ibdl_batch_t b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

}  // extern "C"
