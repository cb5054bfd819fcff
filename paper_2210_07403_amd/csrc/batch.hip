// Batched IBDL solves: many independent scalar Dirichlet problems (Sec. 5.3.2) advanced together.
//
// Problems on the same grid (sizes, box, origin, kappa) form a group.  A group is one
// block-diagonal problem: its markers are concatenated (marker i belongs to problem pid[i]),
// tiles are numbered problem-major, and its grid fields are stored problem after problem, so one
// launch of each FFT pass serves every problem of the group.  In 2-D the spread of all groups is
// one persistent launch over a single queue of busy tiles (longest first across the batch), and
// the interpolation of all groups is one launch.  The spread writes busy tiles only and the
// forward x pass reads only their row segments, so no field is cleared.  The Krylov vectors of
// all problems are concatenated; each GMRES iteration's Gram-Schmidt passes, Givens rotations and
// convergence test run on the device, one workgroup per problem in one launch, with a
// per-problem convergence flag; the host queues the next iteration before it reads the published
// residuals of the current one.  The batched operator apply is captured once in a HIP graph and
// replayed every iteration.  The tile shape of the 2-D spread and the launch shapes of the FFT
// passes are picked per group by timing the candidates on the group's own arrays, and remembered
// in the tuning registry (tune.hip: in memory and in a JSON file).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
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
  int64_t ntot = 0, nxh = 0, nxp = 0, nspec = 0;   // nxp: half-spectrum row pitch (128-byte rows)
  int64_t nib = 0;            // markers of the group
  int64_t aoff = 0;           // offset of the group's first unknown in batch vectors
  double *X = nullptr, *nrm = nullptr, *ds = nullptr, *f = nullptr, *wt = nullptr;
  int *s = nullptr, *pid = nullptr;
  int *tile_count = nullptr, *tile_off = nullptr, *tile_cur = nullptr, *list = nullptr, *list_tmp = nullptr;
  int4* busy = nullptr;
  int4* busy_tmp = nullptr;
  int* busy_off = nullptr;
  int nbusy = 0;
  unsigned long long* seg_all = nullptr;   // busy x-segments of every row of every problem
  bool tiles_tuned = false;
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
  // device-driven GMRES: per-problem segment offsets and lengths, |b|^2, least-squares states
  int64_t *doff = nullptr, *dlen = nullptr;
  int64_t maxlen = 0;
  double* bn2 = nullptr;
  double* gsb = nullptr;
  int64_t gstride = 0;
  int gmx = 0;
  // pointer tables of the per-problem input and output arrays: pinned host staging, device copy
  const double** hptr = nullptr;
  const double** dptr = nullptr;
  // host-mapped, coherent: two publication slots of [nprob][GM_PUB] doubles, then two tags
  double* hmap = nullptr;
  double* hmap_dev = nullptr;
  unsigned seq = 0;
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int gprec = -1;               // precision of the captured graph (0 float, 1 double)
  // 2-D single-launch spread and interpolation over all groups (per working precision: 0 float,
  // 1 double): group descriptors, the work queue of busy tiles, its counters
  struct Queue {
    SpreadGroup* sg = nullptr;
    InterpGroup* ig = nullptr;
    int2* items = nullptr;
    int nitems = 0;
    int blocks = 0;             // workgroups of the persistent spread (0: one per tile)
    bool ready = false;
  } queue[2];
  int spread_blocks = 0;        // workgroups of the persistent spread
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
    if (hmap) (void)hipHostFree(hmap);
    if (hptr) (void)hipHostFree((void*)hptr);
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
  md.nxp = (int)G.nxp;
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
  // the spread wrote the busy tiles only: the x pass reads their row segments and takes the rest
  // of each row as zero (no clearing of the fields)
  RowList rl;
  rl.rpf = rows;
  rl.seg = G.seg_all;
  rl.seg_log2 = __builtin_ctz((unsigned)G.geom.tile[0] / 2);
  fft_x_r2c<T>(W.real, W.spec, G.n[0], rows, W.tab.tw[0], B->st, tn.rpb, rl, G.nxp);
  if (B->dim == 3)
    fft_strided<T>(W.spec, G.n[1], (int64_t)np * G.n[2] * G.nxp, G.nxp, G.nxp * G.n[1], G.nxp, false, W.tab.tw[1],
                   B->st, 0, RowMask(), G.nxh);
  const int last = B->dim - 1;
  fft_fused_last<T>(W.spec, G.n[last], G.nspec / G.n[last], 1, md, W.tab.tw[last], B->st, np, G.nspec, tn.wz);
  if (B->dim == 3)
    fft_strided<T>(W.spec, G.n[1], (int64_t)np * G.n[2] * G.nxp, G.nxp, G.nxp * G.n[1], G.nxp, true, W.tab.tw[1],
                   B->st, 0, RowMask(), G.nxh);
  fft_x_c2r<T>(W.spec, W.real, G.n[0], rows, W.tab.tw[0], B->st, tn.rpb, RowList(), G.nxp);
}

// the group's density q (its slice of a batch vector) -> grid fields u[q] = -L^-1 S~ q per problem
template <typename T> void group_density_to_grid(ibdl_batch_s* B, Group& G, GroupWork<T>& W, const double* q) {
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

// Stencils and tile bins of a group for its current tile shape (geom.tile): candidate lists, busy
// tiles longest first, the busy x-segments of every row; synchronises to read the busy count.
void bin_group(ibdl_batch_s* B, Group& G) {
  const int np = (int)G.probs.size();
  MarkerGeom& g = G.geom;
  for (int d = 0; d < 3; ++d) g.ntile[d] = g.n[d] / g.tile[d];
  const int64_t ntile = (int64_t)g.ntile[0] * g.ntile[1] * g.ntile[2] * np;
  markers_setup(g, B->kernel, G.nib, G.X, G.s, G.f, G.wt, G.tile_count, B->st, G.pid, np);
  markers_bin(g, G.nib, G.s, G.tile_count, G.tile_off, G.tile_cur, G.list, G.list_tmp, G.busy, G.busy_tmp, G.busy_off,
              B->st, G.pid, np);
  markers_row_segments(g, G.tile_off, nullptr, (int64_t)np * G.n[1] * G.n[2], G.seg_all, B->st);
  int nb = 0;
  IBDL_HIP(hipMemcpyAsync(&nb, G.busy_off + ntile, sizeof(int), hipMemcpyDeviceToHost, B->st));
  IBDL_HIP(hipStreamSynchronize(B->st));
  G.nbusy = nb;
}

bool queue_path(const ibdl_batch_s* B) { return B->dim == 2; }

// The work queue of one or all groups' busy tiles, by decreasing candidate count (ties: group, then
// index), read back from the groups' busy lists.
std::vector<int2> queue_items(ibdl_batch_s* B, int only) {
  struct It { int cnt, grp, idx; };
  std::vector<It> all;
  for (int gi = 0; gi < (int)B->groups.size(); ++gi) {
    if (only >= 0 && gi != only) continue;
    Group& G = B->groups[gi];
    std::vector<int4> bt(G.nbusy);
    if (G.nbusy > 0)
      IBDL_HIP(hipMemcpyAsync(bt.data(), G.busy, sizeof(int4) * G.nbusy, hipMemcpyDeviceToHost, B->st));
    IBDL_HIP(hipStreamSynchronize(B->st));
    for (int k = 0; k < G.nbusy; ++k) all.push_back({bt[k].z - bt[k].y, gi, k});
  }
  std::stable_sort(all.begin(), all.end(), [](const It& a, const It& b) { return a.cnt > b.cnt; });
  std::vector<int2> out(all.size());
  for (size_t k = 0; k < all.size(); ++k) out[k] = make_int2(all[k].grp, all[k].idx);
  return out;
}

template <typename T> SpreadGroup spread_group(ibdl_batch_s* B, Group& G, GroupWork<T>& W) {
  SpreadGroup d{};
  SpreadArgs& a = d.a;
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
  a.q = nullptr;
  a.nrm = G.nrm;
  a.ds = G.ds;
  d.wtab = W.wtab;
  d.out = W.real;
  d.qoff = G.aoff;
  d.tx = G.geom.tile[0];
  return d;
}

int prec_index(int bytes) { return bytes == 4 ? 0 : 1; }

// Upload the group descriptors and the merged work queue for precision T (after every group's
// tiles are final).
template <typename T> void build_queue(ibdl_batch_s* B);

// Tile shape of a 2-D group by measurement: 16 x 16, 32 x 8 and 64 x 4 node tiles (at most 64 tiles
// along x), each binned and timed on the group's own spread and forward x pass (two warm-up and five
// timed runs); a shape other than 16 x 16 must be 3% faster.  Remembered per (grid, precision,
// problem count, markers per problem) with the launch shapes.
template <typename T> void tune_tiles(ibdl_batch_s* B, Group& G, GroupWork<T>& W) {
  if (G.tiles_tuned || B->dim != 2) return;
  G.tiles_tuned = true;
  const int np = (int)G.probs.size();
  const TuneKey key{3, B->dim, G.n[0], G.n[1], G.n[2], (int)sizeof(T), pow2_bucket(G.nib / std::max(np, 1)),
                    pow2_bucket(np)};
  LaunchShape got;
  auto use = [&](int tx) {
    G.geom.tile[0] = tx;
    G.geom.tile[1] = 256 / tx;
    bin_group(B, G);
  };
  if (tune_get(key, &got) && got.tile > 0) {
    if (got.tile != G.geom.tile[0]) use(got.tile);
    return;
  }
  const int gi = (int)(&G - &B->groups[0]);
  SpreadGroup* dsg = (SpreadGroup*)B->dalloc(sizeof(SpreadGroup));
  double* q = (double*)B->dalloc(sizeof(double) * G.nib);
  IBDL_HIP(hipMemsetAsync(q, 0, sizeof(double) * G.nib, B->st));
  hipEvent_t e0, e1;
  IBDL_HIP(hipEventCreate(&e0));
  IBDL_HIP(hipEventCreate(&e1));
  int best = 16;
  float best_ms = 1e30f;
  const int64_t rows = (int64_t)np * G.n[1];
  for (int tx : {16, 32, 64}) {
    if (G.n[0] / tx > 64 || G.n[0] < tx || G.n[1] < 256 / tx) continue;
    use(tx);
    const SpreadGroup d = spread_group<T>(B, G, W);
    IBDL_HIP(hipMemcpyAsync(dsg, &d, sizeof(SpreadGroup), hipMemcpyHostToDevice, B->st));
    std::vector<int2> it = queue_items(B, gi);
    for (int2& v : it) v.x = 0;
    int2* ditems = (int2*)B->dalloc(sizeof(int2) * std::max<size_t>(it.size(), 1));
    IBDL_HIP(hipMemcpyAsync(ditems, it.data(), sizeof(int2) * it.size(), hipMemcpyHostToDevice, B->st));
    RowList rl;
    rl.rpf = rows;
    rl.seg = G.seg_all;
    rl.seg_log2 = __builtin_ctz((unsigned)tx / 2);
    auto run = [&]() {
      spread2_queue<T>(dsg, ditems, (int)it.size(), q - G.aoff, B->spread_blocks, B->st);
      fft_x_r2c<T>(W.real, W.spec, G.n[0], rows, W.tab.tw[0], B->st, 0, rl, G.nxp);
    };
    for (int k = 0; k < 2; ++k) run();
    IBDL_HIP(hipEventRecord(e0, B->st));
    for (int k = 0; k < 5; ++k) run();
    IBDL_HIP(hipEventRecord(e1, B->st));
    IBDL_HIP(hipEventSynchronize(e1));
    float ms = 0;
    IBDL_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (tx == 16 ? ms < best_ms : ms < 0.97f * best_ms) {
      best_ms = ms;
      best = tx;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  use(best);
  LaunchShape put;
  put.tile = best;
  tune_put(key, put);
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
  tune_tiles<T>(B, G, W);
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

template <typename T> void build_queue(ibdl_batch_s* B) {
  ibdl_batch_s::Queue& Q = B->queue[prec_index(sizeof(T))];
  if (Q.ready) return;
  const int ng = (int)B->groups.size();
  std::vector<SpreadGroup> sg(ng);
  std::vector<InterpGroup> ig(ng);
  for (int gi = 0; gi < ng; ++gi) {
    Group& G = B->groups[gi];
    GroupWork<T>& W = G.work<T>();
    sg[gi] = spread_group<T>(B, G, W);
    InterpGroup& d = ig[gi];
    d.a = InterpArgs{};
    d.a.g = G.geom;
    d.a.kernel = B->kernel;
    d.a.nf = 1;
    d.a.n_ib = G.nib;
    d.a.s = G.s;
    d.a.f = G.f;
    d.a.wt = G.wt;
    d.a.a = 1.0;
    d.a.b = 0.5;
    d.a.pid = G.pid;
    d.wtab = W.wtab;
    d.u = W.real;
    d.m0 = G.aoff;
  }
  const std::vector<int2> it = queue_items(B, -1);
  Q.sg = (SpreadGroup*)B->dalloc(sizeof(SpreadGroup) * ng);
  Q.ig = (InterpGroup*)B->dalloc(sizeof(InterpGroup) * ng);
  Q.items = (int2*)B->dalloc(sizeof(int2) * std::max<size_t>(it.size(), 1));
  Q.nitems = (int)it.size();
  IBDL_HIP(hipMemcpyAsync(Q.sg, sg.data(), sizeof(SpreadGroup) * ng, hipMemcpyHostToDevice, B->st));
  IBDL_HIP(hipMemcpyAsync(Q.ig, ig.data(), sizeof(InterpGroup) * ng, hipMemcpyHostToDevice, B->st));
  IBDL_HIP(hipMemcpyAsync(Q.items, it.data(), sizeof(int2) * it.size(), hipMemcpyHostToDevice, B->st));
  IBDL_HIP(hipStreamSynchronize(B->st));
  Q.ready = true;
  // Workgroups of the persistent spread by measurement: 2, 4 or 8 per compute unit, or one per tile
  // (two warm-up and five timed runs each; a persistent shape must be 3% faster than one per tile).
  const TuneKey key{4, B->dim, ng, pow2_bucket(Q.nitems), (int)sizeof(T), pow2_bucket(B->N), 0, 0};
  LaunchShape got;
  if (tune_get(key, &got)) {
    Q.blocks = got.blocks;
    return;
  }
  int dev = 0, ncu = 0;
  IBDL_HIP(hipGetDevice(&dev));
  IBDL_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  double* q = (double*)B->dalloc(sizeof(double) * B->N);
  IBDL_HIP(hipMemsetAsync(q, 0, sizeof(double) * B->N, B->st));
  hipEvent_t e0, e1;
  IBDL_HIP(hipEventCreate(&e0));
  IBDL_HIP(hipEventCreate(&e1));
  int best = 0;
  float best_ms = 1e30f;
  for (int nb : {0, 8 * ncu, 4 * ncu, 2 * ncu}) {
    if (nb >= Q.nitems) continue;
    for (int k = 0; k < 2; ++k) spread2_queue<T>(Q.sg, Q.items, Q.nitems, q, nb, B->st);
    IBDL_HIP(hipEventRecord(e0, B->st));
    for (int k = 0; k < 5; ++k) spread2_queue<T>(Q.sg, Q.items, Q.nitems, q, nb, B->st);
    IBDL_HIP(hipEventRecord(e1, B->st));
    IBDL_HIP(hipEventSynchronize(e1));
    float ms = 0;
    IBDL_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (nb == 0 ? ms < best_ms : ms < 0.97f * best_ms) {
      best_ms = ms;
      best = nb;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  Q.blocks = best;
  LaunchShape put;
  put.blocks = best;
  tune_put(key, put);
}

// y = A x for every problem of the batch (Dirichlet: y = S* u[x] + x/2).  2-D: the spread of every
// group in one persistent launch over the merged tile queue, the FFT passes per group, and the
// interpolation of every group in one launch.
template <typename T> void batch_apply(ibdl_batch_s* B, const double* x, double* y) {
  if (queue_path(B)) {
    for (Group& G : B->groups) group_work<T>(B, G);
    build_queue<T>(B);
    ibdl_batch_s::Queue& Q = B->queue[prec_index(sizeof(T))];
    spread2_queue<T>(Q.sg, Q.items, Q.nitems, x, Q.blocks, B->st);
    for (Group& G : B->groups) group_pipeline<T>(B, G, G.work<T>(), G.work<T>().tune);
    interp4_groups<T>(Q.ig, (int)B->groups.size(), B->N, x, y, B->st);
    return;
  }
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
  if (B->gmx < maxit) {
    B->gstride = (int64_t)((kr_gmres_state_doubles(maxit) + 31) / 32 * 32);
    B->gsb = (double*)B->dalloc(sizeof(double) * B->gstride * B->nprob);
    B->gmx = maxit;
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

// The publication slot of the device-driven batch GMRES: wait for its tag (poll 2 ms, then a stream
// synchronisation, after which it must be there).
const volatile double* batch_wait(ibdl_batch_s* B, int slot, unsigned seq) {
  const size_t slot_doubles = (size_t)B->nprob * GM_PUB;
  volatile unsigned* tag = reinterpret_cast<volatile unsigned*>(B->hmap + 2 * slot_doubles) + 16 * slot;
  const auto t0 = std::chrono::steady_clock::now();
  while (*tag != seq) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
      IBDL_HIP(hipStreamSynchronize(B->st));
      if (*tag != seq) throw Error(IBDL_ERR_HIP, "GMRES state did not reach the host");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return B->hmap + slot * slot_doubles;
}

// GMRES per problem (x0 = 0, no restart, CGS2), all problems in lock step and all on the device:
// one launch per step does every problem's Gram-Schmidt passes, least-squares update (Givens
// rotations in double) and normalisation, with a per-problem convergence flag that freezes a
// converged problem.  The host only watches the published residuals: it queues step j + 1 before
// it waits for step j, and stops when every problem has converged.
void batch_gmres(ibdl_batch_s* B, double tol, int maxit, double* x, std::vector<int>& iters,
                 std::vector<double>& relres, std::vector<int>& status, ibdl_info_t* infos) {
  const int np = B->nprob, ld = B->ld;
  const int64_t n = B->N;
  const int mx = B->gmx;
  double* Yd = B->dsmall + np * (2 * ld + 2);
  kb_multidot(B->vb, n, 1, B->vb, B->sg, B->partial, 1, B->bn2, B->st);
  double* xin = B->use_graph ? (ensure_graph(B), B->xin) : nullptr;
  kb_gmres_start(B->vb, B->doff, B->dlen, np, B->bn2, B->V, xin, B->st);
  const size_t slot_doubles = (size_t)np * GM_PUB;
  unsigned* tag_dev = reinterpret_cast<unsigned*>(B->hmap_dev + 2 * slot_doubles);
  unsigned seq[2] = {0, 0};
  auto step = [&](int j) {
    if (B->use_graph) IBDL_HIP(hipGraphLaunch(B->gexec, B->st));
    else apply_any(B, B->V + (int64_t)j * n, B->yout, false);
    kb_arnoldi(B->V, n, j, B->yout, B->doff, B->dlen, np, B->maxlen, B->bn2, B->gsb, B->gstride, mx, tol,
               B->V + (int64_t)(j + 1) * n, xin, B->st);
    const int slot = j & 1;
    seq[slot] = ++B->seq;
    kb_publish(B->gsb, B->gstride, np, B->hmap_dev + slot * slot_doubles, tag_dev + 16 * slot, seq[slot], B->st);
  };
  iters.assign(np, 0);
  relres.assign(np, 0.0);
  status.assign(np, IBDL_OK);
  std::vector<std::vector<double>> rs(np, std::vector<double>(maxit, 1.0));
  std::vector<char> done(np, 0);
  step(0);
  for (int j = 0; j < maxit; ++j) {
    // queue step j + 1 ahead unless every unfinished problem is predicted to converge at step j
    bool ahead = false;
    for (int p = 0; p < np && !ahead; ++p) {
      if (done[p]) continue;
      ahead = j < 2 || rs[p][j - 1] * (rs[p][j - 1] / rs[p][j - 2]) > tol;
    }
    ahead = ahead && j + 1 < maxit;
    if (ahead) step(j + 1);
    const volatile double* hv = batch_wait(B, j & 1, seq[j & 1]);
    bool all = true;
    for (int p = 0; p < np; ++p) {
      const volatile double* v = hv + (size_t)p * GM_PUB;
      if (j == 0 && !std::isfinite((double)v[GM_BETA])) throw Error(IBDL_ERR_NONFINITE, "right-hand side is not finite");
      if (!std::isfinite((double)v[GM_HN]) || !std::isfinite((double)v[GM_RES]))
        throw Error(IBDL_ERR_NONFINITE, "non-finite value in the Arnoldi process");
      if (!done[p]) {
        relres[p] = v[GM_RES];
        iters[p] = (int)v[GM_K];
        rs[p][j] = relres[p];
        if (infos && infos[p].history && j < infos[p].history_cap && v[GM_BETA] > 0) infos[p].history[j] = relres[p];
        done[p] = v[GM_DONE] != 0.0;
      }
      all = all && done[p];
    }
    if (all) break;
    if (!ahead && j + 1 < maxit) step(j + 1);
  }
  int kmax = 0;
  for (int p = 0; p < np; ++p) {
    kmax = std::max(kmax, iters[p]);
    status[p] = relres[p] > tol ? IBDL_NOT_CONVERGED : IBDL_OK;
  }
  kb_gmres_y(B->gsb, B->gstride, np, mx, std::max(kmax, 1), Yd, ld, B->st);
  kb_lincomb(B->V, n, std::max(kmax, 1), Yd, ld, B->sg, x, B->st);
}

template <typename T> void batch_recover(ibdl_batch_s* B, const double* q, void* const* u) {
  if (queue_path(B)) {
    for (Group& G : B->groups) group_work<T>(B, G);
    build_queue<T>(B);
    ibdl_batch_s::Queue& Q = B->queue[prec_index(sizeof(T))];
    spread2_queue<T>(Q.sg, Q.items, Q.nitems, q, Q.blocks, B->st);
  }
  for (Group& G : B->groups) {
    GroupWork<T>& W = group_work<T>(B, G);
    if (queue_path(B)) group_pipeline<T>(B, G, W, W.tune);
    else group_density_to_grid<T>(B, G, W, q + G.aoff);
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
    {   // the persistent spread: four workgroups per compute unit
      int dev = 0, ncu = 0;
      IBDL_HIP(hipGetDevice(&dev));
      IBDL_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      B->spread_blocks = 4 * std::max(ncu, 1);
    }
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
      G.nxp = (G.nxh + 15) / 16 * 16;
      G.nspec = G.nxp * G.n[1] * G.n[2];
      const int64_t ntile = (int64_t)g.ntile[0] * g.ntile[1] * g.ntile[2] * np;
      const int64_t maxlist = G.nib * (dim == 2 ? 6 : 12);   // tiles a 6-node window meets (2-D: 4-row tiles)
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
      G.seg_all = (unsigned long long*)B->dalloc(sizeof(unsigned long long) * np * G.n[1] * G.n[2]);
      bin_group(B.get(), G);
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
    {   // per-problem segments of the batch vectors for the device-driven GMRES
      std::vector<int64_t> hoff(nprob), hlen(nprob);
      for (int p = 0; p < nprob; ++p) {
        hoff[p] = B->aoff[p];
        hlen[p] = n_ib[p];
        B->maxlen = std::max<int64_t>(B->maxlen, n_ib[p]);
      }
      B->doff = (int64_t*)B->dalloc(sizeof(int64_t) * nprob);
      B->dlen = (int64_t*)B->dalloc(sizeof(int64_t) * nprob);
      B->bn2 = (double*)B->dalloc(sizeof(double) * nprob);
      IBDL_HIP(hipMemcpy(B->doff, hoff.data(), sizeof(int64_t) * nprob, hipMemcpyHostToDevice));
      IBDL_HIP(hipMemcpy(B->dlen, hlen.data(), sizeof(int64_t) * nprob, hipMemcpyHostToDevice));
      IBDL_HIP(hipHostMalloc((void**)&B->hptr, sizeof(double*) * 2 * nprob, hipHostMallocDefault));
      B->dptr = (const double**)B->dalloc(sizeof(double*) * 2 * nprob);
      const size_t slot_doubles = (size_t)nprob * GM_PUB;
      IBDL_HIP(hipHostMalloc((void**)&B->hmap, sizeof(double) * (2 * slot_doubles + 32),
                             hipHostMallocMapped | hipHostMallocCoherent));
      IBDL_HIP(hipHostGetDevicePointer((void**)&B->hmap_dev, B->hmap, 0));
      unsigned* tags = reinterpret_cast<unsigned*>(B->hmap + 2 * slot_doubles);
      tags[0] = 0;
      tags[16] = 0;
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
    // the pointer tables of data and q: one staged copy, then one gather launch (the pinned staging
    // is rewritten only after the synchronisation at the end of the previous call)
    const int np = b->nprob;
    for (int p = 0; p < np; ++p) {
      b->hptr[p] = data[p];
      b->hptr[np + p] = q[p];
    }
    IBDL_HIP(hipMemcpyAsync(b->dptr, b->hptr, sizeof(double*) * 2 * np, hipMemcpyHostToDevice, b->st));
    kb_seg_copy(b->dptr, b->doff, b->dlen, np, b->maxlen, b->vb, true, b->st);
    std::vector<int> iters, status;
    std::vector<double> relres;
    batch_gmres(b, tol, maxit, b->xsol, iters, relres, status, infos);
    // true residuals with a double-precision apply; both norms reach the host with one copy
    apply_any(b, b->xsol, b->vr, true);
    kr_axpby(b->vr, 1.0, b->vb, -1.0, b->N, b->st);
    double* nd = b->dsmall + np * (2 * b->ld);   // the two per-problem norm arrays (hn, sc slots)
    kb_multidot(b->vr, b->N, 1, b->vr, b->sg, b->partial, 1, nd, b->st);
    kb_multidot(b->vb, b->N, 1, b->vb, b->sg, b->partial, 1, nd + np, b->st);
    IBDL_HIP(hipMemcpyAsync(b->hsmall, nd, sizeof(double) * 2 * np, hipMemcpyDeviceToHost, b->st));
    kb_seg_copy(b->dptr + np, b->doff, b->dlen, np, b->maxlen, b->xsol, false, b->st);
    if (u) {
      if (b->mixed()) batch_recover<float>(b, b->xsol, u);
      else batch_recover<double>(b, b->xsol, u);
    }
    IBDL_HIP(hipStreamSynchronize(b->st));
    std::vector<double> rn(np), bn(np);
    for (int p = 0; p < np; ++p) {
      rn[p] = sqrt(std::max(b->hsmall[p], 0.0));
      bn[p] = sqrt(std::max(b->hsmall[np + p], 0.0));
    }
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
                               int32_t* n, int32_t* rows_per_block, int32_t* lines_per_block, int32_t* tile_x) {
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
    if (tile_x) *tile_x = G.geom.tile[0];
    return IBDL_OK;
  });
}

const char* ibdl_batch_last_error(ibdl_batch_t b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

}  // extern "C"
