// Periodic grid solve that allocates nothing: the half spectra and the per-axis FFT tables live in a
// file-scope device array instead of a handle's workspaces.  Same passes as ibdl_grid_solve (x
// R2C, y C2C in 3-D, the fused last-axis pass with the multiplier, and back), every row dense.
#include <math.h>

#include <mutex>
#include <string>

#include "../../include/ibdl.h"
#include "kernels.h"

namespace ibdl {
void set_global_error(const std::string& msg);   // ibdl_last_error(NULL) reports it
}

using namespace ibdl;

constexpr size_t kScratchBytes = (size_t)32 << 20;

// The scratch array, one copy per GPU, held until the process ends.  Host code never passes its
// name to a kernel or a copy: in host code the name is a stand-in, not a device address, so every
// use goes through the address looked up below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// The device address of this device's scratch, looked up once per device with it current.
void* scratch_ptr() {
  int dev = 0;
  IBDL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(IBDL_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    IBDL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(IBDL_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Per-axis tables (as the handle's, but formed on the device): twiddles exp(-2 pi i m / n); FD
// symbols sigma = (2 cos(2 pi j / n) - 2) / h^2 = -4 sin^2(pi j / n) / h^2, k~ = sin(2 pi j / n) / h; spectral sigma = -k^2,
// k~ = k (0 at the Nyquist index), k = 2 pi m / L with m the signed index.  Angles through
// sincospi in double, rounded once to T.
template <typename T>
__global__ void k_tables(int n, int len, int fd, double h, double L, cplx<T>* tw, T* sig, T* kt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double s, c;
    sincospi(2.0 * (double)i / (double)n, &s, &c);
    tw[i] = mk<cplx<T>>((T)c, (T)(-s));
  }
  if (i < len) {
    if (fd) {
      // 2 cos(t) - 2 = -4 sin^2(t / 2), free of the cancellation at the low modes
      double s, c, s2, c2;
      sincospi(2.0 * (double)i / (double)n, &s, &c);
      sincospi((double)i / (double)n, &s2, &c2);
      sig[i] = (T)(-4.0 * s2 * s2 / (h * h));
      kt[i] = (T)(s / h);
    } else {
      const int m = i < n / 2 ? i : i - n;
      const double k = 2.0 * M_PI * (double)m / L;
      sig[i] = (T)(-k * k);
      kt[i] = i == n / 2 ? (T)0 : (T)k;
    }
  }
}

struct Layout {
  size_t tw[3], sig[3], kt[3], spec, total;
};

template <typename T> Layout layout(int dim, const int* n, int nf, int64_t nspec) {
  Layout lo{};
  size_t off = 0;
  for (int d = 0; d < 3; ++d) {
    if (d >= dim) {
      lo.tw[d] = lo.sig[d] = lo.kt[d] = 0;
      continue;
    }
    const int len = d == 0 ? n[d] / 2 + 1 : n[d];
    lo.tw[d] = off;
    off += align256(sizeof(cplx<T>) * (size_t)n[d]);
    lo.sig[d] = off;
    off += align256(sizeof(T) * (size_t)len);
    lo.kt[d] = off;
    off += align256(sizeof(T) * (size_t)len);
  }
  lo.spec = off;
  off += align256(sizeof(cplx<T>) * (size_t)nspec * (size_t)nf);
  lo.total = off;
  return lo;
}

template <typename T> void solve_t(const ibdl_config_t& c, const T* rhs, T* u) {
  const int dim = c.dim;
  int n[3] = {1, 1, 1};
  for (int d = 0; d < dim; ++d) n[d] = (int)c.n[d];
  const int64_t ntot = (int64_t)n[0] * n[1] * n[2];
  const int nxh = n[0] / 2 + 1, nxp = (nxh + 15) / 16 * 16;
  const int64_t nspec = (int64_t)nxp * n[1] * n[2];
  const bool stokes = c.pde == IBDL_PDE_STOKES;
  const int nf = stokes ? 2 : 1;
  const Layout lo = layout<T>(dim, n, nf, nspec);
  if (lo.total > kScratchBytes)
    throw Error(IBDL_ERR_UNSUPPORTED, "grid needs " + std::to_string(lo.total) + " bytes of static scratch; the limit is " +
                                          std::to_string(kScratchBytes));
  unsigned char* base = (unsigned char*)scratch_ptr();
  hipStream_t st = (hipStream_t)c.stream;
  const double h = c.L[0] / (double)n[0];
  cplx<T>* tw[3] = {nullptr, nullptr, nullptr};
  T* sig[3] = {nullptr, nullptr, nullptr};
  T* kt[3] = {nullptr, nullptr, nullptr};
  for (int d = 0; d < dim; ++d) {
    tw[d] = (cplx<T>*)(base + lo.tw[d]);
    sig[d] = (T*)(base + lo.sig[d]);
    kt[d] = (T*)(base + lo.kt[d]);
    const int len = d == 0 ? n[d] / 2 + 1 : n[d];
    hipLaunchKernelGGL(k_tables<T>, dim3((unsigned)((n[d] + 255) / 256)), dim3(256), 0, st, n[d], len,
                       c.disc == IBDL_DISC_FD2 ? 1 : 0, h, c.L[d], tw[d], sig[d], kt[d]);
    IBDL_LAUNCH_CHECK();
  }
  cplx<T>* spec = (cplx<T>*)(base + lo.spec);
  MultDesc md{};
  md.dim = dim;
  md.nxh = nxh;
  md.nxp = nxp;
  md.sc = 1.0 / (double)ntot;
  md.mu = c.mu;
  for (int d = 0; d < 3; ++d) {
    md.sig[d] = d < dim ? sig[d] : sig[0];
    md.kt[d] = d < dim ? kt[d] : kt[0];
  }
  const double kap = c.pde == IBDL_PDE_POISSON ? 0.0 : c.kappa;
  if (stokes) {
    md.stokes = 1;
    md.c2 = c.mu;
    md.c0 = kap * kap;
    md.nc = 2;
    md.fk[0] = FK_G1;
    md.fk[1] = FK_G2;
    md.alpha = -1.0;
  } else {
    md.stokes = 0;
    md.c2 = 1.0;
    md.c0 = kap * kap;
    md.nc = 1;
    md.fk[0] = FK_MASS;
    md.alpha = 1.0;
  }
  const int64_t rpf = ntot / n[0];
  RowList rl;
  rl.rpf = rpf;
  fft_x_r2c<T>(rhs, spec, n[0], rpf * nf, tw[0], st, 0, rl, nxp);
  if (dim == 3)
    fft_strided<T>(spec, n[1], (int64_t)nf * n[2] * nxp, nxp, (int64_t)nxp * n[1], nxp, false, tw[1], st, 0, RowMask(),
                   nxh);
  const int last = dim - 1;
  fft_fused_last<T>(spec, n[last], nspec / n[last], nf, md, tw[last], st, 1, 0, 0, RowMask());
  if (dim == 3)
    fft_strided<T>(spec, n[1], (int64_t)nf * n[2] * nxp, nxp, (int64_t)nxp * n[1], nxp, true, tw[1], st, 0, RowMask(),
                   nxh);
  fft_x_c2r<T>(spec, u, n[0], rpf * nf, tw[0], st, 0, rl, nxp);
}

bool pow2_ok(int64_t v) { return v >= 16 && v <= 1024 && (v & (v - 1)) == 0; }

void check(const ibdl_config_t* c) {
  if (!c) throw Error(IBDL_ERR_ARG, "cfg is NULL");
  if (c->dim != 2 && c->dim != 3) throw Error(IBDL_ERR_ARG, "dim must be 2 or 3");
  double h0 = 0.0;
  for (int d = 0; d < c->dim; ++d) {
    if (!pow2_ok(c->n[d])) throw Error(IBDL_ERR_UNSUPPORTED, "grid size must be a power of two in [16, 1024]");
    if (!(c->L[d] > 0) || !std::isfinite(c->L[d])) throw Error(IBDL_ERR_ARG, "box lengths must be positive and finite");
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
  if (c->disc != IBDL_DISC_FD2 && c->disc != IBDL_DISC_SPECTRAL) throw Error(IBDL_ERR_ARG, "unknown disc");
  if (c->precision != IBDL_FP64 && c->precision != IBDL_MIXED) throw Error(IBDL_ERR_ARG, "unknown precision");
}

}  // namespace

extern "C" ibdl_status_t ibdl_grid_solve_static(const ibdl_config_t* cfg, const void* rhs, void* u) {
  try {
    check(cfg);
    if (!rhs || !u) throw Error(IBDL_ERR_ARG, "NULL pointer");
    if (cfg->precision == IBDL_MIXED) solve_t<float>(*cfg, (const float*)rhs, (float*)u);
    else solve_t<double>(*cfg, (const double*)rhs, (double*)u);
    return IBDL_OK;
  } catch (const Error& e) {
    set_global_error(e.what());
    return (ibdl_status_t)e.code;
  } catch (const std::exception& e) {
    set_global_error(e.what());
    return IBDL_ERR_HIP;
  }
}
