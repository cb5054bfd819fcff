// Per-grid constant tables shared by the single-problem and batched runtimes: FFT twiddles and
// the Fourier symbols of the Laplacian (sigma) and of the first derivative (k~) along each axis.
#pragma once

#include <math.h>

#include <vector>

#include "common.h"

namespace ibdl {

template <typename T> struct GridTables {
  cplx<T>* tw[3] = {nullptr, nullptr, nullptr};
  T* sig[3] = {nullptr, nullptr, nullptr};   // axis 0: nx/2 + 1 entries, others n entries
  T* kt[3] = {nullptr, nullptr, nullptr};
};

// FD symbols: sigma = (2 cos(2 pi j / n) - 2) / h^2, k~ = sin(2 pi j / n) / h (centred difference).
// Spectral: sigma = -k^2 and k~ = k with k = 2 pi m / L (m the signed mode index), k~ = 0 at the
// Nyquist index.  Computed in long double and rounded once to T.  dalloc(bytes) returns device
// memory owned by the caller.
template <typename T, typename Alloc>
GridTables<T> make_grid_tables(int dim, const int* n, const double* L, double h, bool fd, Alloc&& dalloc) {
  GridTables<T> G;
  const long double PI = 3.14159265358979323846264338327950288L;
  for (int d = 0; d < dim; ++d) {
    const int nd = n[d];
    std::vector<cplx<T>> tw(nd);
    for (int m = 0; m < nd; ++m) {
      const long double a = 2.0L * PI * (long double)m / (long double)nd;
      tw[m].x = (T)cosl(a);
      tw[m].y = (T)(-sinl(a));
    }
    G.tw[d] = (cplx<T>*)dalloc(sizeof(cplx<T>) * nd);
    IBDL_HIP(hipMemcpy(G.tw[d], tw.data(), sizeof(cplx<T>) * nd, hipMemcpyHostToDevice));
    const int len = (d == 0) ? nd / 2 + 1 : nd;
    std::vector<T> sg(len), kt(len);
    for (int j = 0; j < len; ++j) {
      const long double th = 2.0L * PI * (long double)j / (long double)nd;
      if (fd) {
        sg[j] = (T)((2.0L * cosl(th) - 2.0L) / ((long double)h * h));
        kt[j] = (T)(sinl(th) / (long double)h);
      } else {
        const int m = (j < nd / 2) ? j : j - nd;
        const long double k = 2.0L * PI * (long double)m / (long double)L[d];
        sg[j] = (T)(-k * k);
        kt[j] = (j == nd / 2) ? (T)0 : (T)k;
      }
    }
    G.sig[d] = (T*)dalloc(sizeof(T) * len);
    G.kt[d] = (T*)dalloc(sizeof(T) * len);
    IBDL_HIP(hipMemcpy(G.sig[d], sg.data(), sizeof(T) * len, hipMemcpyHostToDevice));
    IBDL_HIP(hipMemcpy(G.kt[d], kt.data(), sizeof(T) * len, hipMemcpyHostToDevice));
  }
  return G;
}

}  // namespace ibdl
