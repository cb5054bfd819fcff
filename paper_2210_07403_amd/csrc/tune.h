// Launch shapes and radix plans of the FFT passes and tile widths of the batched 2-D spread, chosen by timing;
// remembered for the life of the process and in a JSON file per kind of GPU (tune.hip).
#pragma once

#include <array>

namespace ibdl {

struct LaunchShape {
  int rpb = 0;   // rows per block of the x passes (0: the largest that fits)
  int wy = 0;    // lines per block of the strided y passes
  int wz = 0;    // lines per block of the fused last-axis pass
  int tile = 0;  // 2-D spread tile width along x (batches; 0: not chosen)
  int blocks = 0;  // workgroups of the batched persistent spread (0: not chosen)
  int py = 0;    // radix plan of the strided y passes (fft_line_plans)
  int pz = 0;    // radix plan of the single-field last-axis pass
};

// (kind, dim, n0, n1, n2, bytes per value, fields, size bucket)
using TuneKey = std::array<int, 8>;

bool tune_get(const TuneKey& key, LaunchShape* out);
void tune_put(const TuneKey& key, const LaunchShape& shape);

inline int pow2_bucket(long long v) {
  int b = 1;
  while (b < v && b < (1 << 30)) b *= 2;
  return b;
}

}  // namespace ibdl
