// Process-wide registry of measured launch shapes (see tune.h).
#include <map>
#include <mutex>

#include "tune.h"

namespace ibdl {
namespace {
std::mutex g_mu;
std::map<TuneKey, LaunchShape> g_reg;
}  // namespace

bool tune_get(const TuneKey& key, LaunchShape* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_reg.find(key);
  if (it == g_reg.end()) return false;
  *out = it->second;
  return true;
}

void tune_put(const TuneKey& key, const LaunchShape& shape) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_reg[key] = shape;
}

}  // namespace ibdl
