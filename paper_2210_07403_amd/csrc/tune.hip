// Registry of measured launch shapes and tile widths (see tune.h), kept in memory and persisted to a
// JSON file so that later processes on the same kind of GPU skip the measurements.
//
// File: $IBDL_TUNE_CACHE if set (an empty value turns the file off), else
// $XDG_CACHE_HOME/ibdl/tune.json or $HOME/.cache/ibdl/tune.json.  Layout, one entry per line:
//   {"format": "ibdl-tune-3", "device": "<arch> <CUs>",
//    "entries": [
//     {"key": [k0, ..., k7], "rpb": r, "wy": y, "wz": z, "tile": t, "blocks": b, "py": p, "pz": q},
//     ...
//    ]}
// A file written for another device, or one that does not parse, is ignored (and replaced at the next
// measurement).  Failures to read or write the file are not errors: the cache only saves time.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <filesystem>
#include <map>
#include <mutex>
#include <string>

#include "tune.h"

namespace ibdl {
namespace {

std::mutex g_mu;
std::map<TuneKey, LaunchShape> g_reg;
bool g_loaded = false;

std::string cache_path() {
  const char* e = getenv("IBDL_TUNE_CACHE");
  if (e) return std::string(e);
  const char* x = getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/ibdl/tune.json";
  const char* h = getenv("HOME");
  if (h && *h) return std::string(h) + "/.cache/ibdl/tune.json";
  return std::string();
}

std::string device_id() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  char buf[320];
  snprintf(buf, sizeof(buf), "%s %d", p.gcnArchName, p.multiProcessorCount);
  for (char* c = buf; *c; ++c)
    if (*c == '"' || *c == '\\') *c = '_';
  return std::string(buf);
}

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const std::string path = cache_path();
  if (path.empty()) return;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return;
  const std::string want = "\"device\": \"" + device_id() + "\"";
  char line[1024];
  bool device_ok = false;
  std::map<TuneKey, LaunchShape> got;
  while (fgets(line, sizeof(line), f)) {
    if (strstr(line, "\"format\": \"ibdl-tune-3\"")) {
      device_ok = strstr(line, want.c_str()) != nullptr;
      continue;
    }
    if (!device_ok) break;
    TuneKey k{};
    LaunchShape v;
    const int n = sscanf(line,
                         " {\"key\": [%d, %d, %d, %d, %d, %d, %d, %d], \"rpb\": %d, \"wy\": %d, \"wz\": %d, \"tile\": %d, "
                         "\"blocks\": %d, \"py\": %d, \"pz\": %d}",
                         &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6], &k[7], &v.rpb, &v.wy, &v.wz, &v.tile, &v.blocks,
                         &v.py, &v.pz);
    if (n == 15) got[k] = v;
  }
  fclose(f);
  if (device_ok)
    for (auto& kv : got) g_reg.insert(kv);
}

void save_locked() {
  const std::string path = cache_path();
  if (path.empty()) return;
  std::error_code ec;
  std::filesystem::create_directories(std::filesystem::path(path).parent_path(), ec);
  const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\"format\": \"ibdl-tune-3\", \"device\": \"%s\",\n \"entries\": [\n", device_id().c_str());
  size_t i = 0;
  for (const auto& kv : g_reg) {
    const TuneKey& k = kv.first;
    const LaunchShape& v = kv.second;
    fprintf(f,
            "  {\"key\": [%d, %d, %d, %d, %d, %d, %d, %d], \"rpb\": %d, \"wy\": %d, \"wz\": %d, \"tile\": %d, "
            "\"blocks\": %d, \"py\": %d, \"pz\": %d}%s\n",
            k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7], v.rpb, v.wy, v.wz, v.tile, v.blocks, v.py, v.pz,
            ++i < g_reg.size() ? "," : "");
  }
  fprintf(f, " ]}\n");
  const bool ok = fclose(f) == 0;
  if (ok) std::filesystem::rename(tmp, path, ec);
  if (!ok || ec) std::filesystem::remove(tmp, ec);
}

}  // namespace

bool tune_get(const TuneKey& key, LaunchShape* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  auto it = g_reg.find(key);
  if (it == g_reg.end()) return false;
  *out = it->second;
  return true;
}

void tune_put(const TuneKey& key, const LaunchShape& shape) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  g_reg[key] = shape;
  save_locked();
}

}  // namespace ibdl
