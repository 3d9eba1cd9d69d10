// Autotuner of the KRP sketch tilings (KRP_FLAG_AUTOTUNE).
//
// On the first use of a sketch shape -- (tensor dims, sketched mode, ell,
// arithmetic, storage type, 16-byte alignment of the input) -- the candidate
// tilings (row tiles per wave, waves along the rows, target workgroup count)
// are timed with HIP events on the caller's stream and the fastest is kept.
// Results live in a process-wide table and in a JSON file, one entry per line:
//   {"version": 1, "arch": "gfx950", "entries": {
//   "<key>": {"mt": 4, "wm": 8, "wo": 1, "target_wgs": 256, "us": 123.4},
//   ...
//   }}
// The file is $KRP_TUNE_CACHE, else $HOME/.cache/libkrp/sketch_tiles.json.
// Only tilings whose partial-sum buffer fits the default plan's are
// considered, so workspace sizes queried without the flag remain valid.
// Tuning never runs while the stream is being captured into a graph.
#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

namespace krp {

namespace {

struct Entry {
  SketchTile tile;
  double us = 0.0;
};

std::mutex g_tune_mu;
std::map<std::string, Entry> g_table;
bool g_loaded = false;

std::string cache_path() {
  const char* p = std::getenv("KRP_TUNE_CACHE");
  if (p && *p) return p;
  const char* h = std::getenv("HOME");
  if (!h || !*h) return "";
  return std::string(h) + "/.cache/libkrp/sketch_tiles.json";
}

void make_parent_dirs(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') mkdir(path.substr(0, i).c_str(), 0755);
}

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const std::string path = cache_path();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    const char* q0 = std::strchr(line, '"');
    if (!q0) continue;
    const char* q1 = std::strchr(q0 + 1, '"');
    if (!q1) continue;
    const std::string key(q0 + 1, q1);
    Entry e;
    if (std::sscanf(q1 + 1, " : {\"mt\": %d, \"wm\": %d, \"wo\": %d, \"target_wgs\": %d, \"us\": %lf}",
                    &e.tile.mt, &e.tile.wm, &e.tile.wo, &e.tile.target_wgs, &e.us) == 5)
      g_table[key] = e;
  }
  std::fclose(f);
}

void save_locked() {
  const std::string path = cache_path();
  if (path.empty()) return;
  make_parent_dirs(path);
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\"version\": 1, \"arch\": \"gfx950\", \"entries\": {\n");
  size_t i = 0;
  for (const auto& kv : g_table) {
    const Entry& e = kv.second;
    std::fprintf(f, "\"%s\": {\"mt\": %d, \"wm\": %d, \"wo\": %d, \"target_wgs\": %d, \"us\": %.3f}%s\n",
                 kv.first.c_str(), e.tile.mt, e.tile.wm, e.tile.wo, e.tile.target_wgs, e.us,
                 ++i < g_table.size() ? "," : "");
  }
  std::fprintf(f, "}}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path.c_str());
}

std::string tune_key(const SketchProblem& pb) {
  std::string k = "d=" + std::to_string(pb.d) + " dims=";
  for (int i = 0; i < pb.d; ++i) k += (i ? "x" : "") + std::to_string(pb.dims[i]);
  k += " mode=" + std::to_string(pb.mode) + " ell=" + std::to_string(pb.ell) +
       " prec=" + std::to_string(pb.prec) + " xd=" + std::to_string(pb.x_is_double) +
       " al=" + std::to_string((reinterpret_cast<uintptr_t>(pb.x) & 15) == 0 ? 1 : 0);
  return k;
}

bool same_geometry(const SketchPlan& a, const SketchPlan& b) {
  return a.mt == b.mt && a.wm == b.wm && a.wo == b.wo && a.o_per_wg == b.o_per_wg &&
         a.row_blocks == b.row_blocks && a.f_blocks == b.f_blocks;
}

}  // namespace

SketchTile tuned_tile(const SketchProblem& pb, hipStream_t st) {
  const SketchTile def{};
  if (!pb.x) return def;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return def;
  const std::string key = tune_key(pb);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_locked();
    auto it = g_table.find(key);
    if (it != g_table.end()) return it->second.tile;
  }
  // candidate tilings with distinct geometry, partial sums within the default's
  const SketchPlan base = plan_sketch(pb, def);
  std::vector<std::pair<SketchTile, SketchPlan>> cands;
  cands.emplace_back(def, base);
  for (int mt : {1, 2, 4})
    for (int wm : {0, 2, 4, 8})
      for (int tw : {256, 512, 1024}) {
        SketchTile t;
        t.mt = mt;
        t.wm = wm;
        t.target_wgs = tw;
        const SketchPlan p = plan_sketch(pb, t);
        if (p.partial_bytes > base.partial_bytes) continue;
        bool dup = false;
        for (const auto& c : cands) dup = dup || same_geometry(c.second, p);
        if (!dup) cands.emplace_back(t, p);
      }
  size_t part_max = 0;
  for (const auto& c : cands) part_max = std::max(part_max, c.second.partial_bytes);
  void* part = nullptr;
  double* y64 = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SketchTile best = def;
  double best_us = -1.0;
  bool ok = hipMalloc(&part, std::max<size_t>(part_max, 256)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&y64), (size_t)base.n_rows * pb.ell * sizeof(double)) ==
                hipSuccess &&
            hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  for (size_t i = 0; ok && i < cands.size(); ++i) {
    const SketchPlan& p = cands[i].second;
    ok = launch_sketch(pb, p, part, y64, nullptr, 0, st) == hipSuccess;  // warm-up
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    for (int r = 0; ok && r < 3; ++r) ok = launch_sketch(pb, p, part, y64, nullptr, 0, st) == hipSuccess;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (ok) {
      const double us = ms * 1000.0 / 3.0;
      if (best_us < 0.0 || us < best_us) {
        best_us = us;
        best = cands[i].first;
      }
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (part) hipFree(part);
  if (y64) hipFree(y64);
  (void)hipGetLastError();  // a failed candidate must not leak into the caller's error state
  if (!ok || best_us < 0.0) return def;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_table[key] = Entry{best, best_us};
  save_locked();
  return best;
}

}  // namespace krp
