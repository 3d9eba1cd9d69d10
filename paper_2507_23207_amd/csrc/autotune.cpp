// Autotuner of the KRP sketch and TTM tilings (KRP_FLAG_AUTOTUNE).
//
// On the first use of a sketch shape -- (tensor dims, sketched mode, ell,
// arithmetic, storage type, 16-byte alignment of the input) -- the candidate
// tilings (row tiles per wave, waves along the rows, target workgroup count)
// are timed with HIP events on the caller's stream (median of 11 launches
// each) and the fastest is kept if it beats the default tiling by over 2%.
// Results live in a process-wide table and in a JSON file, one entry per line:
//   {"version": 1, "arch": "gfx950", "entries": {
//   "<key>": {"mt": 4, "wm": 8, "wo": 1, "target_wgs": 256, "us": 123.4},
//   ...
//   }}
// The file is $KRP_TUNE_CACHE, else $HOME/.cache/libkrp/sketch_tiles.json.
// TTM entries (keys starting "ttm ") hold {"split": s, "nt": n, "us": t}: for a
// mode after the first, one wave per item or the split kernel with nt p tiles
// per workgroup, timed the same way on the real input into a scratch output.
// Only sketch tilings whose partial-sum buffer fits the default plan's are
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
  int kind = 0;  // 0 sketch, 1 TTM
  SketchTile tile;
  TtmTile ttile;
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
                    &e.tile.mt, &e.tile.wm, &e.tile.wo, &e.tile.target_wgs, &e.us) == 5) {
      g_table[key] = e;
    } else if (std::sscanf(q1 + 1, " : {\"split\": %d, \"nt\": %d, \"us\": %lf}", &e.ttile.split, &e.ttile.nt,
                           &e.us) == 3) {
      e.kind = 1;
      g_table[key] = e;
    }
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
    const char* sep = ++i < g_table.size() ? "," : "";
    if (e.kind == 1)
      std::fprintf(f, "\"%s\": {\"split\": %d, \"nt\": %d, \"us\": %.3f}%s\n", kv.first.c_str(), e.ttile.split,
                   e.ttile.nt, e.us, sep);
    else
      std::fprintf(f, "\"%s\": {\"mt\": %d, \"wm\": %d, \"wo\": %d, \"target_wgs\": %d, \"us\": %.3f}%s\n",
                   kv.first.c_str(), e.tile.mt, e.tile.wm, e.tile.wo, e.tile.target_wgs, e.us, sep);
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

std::string ttm_key(const TtmProblem& pb) {
  std::string k = "ttm d=" + std::to_string(pb.d) + " dims=";
  for (int i = 0; i < pb.d; ++i) k += (i ? "x" : "") + std::to_string(pb.dims[i]);
  k += " mode=" + std::to_string(pb.mode) + " ell=" + std::to_string(pb.ell) + " prec=" + std::to_string(pb.prec) +
       " gd=" + std::to_string(pb.g_is_double) + " ld=" + std::to_string(pb.out_ld) +
       " al=" + std::to_string((reinterpret_cast<uintptr_t>(pb.g) & 15) == 0 ? 1 : 0);
  return k;
}

bool same_geometry(const SketchPlan& a, const SketchPlan& b) {
  return a.mt == b.mt && a.wm == b.wm && a.wo == b.wo && a.o_per_wg == b.o_per_wg &&
         a.row_blocks == b.row_blocks && a.f_blocks == b.f_blocks;
}

}  // namespace

bool cached_tile(const SketchProblem& pb, SketchTile* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_locked();
  auto it = g_table.find(tune_key(pb));
  if (it == g_table.end() || it->second.kind != 0) return false;
  *out = it->second.tile;
  return true;
}

bool cached_ttm_tile(const TtmProblem& pb, TtmTile* out) {
  TtmTile c[8];
  if (ttm_tile_candidates(pb, c, 8) < 2) {  // a single tiling: nothing to tune
    *out = TtmTile{};
    return true;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_locked();
  auto it = g_table.find(ttm_key(pb));
  if (it == g_table.end() || it->second.kind != 1) return false;
  *out = it->second.ttile;
  return true;
}

TtmTile tuned_ttm_tile(const TtmProblem& pb, hipStream_t st) {
  const TtmTile def{};
  if (!pb.g || !pb.q64) return def;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return def;
  TtmTile hit;
  if (cached_ttm_tile(pb, &hit)) return hit;
  TtmTile cands[8];
  const int nc = ttm_tile_candidates(pb, cands, 8);
  int64_t out_elems = pb.out_ld > 0 ? pb.out_ld : pb.ell;
  for (int k = 0; k < pb.d; ++k)
    if (k != pb.mode) out_elems *= pb.dims[k];
  void* out = nullptr;
  constexpr int kReps = 11;
  hipEvent_t ev[kReps + 1] = {};
  bool ok = hipMalloc(&out, std::max<size_t>((size_t)out_elems * (pb.out_is_double ? 8 : 4), 256)) == hipSuccess;
  for (int i = 0; ok && i <= kReps; ++i) ok = hipEventCreate(&ev[i]) == hipSuccess;
  std::vector<double> med(nc, -1.0);
  for (int i = 0; ok && i < nc; ++i) {
    TtmProblem t = pb;
    t.out = out;
    t.tile = cands[i];
    for (int w = 0; ok && w < 2; ++w) ok = launch_ttm(t, st) == hipSuccess;
    ok = ok && hipEventRecord(ev[0], st) == hipSuccess;
    for (int r = 0; ok && r < kReps; ++r)
      ok = launch_ttm(t, st) == hipSuccess && hipEventRecord(ev[r + 1], st) == hipSuccess;
    ok = ok && hipEventSynchronize(ev[kReps]) == hipSuccess;
    std::vector<double> tm;
    for (int r = 0; ok && r < kReps; ++r) {
      float ms = 0.f;
      ok = hipEventElapsedTime(&ms, ev[r], ev[r + 1]) == hipSuccess;
      tm.push_back(ms * 1000.0);
    }
    if (ok) {
      std::sort(tm.begin(), tm.end());
      med[i] = tm[kReps / 2];
    }
  }
  for (int i = 0; i <= kReps; ++i)
    if (ev[i]) hipEventDestroy(ev[i]);
  if (out) hipFree(out);
  (void)hipGetLastError();
  if (!ok || med[0] < 0.0) return def;
  int best = 0;
  for (int i = 1; i < nc; ++i)
    if (med[i] > 0.0 && med[i] < 0.98 * med[0] && med[i] < med[best]) best = i;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  Entry e;
  e.kind = 1;
  e.ttile = cands[best];
  e.us = med[best];
  g_table[ttm_key(pb)] = e;
  save_locked();
  return cands[best];
}

SketchTile tuned_tile(const SketchProblem& pb, hipStream_t st) {
  const SketchTile def{};
  if (!pb.x) return def;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return def;
  SketchTile hit;
  if (cached_tile(pb, &hit)) return hit;
  const std::string key = tune_key(pb);
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
  // every repetition is bracketed by its own event pair; the median is kept
  constexpr int kReps = 11;
  hipEvent_t ev[kReps + 1] = {};
  bool ok = hipMalloc(&part, std::max<size_t>(part_max, 256)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&y64), (size_t)base.n_rows * pb.ell * sizeof(double)) ==
                hipSuccess;
  for (int i = 0; ok && i <= kReps; ++i) ok = hipEventCreate(&ev[i]) == hipSuccess;
  std::vector<double> med(cands.size(), -1.0);
  for (size_t i = 0; ok && i < cands.size(); ++i) {
    const SketchPlan& p = cands[i].second;
    for (int w = 0; ok && w < 2; ++w) ok = launch_sketch(pb, p, part, y64, nullptr, 0, st) == hipSuccess;
    ok = ok && hipEventRecord(ev[0], st) == hipSuccess;
    for (int r = 0; ok && r < kReps; ++r) {
      ok = launch_sketch(pb, p, part, y64, nullptr, 0, st) == hipSuccess &&
           hipEventRecord(ev[r + 1], st) == hipSuccess;
    }
    ok = ok && hipEventSynchronize(ev[kReps]) == hipSuccess;
    std::vector<double> t;
    for (int r = 0; ok && r < kReps; ++r) {
      float ms = 0.f;
      ok = hipEventElapsedTime(&ms, ev[r], ev[r + 1]) == hipSuccess;
      t.push_back(ms * 1000.0);
    }
    if (ok) {
      std::sort(t.begin(), t.end());
      med[i] = t[kReps / 2];
    }
  }
  for (int i = 0; i <= kReps; ++i)
    if (ev[i]) hipEventDestroy(ev[i]);
  if (part) hipFree(part);
  if (y64) hipFree(y64);
  (void)hipGetLastError();  // a failed candidate must not leak into the caller's error state
  if (!ok || med[0] < 0.0) return def;
  // the default stays unless a candidate beats it by more than 2%
  size_t best = 0;
  for (size_t i = 1; i < cands.size(); ++i)
    if (med[i] > 0.0 && med[i] < 0.98 * med[0] && med[i] < med[best]) best = i;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  Entry e;
  e.tile = cands[best].first;
  e.us = med[best];
  g_table[key] = e;
  save_locked();
  return cands[best].first;
}

}  // namespace krp
