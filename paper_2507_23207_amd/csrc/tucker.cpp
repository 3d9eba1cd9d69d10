// Drivers of krp_sketch, krp_hosvd (Algorithm 7) and krp_sthosvd
// (Algorithm 8): validation, planning, workspace layout and the launch
// sequence (captured into a HIP graph unless KRP_FLAG_NO_GRAPH).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/krp.h"
#include "driver.h"
#include "kernels.h"
#include "truncate.h"

namespace krp {

namespace {

constexpr int kSumScratch = 4096;
constexpr int kMaxEll = 64;

int validate_tensor(const void* X, int dtype, int d, const int64_t* dims, int prec) {
  if (!X) return set_error(KRP_EINVAL, "X is NULL");
  if (dtype != KRP_F64 && dtype != KRP_F32) return set_error(KRP_EINVAL, "unknown dtype %d", dtype);
  if (d < 2 || d > kMaxDims) return set_error(KRP_EINVAL, "order d=%d outside 2..%d", d, kMaxDims);
  if (!dims) return set_error(KRP_EINVAL, "dims is NULL");
  double total = 1.0;
  for (int k = 0; k < d; ++k) {
    if (dims[k] < 1) return set_error(KRP_EINVAL, "dims[%d]=%lld must be >= 1", k, (long long)dims[k]);
    total *= (double)dims[k];
  }
  if (total > 4.0e18) return set_error(KRP_EINVAL, "tensor too large");
  if (prec < KRP_P_FP64 || prec > KRP_P_BF16X3) return set_error(KRP_EINVAL, "unknown precision %d", prec);
  if (dtype == KRP_F64 && prec != KRP_P_FP64)
    return set_error(KRP_EINVAL, "fp64 data requires KRP_P_FP64 arithmetic");
  return KRP_OK;
}

struct TuckerSetup {
  bool sthosvd = false;
  int d = 0, dtype = 0, prec = 0;
  bool out64 = false;  // intermediate cores in fp64
  int64_t dims[kMaxDims]{};
  int rank[kMaxDims]{}, ell[kMaxDims]{}, order[kMaxDims]{};
  int n_sketch = 0;
  SketchProblem spb[kMaxDims];
  SketchPlan spl[kMaxDims];
  int ttm_mode[kMaxDims]{};
  int64_t ttm_in_dims[kMaxDims][kMaxDims]{};
  int64_t ttm_out_elems[kMaxDims]{};
  // workspace layout
  size_t off_status = 0, off_sum = 0, off_norm = 0, off_y64 = 0, off_part = 0;
  size_t off_q64[kMaxDims]{};
  size_t off_core[2]{}, off_err[2]{}, off_trunc = 0;
  size_t total = 0;
  TruncPlan trunc;
  // Algorithm 7 with the all-mode fused sketch: one pass over X leaves every
  // mode's sketch (y64 of mode m at off_y64 + y_off[m] doubles)
  bool fused = false;
  FusedPlan fplan;
  size_t y_off[kMaxDims]{};
  // KRP_FLAG_GAUSSIAN: the dense-Gaussian baselines (RHOSVD / RSTHOSVD)
  bool dense = false;
  DensePlan dpl[kMaxDims];
  // tilings of the core TTMs (KRP_FLAG_AUTOTUNE; default otherwise)
  TtmTile ttile[kMaxDims];
  // STHOSVD: extent the TTM of each step gives its mode (ell, or for mode 1
  // ell padded with zero rows to the vector width of the core's type, so that
  // the later sketches, whose contiguous index it is, load whole vectors);
  // pad0 is the final extent of mode 1 (the core is compacted at the end)
  int64_t ttm_ext[kMaxDims]{};
  int64_t pad0 = 0;
};

// The TTM of step `step` of the core chain (mode order of the sweep) on g.
TtmProblem core_ttm(const TuckerSetup& s, int step, const void* g, bool g64, const double* q64, void* out) {
  TtmProblem tp;
  tp.g = g;
  tp.g_is_double = g64 ? 1 : 0;
  tp.d = s.d;
  for (int k = 0; k < s.d; ++k) tp.dims[k] = s.ttm_in_dims[step][k];
  tp.mode = s.ttm_mode[step];
  tp.ell = s.ell[tp.mode];
  tp.prec = s.prec;
  tp.q64 = q64;
  tp.out = out;
  tp.out_is_double = s.out64 ? 1 : 0;
  tp.tile = s.ttile[step];
  if (s.sthosvd && s.ttm_ext[step] > tp.ell) {
    tp.out_ld = s.ttm_ext[step];
    tp.zero_pad = true;
  }
  return tp;
}

int plan_tucker(bool sthosvd, int dtype, int d, const int64_t* dims, const int32_t* rank,
                int32_t oversample, const krp_opts& o, TuckerSetup& s) {
  s.sthosvd = sthosvd;
  s.d = d;
  s.dtype = dtype;
  s.prec = o.prec;
  s.out64 = (o.prec == KRP_P_FP64);
  if (!rank) return set_error(KRP_EINVAL, "rank is NULL");
  if (oversample < 0) return set_error(KRP_EINVAL, "oversample must be >= 0");
  if (sthosvd && (o.flags & KRP_FLAG_MEMO))
    return set_error(KRP_EINVAL, "KRP_FLAG_MEMO applies to krp_hosvd and krp_sketch, not to krp_sthosvd");
  s.dense = (o.flags & KRP_FLAG_GAUSSIAN) != 0;
  if (s.dense && (o.flags & KRP_FLAG_MEMO))
    return set_error(KRP_EINVAL, "KRP_FLAG_GAUSSIAN and KRP_FLAG_MEMO exclude each other");
  for (int k = 0; k < d; ++k) {
    s.dims[k] = dims[k];
    if (rank[k] < 1) return set_error(KRP_EINVAL, "rank[%d]=%d must be >= 1", k, rank[k]);
    const int64_t l = (int64_t)rank[k] + oversample;
    if (l > dims[k])
      return set_error(KRP_EINVAL, "ell[%d]=%lld exceeds the mode size %lld", k, (long long)l,
                       (long long)dims[k]);
    if (l > kMaxEll) return set_error(KRP_EINVAL, "ell[%d]=%lld exceeds the supported 64", k, (long long)l);
    s.rank[k] = rank[k];
    s.ell[k] = (int)l;
  }
  if (o.order) {
    if (!sthosvd) return set_error(KRP_EINVAL, "a mode order applies to krp_sthosvd only");
    bool seen[kMaxDims] = {false};
    for (int k = 0; k < d; ++k) {
      const int m = o.order[k];
      if (m < 0 || m >= d || seen[m]) return set_error(KRP_EINVAL, "order is not a permutation of 0..d-1");
      seen[m] = true;
      s.order[k] = m;
    }
  } else {
    for (int k = 0; k < d; ++k) s.order[k] = k;
  }
  if (o.truncate != 0 && o.truncate != 1) return set_error(KRP_EINVAL, "truncate must be 0 or 1");

  const size_t cs = s.out64 ? 8 : 4;
  size_t part_max = 0, y_max = 0, core_max = 0, err_max = 0;
  int64_t cur[kMaxDims];
  for (int k = 0; k < d; ++k) cur[k] = dims[k];
  SketchTile tile;
  for (int step = 0; step < d; ++step) {
    const int m = sthosvd ? s.order[step] : step;
    SketchProblem& pb = s.spb[step];
    pb.x_is_double = (step == 0 || !sthosvd) ? (dtype == KRP_F64) : s.out64;
    pb.d = d;
    for (int k = 0; k < d; ++k) pb.dims[k] = sthosvd ? cur[k] : dims[k];
    pb.mode = m;
    pb.ell = s.ell[m];
    pb.prec = o.prec;
    pb.seed = o.seed;
    pb.draw = o.draw;
    pb.sketch_id = (o.flags & KRP_FLAG_MEMO) ? kMemoSketch : (uint32_t)m;
    s.spl[step] = plan_sketch(pb, tile);
    part_max = std::max(part_max, s.spl[step].partial_bytes);
    if (s.dense) {
      s.dpl[step] = plan_dense(pb);
      part_max = std::max(part_max, s.dpl[step].ws_bytes);
    }
    part_max = std::max(part_max, cholqr_split_bytes(pb.dims[m], s.ell[m]));  // reused by the QR
    y_max = std::max(y_max, (size_t)(pb.dims[m] * s.ell[m]));
    if (sthosvd) {
      s.ttm_mode[step] = m;
      for (int k = 0; k < d; ++k) s.ttm_in_dims[step][k] = cur[k];
      // mode 1, compressed before the last step, is padded with zero rows to the
      // vector width (the extra factor rows of later sketches multiply zeros);
      // not for the dense baselines, whose Omega rows follow the core's indexing
      const int64_t vlen = s.out64 ? 2 : 4;
      int64_t ext = s.ell[m];
      if (m == 0 && !s.dense && step + 1 < d) ext = (ext + vlen - 1) / vlen * vlen;
      s.ttm_ext[step] = ext;
      if (m == 0) s.pad0 = ext;
      cur[m] = ext;
      int64_t e = 1;
      for (int k = 0; k < d; ++k) e *= cur[k];
      s.ttm_out_elems[step] = e;
      core_max = std::max(core_max, (size_t)e);
    }
  }
  s.n_sketch = d;
  if (!sthosvd && dtype == KRP_F32 && !s.dense) {
    SketchProblem all[kMaxDims];
    for (int k = 0; k < d; ++k) all[k] = s.spb[k];
    s.fplan = plan_fused(all, d);
    s.fused = s.fplan.ok;
    if (s.fused) {
      part_max = std::max(part_max, s.fplan.ws_bytes);
      size_t yo = 0;
      for (int k = 0; k < d; ++k) {
        s.y_off[k] = yo;
        yo += (size_t)dims[k] * s.ell[k];
      }
      y_max = std::max(y_max, yo);
    }
  }
  // TTM chain of Algorithm 7 (natural order) and of the error check.
  for (int k = 0; k < d; ++k) cur[k] = dims[k];
  for (int step = 0; step < d; ++step) {
    if (!sthosvd) {
      s.ttm_mode[step] = step;
      for (int k = 0; k < d; ++k) s.ttm_in_dims[step][k] = cur[k];
    }
    cur[step] = s.ell[step];
    int64_t e = 1;
    for (int k = 0; k < d; ++k) e *= cur[k];
    if (!sthosvd) {
      s.ttm_out_elems[step] = e;
      core_max = std::max(core_max, (size_t)e);
    }
    err_max = std::max(err_max, (size_t)e);
  }
  size_t off = 0;
  s.off_status = off; off = align_up(off + 64);
  s.off_norm = off; off = align_up(off + 4 * sizeof(double));
  s.off_sum = off; off = align_up(off + kSumScratch * sizeof(double));
  s.off_y64 = off; off = align_up(off + y_max * sizeof(double));
  for (int k = 0; k < d; ++k) {
    s.off_q64[k] = off;
    off = align_up(off + (size_t)dims[k] * s.ell[k] * sizeof(double));
  }
  s.off_part = off; off = align_up(off + part_max);
  s.off_core[0] = off; off = align_up(off + core_max * cs);
  s.off_core[1] = off; off = align_up(off + core_max * cs);
  s.off_err[0] = off; off = align_up(off + err_max * sizeof(double));
  s.off_err[1] = off; off = align_up(off + err_max * sizeof(double));
  // truncation of the ell-sized core (fp64)
  s.trunc = plan_truncate(d, s.ell, s.rank, dims, s.order);
  s.off_trunc = off; off = align_up(off + s.trunc.ws_bytes);
  s.total = off;
  return KRP_OK;
}

std::string plan_key(const SketchPlan& p) {
  return std::to_string(p.mt) + "," + std::to_string(p.wm) + "," + std::to_string(p.wo) + "," +
         std::to_string(p.o_per_wg);
}

std::string tucker_key(const TuckerSetup& s, const krp_opts& o, const void* X, const void* core,
                       void* const* Q, const void* ws, const int* status, bool want_err) {
  std::string k = s.sthosvd ? "sthosvd" : "hosvd";
  k += "|dt=" + std::to_string(s.dtype) + "|p=" + std::to_string(s.prec);
  for (int i = 0; i < s.d; ++i)
    k += "|" + std::to_string(s.dims[i]) + "," + std::to_string(s.rank[i]) + "," +
         std::to_string(s.ell[i]) + "," + std::to_string(s.order[i]) + "," + ptr_key(Q[i]);
  k += "|seed=" + std::to_string(o.seed) + "|draw=" + std::to_string(o.draw) +
       "|memo=" + std::to_string((o.flags & KRP_FLAG_MEMO) ? 1 : 0) + "|tr=" + std::to_string(o.truncate) + "|err=" + std::to_string(want_err ? 1 : 0) +
       "|X=" + ptr_key(X) + "|core=" + ptr_key(core) + "|ws=" + ptr_key(ws) + "|" +
       "|st=" + ptr_key(status);
  for (int i = 0; i < s.n_sketch; ++i) k += "|t=" + plan_key(s.spl[i]);  // tilings (tuned or not)
  k += s.fused ? "|fused" : "";
  k += s.dense ? "|gauss" : "";
  return k;
}

int check(hipError_t e, const char* what) { return e == hipSuccess ? KRP_OK : hip_fail(e, what); }

#define KRP_TRY(expr)            \
  do {                           \
    const int _rc = (expr);      \
    if (_rc != KRP_OK) return _rc; \
  } while (0)

// Enqueues the whole sweep.  With `tune` (a direct, uncaptured call), each
// sketch's tiling is first tuned on its real input -- X or the partial core
// the previous step left -- and the tuned plan replaces the default in `s`.
int enqueue_tucker(TuckerSetup& s, const krp_opts& o, const void* X, void* core,
                   void* const* Q, char* ws, int* status, bool want_err, bool tune,
                   hipStream_t st) {
  const int d = s.d;
  const bool x64 = s.dtype == KRP_F64;
  const bool trunc = o.truncate == 1;
  if (!o.status_dev) KRP_TRY(check(launch_fill_int(status, 0, 1, st), "fill"));
  double* y64 = reinterpret_cast<double*>(ws + s.off_y64);
  void* part = ws + s.off_part;
  void* cores[2] = {ws + s.off_core[0], ws + s.off_core[1]};
  const void* cur = X;
  bool cur64 = x64;
  if (s.fused) {
    // every sketch of Algorithm 7 from one pass over X
    SketchProblem all[kMaxDims];
    double* ys[kMaxDims];
    for (int k = 0; k < d; ++k) {
      all[k] = s.spb[k];
      all[k].x = X;
      ys[k] = y64 + s.y_off[k];
    }
    KRP_TRY(check(launch_fused(s.fplan, all, d, part, ys, nullptr, 0, st), "fused sketch"));
  }
  for (int step = 0; step < d; ++step) {
    const int m = s.spb[step].mode;
    SketchProblem pb = s.spb[step];
    pb.x = s.sthosvd ? cur : X;
    pb.x_is_double = s.sthosvd ? (cur64 ? 1 : 0) : (x64 ? 1 : 0);
    if (s.dense) {
      KRP_TRY(check(launch_dense_sketch(pb, s.dpl[step], reinterpret_cast<char*>(part), y64, nullptr, 0, st),
                    "dense sketch"));
    } else if (s.fused) {
      y64 = reinterpret_cast<double*>(ws + s.off_y64) + s.y_off[m];
    } else {
      if (tune) {
        const SketchPlan t = plan_sketch(pb, tuned_tile(pb, st));
        if (t.partial_bytes <= s.spl[step].partial_bytes) s.spl[step] = t;
      }
      KRP_TRY(check(launch_sketch(pb, s.spl[step], part, y64, nullptr, 0, st), "sketch"));
    }
    double* q64 = reinterpret_cast<double*>(ws + s.off_q64[m]);
    // the partial-sum buffer of the sketch is free again: workspace of the QR
    KRP_TRY(check(launch_cholqr_split(pb.dims[m], s.ell[m], y64, q64, trunc ? nullptr : Q[m], x64 ? 1 : 0,
                                      part, status, st),
                  "cholqr"));
    if (s.sthosvd) {
      TtmProblem tp = core_ttm(s, step, cur, cur64, q64, cores[step & 1]);
      if (tune) tp.tile = s.ttile[step] = tuned_ttm_tile(tp, st);
      KRP_TRY(check(launch_ttm(tp, st), "ttm"));
      cur = tp.out;
      cur64 = s.out64;
    }
  }
  if (!s.sthosvd) {
    cur = X;
    cur64 = x64;
    for (int step = 0; step < d; ++step) {
      TtmProblem tp = core_ttm(s, step, cur, cur64, reinterpret_cast<double*>(ws + s.off_q64[step]),
                               cores[step & 1]);
      if (tune) tp.tile = s.ttile[step] = tuned_ttm_tile(tp, st);
      KRP_TRY(check(launch_ttm(tp, st), "ttm"));
      cur = tp.out;
      cur64 = s.out64;
    }
  }
  // `cur` holds the ell-sized core in the compute type (STHOSVD: mode 1 padded).
  if (s.sthosvd && s.pad0 > s.ell[0]) {
    int64_t rest = 1;
    for (int k = 1; k < d; ++k) rest *= s.ell[k];
    void* dst = (cur == cores[0]) ? cores[1] : cores[0];
    KRP_TRY(check(launch_compact_rows(cur, s.pad0, dst, s.ell[0], rest, cur64 ? 1 : 0, st), "compact core"));
    cur = dst;
  }
  if (trunc) {
    double* qs[kMaxDims];
    for (int k = 0; k < d; ++k) qs[k] = reinterpret_cast<double*>(ws + s.off_q64[k]);
    KRP_TRY(check(launch_truncate(s.trunc, cur, cur64 ? 1 : 0, qs, core, Q, x64 ? 1 : 0,
                                  ws + s.off_trunc, st),
                  "truncate"));
  } else {
    int64_t elems = 1;
    for (int k = 0; k < d; ++k) elems *= s.ell[k];
    KRP_TRY(check(launch_cast(cur, cur64 ? 1 : 0, core, x64 ? 1 : 0, elems, st), "cast core"));
  }
  if (want_err) {
    // ||X||^2 and ||X x_1 Q_1^T ... x_d Q_d^T||^2 in fp64 with the fp64 factors
    // (the projection identity for orthonormal Q_i).
    double* norms = reinterpret_cast<double*>(ws + s.off_norm);
    double* scratch = reinterpret_cast<double*>(ws + s.off_sum);
    int64_t nx = 1;
    for (int k = 0; k < d; ++k) nx *= s.dims[k];
    KRP_TRY(check(launch_sumsq(X, x64 ? 1 : 0, nx, norms + 0, scratch, kSumScratch, st), "sumsq"));
    const void* e_cur = X;
    bool e64 = x64;
    int64_t edims[kMaxDims];
    for (int k = 0; k < d; ++k) edims[k] = s.dims[k];
    int64_t elems = 0;
    for (int step = 0; step < d; ++step) {
      const int r = trunc ? s.rank[step] : s.ell[step];
      TtmProblem tp;
      tp.g = e_cur;
      tp.g_is_double = e64 ? 1 : 0;
      tp.d = d;
      for (int k = 0; k < d; ++k) tp.dims[k] = edims[k];
      tp.mode = step;
      tp.ell = r;
      tp.prec = KRP_P_FP64;
      tp.q64 = trunc ? truncated_q64(s.trunc, ws + s.off_trunc, step)
                     : reinterpret_cast<double*>(ws + s.off_q64[step]);
      tp.out = ws + s.off_err[step & 1];
      tp.out_is_double = 1;
      KRP_TRY(check(launch_ttm(tp, st), "ttm(err)"));
      e_cur = tp.out;
      e64 = true;
      edims[step] = r;
    }
    elems = 1;
    for (int k = 0; k < d; ++k) elems *= edims[k];
    KRP_TRY(check(launch_sumsq(e_cur, 1, elems, norms + 1, scratch, kSumScratch, st), "sumsq"));
  }
  return KRP_OK;
}

// Tilings the tuning table already holds replace the default plans (only
// when their partial sums fit the default plan's, so workspace sizes queried
// without the flag stay valid).  Returns true when some sketch of the sweep
// has no entry yet.  Launches nothing.
bool apply_cached_tiles(TuckerSetup& s, const void* X, char* ws) {
  if (s.fused || s.dense) return false;  // the fused pass and the dense sketches have no tiling to tune
  bool missing = false;
  for (int step = 0; step < s.n_sketch; ++step) {
    SketchProblem pb = s.spb[step];
    // the input of the sketch: X, or the partial core of the previous step
    pb.x = (step == 0 || !s.sthosvd) ? X : static_cast<const void*>(ws + s.off_core[(step - 1) & 1]);
    SketchTile t;
    if (!cached_tile(pb, &t)) {
      missing = true;
      continue;
    }
    const SketchPlan p = plan_sketch(pb, t);
    if (p.partial_bytes <= s.spl[step].partial_bytes) s.spl[step] = p;
  }
  return missing;
}

// The same for the core TTMs: cached tilings go into s.ttile; true when some
// TTM of the chain has no entry yet.  Launches nothing.
bool apply_cached_ttm_tiles(TuckerSetup& s, const void* X, char* ws) {
  bool missing = false;
  bool g64 = s.dtype == KRP_F64;
  for (int step = 0; step < s.d; ++step) {
    const void* g = step == 0 ? X : static_cast<const void*>(ws + s.off_core[(step - 1) & 1]);
    TtmProblem tp = core_ttm(s, step, g, step == 0 ? g64 : s.out64, nullptr, ws + s.off_core[step & 1]);
    TtmTile t;
    if (cached_ttm_tile(tp, &t))
      s.ttile[step] = t;
    else
      missing = true;
  }
  return missing;
}

std::string ttm_tiles_key(const TuckerSetup& s) {
  std::string k = "|ttm=";
  for (int step = 0; step < s.d; ++step) k += std::to_string(s.ttile[step].split) + "." + std::to_string(s.ttile[step].nt) + ",";
  return k;
}

bool stream_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

int tucker_entry(bool sthosvd, const void* X, int dtype, int d, const int64_t* dims,
                 const int32_t* rank, int32_t oversample, const krp_opts* opts, void* core,
                 void* const* Q, int64_t* core_dims, void* stream) {
  krp_opts o;
  if (opts)
    o = *opts;
  else
    krp_opts_default(&o);
  KRP_TRY(validate_tensor(X, dtype, d, dims, o.prec));
  if (!core) return set_error(KRP_EINVAL, "core is NULL");
  if (!Q) return set_error(KRP_EINVAL, "Q is NULL");
  for (int k = 0; k < d; ++k)
    if (!Q[k]) return set_error(KRP_EINVAL, "Q[%d] is NULL", k);
  TuckerSetup s;
  KRP_TRY(plan_tucker(sthosvd, dtype, d, dims, rank, oversample, o, s));
  if (s.fused && (reinterpret_cast<uintptr_t>(X) & 15) != 0) s.fused = false;  // the fused pass loads 16-byte rows
  if (core_dims)
    for (int k = 0; k < d; ++k) core_dims[k] = o.truncate ? s.rank[k] : s.ell[k];
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = nullptr;
  KRP_TRY(acquire_workspace(&o, s.total, st, &ws));
  int* status = o.status_dev ? o.status_dev : reinterpret_cast<int*>(ws + s.off_status);
  const bool want_err = o.rel_err != nullptr;
  // Autotuning: cached tilings are used as they are; a sweep with untuned
  // sketches runs once directly (not captured), tuning each sketch on its real
  // input.  Nothing is tuned, allocated or synchronised while the caller's
  // stream is being captured.
  bool tune_now = false;
  if (o.flags & KRP_FLAG_AUTOTUNE) {
    const bool sk_missing = apply_cached_tiles(s, X, ws);
    const bool ttm_missing = !s.dense && apply_cached_ttm_tiles(s, X, ws);
    tune_now = (sk_missing || ttm_missing) && !stream_capturing(st);
  }
  if (tune_now) {
    KRP_TRY(enqueue_tucker(s, o, X, core, Q, ws, status, want_err, true, st));
  } else {
    const std::string key = tucker_key(s, o, X, core, Q, ws, status, want_err) + ttm_tiles_key(s);
    KRP_TRY(run_maybe_graph(key, !(o.flags & KRP_FLAG_NO_GRAPH), st, [&](hipStream_t cs) {
      return enqueue_tucker(s, o, X, core, Q, ws, status, want_err, false, cs);
    }));
  }
  int rc = KRP_OK;
  if (!o.status_dev) rc = finish_status(status, st);
  if (want_err) {
    double nrm[2] = {0.0, 0.0};
    hipError_t e = hipMemcpyAsync(nrm, ws + s.off_norm, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "read norms");
    *o.rel_err = nrm[0] > 0 ? std::sqrt(std::max(0.0, nrm[0] - nrm[1]) / nrm[0]) : 0.0;
  }
  return rc;
}

}  // namespace

int prepare_sketches(const void* X, int dtype, int d, const int64_t* dims, int nmodes,
                     const int32_t* modes, const int32_t* ell, void* const* Y, const krp_opts& o,
                     bool tune, hipStream_t st, SketchSet* out) {
  KRP_TRY(validate_tensor(X, dtype, d, dims, o.prec));
  if (nmodes < 1 || nmodes > d) return set_error(KRP_EINVAL, "nmodes=%d outside 1..d", nmodes);
  if (!modes || !ell || !Y) return set_error(KRP_EINVAL, "modes, ell and Y must not be NULL");
  bool seen[kMaxDims] = {false};
  SketchSet& ss = *out;
  ss.nmodes = nmodes;
  ss.out_double = dtype == KRP_F64 ? 1 : 0;
  ss.dense = (o.flags & KRP_FLAG_GAUSSIAN) != 0;
  if (ss.dense && (o.flags & KRP_FLAG_MEMO))
    return set_error(KRP_EINVAL, "KRP_FLAG_GAUSSIAN and KRP_FLAG_MEMO exclude each other");
  if (ss.dense) tune = false;
  size_t part = 0;
  for (int j = 0; j < nmodes; ++j) {
    const int m = modes[j];
    if (m < 0 || m >= d || seen[m]) return set_error(KRP_EINVAL, "modes must be distinct values in 0..d-1");
    seen[m] = true;
    if (ell[j] < 1 || ell[j] > kMaxEll) return set_error(KRP_EINVAL, "ell[%d]=%d outside 1..64", j, ell[j]);
    if (!Y[j]) return set_error(KRP_EINVAL, "Y[%d] is NULL", j);
    SketchProblem& pb = ss.pb[j];
    pb.x = X;
    pb.x_is_double = dtype == KRP_F64;
    pb.d = d;
    for (int k = 0; k < d; ++k) pb.dims[k] = dims[k];
    pb.mode = m;
    pb.ell = ell[j];
    pb.prec = o.prec;
    pb.seed = o.seed;
    pb.draw = o.draw;
    pb.sketch_id = (o.flags & KRP_FLAG_MEMO) ? kMemoSketch : (uint32_t)m;
    ss.pl[j] = plan_sketch(pb, SketchTile{});
    if (tune) {
      const SketchPlan t = plan_sketch(pb, tuned_tile(pb, st));
      if (t.partial_bytes <= ss.pl[j].partial_bytes) ss.pl[j] = t;
    }
    part = std::max(part, ss.pl[j].partial_bytes);
    if (ss.dense) {
      ss.dp[j] = plan_dense(pb);
      part = std::max(part, ss.dp[j].ws_bytes);
    }
  }
  // several modes of the same tensor: one fused pass over X when it applies
  ss.fused = false;
  if (nmodes >= 2 && !ss.dense) {
    ss.fplan = plan_fused(ss.pb, nmodes);
    if (ss.fplan.ok) {
      ss.fused = true;
      part = ss.fplan.ws_bytes;
    }
  }
  ss.ws_bytes = align_up(part);
  return KRP_OK;
}

int enqueue_sketches(const SketchSet& ss, char* ws, void* const* Y, hipStream_t st) {
  if (ss.dense) {
    for (int j = 0; j < ss.nmodes; ++j)
      KRP_TRY(check(launch_dense_sketch(ss.pb[j], ss.dp[j], ws, nullptr, Y[j], ss.out_double, st), "dense sketch"));
    return KRP_OK;
  }
  if (ss.fused) return check(launch_fused(ss.fplan, ss.pb, ss.nmodes, ws, nullptr, Y, ss.out_double, st), "fused sketch");
  for (int j = 0; j < ss.nmodes; ++j)
    KRP_TRY(check(launch_sketch(ss.pb[j], ss.pl[j], ws, nullptr, Y[j], ss.out_double, st), "sketch"));
  return KRP_OK;
}

}  // namespace krp

using namespace krp;

extern "C" {

int krp_sketch(const void* X, int dtype, int d, const int64_t* dims, int nmodes, const int32_t* modes,
               const int32_t* ell, const krp_opts* opts, void* const* Y, void* stream) {
  krp_opts o;
  if (opts)
    o = *opts;
  else
    krp_opts_default(&o);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  SketchSet ss;
  KRP_TRY(prepare_sketches(X, dtype, d, dims, nmodes, modes, ell, Y, o, (o.flags & KRP_FLAG_AUTOTUNE) != 0,
                           st, &ss));
  char* ws = nullptr;
  KRP_TRY(acquire_workspace(&o, ss.ws_bytes, st, &ws));
  std::string key = "sketch|dt=" + std::to_string(dtype) + "|p=" + std::to_string(o.prec) +
                    "|seed=" + std::to_string(o.seed) + "|draw=" + std::to_string(o.draw) +
                    "|X=" + ptr_key(X) + "|ws=" + ptr_key(ws) + "|";
  for (int k = 0; k < d; ++k) key += std::to_string(dims[k]) + ",";
  for (int j = 0; j < nmodes; ++j)
    key += "|" + std::to_string(modes[j]) + "," + std::to_string(ell[j]) + "," + ptr_key(Y[j]) + ",t=" +
           plan_key(ss.pl[j]);
  key += ss.fused ? "|fused" : "";
  key += (o.flags & KRP_FLAG_MEMO) ? "|memo" : "";
  key += ss.dense ? "|gauss" : "";
  return run_maybe_graph(key, !(o.flags & KRP_FLAG_NO_GRAPH), st,
                         [&](hipStream_t cs) -> int { return enqueue_sketches(ss, ws, Y, cs); });
}

int krp_range_factors(const void* X, int dtype, int d, const int64_t* dims, int nmodes, const int32_t* modes,
                      const int32_t* ell, const krp_opts* opts, void* const* Q, void* stream) {
  krp_opts o;
  if (opts)
    o = *opts;
  else
    krp_opts_default(&o);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  SketchSet ss;
  // Q stands in for the sketch outputs in the validation; the sketches go to
  // fp64 workspace buffers
  KRP_TRY(prepare_sketches(X, dtype, d, dims, nmodes, modes, ell, Q, o, false, st, &ss));
  for (int j = 0; j < nmodes; ++j)
    if (ell[j] > dims[modes[j]])
      return set_error(KRP_EINVAL, "ell[%d]=%d exceeds the mode size %lld", j, ell[j], (long long)dims[modes[j]]);
  // workspace: status | y64 of every mode | q64 of every mode | partial sums / QR scratch
  size_t off = align_up(64), y_off[kMaxDims], q_off[kMaxDims], part = ss.ws_bytes;
  for (int j = 0; j < nmodes; ++j) {
    y_off[j] = off;
    off = align_up(off + (size_t)dims[modes[j]] * ell[j] * sizeof(double));
  }
  for (int j = 0; j < nmodes; ++j) {
    q_off[j] = off;
    off = align_up(off + (size_t)dims[modes[j]] * ell[j] * sizeof(double));
    part = std::max(part, cholqr_split_bytes(dims[modes[j]], ell[j]));
  }
  const size_t part_off = off;
  off = align_up(off + part);
  char* ws = nullptr;
  KRP_TRY(acquire_workspace(&o, off, st, &ws));
  int* status = o.status_dev ? o.status_dev : reinterpret_cast<int*>(ws);
  std::string key = "range|dt=" + std::to_string(dtype) + "|p=" + std::to_string(o.prec) +
                    "|seed=" + std::to_string(o.seed) + "|draw=" + std::to_string(o.draw) +
                    "|X=" + ptr_key(X) + "|ws=" + ptr_key(ws) + "|st=" + ptr_key(status) + "|";
  for (int k = 0; k < d; ++k) key += std::to_string(dims[k]) + ",";
  for (int j = 0; j < nmodes; ++j)
    key += "|" + std::to_string(modes[j]) + "," + std::to_string(ell[j]) + "," + ptr_key(Q[j]);
  key += ss.fused ? "|fused" : "";
  key += (o.flags & KRP_FLAG_MEMO) ? "|memo" : "";
  key += ss.dense ? "|gauss" : "";
  const int out_double = dtype == KRP_F64 ? 1 : 0;
  KRP_TRY(run_maybe_graph(key, !(o.flags & KRP_FLAG_NO_GRAPH), st, [&](hipStream_t cs) -> int {
    if (!o.status_dev) KRP_TRY(check(launch_fill_int(status, 0, 1, cs), "fill"));
    double* ys[kMaxDims];
    for (int j = 0; j < nmodes; ++j) ys[j] = reinterpret_cast<double*>(ws + y_off[j]);
    void* pw = ws + part_off;
    if (ss.dense) {
      for (int j = 0; j < nmodes; ++j)
        KRP_TRY(check(launch_dense_sketch(ss.pb[j], ss.dp[j], reinterpret_cast<char*>(pw), ys[j], nullptr, 0, cs),
                      "dense sketch"));
    } else if (ss.fused) {
      KRP_TRY(check(launch_fused(ss.fplan, ss.pb, nmodes, pw, ys, nullptr, 0, cs), "fused sketch"));
    } else {
      for (int j = 0; j < nmodes; ++j)
        KRP_TRY(check(launch_sketch(ss.pb[j], ss.pl[j], pw, ys[j], nullptr, 0, cs), "sketch"));
    }
    for (int j = 0; j < nmodes; ++j)
      KRP_TRY(check(launch_cholqr_split(dims[modes[j]], ell[j], ys[j], reinterpret_cast<double*>(ws + q_off[j]),
                                        Q[j], out_double, pw, status, cs),
                    "cholqr"));
    return KRP_OK;
  }));
  if (!o.status_dev) return finish_status(status, st);
  return KRP_OK;
}

int krp_hosvd(const void* X, int dtype, int d, const int64_t* dims, const int32_t* rank,
              int32_t oversample, const krp_opts* opts, void* core, void* const* Q, int64_t* core_dims,
              void* stream) {
  return tucker_entry(false, X, dtype, d, dims, rank, oversample, opts, core, Q, core_dims, stream);
}

int krp_sthosvd(const void* X, int dtype, int d, const int64_t* dims, const int32_t* rank,
                int32_t oversample, const krp_opts* opts, void* core, void* const* Q, int64_t* core_dims,
                void* stream) {
  return tucker_entry(true, X, dtype, d, dims, rank, oversample, opts, core, Q, core_dims, stream);
}

int krp_workspace_size(int which, int dtype, int d, const int64_t* dims, const int32_t* rank,
                       int32_t oversample, int prec, size_t* bytes) {
  if (!bytes) return set_error(KRP_EINVAL, "bytes is NULL");
  if (dtype != KRP_F64 && dtype != KRP_F32) return set_error(KRP_EINVAL, "unknown dtype %d", dtype);
  if (d < 2 || d > kMaxDims || !dims || !rank) return set_error(KRP_EINVAL, "bad shape arguments");
  if (prec < 0 || prec > 3 || (dtype == KRP_F64 && prec != KRP_P_FP64))
    return set_error(KRP_EINVAL, "bad precision");
  for (int k = 0; k < d; ++k)
    if (dims[k] < 1) return set_error(KRP_EINVAL, "dims[%d] must be >= 1", k);
  krp_opts o;
  krp_opts_default(&o);
  o.prec = prec;
  const bool gauss = which >= 3 && which <= 5;
  if (gauss) {
    o.flags |= KRP_FLAG_GAUSSIAN;
    which -= 3;
  }
  if (which == 0) {
    size_t part = 0;
    SketchProblem all[kMaxDims];
    for (int m = 0; m < d; ++m) {
      if (rank[m] < 1 || rank[m] > kMaxEll) return set_error(KRP_EINVAL, "ell[%d] outside 1..64", m);
      SketchProblem& pb = all[m];
      pb.x_is_double = dtype == KRP_F64;
      pb.d = d;
      for (int k = 0; k < d; ++k) pb.dims[k] = dims[k];
      pb.mode = m;
      pb.ell = rank[m];
      pb.prec = prec;
      pb.sketch_id = (uint32_t)m;
      part = std::max(part, plan_sketch(pb, SketchTile{}).partial_bytes);
      if (gauss) part = std::max(part, plan_dense(pb).ws_bytes);
    }
    const FusedPlan fp = plan_fused(all, d);  // the call with all modes takes the fused pass
    if (fp.ok && !gauss) part = std::max(part, fp.ws_bytes);
    *bytes = align_up(part);
    return KRP_OK;
  }
  if (which != 1 && which != 2) return set_error(KRP_EINVAL, "which must be 0..5");
  TuckerSetup s;
  KRP_TRY(plan_tucker(which == 2, dtype, d, dims, rank, oversample, o, s));
  *bytes = s.total;
  return KRP_OK;
}

}  // extern "C"
