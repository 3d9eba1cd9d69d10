// Drivers of krp_sensor_select, krp_sensor_measure and krp_sensor_reconstruct
// (the training and test phases of the sensor placement of Section 6):
// validation, workspace layout and launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/krp.h"
#include "driver.h"
#include "kernels.h"
#include "sensor.h"

namespace krp {
namespace {

constexpr int kSensorMaxEll = 64;
constexpr int64_t kTtmChunk = 64;  // output columns per TTM launch

krp_opts opts_or_default(const krp_opts* opts) {
  krp_opts o;
  if (opts)
    o = *opts;
  else
    krp_opts_default(&o);
  return o;
}

int check_dtype(int dtype) {
  if (dtype != KRP_F64 && dtype != KRP_F32) return set_error(KRP_EINVAL, "unknown dtype %d", dtype);
  return KRP_OK;
}

// Spatial modes d (the snapshot mode comes on top of them).
int check_grid(int d, const int64_t* dims, const int32_t* ell) {
  if (d < 1 || d > kMaxDims - 1) return set_error(KRP_EINVAL, "d=%d outside 1..%d", d, kMaxDims - 1);
  if (!dims || !ell) return set_error(KRP_EINVAL, "dims and ell must not be NULL");
  for (int i = 0; i < d; ++i) {
    if (dims[i] < 1) return set_error(KRP_EINVAL, "dims[%d] must be >= 1", i);
    if (ell[i] < 1 || ell[i] > dims[i])
      return set_error(KRP_EINVAL, "ell[%d]=%d outside 1..dims[%d]", i, ell[i], i);
  }
  return KRP_OK;
}

struct SelectLayout {
  size_t w[kMaxDims], taken[kMaxDims], minv[kMaxDims], status, total;
};

SelectLayout select_layout(int nmodes, const int64_t* n, const int32_t* ell) {
  SelectLayout l{};
  size_t off = 0;
  for (int j = 0; j < nmodes; ++j) {
    l.w[j] = off;
    off = align_up(off + (size_t)n[j] * ell[j] * sizeof(double));
    l.taken[j] = off;
    off = align_up(off + (size_t)n[j]);
    l.minv[j] = off;
    off = align_up(off + (size_t)ell[j] * ell[j] * sizeof(double));
  }
  l.status = off;
  off = align_up(off + 64);
  l.total = off;
  return l;
}

struct ReconLayout {
  size_t at[kMaxDims], buf[2], total;
  int64_t elems_max;
};

// Order of the reconstruction chain: smallest expansion dims_i / ell_i first
// (ties: lower mode first), so the intermediate tensors stay small and the
// widest expansion produces the output.  Any order gives the same product.
void recon_order(int d, const int64_t* dims, const int32_t* ell, int* order) {
  for (int i = 0; i < d; ++i) order[i] = i;
  std::stable_sort(order, order + d, [&](int a, int b) { return dims[a] * ell[b] < dims[b] * ell[a]; });
}
// Sizes of the reconstruction chain (mode order[s] expands ell -> dims at
// step s); the last step writes the caller's output.
ReconLayout recon_layout(int d, const int64_t* dims, const int32_t* ell, int64_t snaps, size_t esz) {
  ReconLayout l{};
  size_t off = 0;
  for (int i = 0; i < d; ++i) {  // fp64 transposed factors of the modes that take the TTM path
    l.at[i] = off;
    if (ell[i] > kExpandMaxEll) off = align_up(off + (size_t)dims[i] * ell[i] * sizeof(double));
  }
  int order[kMaxDims];
  recon_order(d, dims, ell, order);
  int64_t cur[kMaxDims];
  for (int i = 0; i < d; ++i) cur[i] = ell[i];
  l.elems_max = 0;
  for (int s = 0; s + 1 < d; ++s) {
    cur[order[s]] = dims[order[s]];
    int64_t e = snaps;
    for (int k = 0; k < d; ++k) e *= cur[k];
    l.elems_max = std::max(l.elems_max, e);
  }
  for (int b = 0; b < 2; ++b) {
    l.buf[b] = off;
    off = align_up(off + (size_t)l.elems_max * esz);
  }
  l.total = off;
  return l;
}

}  // namespace
}  // namespace krp

using namespace krp;

extern "C" {

int krp_sensor_select(int nmodes, const int64_t* n, const int32_t* ell, int dtype, const void* const* Q,
                      const krp_opts* opts, int32_t* const* idx, void* const* A, void* stream) {
  const krp_opts o = opts_or_default(opts);
  int rc = check_dtype(dtype);
  if (rc != KRP_OK) return rc;
  if (nmodes < 1 || nmodes > kMaxDims) return set_error(KRP_EINVAL, "nmodes=%d outside 1..%d", nmodes, kMaxDims);
  if (!n || !ell) return set_error(KRP_EINVAL, "n and ell must not be NULL");
  for (int j = 0; j < nmodes; ++j)
    if (n[j] < 1 || ell[j] < 1 || ell[j] > n[j] || ell[j] > kSensorMaxEll)
      return set_error(KRP_EINVAL, "mode %d: need 1 <= ell=%d <= min(n=%lld, %d)", j, ell[j], (long long)n[j],
                       kSensorMaxEll);
  if (!Q || !idx || !A) return set_error(KRP_EINVAL, "Q, idx and A must not be NULL");
  for (int j = 0; j < nmodes; ++j)
    if (!Q[j] || !idx[j] || !A[j]) return set_error(KRP_EINVAL, "Q[%d], idx[%d] or A[%d] is NULL", j, j, j);
  const SelectLayout l = select_layout(nmodes, n, ell);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = nullptr;
  rc = acquire_workspace(&o, l.total, st, &ws);
  if (rc != KRP_OK) return rc;
  int* status = o.status_dev ? o.status_dev : reinterpret_cast<int*>(ws + l.status);
  SensorSelectArgs a{};
  a.nmodes = nmodes;
  a.status = status;
  std::string key = "sensor_select|dt=" + std::to_string(dtype) + "|ws=" + ptr_key(ws) + "|st=" + ptr_key(status);
  for (int j = 0; j < nmodes; ++j) {
    SensorMode& m = a.mode[j];
    m.q = Q[j];
    m.a = A[j];
    m.w = reinterpret_cast<double*>(ws + l.w[j]);
    m.taken = reinterpret_cast<unsigned char*>(ws + l.taken[j]);
    m.minv = reinterpret_cast<double*>(ws + l.minv[j]);
    m.idx = idx[j];
    m.n = n[j];
    m.ell = ell[j];
    key += "|" + std::to_string(n[j]) + "," + std::to_string(ell[j]) + "," + ptr_key(Q[j]) + "," +
           ptr_key(idx[j]) + "," + ptr_key(A[j]);
  }
  rc = run_maybe_graph(key, !(o.flags & KRP_FLAG_NO_GRAPH), st, [&](hipStream_t cs) -> int {
    if (!o.status_dev) {
      const hipError_t e = launch_fill_int(status, 0, 1, cs);
      if (e != hipSuccess) return hip_fail(e, "fill");
    }
    const hipError_t e = launch_sensor_select(a, dtype == KRP_F64 ? 1 : 0, cs);
    return e == hipSuccess ? KRP_OK : hip_fail(e, "sensor select kernels");
  });
  if (rc != KRP_OK) return rc;
  if (!o.status_dev) return finish_status(status, st);
  return KRP_OK;
}

int krp_sensor_measure(const void* T, int dtype, int d, const int64_t* dims, int64_t snapshots,
                       const int32_t* ell, const int32_t* const* idx, void* T_hat, void* stream) {
  int rc = check_dtype(dtype);
  if (rc != KRP_OK) return rc;
  rc = check_grid(d, dims, ell);
  if (rc != KRP_OK) return rc;
  if (snapshots < 1) return set_error(KRP_EINVAL, "snapshots must be >= 1");
  if (!T || !T_hat || !idx) return set_error(KRP_EINVAL, "T, T_hat and idx must not be NULL");
  SensorMeasureArgs a{};
  a.t = T;
  a.out = T_hat;
  a.d = d;
  a.total = snapshots;
  for (int i = 0; i < d; ++i) {
    if (!idx[i]) return set_error(KRP_EINVAL, "idx[%d] is NULL", i);
    a.dims[i] = dims[i];
    a.ell[i] = ell[i];
    a.idx[i] = idx[i];
    a.total *= ell[i];
  }
  const hipError_t e = launch_sensor_measure(a, dtype == KRP_F64 ? 1 : 0, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? KRP_OK : hip_fail(e, "sensor measure kernel");
}

int krp_sensor_reconstruct(const void* T_hat, int dtype, int d, const int64_t* dims, int64_t snapshots,
                           const int32_t* ell, const void* const* A, const krp_opts* opts, void* T_out,
                           void* stream) {
  const krp_opts o = opts_or_default(opts);
  int rc = check_dtype(dtype);
  if (rc != KRP_OK) return rc;
  rc = check_grid(d, dims, ell);
  if (rc != KRP_OK) return rc;
  if (snapshots < 1) return set_error(KRP_EINVAL, "snapshots must be >= 1");
  if (!T_hat || !T_out || !A) return set_error(KRP_EINVAL, "T_hat, T_out and A must not be NULL");
  for (int i = 0; i < d; ++i)
    if (!A[i]) return set_error(KRP_EINVAL, "A[%d] is NULL", i);
  const bool x64 = dtype == KRP_F64;
  const size_t esz = x64 ? 8 : 4;
  const ReconLayout l = recon_layout(d, dims, ell, snapshots, esz);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = nullptr;
  rc = acquire_workspace(&o, l.total, st, &ws);
  if (rc != KRP_OK) return rc;
  std::string key = "sensor_recon|dt=" + std::to_string(dtype) + "|s=" +
                    std::to_string(snapshots) + "|in=" + ptr_key(T_hat) + "|out=" + ptr_key(T_out) +
                    "|ws=" + ptr_key(ws);
  for (int i = 0; i < d; ++i)
    key += "|" + std::to_string(dims[i]) + "," + std::to_string(ell[i]) + "," + ptr_key(A[i]);
  return run_maybe_graph(key, !(o.flags & KRP_FLAG_NO_GRAPH), st, [&](hipStream_t cs) -> int {
    int order[kMaxDims];
    recon_order(d, dims, ell, order);
    int64_t cur[kMaxDims];
    for (int i = 0; i < d; ++i) cur[i] = ell[i];
    cur[d] = snapshots;
    const void* in = T_hat;
    for (int s = 0; s < d; ++s) {
      const int i = order[s];
      char* out = s + 1 == d ? reinterpret_cast<char*>(T_out) : ws + l.buf[s & 1];
      int64_t before = 1;  // elements of the modes ahead of mode i (already expanded)
      for (int k = 0; k < i; ++k) before *= cur[k];
      int64_t after = 1;
      for (int k = i + 1; k <= d; ++k) after *= cur[k];
      if (ell[i] <= kExpandMaxEll) {
        SensorExpandArgs ea{};
        ea.g = in;
        ea.a = A[i];
        ea.out = out;
        ea.p = before;
        ea.n = dims[i];
        ea.q = after;
        ea.ell = ell[i];
        const hipError_t e = launch_sensor_expand(ea, x64 ? 1 : 0, cs);
        if (e != hipSuccess) return hip_fail(e, "sensor expansion kernel");
        cur[i] = dims[i];
        in = out;
        continue;
      }
      // wider reductions: TTM with the factor transposed to fp64, 64 output columns at a time
      double* at = reinterpret_cast<double*>(ws + l.at[i]);
      hipError_t e = launch_sensor_transpose(A[i], x64 ? 1 : 0, dims[i], ell[i], at, cs);
      if (e != hipSuccess) return hip_fail(e, "sensor transpose kernel");
      for (int64_t c0 = 0; c0 < dims[i]; c0 += kTtmChunk) {
        TtmProblem tp;
        tp.g = in;
        tp.g_is_double = x64 ? 1 : 0;
        tp.d = d + 1;
        for (int k = 0; k <= d; ++k) tp.dims[k] = cur[k];
        tp.mode = i;
        tp.ell = (int)std::min<int64_t>(kTtmChunk, dims[i] - c0);
        tp.prec = x64 ? KRP_P_FP64 : KRP_P_FP32;
        tp.q64 = at + (size_t)ell[i] * c0;
        tp.out = out + (size_t)(c0 * before) * esz;
        tp.out_is_double = x64 ? 1 : 0;
        tp.out_ld = dims[i];
        e = launch_ttm(tp, cs);
        if (e != hipSuccess) return hip_fail(e, "sensor reconstruction ttm");
      }
      cur[i] = dims[i];
      in = out;
    }
    return KRP_OK;
  });
}

int krp_sensor_workspace_size(int which, int d, const int64_t* dims, const int32_t* ell, int64_t snapshots,
                              int dtype, size_t* bytes) {
  if (!bytes) return set_error(KRP_EINVAL, "bytes is NULL");
  int rc = check_dtype(dtype);
  if (rc != KRP_OK) return rc;
  if (which == 0) {
    if (d < 1 || d > kMaxDims || !dims || !ell) return set_error(KRP_EINVAL, "bad shape arguments");
    for (int j = 0; j < d; ++j)
      if (dims[j] < 1 || ell[j] < 1 || ell[j] > dims[j] || ell[j] > kSensorMaxEll)
        return set_error(KRP_EINVAL, "mode %d: need 1 <= ell <= min(n, %d)", j, kSensorMaxEll);
    *bytes = select_layout(d, dims, ell).total;
    return KRP_OK;
  }
  if (which != 1) return set_error(KRP_EINVAL, "which must be 0 (select) or 1 (reconstruct)");
  rc = check_grid(d, dims, ell);
  if (rc != KRP_OK) return rc;
  if (snapshots < 1) return set_error(KRP_EINVAL, "snapshots must be >= 1");
  *bytes = recon_layout(d, dims, ell, snapshots, dtype == KRP_F64 ? 8 : 4).total;
  return KRP_OK;
}

}  // extern "C"
