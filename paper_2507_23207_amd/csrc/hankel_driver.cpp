// Driver of krp_hankel_lowrank (Algorithm 6 on block-Hankel matrices):
// validation, grouping of the batch, workspace and graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/krp.h"
#include "driver.h"
#include "hankel.h"
#include "kernels.h"

namespace krp {
namespace {

struct Group {
  int first, count;
  int64_t h_off, u_off, v_off, s_off;
  HankelPlan plan;
  size_t ws_off;
};

int plan_groups(int batch, const int64_t* s, int m, int n, int r, int ell_r, int ell_l, int is_double,
                std::vector<Group>& groups, size_t& total) {
  groups.clear();
  total = 0;
  int64_t h_off = 0, u_off = 0, v_off = 0;
  for (int first = 0; first < batch; first += kHankelGroup) {
    Group g;
    g.first = first;
    g.count = std::min(kHankelGroup, batch - first);
    g.h_off = h_off;
    g.u_off = u_off;
    g.v_off = v_off;
    g.s_off = (int64_t)first * r;
    g.plan = plan_hankel(g.count, s + first, m, n, r, ell_r, ell_l, is_double);
    if (g.plan.sketch_lds > hankel_lds_limit())
      return set_error(KRP_EINVAL, "block count s=%lld is too large for the LDS-resident sketch",
                       (long long)g.plan.s_max);
    g.ws_off = total;
    total = align_up(total + g.plan.ws_bytes);
    for (int b = first; b < first + g.count; ++b) {
      h_off += (2 * s[b] - 1) * (int64_t)m * n;
      u_off += (int64_t)m * s[b] * r;
      v_off += (int64_t)n * s[b] * r;
    }
    groups.push_back(g);
  }
  total = align_up(total + 64);  // shared status word
  return KRP_OK;
}

int validate(int batch, const int64_t* s, int m, int n, int r, int ell_r, int& ell_l) {
  if (batch < 1) return set_error(KRP_EINVAL, "batch must be >= 1");
  if (!s) return set_error(KRP_EINVAL, "s is NULL");
  if (m < 1 || n < 1 || m > kHankelMaxBlock || n > kHankelMaxBlock)
    return set_error(KRP_EINVAL, "block sizes m=%d, n=%d outside 1..%d", m, n, kHankelMaxBlock);
  if (ell_l == 0) ell_l = (3 * ell_r + 1) / 2;
  if (r < 1 || r > ell_r) return set_error(KRP_EINVAL, "need 1 <= r <= ell_r");
  if (ell_r > ell_l) return set_error(KRP_EINVAL, "need ell_r <= ell_l");
  if (ell_l > kHankelMaxEll) return set_error(KRP_EINVAL, "ell_l=%d exceeds the supported %d", ell_l, kHankelMaxEll);
  for (int b = 0; b < batch; ++b) {
    if (s[b] < 1) return set_error(KRP_EINVAL, "s[%d] must be >= 1", b);
    if ((int64_t)m * s[b] < ell_r || (int64_t)n * s[b] < ell_r)
      return set_error(KRP_EINVAL, "instance %d: ell_r=%d exceeds m s or n s", b, ell_r);
    if (s[b] > (1 << 20)) return set_error(KRP_EINVAL, "s[%d] too large", b);
  }
  return KRP_OK;
}

}  // namespace
}  // namespace krp

using namespace krp;

extern "C" {

int krp_hankel_lowrank(int batch, const int64_t* s, int m, int n, const void* h, int dtype, int r,
                       int ell_r, int ell_l, const krp_opts* opts, void* U, void* S, void* V,
                       void* stream) {
  krp_opts o;
  if (opts)
    o = *opts;
  else
    krp_opts_default(&o);
  int rc = validate(batch, s, m, n, r, ell_r, ell_l);
  if (rc != KRP_OK) return rc;
  if (!h || !U || !S || !V) return set_error(KRP_EINVAL, "h, U, S and V must not be NULL");
  if (dtype != KRP_F64 && dtype != KRP_F32) return set_error(KRP_EINVAL, "unknown dtype %d", dtype);
  if (o.prec < KRP_P_FP64 || o.prec > KRP_P_BF16X3) return set_error(KRP_EINVAL, "unknown precision");
  const int is_double = dtype == KRP_F64;
  if (is_double && o.prec != KRP_P_FP64) return set_error(KRP_EINVAL, "fp64 data requires KRP_P_FP64");
  if (!is_double && o.prec != KRP_P_FP32)
    return set_error(KRP_EINVAL, "the Hankel sketch of fp32 data runs in fp32: opts->prec must be KRP_P_FP32");
  std::vector<Group> groups;
  size_t total = 0;
  rc = plan_groups(batch, s, m, n, r, ell_r, ell_l, is_double, groups, total);
  if (rc != KRP_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = nullptr;
  rc = acquire_workspace(&o, total, st, &ws);
  if (rc != KRP_OK) return rc;
  int* status = o.status_dev ? o.status_dev : reinterpret_cast<int*>(ws + total - 64);
  std::string key = "hankel|" + std::to_string(batch) + "|" + std::to_string(m) + "," + std::to_string(n) +
                    "," + std::to_string(r) + "," + std::to_string(ell_r) + "," + std::to_string(ell_l) +
                    "|dt=" + std::to_string(dtype) + "|seed=" + std::to_string(o.seed) +
                    "|draw=" + std::to_string(o.draw) + "|h=" + ptr_key(h) + "|U=" + ptr_key(U) +
                    "|S=" + ptr_key(S) + "|V=" + ptr_key(V) + "|ws=" + ptr_key(ws) + "|st=" + ptr_key(status) + "|s=";
  for (int b = 0; b < batch; ++b) key += std::to_string(s[b]) + ",";
  const size_t esz = is_double ? 8 : 4;
  rc = run_maybe_graph(key, !(o.flags & KRP_FLAG_NO_GRAPH), st, [&](hipStream_t cs) -> int {
    if (!o.status_dev) {
      hipError_t e = launch_fill_int(status, 0, 1, cs);
      if (e != hipSuccess) return hip_fail(e, "fill");
    }
    for (const Group& g : groups) {
      const hipError_t e = launch_hankel(
          g.plan, s + g.first, reinterpret_cast<const char*>(h) + g.h_off * esz, o.seed, o.draw,
          reinterpret_cast<char*>(U) + g.u_off * esz, reinterpret_cast<char*>(S) + g.s_off * esz,
          reinterpret_cast<char*>(V) + g.v_off * esz, ws + g.ws_off, status, cs);
      if (e != hipSuccess) return hip_fail(e, "hankel kernels");
    }
    return KRP_OK;
  });
  if (rc != KRP_OK) return rc;
  if (!o.status_dev) return finish_status(status, st);
  return KRP_OK;
}

int krp_hankel_workspace_size(int batch, const int64_t* s, int m, int n, int r, int ell_r, int ell_l,
                              size_t* bytes) {
  if (!bytes) return set_error(KRP_EINVAL, "bytes is NULL");
  int rc = validate(batch, s, m, n, r, ell_r, ell_l);
  if (rc != KRP_OK) return rc;
  std::vector<Group> groups;
  size_t total = 0;
  rc = plan_groups(batch, s, m, n, r, ell_r, ell_l, 0, groups, total);
  if (rc != KRP_OK) return rc;
  *bytes = total;  // the fp64 buffers of the pipeline do not depend on the storage type
  return KRP_OK;
}

}  // extern "C"
