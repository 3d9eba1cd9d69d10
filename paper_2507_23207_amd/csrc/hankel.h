// Batched block-Hankel single-pass SVD (Algorithm 6): plan and launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace krp {

constexpr int kHankelGroup = 512;   // instances per launch group (s[] travels by value)
constexpr int kHankelMaxEll = 48;   // ell_r, ell_l limit of the completion kernels
constexpr int kHankelMaxBlock = 64; // m, n limit

// Device tables built by the setup kernel (all in the workspace).
struct HankelTables {
  int64_t* s;
  int64_t* h_off;
  int64_t* y_off;
  int64_t* z_off;
  int64_t* w_off;
  int64_t* u_off;
  int64_t* v_off;
  int64_t* y_rows;
  int32_t* order;   // instances by decreasing s (ties: lower index first)
};

struct HankelPlan {
  int batch, m, n, r, ell_r, ell_l, is_double;
  int64_t s_max, s_sum;
  int nc[2], nrho[2], cchunks[2], rchunks[2];
  int items_side0, items_per_inst;
  size_t lds[2], lds_max;
  size_t off_tab, off_y, off_z, off_w, off_gw, off_uw, off_ev, off_status, ws_bytes;
};

HankelPlan plan_hankel(int batch, const int64_t* s, int m, int n, int r, int ell_r, int ell_l,
                       int is_double);
HankelTables hankel_tables(const HankelPlan& p, char* ws);
// Enqueues the whole pipeline for one group of at most kHankelGroup instances.
hipError_t launch_hankel(const HankelPlan& p, const int64_t* s_host, const void* h, uint64_t seed,
                         uint32_t draw, void* U, void* S, void* V, char* ws, int* status,
                         hipStream_t st);

}  // namespace krp
