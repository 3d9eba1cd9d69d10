// Batched block-Hankel single-pass SVD (Algorithm 6): plan and launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace krp {

constexpr int kHankelGroup = 512;   // instances per launch group (s[] travels by value)
constexpr int kHankelMaxEll = 48;   // ell_r, ell_l limit of the completion kernels
constexpr int kHankelMaxBlock = 64; // m, n limit
constexpr int kHankelChRows = 256;  // rows of Y and of Z per completion chunk
constexpr int kHankelPasses = 5;    // CholeskyQR passes at most (shifted CholeskyQR3 included)

// Device tables built by the setup kernel (all in the workspace).
struct HankelTables {
  int64_t* s;
  int64_t* h_off;   // first element of instance b's blocks
  int64_t* y_off;   // Y_b (m s x ell_r, column-major) in the Y buffer
  int64_t* z_off;   // Z_b (n s x ell_l)
  int64_t* u_off;   // U_b (m s x r) in the output
  int64_t* v_off;   // V_b (n s x r)
  int64_t* ch_off;  // first completion chunk of instance b
  int64_t* p_off;   // P sequences of instance b (both sides) in the P buffer
  int64_t* f_off;   // filter columns (Omega1, then Psi1) of instance b
  int32_t* order;   // instances by decreasing s (ties: lower index first)
  int32_t* chunk_inst;  // instance of each completion chunk
  int32_t* state;   // CholeskyQR pass state of each instance
  int32_t* queue;   // work counter of the persistent sketch launch
};

struct HankelPlan {
  int batch, m, n, r, ell_r, ell_l, is_double;
  int64_t s_max, s_sum;
  int n_chunks;
  // sketch items: per side (0: Y, 1: Z), rows of a block per item (rp),
  // output shift groups per MFMA tile (hs) and row chunks per block (ach)
  int rp[2], hs[2], ach[2];
  int items_side0, items_per_inst;
  int fl_cap, kp_cap;
  size_t sketch_lds;
  int sketch_grid;
  int pseq_kc, pseq_chunks;  // P-sequence kernel: blocks per workgroup, workgroups per instance
  size_t pseq_lds;
  size_t off_tab, off_pall, off_filt, off_y, off_z, off_part, off_rinv, off_t, off_gz, off_k, off_mp, off_uw, off_ev, off_bu,
      off_bv, off_am, ws_bytes;
};

HankelPlan plan_hankel(int batch, const int64_t* s, int m, int n, int r, int ell_r, int ell_l,
                       int is_double);
// Largest dynamic LDS the sketch launch may use (bytes).
size_t hankel_lds_limit();
HankelTables hankel_tables(const HankelPlan& p, char* ws);
// Enqueues the whole pipeline for one group of at most kHankelGroup instances.
hipError_t launch_hankel(const HankelPlan& p, const int64_t* s_host, const void* h, uint64_t seed,
                         uint32_t draw, void* U, void* S, void* V, char* ws, int* status,
                         hipStream_t st);

}  // namespace krp
