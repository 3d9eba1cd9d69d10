// Host-side launch interfaces of the libkrp HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace krp {

constexpr int kMaxDims = 8;

// Tiling of one mode sketch (chosen by the planner or the autotuner).
struct SketchTile {
  int mt = 4;         // 16-row M tiles per wave
  int wm = 0;         // waves along the rows (0: derived from the row count)
  int wo = 0;         // waves splitting the outer iterations (0: derived)
  int64_t o_per_wg = 0;  // outer iterations per workgroup (0: derived)
  int target_wgs = 256;  // workgroups aimed for when deriving o_per_wg
  int waves = 8;         // waves per workgroup (wm * wo <= waves)
};

// Problem description of a single-mode MTTKRP sketch
//   Y[a, c] = sum_{all i_k, k != mode; i_mode = a} x[i] prod_{k != mode} Omega_k[i_k, c]
// for a dense tensor in Kolda order (mode 0 fastest).
struct SketchProblem {
  const void* x = nullptr;
  int x_is_double = 0;
  int d = 0;
  int64_t dims[kMaxDims] = {0};
  int mode = 0;
  int ell = 0;
  int prec = 0;               // Prec
  uint64_t seed = 0;
  uint32_t draw = 0;
  uint32_t sketch_id = 0;     // counter field "sketch" (normally == mode; kMemoSketch: shared set)
};

// Counter field "sketch" of the shared factor set of RHOSVD-KRP-MEMO.
constexpr uint32_t kMemoSketch = 0xFFFF;

struct SketchPlan {
  int fmode, n_out;
  int64_t n_rows, s_row, n_f, s_f;
  int64_t o_size[kMaxDims], o_stride[kMaxDims];
  int o_fid[kMaxDims];
  int64_t o_total, o_per_wg;
  int o_ranges, f_blocks, row_blocks, col_chunks;
  int mt, nt, wm, wo, kvec, kvec2, rowvec;  // kvec2: 8-byte loads along f (fp32, even n_f)
  int cpad, nparts;       // nparts: one partial per workgroup (f block, o range)
  int nseg;               // level-1 segments of the reduction (1: single level)
  int lds_rows;           // factor-table rows the LDS allocation holds
  size_t lds_bytes;
  size_t lvl_off;         // byte offset of the level-1 sums (nseg > 1)
  size_t partial_bytes;   // bytes of the partial-sum buffer (and level-1 sums)
};

SketchPlan plan_sketch(const SketchProblem& pb, const SketchTile& tile);

// The fastest tiling of this sketch shape: from the tuning table (memory, then
// the JSON cache file), else timed now on pb.x over the candidate tilings on
// `st` (median of repeated launches; a candidate replaces the default tiling
// only when it is faster by a margin).  Never while `st` is capturing: the
// default tile is returned then.
SketchTile tuned_tile(const SketchProblem& pb, hipStream_t st);
// The tuned tiling of this shape if the table (memory or cache file) holds
// one; never launches anything.
bool cached_tile(const SketchProblem& pb, SketchTile* out);

// Launches the sketch of one mode: partial sums into `partial` (workspace of
// plan.partial_bytes), then the deterministic reduction into y64 (fp64,
// n_rows x ell column-major) and, if y_out is not null, into y_out in the
// storage type (double when out_is_double).
hipError_t launch_sketch(const SketchProblem& pb, const SketchPlan& plan, void* partial,
                         double* y64, void* y_out, int out_is_double, hipStream_t st);

// Deterministic fp64 reduction of per-workgroup partial sums: `partial` holds,
// per column chunk z of width cp, nparts blocks of n_rows x ncz_z values
// (ncz_z = min(cp, ell - z cp)), fp32 (acc_double: fp64); Y (n_rows x ell,
// column-major) goes to y64 and/or y_out.  `lvl` holds
// partial_reduce_lvl_bytes() bytes of level-1 sums.
size_t partial_reduce_lvl_bytes(int nparts, int64_t n_rows, int cp, int col_chunks);
hipError_t launch_partial_reduce(const void* partial, bool acc_double, int nparts, int64_t n_rows, int ell,
                                 int cp, int col_chunks, void* lvl, double* y64, void* y_out,
                                 int out_is_double, hipStream_t st);

// One pass over X for several mode sketches of the same tensor (all-mode
// fused kernel); see fused.hip.
struct FusedPlan {
  bool ok = false;
  alignas(8) unsigned char args[2560];
  size_t args_bytes = 0;
  int nt = 0;
  size_t lds = 0;
  int64_t grid_x = 0;
  int grid_y = 0;
  int64_t nparts[kMaxDims] = {0};
  size_t part_off[kMaxDims] = {0}, lvl_off[kMaxDims] = {0};
  size_t ws_bytes = 0;
};
FusedPlan plan_fused(const SketchProblem* pbs, int nmodes);
// y64[j] / y_out[j] (either may be null, or the arrays themselves) receive the
// sketch of pbs[j]; ws holds fp.ws_bytes.
hipError_t launch_fused(const FusedPlan& fp, const SketchProblem* pbs, int nmodes, void* ws,
                        double* const* y64, void* const* y_out, int out_is_double, hipStream_t st);

// Fills out (rows x cols, column-major) with the factor entries of the RNG
// spec in precision prec (0 fp64, 1 fp32, 2 bf16 bits, 3 bf16 hi plane then
// lo plane).
hipError_t launch_gaussian(uint64_t seed, uint64_t w2, uint64_t instance, int64_t rows,
                           int64_t cols, int prec, void* out, hipStream_t st);

// Batched CholeskyQR2 of column-major fp64 matrices Y_b (n_b x ell), with a
// shifted CholeskyQR3 fallback.  q64 receives Q_b in fp64 (may alias y64),
// q_out (optional) in the storage type.  offsets[b] is the element offset of
// matrix b (device array, or null for a single matrix at offset 0), nrows[b]
// its row count (device array, or null: all have n rows).
hipError_t launch_cholqr(int batch, int64_t n, int ell, const double* y64, double* q64,
                         void* q_out, int out_is_double, const int64_t* offsets,
                         const int64_t* nrows, int* status, hipStream_t st);

// The same for one matrix (q64 distinct from y64), with the streaming passes
// split over workgroups of row chunks; ws holds cholqr_split_bytes(n, ell)
// bytes.  Small n falls back to launch_cholqr.
size_t cholqr_split_bytes(int64_t n, int ell);
hipError_t launch_cholqr_split(int64_t n, int ell, const double* y64, double* q64, void* q_out,
                               int out_is_double, void* ws, int* status, hipStream_t st);

// TTM G_new = G x_mode Q^T for a tensor in Kolda order with current sizes
// dims (dims[mode] = n rows of Q), Q (n x ell, fp64 column-major).  With
// out_ld > ell the output mode has extent out_ld and these ell columns are a
// chunk of it: `out` then points at the chunk's first column (element offset
// c0 for mode 0, c0 * prod(dims before mode) otherwise).
// Tiling of a TTM of a mode after the first (the autotuner's choice):
// split < 0 keeps the planner's choice, 0 one wave per item, 1 the split
// kernel (the reduction spread over the waves of a workgroup) with nt p tiles
// per workgroup (0: the planner's).  Mode 1 has a single tiling.
struct TtmTile {
  int split = -1;
  int nt = 0;
};

struct TtmProblem {
  const void* g = nullptr;
  int g_is_double = 0;
  void* out = nullptr;
  int out_is_double = 0;
  int d = 0;
  int64_t dims[kMaxDims] = {0};
  int mode = 0;
  int ell = 0;
  int prec = 0;
  const double* q64 = nullptr;
  int64_t out_ld = 0;  // 0: ell
  TtmTile tile;
  // mode 1 only: write zeros to the output columns ell..out_ld-1 (a padded
  // extent of the compressed mode)
  bool zero_pad = false;
};
hipError_t launch_ttm(const TtmProblem& pb, hipStream_t st);
// Candidate tilings of a TTM problem (the default first); mode 1 has one.
int ttm_tile_candidates(const TtmProblem& pb, TtmTile* out, int max);
// The fastest TTM tiling of this shape (tuning table, else timed now on
// pb.g / pb.q64 into a scratch output, median of repeated launches, kept only
// when faster than the default by a margin); never while `st` is capturing.
TtmTile tuned_ttm_tile(const TtmProblem& pb, hipStream_t st);
bool cached_ttm_tile(const TtmProblem& pb, TtmTile* out);

// Casts between storage types (count elements).
hipError_t launch_cast(const void* in, int in_is_double, void* out, int out_is_double,
                       int64_t count, hipStream_t st);
// Sum of squares of a storage-type array into *acc (fp64, cleared first).
hipError_t launch_sumsq(const void* x, int is_double, int64_t count, double* acc,
                        double* scratch, int scratch_len, hipStream_t st);
// dst (rows x cols, leading dimension rows) = the first rows rows of src
// (leading dimension src_ld): removes the padding of a tensor's first mode.
hipError_t launch_compact_rows(const void* src, int64_t src_ld, void* dst, int64_t rows, int64_t cols, int is_double,
                               hipStream_t st);
// Fills count ints with value (graph-safe replacement for memset).
hipError_t launch_fill_int(int* p, int value, int64_t count, hipStream_t st);

}  // namespace krp
