// KRP sketch of one mode unfolding of a dense tensor (the MTTKRP of
// Algorithm 7, step 3 and Algorithm 8, step 4):
//   Y_(i) = X_(i) (Omega_d kr ... kr Omega_{i+1} kr Omega_{i-1} kr ... kr Omega_1).
// The Khatri-Rao product is never formed.  The tensor is viewed as
//   x[i_f, a, o]   (a = i_mode, f = fastest other mode, o = remaining modes)
// and every column of the KRP factorises as Omega_f[i_f, c] * W[o, c] with
// W[o, c] = prod_{k in o} Omega_k[o_k, c].  A workgroup owns a 32-wide block
// of i_f, a range of o and all (or a block of) rows a; it draws the factor rows
// it needs into LDS with the counter-based generator, then streams its slab of
// X once: each 16-row x 32-deep slice of X is an MFMA A fragment, the matching
// KRP weights (Omega_f slice times W[o, :]) the B fragment.  Per-workgroup
// partial sums are reduced deterministically (fixed order, fp64) by a second
// kernel.
#include "sketch_kernel.h"

#include <algorithm>

namespace krp {

namespace {

using skdetail::SketchArgs;
using skdetail::kLoadScalar;
using skdetail::kLoadVecF;
using skdetail::kLoadXpose;

// Y[a, c] = sum_p partial[z][p][a][c mod CP] (z = c / CP; rows of a chunk
// hold its real columns only), summed in fp64.
// A workgroup owns kRedRows rows of one column chunk; its threads are split
// into `tpe` groups that sum interleaved subsets of the partials, combined in
// LDS in a fixed order, so the result does not depend on scheduling.
constexpr int kRedThreads = 512;
constexpr int kRedRows = 1;

template <typename AccT>
__global__ __launch_bounds__(kRedThreads) void sketch_reduce_kernel(
    const AccT* __restrict__ partial, int nparts, int64_t n_rows, int ell, int cp,
    double* __restrict__ y64, void* yout, int out_double) {
  __shared__ double red[kRedThreads];
  const int z = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * kRedRows;
  const int cpz = min(cp, ell - z * cp);  // real columns of this chunk (the partials' row stride)
  const int E = kRedRows * cpz;       // elements of this block (<= 64)
  const int tpe = kRedThreads / E;    // threads per element (>= 8)
  const int t = threadIdx.x;
  const int e = t % E, sub = t / E;
  const int64_t a = r0 + e / cpz;
  const int cc = e % cpz;
  const int64_t stride = n_rows * cpz;
  double s = 0.0;
  if (sub < tpe && a < n_rows) {
    const AccT* p = partial + (int64_t)z * nparts * n_rows * cp + a * cpz + cc;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = sub;
    for (; q + 7 * tpe < nparts; q += 8 * tpe) {
      const double v0 = (double)p[(int64_t)q * stride];
      const double v1 = (double)p[(int64_t)(q + tpe) * stride];
      const double v2 = (double)p[(int64_t)(q + 2 * tpe) * stride];
      const double v3 = (double)p[(int64_t)(q + 3 * tpe) * stride];
      const double v4 = (double)p[(int64_t)(q + 4 * tpe) * stride];
      const double v5 = (double)p[(int64_t)(q + 5 * tpe) * stride];
      const double v6 = (double)p[(int64_t)(q + 6 * tpe) * stride];
      const double v7 = (double)p[(int64_t)(q + 7 * tpe) * stride];
      s0 += v0 + v4;
      s1 += v1 + v5;
      s2 += v2 + v6;
      s3 += v3 + v7;
    }
    for (; q < nparts; q += tpe) s0 += (double)p[(int64_t)q * stride];
    s = (s0 + s1) + (s2 + s3);
  }
  red[t] = s;
  __syncthreads();
  if (sub == 0 && a < n_rows) {
    double tot = red[e];
    for (int k = 1; k < tpe; ++k) tot += red[e + k * E];
    const int c = z * cp + cc;
    if (c < ell) {
      const int64_t o = a + n_rows * c;
      if (y64) y64[o] = tot;
      if (yout) {
        if (out_double)
          reinterpret_cast<double*>(yout)[o] = tot;
        else
          reinterpret_cast<float*>(yout)[o] = (float)tot;
      }
    }
  }
}

__global__ void gaussian_kernel(uint64_t seed, uint64_t w2, uint64_t instance, int64_t rows,
                                int64_t cols, int prec, void* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t r = idx % rows, c = idx / rows;
  const double gv = gauss_entry(seed, w2, instance, (uint64_t)r, (uint64_t)c);
  if (prec == kFP64) {
    reinterpret_cast<double*>(out)[idx] = gv;
  } else if (prec == kFP32) {
    reinterpret_cast<float*>(out)[idx] = (float)gv;
  } else {
    const float x = (float)gv;
    const __bf16 h = (__bf16)x;
    reinterpret_cast<__bf16*>(out)[idx] = h;
    if (prec == kBF16X3) reinterpret_cast<__bf16*>(out)[rows * cols + idx] = (__bf16)(x - (float)h);
  }
}

}  // namespace

constexpr int64_t kMaxWaveSteps = 64;

SketchPlan plan_sketch(const SketchProblem& pb, const SketchTile& tile) {
  SketchPlan p{};
  int64_t stride[kMaxDims];
  int64_t s = 1;
  for (int k = 0; k < pb.d; ++k) {
    stride[k] = s;
    s *= pb.dims[k];
  }
  const int i = pb.mode;
  p.fmode = (i == 0) ? 1 : 0;
  p.n_rows = pb.dims[i];
  p.s_row = stride[i];
  p.n_f = pb.dims[p.fmode];
  p.s_f = stride[p.fmode];
  p.n_out = 0;
  p.o_total = 1;
  for (int k = 0; k < pb.d; ++k) {
    if (k == i || k == p.fmode) continue;
    p.o_size[p.n_out] = pb.dims[k];
    p.o_stride[p.n_out] = stride[k];
    p.o_fid[p.n_out] = k;
    p.o_total *= pb.dims[k];
    ++p.n_out;
  }
  const bool fp64 = pb.prec == kFP64;
  const size_t tsz = fp64 ? 8 : 4;
  p.nt = pb.ell >= 64 ? 4 : (pb.ell + 15) / 16;
  p.cpad = 16 * p.nt;
  p.col_chunks = (pb.ell + p.cpad - 1) / p.cpad;
  int mt = tile.mt;
  if (mt != 1 && mt != 2) mt = 4;
  while (mt > 1 && 16 * (mt / 2) >= p.n_rows) mt /= 2;
  // Mode 0 reads rows along the contiguous index.  Scalar (strided) loads
  // need one 64-bit address per element: keep the register budget within two
  // waves per SIMD by halving the row tiles.  The staged 16-byte path
  // (fp32 storage, 16-byte aligned data, n_0 a multiple of 4) keeps 64 rows.
  const int64_t vlen = 16 / (pb.x_is_double ? 8 : 4);
  const bool x_aligned = (reinterpret_cast<uintptr_t>(pb.x) & 15) == 0;
  p.xpose = (i == 0) && pb.d >= 2 && (p.n_rows % vlen == 0);
  if (i == 0 && mt > 2 && !(p.xpose && x_aligned && !pb.x_is_double)) mt = 2;
  if (fp64 && mt > 2 && p.nt >= 3) mt = 2;  // register budget of fp64 fragments
  p.mt = mt;
  const int64_t wave_rows = 16 * mt;
  int wm = tile.wm > 0 ? tile.wm : (int)std::min<int64_t>(8, (p.n_rows + wave_rows - 1) / wave_rows);
  p.wm = std::max(1, std::min(8, wm));
  p.row_blocks = (int)((p.n_rows + wave_rows * p.wm - 1) / (wave_rows * p.wm));
  int wo = tile.wo > 0 ? tile.wo : std::max(1, 8 / p.wm);
  while (p.wm * wo > 8) --wo;
  p.wo = std::max(1, wo);
  p.f_blocks = (int)((p.n_f + 31) / 32);
  p.kvec = (i != 0) && (p.n_f % vlen == 0);

  int64_t o_per = tile.o_per_wg;
  if (o_per <= 0) {
    const int64_t per_o = (int64_t)p.f_blocks * p.row_blocks * p.col_chunks;
    int64_t ranges = std::max<int64_t>(1, tile.target_wgs / std::max<int64_t>(1, per_o));
    ranges = std::min(ranges, p.o_total);
    o_per = (p.o_total + ranges - 1) / ranges;
  }
  o_per = std::max<int64_t>(1, std::min(o_per, p.o_total));
  // A wave accumulates at most kMaxWaveSteps outer steps in its fp32 (or
  // policy) accumulators before the partial goes to the fp64 reduction: the
  // rounding error of a long fp32 sum grows with its length, and long sums
  // (e.g. 64^5 tensors, 64^4 terms per output) would otherwise cost accuracy.
  o_per = std::min<int64_t>(o_per, (int64_t)kMaxWaveSteps * p.wo);
  // Keep the LDS factor tables under 64 KiB.
  for (;;) {
    int64_t rows = 32, period = 1;
    for (int k = 0; k < p.n_out; ++k) {
      rows += std::min<int64_t>(p.o_size[k], (o_per + period - 1) / period + 1);
      period *= p.o_size[k];
    }
    p.lds_rows = (int)rows;
    p.lds_bytes = (size_t)rows * p.cpad * tsz;
    if (p.lds_bytes <= 65536 || o_per == 1) break;
    o_per = (o_per + 1) / 2;
  }
  p.o_per_wg = o_per;
  p.stage_bytes = (size_t)8 * 32 * (16 * p.mt + 2) * (pb.x_is_double ? 8 : 4);  // 8 waves (upper bound)
  p.o_ranges = (int)((p.o_total + o_per - 1) / o_per);
  p.nparts = p.f_blocks * p.o_ranges * p.wo;
  p.partial_bytes = (size_t)p.col_chunks * p.nparts * p.n_rows * p.cpad * tsz;
  return p;
}

hipError_t launch_sketch(const SketchProblem& pb, const SketchPlan& p, void* partial, double* y64,
                         void* y_out, int out_is_double, hipStream_t st) {
  SketchArgs a{};
  a.x = pb.x;
  a.partial = partial;
  a.n_rows = p.n_rows;
  a.s_row = p.s_row;
  a.n_f = p.n_f;
  a.s_f = p.s_f;
  int64_t period = 1;
  for (int k = 0; k < kMaxDims; ++k) {
    a.o_size[k] = k < p.n_out ? p.o_size[k] : 1;
    a.o_stride[k] = k < p.n_out ? p.o_stride[k] : 0;
    a.o_fid[k] = k < p.n_out ? p.o_fid[k] : 0;
    a.o_period[k] = period;
    if (k < p.n_out) period *= p.o_size[k];
  }
  a.n_out = p.n_out;
  a.o_total = p.o_total;
  a.o_per_wg = p.o_per_wg;
  a.f_blocks = p.f_blocks;
  a.ell = pb.ell;
  a.nparts = p.nparts;
  a.wm = p.wm;
  a.wo = p.wo;
  a.rows_per_wg = 16 * p.mt * p.wm;
  a.fid_f = p.fmode;
  a.lds_rows = p.lds_rows;
  a.seed = pb.seed;
  a.w2_base = counter_word2(pb.draw, pb.sketch_id, 0);

  // Vector loads need 16-byte aligned rows; misaligned views take the scalar path.
  const bool aligned = (reinterpret_cast<uintptr_t>(pb.x) & 15) == 0;
  int lm = kLoadScalar;
  if (aligned && p.kvec) lm = kLoadVecF;
  if (aligned && p.xpose) lm = kLoadXpose;
  size_t lds = p.lds_bytes;
  a.stage_off = (int64_t)((lds + 15) / 16 * 16);
  if (lm == kLoadXpose) lds = (size_t)a.stage_off + p.stage_bytes;
  const dim3 grid((unsigned)(p.f_blocks * p.o_ranges), (unsigned)p.row_blocks, (unsigned)p.col_chunks);
  const int threads = 64 * p.wm * p.wo;
  hipError_t e;
  if (pb.x_is_double) {
    if (pb.prec != kFP64) return hipErrorInvalidValue;
    e = skdetail::dispatch_fp64(true, lm, p.mt, p.nt, a, grid, threads, lds, st);
  } else {
    switch (pb.prec) {
      case kFP64: e = skdetail::dispatch_fp64(false, lm, p.mt, p.nt, a, grid, threads, lds, st); break;
      case kFP32: e = skdetail::dispatch_fp32(lm, p.mt, p.nt, a, grid, threads, lds, st); break;
      case kBF16: e = skdetail::dispatch_bf16(lm, p.mt, p.nt, a, grid, threads, lds, st); break;
      default: e = skdetail::dispatch_bf16x3(lm, p.mt, p.nt, a, grid, threads, lds, st); break;
    }
  }
  if (e != hipSuccess) return e;
  const dim3 rg((unsigned)((p.n_rows + kRedRows - 1) / kRedRows), (unsigned)p.col_chunks);
  if (pb.prec == kFP64)
    hipLaunchKernelGGL(sketch_reduce_kernel<double>, rg, dim3(kRedThreads), 0, st,
                       reinterpret_cast<const double*>(partial), p.nparts, p.n_rows, pb.ell, p.cpad,
                       y64, y_out, out_is_double);
  else
    hipLaunchKernelGGL(sketch_reduce_kernel<float>, rg, dim3(kRedThreads), 0, st,
                       reinterpret_cast<const float*>(partial), p.nparts, p.n_rows, pb.ell, p.cpad,
                       y64, y_out, out_is_double);
  return hipGetLastError();
}

hipError_t launch_gaussian(uint64_t seed, uint64_t w2, uint64_t instance, int64_t rows, int64_t cols,
                           int prec, void* out, hipStream_t st) {
  const int64_t n = rows * cols;
  if (n == 0) return hipSuccess;
  const int t = 256;
  hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)((n + t - 1) / t)), dim3(t), 0, st, seed, w2,
                     instance, rows, cols, prec, out);
  return hipGetLastError();
}

}  // namespace krp
