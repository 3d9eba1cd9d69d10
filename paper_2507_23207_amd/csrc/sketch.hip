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
using skdetail::kLoadRowVec;

// Deterministic fp64 reduction of the per-workgroup partial sums.  Chunk z
// of the columns holds nparts partials of E_z = n_rows * ncz_z values (ncz_z
// its real columns), one after the other.  Level 1: workgroup (element block,
// segment, chunk) sums the partials of its segment, in order, one thread per
// element (coalesced across threads); with a single segment it writes Y
// directly, otherwise its fp64 sums go to `lvl`, and level 2 adds the
// segments in order.  The summation order is fixed, so the result does not
// depend on scheduling.
constexpr int kRedThreads = 256;
constexpr int kRedSeg = 32;  // partials per level-1 segment

__device__ __forceinline__ void store_y(int64_t e, int ncz, int64_t n_rows, int col0, double v, double* y64,
                                        void* yout, int out_double) {
  const int64_t a = e / ncz;
  const int c = col0 + (int)(e - a * ncz);
  const int64_t o = a + n_rows * c;
  if (y64) y64[o] = v;
  if (yout) {
    if (out_double)
      reinterpret_cast<double*>(yout)[o] = v;
    else
      reinterpret_cast<float*>(yout)[o] = (float)v;
  }
}

template <typename AccT>
__global__ __launch_bounds__(kRedThreads) void sketch_reduce1_kernel(
    const AccT* __restrict__ partial, int nparts, int64_t n_rows, int ell, int cp, double* __restrict__ lvl,
    int nseg, double* __restrict__ y64, void* yout, int out_double) {
  const int z = blockIdx.z;
  const int ncz = min(cp, ell - z * cp);
  const int64_t E = n_rows * ncz;
  const int64_t e = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
  if (e >= E) return;
  const int seg = blockIdx.y;
  const int p0 = seg * kRedSeg, p1 = min(nparts, p0 + kRedSeg);
  const AccT* src = partial + (int64_t)z * nparts * n_rows * cp + e;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int q = p0;
  for (; q + 7 < p1; q += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (double)src[(int64_t)(q + u) * E];
    s0 += v[0] + v[4];
    s1 += v[1] + v[5];
    s2 += v[2] + v[6];
    s3 += v[3] + v[7];
  }
  for (; q < p1; ++q) s0 += (double)src[(int64_t)q * E];
  const double s = (s0 + s1) + (s2 + s3);
  if (nseg == 1)
    store_y(e, ncz, n_rows, z * cp, s, y64, yout, out_double);
  else
    lvl[((int64_t)z * nseg + seg) * n_rows * cp + e] = s;
}

// Level 2: a workgroup owns 64 elements; its four thread groups sum
// consecutive quarters of the segments, and the quarters are added in order.
__global__ __launch_bounds__(kRedThreads) void sketch_reduce2_kernel(const double* __restrict__ lvl, int nseg,
                                                                     int64_t n_rows, int ell, int cp,
                                                                     double* __restrict__ y64, void* yout,
                                                                     int out_double) {
  __shared__ double part[kRedThreads];
  const int z = blockIdx.y;
  const int ncz = min(cp, ell - z * cp);
  const int64_t E = n_rows * ncz;
  const int el = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + el;
  const int per = (nseg + 3) / 4;
  const int q0 = grp * per, q1 = min(nseg, q0 + per);
  double s = 0.0;
  if (e < E) {
    const double* src = lvl + (int64_t)z * nseg * n_rows * cp + e;
    const int64_t st = n_rows * cp;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = q0;
    for (; q + 3 < q1; q += 4) {
      s0 += src[(int64_t)q * st];
      s1 += src[(int64_t)(q + 1) * st];
      s2 += src[(int64_t)(q + 2) * st];
      s3 += src[(int64_t)(q + 3) * st];
    }
    for (; q < q1; ++q) s0 += src[(int64_t)q * st];
    s = (s0 + s1) + (s2 + s3);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (grp == 0 && e < E)
    store_y(e, ncz, n_rows, z * cp, ((part[el] + part[64 + el]) + part[128 + el]) + part[192 + el], y64, yout,
            out_double);
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
  const size_t xsz = pb.x_is_double ? 8 : 4;
  const int64_t vlen = 16 / (int64_t)xsz;
  if (fp64 && mt > 2 && p.nt >= 3) mt = 2;  // register budget of fp64 fragments
  // Mode 0 reads rows along the contiguous index: each lane loads mt
  // consecutive rows as one vector (at most 16 bytes, aligned), which needs
  // n_0 to be a multiple of mt.  Otherwise the loads are scalar (one 64-bit
  // address per element): the row tiles are halved to keep the register
  // budget within two waves per SIMD.
  if (i == 0 && pb.x_is_double && mt > 2) mt = 2;
  while (i == 0 && mt > 1 && p.n_rows % mt != 0) mt /= 2;
  p.rowvec = (i == 0) && (reinterpret_cast<uintptr_t>(pb.x) % ((uintptr_t)mt * xsz) == 0);
  if (i == 0 && mt > 2 && !p.rowvec) mt = 2;
  p.mt = mt;
  const int64_t wave_rows = 16 * mt;
  const int wmax = std::max(1, std::min(8, tile.waves));
  int wm = tile.wm > 0 ? tile.wm : (int)std::min<int64_t>(wmax, (p.n_rows + wave_rows - 1) / wave_rows);
  p.wm = std::max(1, std::min(wmax, wm));
  p.row_blocks = (int)((p.n_rows + wave_rows * p.wm - 1) / (wave_rows * p.wm));
  int wo = tile.wo > 0 ? tile.wo : std::max(1, wmax / p.wm);
  while (p.wm * wo > wmax) --wo;
  p.wo = std::max(1, wo);
  p.f_blocks = (int)((p.n_f + 31) / 32);
  p.kvec = (i != 0) && (p.n_f % vlen == 0);
  p.kvec2 = (i != 0) && !p.kvec && !pb.x_is_double && (p.n_f % 2 == 0);

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
  // the end-of-kernel wave reduction reuses the table's LDS
  p.lds_bytes = std::max(p.lds_bytes, skdetail::wave_reduce_lds(p.wm, p.wo, p.mt, p.nt));
  p.o_per_wg = o_per;
  p.o_ranges = (int)((p.o_total + o_per - 1) / o_per);
  p.nparts = p.f_blocks * p.o_ranges;  // one partial per workgroup
  p.nseg = (p.nparts + kRedSeg - 1) / kRedSeg;
  p.partial_bytes = (size_t)p.col_chunks * p.nparts * p.n_rows * p.cpad * tsz;
  p.lvl_off = (p.partial_bytes + 255) / 256 * 256;
  if (p.nseg > 1) p.partial_bytes = p.lvl_off + (size_t)p.col_chunks * p.nseg * p.n_rows * p.cpad * sizeof(double);
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

  // Vector loads need aligned rows; misaligned views take the scalar path.
  const uintptr_t xa = reinterpret_cast<uintptr_t>(pb.x);
  const size_t xsz = pb.x_is_double ? 8 : 4;
  int lm = kLoadScalar;
  if ((xa & 15) == 0 && p.kvec) lm = kLoadVecF;
  if ((xa & 7) == 0 && p.kvec2) lm = skdetail::kLoadVecF2;
  if (p.rowvec && xa % ((uintptr_t)p.mt * xsz) == 0) lm = kLoadRowVec;
  const size_t lds = p.lds_bytes;
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
  return launch_partial_reduce(partial, pb.prec == kFP64, p.nparts, p.n_rows, pb.ell, p.cpad, p.col_chunks,
                               reinterpret_cast<char*>(partial) + p.lvl_off, y64, y_out, out_is_double, st);
}

size_t partial_reduce_lvl_bytes(int nparts, int64_t n_rows, int cp, int col_chunks) {
  const int nseg = (nparts + kRedSeg - 1) / kRedSeg;
  return nseg > 1 ? (size_t)col_chunks * nseg * n_rows * cp * sizeof(double) : 0;
}

hipError_t launch_partial_reduce(const void* partial, bool acc_double, int nparts, int64_t n_rows, int ell,
                                 int cp, int col_chunks, void* lvl_buf, double* y64, void* y_out,
                                 int out_is_double, hipStream_t st) {
  const int nseg = (nparts + kRedSeg - 1) / kRedSeg;
  const int64_t emax = n_rows * std::min(cp, ell);
  const unsigned eblk = (unsigned)((emax + kRedThreads - 1) / kRedThreads);
  double* lvl = nseg > 1 ? reinterpret_cast<double*>(lvl_buf) : nullptr;
  const dim3 g1(eblk, (unsigned)nseg, (unsigned)col_chunks);
  if (acc_double)
    hipLaunchKernelGGL(sketch_reduce1_kernel<double>, g1, dim3(kRedThreads), 0, st,
                       reinterpret_cast<const double*>(partial), nparts, n_rows, ell, cp, lvl, nseg, y64, y_out,
                       out_is_double);
  else
    hipLaunchKernelGGL(sketch_reduce1_kernel<float>, g1, dim3(kRedThreads), 0, st,
                       reinterpret_cast<const float*>(partial), nparts, n_rows, ell, cp, lvl, nseg, y64, y_out,
                       out_is_double);
  if (nseg > 1) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sketch_reduce2_kernel, dim3((unsigned)((emax + 63) / 64), (unsigned)col_chunks),
                       dim3(kRedThreads), 0, st, lvl, nseg, n_rows, ell, cp, y64, y_out, out_is_double);
  }
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
