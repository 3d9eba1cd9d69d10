// Dense-Gaussian sketch of a mode unfolding, Y = X_(i) Omega with Omega of
// size prod_{j != i} n_j x ell: the randomized HOSVD / STHOSVD baselines
// (RHOSVD, RSTHOSVD) that Section 5.3 compares the KRP sketches with.
//
// Three stages, as the baseline itself is defined: (1) Omega is drawn into
// HBM (row k holds the ell entries of the unfolding's column k, four per
// generator call, rows padded to a multiple of four); (2) for a mode other
// than the first, X is unfolded into a copy with that mode first (tiled
// transposes through LDS); (3) Y = X_(i) Omega as a split-K product on the
// matrix cores, one fp32 (fp64) partial block per workgroup, summed in a fixed
// order in fp64 by the sketch's reduction kernels.
#include "dense.h"
#include "driver.h"
#include "device_common.h"
#include "philox.h"

#include <algorithm>

namespace krp {

namespace {

constexpr int kDenseWaves = 4;
constexpr int kDenseMT = 4;  // 16-row tiles per wave: 64 rows
constexpr int kTrTile = 32;  // unfolding transpose tile

template <typename T>
__global__ __launch_bounds__(256) void dense_omega_kernel(uint64_t seed, uint64_t w2, int64_t rows, int ell, int lp,
                                                          T* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int quads = lp / 4;
  if (e >= rows * quads) return;
  const int64_t k = e / quads;
  const int j = (int)(e - k * quads);
  double g[4];
  gauss_quad(seed, w2, 0, (uint64_t)k, (uint64_t)j, g);
  T* o = out + k * lp + 4 * j;
#pragma unroll
  for (int u = 0; u < 4; ++u) o[u] = 4 * j + u < ell ? (T)g[u] : (T)0;
}

// xu[a + n (p + P q)] = x[p + P (a + n q)]: a P x n -> n x P transpose per q.
template <typename T>
__global__ __launch_bounds__(256) void dense_unfold_kernel(const T* __restrict__ x, T* __restrict__ xu, int64_t P,
                                                           int64_t n, int64_t tiles_p, int64_t tiles_a) {
  __shared__ T tile[kTrTile][kTrTile + 1];
  int64_t b = blockIdx.x;
  const int64_t tp = b % tiles_p;
  b /= tiles_p;
  const int64_t ta = b % tiles_a;
  const int64_t q = b / tiles_a;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t p0 = tp * kTrTile, a0 = ta * kTrTile;
  const T* src = x + P * n * q;
#pragma unroll
  for (int r = 0; r < kTrTile; r += 8) {
    const int64_t a = a0 + ty + r, p = p0 + tx;
    if (a < n && p < P) tile[ty + r][tx] = src[p + P * a];
  }
  __syncthreads();
  T* dst = xu + n * P * q;
#pragma unroll
  for (int r = 0; r < kTrTile; r += 8) {
    const int64_t p = p0 + ty + r, a = a0 + tx;
    if (a < n && p < P) dst[a + n * p] = tile[tx][ty + r];
  }
}

// Split-K product: workgroup (row block rb, part z) sums over its k range
//   Y[a, c] = sum_k xu[a + n k] omega[k lp + c]
// for a in the row block; wave w takes rows 64 (w % wr) .. and every wk-th
// 32-wide k step.  Lane (m, g) of a fragment holds row/column m and the
// reduction slots k0 + 8 g + j (j = 0..7) of the policy's fragments.
template <typename Tin, int P, int NT>
__global__ __launch_bounds__(64 * kDenseWaves) void dense_gemm_kernel(DenseArgs a) {
  using Pol = Policy<P>;
  using T = typename Pol::T;
  using AccT = typename Pol::AccT;
  extern __shared__ __align__(16) unsigned char dense_smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ln = lane & 15, g = lane >> 4;
  const int wr = a.wr, wk = kDenseWaves / a.wr;
  const int wrow = wave % wr, wkk = wave / wr;
  const int64_t z = blockIdx.x;
  const int64_t rb = blockIdx.y;
  const int64_t row0 = rb * 64 * wr + 64 * wrow;
  const int64_t k_begin = z * a.kc, k_end = min(a.K, k_begin + a.kc);
  const Tin* __restrict__ xu = reinterpret_cast<const Tin*>(a.xu);
  const T* __restrict__ om = reinterpret_cast<const T*>(a.omega);

  typename Pol::Acc acc[kDenseMT][NT];
#pragma unroll
  for (int m = 0; m < kDenseMT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = Pol::zero();

  // rows clamped to n - 1 (their sums are never stored), columns to lp - 1
  // (zeroed), k to K - 1 (zeroed through the omega operand)
  int64_t arow[kDenseMT];
#pragma unroll
  for (int m = 0; m < kDenseMT; ++m) arow[m] = min(row0 + 16 * m + ln, a.n - 1);
  int bcol[NT];
  bool bval[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = 16 * t + ln;
    bval[t] = c < a.lp;
    bcol[t] = min(c, a.lp - 1);
  }
  for (int64_t k0 = k_begin + 32 * wkk; k0 < k_end; k0 += 32 * wk) {
    T av[kDenseMT][8], bv[NT][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t k = k0 + 8 * g + j;
      const bool kv = k < k_end;
      const int64_t kc = kv ? k : k_end - 1;
#pragma unroll
      for (int m = 0; m < kDenseMT; ++m) av[m][j] = (T)xu[arow[m] + a.n * kc];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const T v = om[kc * a.lp + bcol[t]];
        bv[t][j] = (kv && bval[t]) ? v : (T)0;
      }
    }
    typename Pol::Frag af[kDenseMT], bf[NT];
#pragma unroll
    for (int m = 0; m < kDenseMT; ++m) af[m] = Pol::make(av[m]);
#pragma unroll
    for (int t = 0; t < NT; ++t) bf[t] = Pol::make(bv[t]);
#pragma unroll
    for (int m = 0; m < kDenseMT; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) Pol::mma(acc[m][t], af[m], bf[t]);
  }

  // waves that split k add up through LDS (fixed order), then one partial
  // block per workgroup: partial[z][row][c] (c fastest), the layout of the
  // sketch's reduction kernels
  AccT* red = reinterpret_cast<AccT*>(dense_smem);
  if (wk > 1) {
#pragma unroll
    for (int m = 0; m < kDenseMT; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(wave * kDenseMT * NT + m * NT + t) * 256 + r * 64 + lane] = acc[m][t][r];
    __syncthreads();
    if (wkk != 0) return;
#pragma unroll
    for (int m = 0; m < kDenseMT; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double s = 0.0;
          for (int w = 0; w < wk; ++w)
            s += (double)red[((wrow + w * wr) * kDenseMT * NT + m * NT + t) * 256 + r * 64 + lane];
          acc[m][t][r] = (AccT)s;
        }
  }
  AccT* part = reinterpret_cast<AccT*>(a.partial) + z * a.n * a.ell;
#pragma unroll
  for (int m = 0; m < kDenseMT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + 16 * m + Pol::out_row(g, r);
        const int c = 16 * t + ln;
        if (row < a.n && c < a.ell) part[row * a.ell + c] = acc[m][t][r];
      }
}

template <typename Tin, int P, int NT>
hipError_t gemm_go(const DenseArgs& a, const DensePlan& p, hipStream_t st) {
  using AccT = typename Policy<P>::AccT;
  const size_t lds = (size_t)kDenseWaves * kDenseMT * NT * 256 * sizeof(AccT);
  auto kern = dense_gemm_kernel<Tin, P, NT>;
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)p.nparts, (unsigned)p.row_blocks), dim3(64 * kDenseWaves),
                     p.wr < kDenseWaves ? lds : 0, st, a);
  return hipGetLastError();
}

template <typename Tin, int P>
hipError_t gemm_nt(const DenseArgs& a, const DensePlan& p, hipStream_t st) {
  switch ((p.ell + 15) / 16) {
    case 1: return gemm_go<Tin, P, 1>(a, p, st);
    case 2: return gemm_go<Tin, P, 2>(a, p, st);
    case 3: return gemm_go<Tin, P, 3>(a, p, st);
    default: return gemm_go<Tin, P, 4>(a, p, st);
  }
}

}  // namespace

DensePlan plan_dense(const SketchProblem& pb) {
  DensePlan p{};
  const int i = pb.mode;
  p.n = pb.dims[i];
  p.P = 1;
  for (int k = 0; k < i; ++k) p.P *= pb.dims[k];
  p.Q = 1;
  for (int k = i + 1; k < pb.d; ++k) p.Q *= pb.dims[k];
  p.K = p.P * p.Q;
  p.ell = pb.ell;
  p.lp = (pb.ell + 3) / 4 * 4;
  const bool w64 = pb.prec == kFP64;
  const size_t tsz = w64 ? 8 : 4;  // omega and accumulators
  const size_t xsz = pb.x_is_double ? 8 : 4;
  // waves along the rows: enough for n (up to 256 rows per workgroup)
  p.wr = p.n <= 64 ? 1 : (p.n <= 128 ? 2 : kDenseWaves);
  p.row_blocks = (int)((p.n + 64 * p.wr - 1) / (64 * p.wr));
  // parts along k: about 1024 workgroups, partial sums at most 32 MiB, at
  // least 32 k per wave step
  const int64_t step = 32 * (kDenseWaves / p.wr);
  int64_t parts = std::max<int64_t>(1, 1024 / p.row_blocks);
  const int64_t cap = std::max<int64_t>(1, (int64_t)(32ll << 20) / (int64_t)(p.n * p.ell * tsz));
  parts = std::min(parts, cap);
  parts = std::min(parts, (p.K + step - 1) / step);
  p.kc = (p.K + parts - 1) / parts;
  p.kc = (p.kc + step - 1) / step * step;
  p.nparts = (int)((p.K + p.kc - 1) / p.kc);
  size_t off = 0;
  p.off_omega = off;
  off = align_up(off + (size_t)p.K * p.lp * tsz);
  p.off_xu = off;
  if (i != 0 && p.P > 1) off = align_up(off + (size_t)p.n * p.K * xsz);
  p.off_part = off;
  off = align_up(off + (size_t)p.nparts * p.n * p.ell * tsz);
  p.off_lvl = off;
  off = align_up(off + partial_reduce_lvl_bytes(p.nparts, p.n, p.ell, 1));
  p.ws_bytes = off;
  return p;
}

hipError_t launch_dense_sketch(const SketchProblem& pb, const DensePlan& p, char* ws, double* y64, void* y_out,
                               int out_is_double, hipStream_t st) {
  const bool w64 = pb.prec == kFP64;
  if (pb.x_is_double && !w64) return hipErrorInvalidValue;
  const uint64_t w2 = counter_word2(pb.draw, pb.sketch_id, kDenseFactor);
  void* omega = ws + p.off_omega;
  const int64_t nq = p.K * (p.lp / 4);
  if (nq > 0) {
    const unsigned grid = (unsigned)((nq + 255) / 256);
    if (w64)
      hipLaunchKernelGGL(dense_omega_kernel<double>, dim3(grid), dim3(256), 0, st, pb.seed, w2, p.K, p.ell, p.lp,
                         reinterpret_cast<double*>(omega));
    else
      hipLaunchKernelGGL(dense_omega_kernel<float>, dim3(grid), dim3(256), 0, st, pb.seed, w2, p.K, p.ell, p.lp,
                         reinterpret_cast<float*>(omega));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const void* xu = pb.x;
  if (pb.mode != 0 && p.P > 1) {
    void* dst = ws + p.off_xu;
    const int64_t tp = (p.P + kTrTile - 1) / kTrTile, ta = (p.n + kTrTile - 1) / kTrTile;
    const int64_t blocks = tp * ta * p.Q;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (pb.x_is_double)
      hipLaunchKernelGGL(dense_unfold_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                         reinterpret_cast<const double*>(pb.x), reinterpret_cast<double*>(dst), p.P, p.n, tp, ta);
    else
      hipLaunchKernelGGL(dense_unfold_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                         reinterpret_cast<const float*>(pb.x), reinterpret_cast<float*>(dst), p.P, p.n, tp, ta);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    xu = dst;
  }
  DenseArgs a{};
  a.xu = xu;
  a.omega = omega;
  a.partial = ws + p.off_part;
  a.n = p.n;
  a.K = p.K;
  a.kc = p.kc;
  a.ell = p.ell;
  a.lp = p.lp;
  a.wr = p.wr;
  hipError_t e;
  if (pb.x_is_double) {
    e = gemm_nt<double, kFP64>(a, p, st);
  } else {
    switch (pb.prec) {
      case kFP64: e = gemm_nt<float, kFP64>(a, p, st); break;
      case kFP32: e = gemm_nt<float, kFP32>(a, p, st); break;
      case kBF16: e = gemm_nt<float, kBF16>(a, p, st); break;
      default: e = gemm_nt<float, kBF16X3>(a, p, st); break;
    }
  }
  if (e != hipSuccess) return e;
  return launch_partial_reduce(ws + p.off_part, w64, p.nparts, p.n, p.ell, p.ell, 1, ws + p.off_lvl, y64, y_out,
                               out_is_double, st);
}

}  // namespace krp
