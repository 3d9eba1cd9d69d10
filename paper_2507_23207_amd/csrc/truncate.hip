// FP64 truncation of the ell-sized core: for each mode i (in the sweep
// order) the r_i leading left singular vectors W_i of the current core's
// mode-i unfolding are the leading eigenvectors of its Gram matrix; the core
// is projected (G <- G x_i W_i^T) before the next mode, and the factors
// become Q_i W_i.  Eigenvectors come from a cyclic (round-robin parallel)
// Jacobi method in one workgroup.
#include "device_common.h"
#include "kernels.h"
#include "truncate.h"

#include <algorithm>

namespace krp {

namespace {

constexpr int kEigThreads = 512;
constexpr int kEigMax = 64;

// Small tensors (one mode): one workgroup per entry pair a <= b of the Gram
// matrix, summing g[p, a, q] g[p, b, q] over p, q (more workgroups than the
// column split would have, each with few loads).
constexpr int kGramThreads = 256;
constexpr int64_t kGramPairMaxElems = 1 << 18;
__device__ void mode_gram_pair(const double* __restrict__ g, int64_t P, int l, int64_t Q,
                               double* __restrict__ gram, int pair, double* red) {
  int b = 0;
  while ((b + 1) * (b + 2) / 2 <= pair) ++b;
  const int a = pair - b * (b + 1) / 2;
  double s = 0.0;
  const int64_t total = P * Q;
  // eight (p, q) positions per thread and batch, their loads in flight together
  for (int64_t e0 = threadIdx.x; e0 < total; e0 += 8 * (int64_t)blockDim.x) {
    double x[8], y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t e = e0 + u * (int64_t)blockDim.x;
      x[u] = 0.0;
      y[u] = 0.0;
      if (e < total) {
        const int64_t q = e / P, p = e - q * P;
        x[u] = g[p + P * (a + (int64_t)l * q)];
        y[u] = g[p + P * (b + (int64_t)l * q)];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += x[u] * y[u];
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    gram[a + (int64_t)l * b] = t;
    gram[b + (int64_t)l * a] = t;
  }
}

__global__ void mode_gram_kernel(const double* __restrict__ g, int64_t P, int l, int64_t Q,
                                 double* __restrict__ gram) {
  __shared__ double red[kGramThreads / 64];
  mode_gram_pair(g, P, l, Q, gram, blockIdx.x, red);
}

// Gram matrices of mode unfoldings of a fp64 tensor viewed as g[p, a, q]
// (P x l x Q): gram[a + l b] = sum over the columns k = p + P q of
// g[p, a, q] g[p, b, q].  The columns of each mode are split into nparts
// contiguous ranges, one workgroup each: it streams its range in chunks of
// kGramCh columns through LDS (column-major in k: xs[k][a]) and accumulates
// the 16 x 16 tiles of the upper triangle on the fp64 matrix cores, each
// tile's chunk split over several waves when there are few tiles; the tile
// accumulators are summed in wave order and the workgroup's partial Gram
// matrix (both triangles) goes to part[w][l][l].  A second kernel adds the
// partials of each entry in workgroup order.  Every sum has a fixed order.
constexpr int kGramCh = 64;
constexpr int kGramPitch = kEigMax + 1;
constexpr int kGramWgThreads = 512;
constexpr int kGramMaxParts = 256;

struct GramJobs {
  int64_t P[kMaxDims], Q[kMaxDims];
  int l[kMaxDims];
  double* part[kMaxDims];  // nparts x l x l partial Gram matrices
  double* gram[kMaxDims];  // l x l result
  int nparts[kMaxDims];
  int first[kMaxDims + 1];  // workgroups [first[m], first[m + 1]) take mode m
  int n;
};

// Column ranges per mode: one chunk per workgroup up to kGramMaxParts
// workgroups (small cores: every chunk at once), and at most 2^19 partial
// entries.
int gram_parts(int64_t K, int l) {
  int64_t np = (K + kGramCh - 1) / kGramCh;
  np = std::min<int64_t>(np, kGramMaxParts);
  np = std::min<int64_t>(np, std::max<int64_t>(1, (int64_t)(1 << 19) / ((int64_t)l * l)));
  return (int)std::max<int64_t>(1, np);
}

__global__ __launch_bounds__(kGramWgThreads) void gram_part_kernel(const double* __restrict__ g, GramJobs jobs) {
  __shared__ double xs[kGramCh * kGramPitch];
  int m = 0;
  while (m + 1 < jobs.n && (int)blockIdx.x >= jobs.first[m + 1]) ++m;
  const int w = (int)blockIdx.x - jobs.first[m];
  const int64_t P = jobs.P[m], Q = jobs.Q[m];
  const int l = jobs.l[m], np = jobs.nparts[m];
  const int64_t K = P * Q;
  const int64_t kb = K * w / np, ke = K * (w + 1) / np;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nl = lane & 15, gq = lane >> 4;
  const int T = (l + 15) / 16, lp = 16 * T;
  const int pairs = T * (T + 1) / 2;
  // tasks: tile pairs x splits of the chunk's 16 column quads over the waves
  const int ks = pairs == 1 ? 8 : pairs <= 2 ? 4 : pairs <= 4 ? 2 : 1;
  const int tasks = pairs * ks, qper = 16 / ks;
  int ti[2] = {0, 0}, tj[2] = {0, 0};
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int pr = (wave + u * 8) % pairs;
    int cnt = 0;
    for (int a = 0; a < T; ++a)
      for (int b = a; b < T; ++b) {
        if (cnt == pr) {
          ti[u] = a;
          tj[u] = b;
        }
        ++cnt;
      }
  }
  doublex4 acc[2] = {doublex4{0.0, 0.0, 0.0, 0.0}, doublex4{0.0, 0.0, 0.0, 0.0}};
  // chunk loads, coalesced along the contiguous index: a for mode 0 (P = 1),
  // the column k (p fastest) otherwise; zeros past the range and past l.  The
  // next chunk's loads are in flight while the current one is multiplied.
  constexpr int kPer = kGramCh * kEigMax / kGramWgThreads;
  double pre[kPer];
  auto slot = [&](int e, int& kk, int& a) {
    if (P == 1) {
      kk = e / lp;
      a = e - kk * lp;
    } else {
      a = e >> 6;  // kGramCh = 64 columns per a
      kk = e & 63;
    }
  };
  // column k0 of the chunk as (q0, p0), advanced chunk by chunk (uniform);
  // within the chunk column k0 + kk is (q0 + x / P, x % P), x = p0 + kk < P + 64
  int64_t q0 = P == 1 ? kb : kb / P;
  int64_t p0 = P == 1 ? 0 : kb - q0 * P;
  const float rcp_p = 1.0f / (float)min(P, (int64_t)64);
  auto load = [&](int64_t k0) {
    const int kc = (int)min((int64_t)kGramCh, ke - k0);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * kGramWgThreads;
      int kk, a;
      slot(e, kk, a);
      double v = 0.0;
      if (e < kGramCh * lp && kk < kc && a < l) {
        int64_t off;
        if (P == 1) {
          off = a + (int64_t)l * (k0 + kk);
        } else {
          const int64_t x = p0 + kk;
          int64_t qd, pr;
          if (P >= 64) {
            qd = x >= P ? 1 : 0;
          } else {  // x < 128: the float quotient is exact or one off
            qd = (int64_t)((float)x * rcp_p);
            if (qd * P > x) --qd;
            else if ((qd + 1) * P <= x) ++qd;
          }
          pr = x - qd * P;
          off = pr + P * (a + (int64_t)l * (q0 + qd));
        }
        v = g[off];
      }
      pre[u] = v;
    }
  };
  auto advance = [&]() {
    if (P == 1) return;
    p0 += kGramCh;
    while (p0 >= P) {
      p0 -= P;
      ++q0;
    }
  };
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kGramCh) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * kGramWgThreads;
      int kk, a;
      slot(e, kk, a);
      if (e < kGramCh * lp) xs[kk * kGramPitch + a] = pre[u];
    }
    __syncthreads();
    advance();
    if (k0 + kGramCh < ke) load(k0 + kGramCh);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int task = wave + u * 8;
      if (task < tasks) {
        const int kh = task / pairs;
        double av[4], bv[4];
#pragma unroll 1
        for (int s0 = 0; s0 < qper; s0 += 4) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int kk = 4 * (kh * qper + min(s0 + s, qper - 1)) + gq;
            av[s] = xs[kk * kGramPitch + 16 * ti[u] + nl];
            bv[s] = xs[kk * kGramPitch + 16 * tj[u] + nl];
          }
#pragma unroll
          for (int s = 0; s < 4; ++s)
            if (s0 + s < qper) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc[u], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // tile accumulators of each task into LDS, then the splits of a tile pair
  // in order (16 tasks x 256 entries fit the chunk buffer)
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int task = wave + u * 8;
    if (task < tasks) {
#pragma unroll
      for (int r = 0; r < 4; ++r) xs[task * 256 + (4 * r + gq) * 16 + nl] = acc[u][r];
    }
  }
  __syncthreads();
  double* out = jobs.part[m] + (int64_t)w * l * l;
  for (int e = tid; e < pairs * 256; e += kGramWgThreads) {
    const int pr = e / 256, i = (e % 256) / 16, j = e % 16;
    int a0 = 0, b0 = 0, cnt = 0;
    for (int a = 0; a < T; ++a)
      for (int b = a; b < T; ++b) {
        if (cnt == pr) {
          a0 = a;
          b0 = b;
        }
        ++cnt;
      }
    double v = 0.0;
    for (int kh = 0; kh < ks; ++kh) v += xs[(pr + pairs * kh) * 256 + i * 16 + j];
    const int ga = 16 * a0 + i, gb = 16 * b0 + j;
    if (ga < l && gb < l) {
      out[ga + (int64_t)l * gb] = v;
      out[gb + (int64_t)l * ga] = v;
    }
  }
}

// gram[e] = sum of the partials' entry e in workgroup order: a workgroup owns
// 16 entries of one mode (blockIdx.y), its 16 thread groups sum consecutive
// sixteenths of the partials, and those are added in order.
__global__ __launch_bounds__(256) void gram_sum_kernel(GramJobs jobs) {
  __shared__ double red[256];
  const int m = blockIdx.y;
  const int l = jobs.l[m], np = jobs.nparts[m];
  const int64_t E = (int64_t)l * l;
  const int el = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + el;
  const int per = (np + 15) / 16, q0 = grp * per, q1 = min(np, q0 + per);
  double s = 0.0;
  if (e < E) {
    const double* src = jobs.part[m] + e;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = q0;
    for (; q + 3 < q1; q += 4) {
      s0 += src[(int64_t)q * E];
      s1 += src[(int64_t)(q + 1) * E];
      s2 += src[(int64_t)(q + 2) * E];
      s3 += src[(int64_t)(q + 3) * E];
    }
    for (; q < q1; ++q) s0 += src[(int64_t)q * E];
    s = (s0 + s1) + (s2 + s3);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (grp == 0 && e < E) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += red[16 * k + el];
    jobs.gram[m][e] = t;
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cyclic Jacobi with a round-robin parallel ordering kept in "position
// space": the np (even) indices occupy positions, every round rotates the
// pairs of positions (2k, 2k+1) at once, and the rotated matrix is stored
// with its positions moved by a fixed permutation sigma (the circle method
// of round-robin scheduling: position 0 stays, the even positions advance,
// the odd ones fall back), so that after np - 1 rounds every pair of
// indices has met once.  Both A and the accumulated V = J_1 J_2 ... are
// kept in position order (V's rows stay in index order), double-buffered in
// LDS: a thread reads the 2x2 block {2k1, 2k1+1} x {2k2, 2k2+1} of A (two
// aligned 16-byte loads, consecutive across lanes), forms J^T A J for it and
// stores the four values at their permuted positions.  Every wave computes
// the round's rotations itself, so a round costs one workgroup barrier.
// Sweeps stop when the off-diagonal Frobenius norm is below 1e-13 of the
// diagonal's.  With v_init, the iteration starts from A = V0^T A_in V0,
// V = V0 (a warm start from the eigenvectors of a nearby matrix).
constexpr int kJTasks = 2;  // 2x2 tasks per thread: ceil(32 / (512 / 32))
constexpr int kJPitch = kEigMax + 2;  // even, so 2-element pairs are 16-byte aligned

// 1 / sqrt(x) and 1 / x for positive normal x: hardware estimate plus two
// Newton steps (relative error within a few ulp).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}
// One Newton step each, for quantities that need not be exact.
__device__ __forceinline__ double rsqrt_nr1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ double rcp_nr1(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}

__device__ __forceinline__ int jacobi_sigma(int x, int half) {
  if (x == 0) return 0;
  if (x & 1) return x == 1 ? (half > 1 ? 2 : 1) : x - 2;
  return (x >> 1) == half - 1 ? x + 1 : x + 2;
}

__global__ __launch_bounds__(kEigThreads) void jacobi_eig_kernel(int ell, int r, const double* a_in,
                                                                 int64_t a_stride, const double* v_init,
                                                                 int64_t v_stride, double* w,
                                                                 int64_t w_stride, double* evals,
                                                                 int64_t ev_stride, int njobs,
                                                                 EigJobs jobs) {
  constexpr int P = kJPitch;
  constexpr int NW = kEigThreads / 64;
  __shared__ __align__(16) double A[2][kEigMax * P];
  __shared__ __align__(16) double VT[2][kEigMax * P];  // V^T: row = position, column = index
  __shared__ double2 rcs[NW][kEigMax / 2];
  __shared__ double red[2][NW];
  __shared__ int order_idx[kEigMax];

  int b = blockIdx.x;
  if (njobs > 0) {  // independent problems of their own sizes
    const EigJob& jb = jobs.job[b];
    ell = jb.ell;
    r = jb.r;
    a_in = jb.a;
    v_init = jb.v_init;
    w = jb.w;
    evals = jb.evals;
    b = 0;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int np = ell + (ell & 1);
  const int half = np / 2;
  const int cpp = kEigThreads / half;  // task rows per pass (>= 8)
  const bool active = tid < half * cpp;
  const int k2 = tid % half, kb = tid / half;
  const double* ain = a_in + b * a_stride;
  // A[0] <- input (padding index: -1 on the diagonal, decoupled, sorts last
  // since the input is positive semi-definite); VT[0] <- identity or V0^T.
  for (int e = tid; e < np * np; e += kEigThreads) {
    const int i = e % np, j = e / np;
    double v = 0.0;
    if (i < ell && j < ell) v = ain[i + (int64_t)ell * j];
    else if (i == j) v = -1.0;
    double v0 = (i == j) ? 1.0 : 0.0;
    if (v_init && i < ell && j < ell) v0 = v_init[b * v_stride + i + (int64_t)ell * j];
    A[0][i * P + j] = v;
    VT[0][j * P + i] = v0;
  }
  __syncthreads();
  int cur = 0;
  // position of the padding index (odd ell); every round moves it by sigma
  int pad = (ell & 1) ? np - 1 : -1;
  if (v_init) {
    // Dot product of two rows (16-byte aligned, np even): pairs of entries per
    // load, four independent partial sums.
    auto row_dot = [&](const double* x, const double* y) {
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < np; k0 += 8) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 2 * u;
          if (k < np) {
            const double2 a = *reinterpret_cast<const double2*>(x + k);
            const double2 c = *reinterpret_cast<const double2*>(y + k);
            s4[u] = fma(a.x, c.x, s4[u]);
            s4[u] = fma(a.y, c.y, s4[u]);
          }
        }
      }
      return (s4[0] + s4[1]) + (s4[2] + s4[3]);
    };
    // T = A_in V0, stored transposed in A[1] (row j = column j of T), then
    // A[0] = V0^T T: both products read rows of their operands.
    for (int e = tid; e < np * np; e += kEigThreads) {
      const int i = e % np, j = e / np;
      A[1][j * P + i] = row_dot(&A[0][i * P], &VT[0][j * P]);
    }
    __syncthreads();
    for (int e = tid; e < np * np; e += kEigThreads) {
      const int i = e % np, j = e / np;
      A[0][i * P + j] = row_dot(&VT[0][i * P], &A[1][j * P]);
    }
    __syncthreads();
  }
  for (int sweep = 0; sweep < 60; ++sweep) {
    // Sums over the real indices only: the padding entry of an odd ell (-1 on
    // the diagonal, at position pad) must not set the scale of the relative
    // stopping test.
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < np * np; e += kEigThreads) {
      const int i = e % np, j = e / np;
      const double v = A[cur][i * P + j];
      if (i != pad && j != pad) {
        if (i != j) off += v * v;
        else dia += v * v;
      }
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    if (lane == 0) {
      red[0][wave] = off;
      red[1][wave] = dia;
    }
    __syncthreads();
    double to = 0.0, td = 0.0;
    for (int k = 0; k < NW; ++k) {
      to += red[0][k];
      td += red[1][k];
    }
    __syncthreads();
    if (to <= 1e-26 * td) break;
    for (int round = 0; round < np - 1; ++round) {
      const double* Ac = A[cur];
      double* An = A[cur ^ 1];
      const double* Vc = VT[cur];
      double* Vn = VT[cur ^ 1];
      // loads of this thread's tasks first: they do not depend on the rotations
      double2 ra[kJTasks], rb[kJTasks], va[kJTasks], vb[kJTasks];
      if (active) {
#pragma unroll
        for (int u = 0; u < kJTasks; ++u) {
          const int k1 = kb + u * cpp;
          if (k1 < half) {
            ra[u] = *reinterpret_cast<const double2*>(&Ac[(2 * k1) * P + 2 * k2]);
            rb[u] = *reinterpret_cast<const double2*>(&Ac[(2 * k1 + 1) * P + 2 * k2]);
            va[u] = *reinterpret_cast<const double2*>(&Vc[(2 * k1) * P + 2 * k2]);
            vb[u] = *reinterpret_cast<const double2*>(&Vc[(2 * k1 + 1) * P + 2 * k2]);
          }
        }
      }
      if (lane < half) {
        // rotation of positions (2k, 2k+1) zeroing their off-diagonal entry:
        // t = tan(phi) = sign(d) 2 apq / (|d| + sqrt(d^2 + 4 apq^2)), d = aqq - app
        // t only has to be close to the exact angle (c and s stay exactly
        // normalised by c = 1 / sqrt(1 + t^2), s = t c): its reciprocal
        // square root and reciprocal take the hardware estimates and one
        // Newton step each, c's two, which keeps the dependent chain short.
        const int p = 2 * lane;
        const double app = Ac[p * P + p], apq = Ac[p * P + p + 1], aqq = Ac[(p + 1) * P + p + 1];
        const double d = aqq - app;
        double t = 0.0;
        const double num = 2.0 * apq;
        const double x = fma(d, d, num * num);
        if (apq != 0.0 && x >= 0x1.0p-1000) {  // (entries below ~1e-150 count as zero)
          const double hyp = x * rsqrt_nr1(x);
          t = num * rcp_nr1(fabs(d) + hyp);
          if (d < 0.0) t = -t;
        }
        const double c = rsqrt_nr(fma(t, t, 1.0));
        rcs[wave][lane] = make_double2(c, t * c);
      }
      wave_sync();
      if (active) {
        const double2 r2 = rcs[wave][k2];
        const double c2 = r2.x, s2 = r2.y;
        const int cp = jacobi_sigma(2 * k2, half), cq = jacobi_sigma(2 * k2 + 1, half);
#pragma unroll
        for (int u = 0; u < kJTasks; ++u) {
          const int k1 = kb + u * cpp;
          if (k1 < half) {
            const double2 r1 = rcs[wave][k1];
            const double c1 = r1.x, s1 = r1.y;
            // columns: (A J)[:, p] = c A[:, p] - s A[:, q], (A J)[:, q] = s A[:, p] + c A[:, q]
            const double t00 = c2 * ra[u].x - s2 * ra[u].y, t01 = s2 * ra[u].x + c2 * ra[u].y;
            const double t10 = c2 * rb[u].x - s2 * rb[u].y, t11 = s2 * rb[u].x + c2 * rb[u].y;
            // rows: J^T (A J)
            double n00 = c1 * t00 - s1 * t10, n01 = c1 * t01 - s1 * t11;
            double n10 = s1 * t00 + c1 * t10, n11 = s1 * t01 + c1 * t11;
            if (k1 == k2) {
              n01 = 0.0;
              n10 = 0.0;
            }
            const int rp = jacobi_sigma(2 * k1, half), rq = jacobi_sigma(2 * k1 + 1, half);
            An[rp * P + cp] = n00;
            An[rp * P + cq] = n01;
            An[rq * P + cp] = n10;
            An[rq * P + cq] = n11;
            // V^T <- J^T V^T on rows (2 k1, 2 k1 + 1), columns 2 k2 and 2 k2 + 1
            double2 w0, w1;
            w0.x = c1 * va[u].x - s1 * vb[u].x;
            w0.y = c1 * va[u].y - s1 * vb[u].y;
            w1.x = s1 * va[u].x + c1 * vb[u].x;
            w1.y = s1 * va[u].y + c1 * vb[u].y;
            *reinterpret_cast<double2*>(&Vn[rp * P + 2 * k2]) = w0;
            *reinterpret_cast<double2*>(&Vn[rq * P + 2 * k2]) = w1;
          }
        }
      }
      __syncthreads();
      cur ^= 1;
      if (pad >= 0) pad = jacobi_sigma(pad, half);
    }
  }
  // descending eigenvalues by ranking (ties keep the lower position first)
  if (tid < np) order_idx[tid] = tid;
  __syncthreads();
  if (tid < np) {
    const double li = A[cur][tid * (P + 1)];
    int rank = 0;
    for (int j = 0; j < np; ++j) {
      const double lj = A[cur][j * (P + 1)];
      rank += (lj > li || (lj == li && j < tid)) ? 1 : 0;
    }
    order_idx[rank] = tid;
  }
  __syncthreads();
  double* wout = w + b * w_stride;
  for (int j = tid; j < r; j += kEigThreads) {
    const int c = order_idx[j];
    const double* vc = &VT[cur][c * P];
    int imax = 0;
    double vmax = -1.0;
    for (int i = 0; i < ell; ++i) {
      const double v = fabs(vc[i]);
      if (v > vmax) {
        vmax = v;
        imax = i;
      }
    }
    const double sgn = vc[imax] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < ell; ++i) wout[i + (int64_t)ell * j] = sgn * vc[i];
    if (evals) evals[b * ev_stride + j] = A[cur][c * (P + 1)];
  }
}

// out = q (n x l) * w (l x r), fp64; also in the storage type if out_s.
__global__ void small_gemm_kernel(const double* __restrict__ q, int64_t n, int l,
                                  const double* __restrict__ w, int r, double* out64, void* out_s,
                                  int out_double) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * r) return;
  const int64_t i = idx % n;
  const int j = (int)(idx / n);
  double s = 0.0;
  for (int k0 = 0; k0 < l; k0 += 8) {
    double x[8], y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u;
      x[u] = k < l ? q[i + n * k] : 0.0;
      y[u] = k < l ? w[k + (int64_t)l * j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += x[u] * y[u];
  }
  if (out64) out64[idx] = s;
  if (out_s) {
    if (out_double)
      reinterpret_cast<double*>(out_s)[idx] = s;
    else
      reinterpret_cast<float*>(out_s)[idx] = (float)s;
  }
}

}  // namespace

TruncPlan plan_truncate(int d, const int* ell, const int* rank, const int64_t* dims, const int* order) {
  TruncPlan p;
  p.d = d;
  int64_t elems = 1;
  for (int k = 0; k < d; ++k) {
    p.ell[k] = ell[k];
    p.rank[k] = rank[k];
    p.order[k] = order[k];
    p.dims[k] = dims[k];
    elems *= ell[k];
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  p.off_g[0] = take(elems * sizeof(double));
  p.off_g[1] = take(elems * sizeof(double));
  for (int k = 0; k < d; ++k) p.off_gram[k] = take((size_t)ell[k] * ell[k] * sizeof(double));
  // partial Gram matrices: the ell-core has the most columns per mode, so its
  // partition also bounds those of the partially truncated cores
  for (int k = 0; k < d; ++k)
    p.off_part[k] = take((size_t)gram_parts(elems / ell[k], ell[k]) * ell[k] * ell[k] * sizeof(double));
  for (int k = 0; k < d; ++k) p.off_v0[k] = take((size_t)ell[k] * ell[k] * sizeof(double));
  for (int k = 0; k < d; ++k) p.off_w[k] = take((size_t)ell[k] * rank[k] * sizeof(double));
  for (int k = 0; k < d; ++k) p.off_qt[k] = take((size_t)dims[k] * rank[k] * sizeof(double));
  p.ws_bytes = off;
  return p;
}

double* truncated_q64(const TruncPlan& p, char* ws, int k) {
  return reinterpret_cast<double*>(ws + p.off_qt[k]);
}

hipError_t launch_sym_eig(int batch, int ell, int r, const double* a, int64_t a_stride, double* w,
                          int64_t w_stride, double* evals, int64_t ev_stride, hipStream_t st,
                          const double* v_init, int64_t v_stride) {
  if (ell < 1 || ell > kEigMax || r < 1 || r > ell) return hipErrorInvalidValue;
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_eig_kernel, dim3(batch), dim3(kEigThreads), 0, st, ell, r, a, a_stride,
                     v_init, v_stride, w, w_stride, evals, ev_stride, 0, EigJobs{});
  return hipGetLastError();
}

hipError_t launch_sym_eig_jobs(int njobs, const EigJob* jobs, hipStream_t st) {
  if (njobs < 1 || njobs > kMaxDims) return hipErrorInvalidValue;
  EigJobs t{};
  for (int k = 0; k < njobs; ++k) {
    const EigJob& j = jobs[k];
    if (j.ell < 1 || j.ell > kEigMax || j.r < 1 || j.r > j.ell) return hipErrorInvalidValue;
    t.job[k] = j;
  }
  hipLaunchKernelGGL(jacobi_eig_kernel, dim3(njobs), dim3(kEigThreads), 0, st, 0, 0, nullptr, 0,
                     nullptr, 0, nullptr, 0, nullptr, 0, njobs, t);
  return hipGetLastError();
}

hipError_t launch_truncate(const TruncPlan& p, const void* core, int core_double, double* const* q64,
                           void* core_out, void* const* q_out, int out_double, char* ws,
                           hipStream_t st) {
  const int d = p.d;
  int64_t cur[kMaxDims];
  int64_t elems = 1;
  for (int k = 0; k < d; ++k) {
    cur[k] = p.ell[k];
    elems *= cur[k];
  }
  double* g[2] = {reinterpret_cast<double*>(ws + p.off_g[0]), reinterpret_cast<double*>(ws + p.off_g[1])};
  hipError_t e = launch_cast(core, core_double, g[0], 1, elems, st);
  if (e != hipSuccess) return e;
  // Gram matrices of the modes `modes` of the tensor src (sizes cur)
  auto grams_of = [&](const double* src, int nm, const int* modes) -> hipError_t {
    GramJobs gj{};
    gj.n = nm;
    gj.first[0] = 0;
    int lmax = 1;
    for (int j = 0; j < nm; ++j) {
      const int i = modes[j];
      int64_t P = 1, Q = 1;
      for (int k = 0; k < i; ++k) P *= cur[k];
      for (int k = i + 1; k < d; ++k) Q *= cur[k];
      const int l = (int)cur[i];
      gj.P[j] = P;
      gj.Q[j] = Q;
      gj.l[j] = l;
      gj.nparts[j] = gram_parts(P * Q, l);
      gj.part[j] = reinterpret_cast<double*>(ws + p.off_part[i]);
      gj.gram[j] = reinterpret_cast<double*>(ws + p.off_gram[i]);
      gj.first[j + 1] = gj.first[j] + gj.nparts[j];
      lmax = std::max(lmax, l);
    }
    hipLaunchKernelGGL(gram_part_kernel, dim3(gj.first[nm]), dim3(kGramWgThreads), 0, st, src, gj);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(gram_sum_kernel, dim3((unsigned)((lmax * lmax + 15) / 16), (unsigned)nm), dim3(256), 0, st,
                       gj);
    return hipGetLastError();
  };
  // The Gram matrices of all modes of the ell-core, and their complete
  // eigenbases in one launch (the modes are independent problems).  The first
  // mode of the order uses them as they are; every later mode's Gram matrix
  // (of the partially truncated core) differs from its ell-core counterpart
  // only by the discarded components, so its Jacobi iteration starts from
  // that basis and needs few sweeps.
  EigJob jobs[kMaxDims];
  int all[kMaxDims];
  for (int i = 0; i < d; ++i) {
    all[i] = i;
    jobs[i] = EigJob{reinterpret_cast<double*>(ws + p.off_gram[i]), nullptr,
                     reinterpret_cast<double*>(ws + p.off_v0[i]), nullptr, p.ell[i], p.ell[i]};
  }
  e = grams_of(g[0], d, all);
  if (e != hipSuccess) return e;
  e = launch_sym_eig_jobs(d, jobs, st);
  if (e != hipSuccess) return e;
  for (int s = 0; s < d; ++s) {
    const int i = p.order[s];
    const int l = (int)cur[i];
    double* wi = reinterpret_cast<double*>(ws + p.off_w[i]);
    const double* v0 = reinterpret_cast<const double*>(ws + p.off_v0[i]);
    if (s == 0) {
      // leading r columns of the (sorted, sign-normalised) eigenbasis
      e = launch_cast(v0, 1, wi, 1, (int64_t)l * p.rank[i], st);
    } else {
      double* gram = reinterpret_cast<double*>(ws + p.off_gram[i]);
      int64_t P = 1, Q = 1;
      for (int k = 0; k < i; ++k) P *= cur[k];
      for (int k = i + 1; k < d; ++k) Q *= cur[k];
      if (P * Q * l <= kGramPairMaxElems) {
        hipLaunchKernelGGL(mode_gram_kernel, dim3(l * (l + 1) / 2), dim3(kGramThreads), 0, st, g[s & 1], P, l,
                           Q, gram);
        e = hipGetLastError();
      } else {
        e = grams_of(g[s & 1], 1, &i);
      }
      if (e != hipSuccess) return e;
      e = launch_sym_eig(1, l, p.rank[i], gram, 0, wi, 0, nullptr, 0, st, v0, 0);
    }
    if (e != hipSuccess) return e;
    TtmProblem tp;
    tp.g = g[s & 1];
    tp.g_is_double = 1;
    tp.d = d;
    for (int k = 0; k < d; ++k) tp.dims[k] = cur[k];
    tp.mode = i;
    tp.ell = p.rank[i];
    tp.prec = kFP64;
    tp.q64 = wi;
    tp.out = g[(s + 1) & 1];
    tp.out_is_double = 1;
    e = launch_ttm(tp, st);
    if (e != hipSuccess) return e;
    cur[i] = p.rank[i];
  }
  for (int k = 0; k < d; ++k) {
    const int64_t n = p.dims[k];
    const int64_t cnt = n * p.rank[k];
    const unsigned grid = (unsigned)((cnt + 255) / 256);
    hipLaunchKernelGGL(small_gemm_kernel, dim3(grid), dim3(256), 0, st, q64[k], n, p.ell[k],
                       reinterpret_cast<const double*>(ws + p.off_w[k]), p.rank[k],
                       reinterpret_cast<double*>(ws + p.off_qt[k]), q_out[k], out_double);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  int64_t relems = 1;
  for (int k = 0; k < d; ++k) relems *= p.rank[k];
  return launch_cast(g[d & 1], 1, core_out, out_double, relems, st);
}

}  // namespace krp
