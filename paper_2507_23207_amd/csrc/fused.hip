// All-mode KRP sketch from one pass over X (Algorithm 7, step 3 for every
// mode at once; each sketch keeps its own fresh factors, or all share one
// set in the memoised variant of Section 5.1).
//
// The tensor is viewed as slabs S_o[i0, i1] (modes 1 and 2 of the paper) over
// the outer index o = (i2, ..., i_{d-1}).  A workgroup owns a 64-row block of
// i0, a 32-wide block of i1 and a box of outer indices; its eight waves take
// the steps of the box in turn, each loading its 64 x 32 slab as row vectors
// (as the mode-1 sketch does).  From the same registers every wave feeds:
//   mode 0:  Y0[i0, c] += sum_i1 S[i0, i1] Omega^(0)_1[i1, c] W^(0)[o, c]
//            (MFMA, A = S, weights of the step in the B fragment);
//   mode m >= 2 (outer): t[c] = sum_{i0, i1} S[i0, i1] Omega^(m)_0[i0, c]
//            Omega^(m)_1[i1, c] (MFMA over i1, then a weighted sum over the
//            wave's rows and its lane groups), added with the weight of the
//            other outer digits to row o_m of a per-wave accumulator in LDS;
//   mode 1:  Y1[i1, c] += sum_i0 Omega^(1)_0[i0, c] W^(1)[o, c] S[i0, i1]
//            (MFMA with the slab as B operand, reduced over i0: the slab goes
//            through a per-wave LDS staging region to get i0 into the
//            fragments' reduction slots).
// W^(m)[o, c] is the product of the outer factors' rows of the step.  With
// one shared factor set (RHOSVD-KRP-MEMO) the slab's product with the mode-2
// factor is the same for mode 0 and every outer mode, so the outer modes'
// weighted sums take mode 0's product instead of an MFMA of their own (the
// memoised partial MTTKRP: half the matrix-core work for four modes).  Each
// workgroup leaves one partial block per mode (its waves summed in fp64 in
// wave order); the partials are reduced by the fixed-order reduction of the
// single-mode sketch.  The factor rows a workgroup needs are drawn into LDS
// by the counter-based generator; no factor is stored in HBM.
#include "device_common.h"
#include "kernels.h"
#include "philox.h"

#include <algorithm>
#include <cstring>

namespace krp {

namespace {

constexpr int kFuWaves = 8;
constexpr int kFuMaxSeg = 64;
constexpr int kStagePitch = 36;  // floats per staged i1 column: 32 rows of i0 + 4
constexpr size_t kFuLdsMax = 160 * 1024;

struct FusedArgs {
  const float* x;
  int64_t n0, n1;
  int n_out;  // outer modes: tensor modes 2..d-1
  int64_t o_size[kMaxDims], o_stride[kMaxDims];
  int box[kMaxDims], nbox[kMaxDims];
  int f_blocks, row_blocks;
  int want;  // bit m: mode m is sketched
  int ell[kMaxDims];
  uint64_t seed;
  uint32_t draw;
  int memo;   // one shared factor set (counter field "sketch" = kMemoSketch for every factor)
  int reuse;  // outer modes take the mode-0 product of the slab (shared factors, ell_0 = max ell)
  // factor-table segments (rows of CP columns in LDS)
  int nseg, tab_rows;
  int seg_off[kFuMaxSeg], seg_rows[kFuMaxSeg];
  int seg_kind[kFuMaxSeg];    // 0: rows of the i1 block, 1: rows of the i0 block, 2 + k: outer mode k
  int seg_sketch[kFuMaxSeg];  // sketched mode the factor belongs to
  int seg_factor[kFuMaxSeg];  // tensor mode of the factor
  int off_f[kMaxDims];        // per sketch m: Omega^(m)_1 rows (i1 block)
  int off_r[kMaxDims];        // per sketch m: Omega^(m)_0 rows (i0 block)
  int off_o[kMaxDims][kMaxDims];  // per sketch m and outer mode k: Omega^(m)_{k+2} rows (box)
  int frag_off, stage_off, acc_off, acc_rows;
  int acc_row0[kMaxDims];     // per outer mode k sketched: first accumulator row
  float* part[kMaxDims];      // per sketch m: partial sums [part][n_m][ell_m]
};

// Fragments of the factor operands that do not change along the outer loop
// (Omega^(0)_1, Omega^(m)_1 for outer m, Omega^(1)_0) are split once into the
// policy's MFMA fragments and kept in LDS as 16-byte chunks [frag][chunk][lane].
template <int P>
struct FragStore {
  using Frag = typename Policy<P>::Frag;
  static constexpr int NC = (int)(sizeof(Frag) / 16);
  static_assert(sizeof(Frag) % 16 == 0, "fragments are whole 16-byte chunks");
  __device__ static void put(unsigned char* base, int id, int lane, const Frag& f) {
    uint4 c[NC];
    __builtin_memcpy(c, &f, sizeof(Frag));
#pragma unroll
    for (int k = 0; k < NC; ++k) reinterpret_cast<uint4*>(base)[(id * NC + k) * 64 + lane] = c[k];
  }
  __device__ static Frag get(const unsigned char* base, int id, int lane) {
    uint4 c[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) c[k] = reinterpret_cast<const uint4*>(base)[(id * NC + k) * 64 + lane];
    Frag f;
    __builtin_memcpy(&f, c, sizeof(Frag));
    return f;
  }
};

template <int P, int NT, int NOUT>
__global__ __launch_bounds__(512) void fused_sketch_kernel(FusedArgs a) {
  using Pol = Policy<P>;
  using T = typename Pol::T;
  using FS = FragStore<P>;
  static_assert(sizeof(T) == 4, "fp32, bf16 and split-bf16 policies");
  constexpr int MT = 4;
  constexpr int CP = 16 * NT;
  constexpr int TP = CP + 1;  // table pitch: the lane groups' row reads fall on distinct banks
  extern __shared__ __align__(16) unsigned char smem[];
  T* tab = reinterpret_cast<T*>(smem);
  unsigned char* frg = smem + a.frag_off;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = lane & 15, g = lane >> 4;
  const int fb = blockIdx.x % a.f_blocks;
  const int64_t box_id = blockIdx.x / a.f_blocks;
  const int rb = blockIdx.y;
  const int64_t f0 = (int64_t)fb * 32, a0 = (int64_t)rb * 64;
  float* stage = reinterpret_cast<float*>(smem + a.stage_off) + wave * 32 * kStagePitch;
  float* accl = reinterpret_cast<float*>(smem + a.acc_off) + wave * a.acc_rows * CP;

  // the workgroup's box of outer indices: [lo_k, lo_k + rr_k) per outer mode
  int lo[NOUT + 1], rr[NOUT + 1], bc[NOUT + 1];
  int nsteps = 1;
  {
    int64_t rem = box_id;
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
      bc[k] = (int)(rem % a.nbox[k]);
      rem /= a.nbox[k];
      lo[k] = bc[k] * a.box[k];
      rr[k] = (int)min((int64_t)a.box[k], a.o_size[k] - lo[k]);
      nsteps *= rr[k];
    }
  }

  // Factor rows, four columns per generator call; zeros outside the factor.
  constexpr int NQ = CP / 4;
  for (int e = threadIdx.x; e < a.tab_rows * NQ; e += blockDim.x) {
    const int r = e / NQ, q = e - (e / NQ) * NQ;
    int s = 0;
    while (s + 1 < a.nseg && r >= a.seg_off[s + 1]) ++s;
    const int kind = a.seg_kind[s];
    const int idx = r - a.seg_off[s];
    int64_t row = 0, limit = 0;
    bool inbox = true;
    if (kind == 0) {
      row = f0 + idx;
      limit = a.n1;
    } else if (kind == 1) {
      row = a0 + idx;
      limit = a.n0;
    } else {
#pragma unroll
      for (int k = 0; k < NOUT; ++k)
        if (k == kind - 2) {
          row = lo[k] + idx;
          limit = a.o_size[k];
          inbox = idx < rr[k];
        }
    }
    const int m = a.seg_sketch[s];
    double gq[4];
    gauss_quad(a.seed, counter_word2(a.draw, a.memo ? kMemoSketch : (uint32_t)m, (uint32_t)a.seg_factor[s]), 0,
               (uint64_t)row,
               (uint64_t)q, gq);
    const bool live = inbox && row < limit;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = 4 * q + u;
      tab[r * TP + c] = (live && c < a.ell[m]) ? (T)gq[u] : (T)0;
    }
  }
  for (int e = lane; e < a.acc_rows * CP; e += 64) accl[e] = 0.f;
  __syncthreads();
  // Static fragments: frag ids  [0, NT) mode 0's B (Omega^(0)_1),
  // [NT (1 + k), NT (2 + k)) outer sketch k's B (Omega^(k+2)_1),
  // [NT (1 + NOUT) + 2 t + kc] mode 1's A (Omega^(1)_0, i0 chunk kc).
  const bool want0 = a.want & 1, want1 = (a.want >> 1) & 1;
  for (int e = threadIdx.x; e < NT * (3 + NOUT) * 64; e += blockDim.x) {
    const int id = e / 64, l = e % 64;
    const int ln = l & 15, lg = l >> 4;
    T v[8];
    int base = -1, t = 0, kc = 0;
    bool amode = false;
    if (id < NT) {
      if (want0) base = a.off_f[0];
      t = id;
    } else if (id < NT * (1 + NOUT)) {
      const int k = id / NT - 1;
      if ((a.want >> (k + 2)) & 1) base = a.off_f[k + 2];
      t = id % NT;
    } else {
      const int j2 = id - NT * (1 + NOUT);
      t = j2 / 2;
      kc = j2 % 2;
      amode = true;
      if (want1) base = a.off_r[1];
    }
    if (base < 0) continue;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      v[j] = amode ? tab[(base + 32 * kc + 8 * lg + j) * TP + 16 * t + ln] : tab[(base + 8 * lg + j) * TP + 16 * t + ln];
    FS::put(frg, id, l, Pol::make(v));
  }

  const float* X = a.x;
  // lane (n, g): rows a0 + 4 n .. a0 + 4 n + 3 of i1 = f0 + 8 g + j (clamped:
  // rows past n0 and columns past n1 meet zero factor rows or are not stored)
  const int64_t lrow = min(a0 + 4 * n, a.n0 - 4);
  auto load = [&](float (&buf)[MT][8], int64_t off) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t kk = min(f0 + 8 * g + j, a.n1 - 1);
      const float4 v = *reinterpret_cast<const float4*>(X + off + lrow + kk * a.n0);
      buf[0][j] = v.x;
      buf[1][j] = v.y;
      buf[2][j] = v.z;
      buf[3][j] = v.w;
    }
  };
  // step odometer over the box (digits dig_k in [0, rr_k)), uniform
  struct Odo {
    int s;
    int64_t off;
    int dig[NOUT + 1];
  };
  auto odo_init = [&](int s) {
    Odo z;
    z.s = s;
    z.off = 0;
    int rem = s;
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
      z.dig[k] = rem % rr[k];
      rem /= rr[k];
      z.off += (int64_t)(lo[k] + z.dig[k]) * a.o_stride[k];
    }
    return z;
  };
  auto odo_step = [&](Odo& z, int by) {
    z.s += by;
    int carry = by;
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
      int dn = z.dig[k] + carry;
      carry = 0;
      while (dn >= rr[k]) {
        dn -= rr[k];
        ++carry;
      }
      z.off += (int64_t)(dn - z.dig[k]) * a.o_stride[k];
      z.dig[k] = dn;
    }
  };
  // product over the outer modes (except `skip`) of sketch m's factor rows at column col
  auto outer_weight = [&](const Odo& z, int m, int skip, int col) {
    float w = 1.f;
#pragma unroll
    for (int k = 0; k < NOUT; ++k)
      if (k != skip) w *= (float)tab[(a.off_o[m][k] + z.dig[k]) * TP + col];
    return w;
  };

  typename Pol::Acc acc0[MT][NT];
  typename Pol::Acc acc1[NT][2];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int m = 0; m < MT; ++m) acc0[m][t] = Pol::zero();
    acc1[t][0] = Pol::zero();
    acc1[t][1] = Pol::zero();
  }

  auto compute = [&](const float (&buf)[MT][8], const Odo& z) {
    typename Pol::Frag af[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      T v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (T)buf[m][j];
      af[m] = Pol::make(v);
    }
    if (want0) {
      // the step's weight is applied to the product: acc += W^(0)[o, c] (S Omega^(0)_1);
      // with shared factors the same product also feeds the outer modes'
      // weighted row sums (the memoised partial MTTKRP)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const typename Pol::Frag bf = FS::get(frg, t, lane);
        const float w = outer_weight(z, 0, -1, 16 * t + n);
        float ts[NOUT];
#pragma unroll
        for (int k = 0; k < NOUT; ++k) ts[k] = 0.f;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          typename Pol::Acc u = Pol::zero();
          Pol::mma(u, af[m], bf);
#pragma unroll
          for (int r = 0; r < 4; ++r) acc0[m][t][r] += w * u[r];
          if (a.reuse) {
#pragma unroll
            for (int k = 0; k < NOUT; ++k)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                ts[k] += u[r] * (float)tab[(a.off_r[k + 2] + 4 * Pol::out_row(g, r) + m) * TP + 16 * t + n];
          }
        }
        if (a.reuse) {
#pragma unroll
          for (int k = 0; k < NOUT; ++k) {
            if (!((a.want >> (k + 2)) & 1)) continue;
            float tk = ts[k];
            tk += __shfl_xor(tk, 16, 64);
            tk += __shfl_xor(tk, 32, 64);
            if (g == 0) {
              float* dst = &accl[(a.acc_row0[k] + z.dig[k]) * CP + 16 * t + n];
              *dst += tk * outer_weight(z, k + 2, k, 16 * t + n);
            }
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
      if (a.reuse) break;
      const int ms = k + 2;
      if (!((a.want >> ms) & 1)) continue;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const typename Pol::Frag bf = FS::get(frg, NT * (1 + k) + t, lane);
        float ts = 0.f;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          typename Pol::Acc u = Pol::zero();
          Pol::mma(u, af[m], bf);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            ts += u[r] * (float)tab[(a.off_r[ms] + 4 * Pol::out_row(g, r) + m) * TP + 16 * t + n];
        }
        ts += __shfl_xor(ts, 16, 64);
        ts += __shfl_xor(ts, 32, 64);
        if (g == 0) {
          float* dst = &accl[(a.acc_row0[k] + z.dig[k]) * CP + 16 * t + n];
          *dst += ts * outer_weight(z, ms, k, 16 * t + n);
        }
      }
    }
    if (want1) {
      // the slab, half at a time (i0 rows 32 kc .. 32 kc + 31), into the
      // wave's staging region as [i1][i0]; the lanes holding those rows write
      typename Pol::Acc u1[NT][2];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        u1[t][0] = Pol::zero();
        u1[t][1] = Pol::zero();
      }
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) {
        if ((n >> 3) == kc) {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            *reinterpret_cast<float4*>(&stage[(8 * g + j) * kStagePitch + 4 * (n & 7)]) =
                make_float4(buf[0][j], buf[1][j], buf[2][j], buf[3][j]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        typename Pol::Frag bs[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          const float* src = &stage[(16 * nt + n) * kStagePitch + 8 * g];
          const float4 p0 = *reinterpret_cast<const float4*>(src);
          const float4 p1 = *reinterpret_cast<const float4*>(src + 4);
          const T v[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
          bs[nt] = Pol::make(v);
        }
        // the next half's staging writes must not overtake these reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const typename Pol::Frag aw = FS::get(frg, NT * (1 + NOUT) + 2 * t + kc, lane);
          Pol::mma(u1[t][0], aw, bs[0]);
          Pol::mma(u1[t][1], aw, bs[1]);
        }
      }
      // acc1 += W^(1)[o, c] (Omega^(1)_0^T S), row c of the product = 16 t + out_row(g, r)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float w = outer_weight(z, 1, -1, 16 * t + Pol::out_row(g, r));
          acc1[t][0][r] += w * u1[t][0][r];
          acc1[t][1][r] += w * u1[t][1][r];
        }
    }
  };

  float bufA[MT][8], bufB[MT][8];
  Odo cur = odo_init(wave);
  load(bufA, cur.s < nsteps ? cur.off : 0);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  while (cur.s < nsteps) {
    Odo nxt = cur;
    odo_step(nxt, kFuWaves);
    load(bufB, nxt.s < nsteps ? nxt.off : cur.off);
    compute(bufA, cur);
    cur = nxt;
    if (cur.s >= nsteps) break;
    odo_step(nxt, kFuWaves);
    load(bufA, nxt.s < nsteps ? nxt.off : cur.off);
    compute(bufB, cur);
    cur = nxt;
  }

  // --- partial sums of the workgroup, its waves summed in fp64 in wave order ---
  double* red = reinterpret_cast<double*>(smem + a.stage_off);
  __syncthreads();
  if (want0) {
    for (int w = 0; w < kFuWaves; ++w) {
      if (wave == w) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              double* d = &red[((m * NT + t) * 4 + r) * 64 + lane];
              *d = (w == 0 ? 0.0 : *d) + (double)acc0[m][t][r];
            }
      }
      __syncthreads();
    }
    if (wave == 0) {
      const int l0 = a.ell[0];
      float* p = a.part[0] + (int64_t)blockIdx.x * a.n0 * l0;
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = a0 + 4 * Pol::out_row(g, r) + m;
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const int c = 16 * t + n;
            if (row < a.n0 && c < l0) p[row * l0 + c] = (float)red[((m * NT + t) * 4 + r) * 64 + lane];
          }
        }
    }
    __syncthreads();
  }
  if (want1) {
    for (int w = 0; w < kFuWaves; ++w) {
      if (wave == w) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              double* d = &red[((t * 2 + nt) * 4 + r) * 64 + lane];
              *d = (w == 0 ? 0.0 : *d) + (double)acc1[t][nt][r];
            }
      }
      __syncthreads();
    }
    if (wave == 0) {
      const int l1 = a.ell[1];
      float* p = a.part[1] + ((int64_t)rb + (int64_t)a.row_blocks * box_id) * a.n1 * l1;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = 16 * t + Pol::out_row(g, r);
            const int64_t i1 = f0 + 16 * nt + n;
            if (i1 < a.n1 && c < l1) p[i1 * l1 + c] = (float)red[((t * 2 + nt) * 4 + r) * 64 + lane];
          }
    }
    __syncthreads();
  }
  // outer modes: the waves' accumulator rows, summed in wave order
#pragma unroll
  for (int k = 0; k < NOUT; ++k) {
    const int ms = k + 2;
    if (!((a.want >> ms) & 1)) continue;
    const int lm = a.ell[ms];
    // partial index: (row block, i1 block, box coordinates other than k)
    int64_t pbox = 0, mul = 1;
#pragma unroll
    for (int kk = 0; kk < NOUT; ++kk) {
      if (kk == k) continue;
      pbox += bc[kk] * mul;
      mul *= a.nbox[kk];
    }
    const int64_t part = rb + (int64_t)a.row_blocks * (fb + (int64_t)a.f_blocks * pbox);
    float* p = a.part[ms] + part * a.o_size[k] * lm;
    const float* base = reinterpret_cast<const float*>(smem + a.acc_off);
    for (int e = threadIdx.x; e < rr[k] * lm; e += blockDim.x) {
      const int dr = e / lm, c = e - (e / lm) * lm;
      double s = 0.0;
      for (int w = 0; w < kFuWaves; ++w) s += (double)base[(w * a.acc_rows + a.acc_row0[k] + dr) * CP + c];
      p[(int64_t)(lo[k] + dr) * lm + c] = (float)s;
    }
  }
}

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

template <int P, int NOUT>
hipError_t fused_go_nout(int nt, const FusedArgs& a, dim3 grid, size_t lds, hipStream_t st) {
  auto pick = [&](auto kern) -> hipError_t {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(64 * kFuWaves), lds, st, a);
    return hipGetLastError();
  };
  switch (nt) {
    case 1: return pick(fused_sketch_kernel<P, 1, NOUT>);
    case 2: return pick(fused_sketch_kernel<P, 2, NOUT>);
    case 3: return pick(fused_sketch_kernel<P, 3, NOUT>);
    default: return pick(fused_sketch_kernel<P, 4, NOUT>);
  }
}

template <int P>
hipError_t fused_go(int nt, const FusedArgs& a, dim3 grid, size_t lds, hipStream_t st) {
  switch (a.n_out) {
    case 1: return fused_go_nout<P, 1>(nt, a, grid, lds, st);
    case 2: return fused_go_nout<P, 2>(nt, a, grid, lds, st);
    case 3: return fused_go_nout<P, 3>(nt, a, grid, lds, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Plan of the fused pass for the sketches of `pbs` (all of the same tensor,
// seed and draw).  ok = false when the fused kernel does not apply (fp64
// storage or arithmetic, n_0 not a multiple of 4, misaligned X, fewer than
// two modes, or no box of at least 64 steps fits the LDS).
FusedPlan plan_fused(const SketchProblem* pbs, int nmodes) {
  FusedPlan fp{};
  fp.ok = false;
  if (nmodes < 2) return fp;
  if (pbs[0].d < 3 || pbs[0].d > 5) return fp;  // one to three outer modes
  const SketchProblem& p0 = pbs[0];
  const int d = p0.d;
  if (p0.x_is_double || p0.prec == kFP64) return fp;
  if (p0.dims[0] % 4 != 0) return fp;
  if (p0.x && (reinterpret_cast<uintptr_t>(p0.x) & 15) != 0) return fp;
  int ell[kMaxDims] = {0};
  int want = 0, lmax = 0;
  for (int j = 0; j < nmodes; ++j) {
    const SketchProblem& pb = pbs[j];
    if (pb.prec != p0.prec || pb.seed != p0.seed || pb.draw != p0.draw || pb.d != d) return fp;
    const bool memo_pb = pb.sketch_id == kMemoSketch;
    if (!memo_pb && pb.sketch_id != (uint32_t)pb.mode) return fp;
    if (memo_pb != (p0.sketch_id == kMemoSketch)) return fp;
    want |= 1 << pb.mode;
    ell[pb.mode] = pb.ell;
    lmax = std::max(lmax, pb.ell);
  }
  const int nt = (lmax + 15) / 16;
  const int cp = 16 * nt;
  const int n_out = d - 2;
  int64_t o_size[kMaxDims] = {0};
  for (int k = 0; k < n_out; ++k) o_size[k] = p0.dims[k + 2];
  const int row_blocks = (int)((p0.dims[0] + 63) / 64);
  const int f_blocks = (int)((p0.dims[1] + 31) / 32);
  // boxes: halve the largest extent until a box has at most 512 steps (eight
  // waves, at most 64 fp32-accumulated steps each) and the grid has at least
  // 256 workgroups, then until the LDS fits
  int box[kMaxDims];
  for (int k = 0; k < n_out; ++k) box[k] = (int)o_size[k];
  auto steps = [&] {
    int64_t s = 1;
    for (int k = 0; k < n_out; ++k) s *= box[k];
    return s;
  };
  auto nboxes = [&] {
    int64_t s = 1;
    for (int k = 0; k < n_out; ++k) s *= (o_size[k] + box[k] - 1) / box[k];
    return s;
  };
  // halves the largest extent unless that leaves fewer than 64 steps
  auto halve_largest = [&] {
    int kb = -1;
    for (int k = 0; k < n_out; ++k)
      if (box[k] > 1 && (kb < 0 || box[k] > box[kb])) kb = k;
    if (kb < 0) return false;
    const int keep = box[kb];
    box[kb] = (box[kb] + 1) / 2;
    if (steps() < 64) {
      box[kb] = keep;
      return false;
    }
    return true;
  };
  while (steps() > 512 || nboxes() * row_blocks * f_blocks < 256)
    if (!halve_largest()) break;
  const bool want1 = (want >> 1) & 1;
  auto layout = [&](FusedArgs& a) {
    int rows = 0, ns = 0;
    auto seg = [&](int kind, int nrows, int sketch, int factor) {
      a.seg_off[ns] = rows;
      a.seg_rows[ns] = nrows;
      a.seg_kind[ns] = kind;
      a.seg_sketch[ns] = sketch;
      a.seg_factor[ns] = factor;
      ++ns;
      const int off = rows;
      rows += nrows;
      return off;
    };
    int acc_rows = 0;
    for (int m = 0; m < d; ++m) {
      if (!((want >> m) & 1)) continue;
      if (m != 1) a.off_f[m] = seg(0, 32, m, 1);
      if (m != 0) a.off_r[m] = seg(1, 64, m, 0);
      for (int k = 0; k < n_out; ++k)
        if (k + 2 != m) a.off_o[m][k] = seg(2 + k, box[k], m, k + 2);
      if (m >= 2) {
        a.acc_row0[m - 2] = acc_rows;
        acc_rows += box[m - 2];
      }
    }
    a.nseg = ns;
    a.tab_rows = rows;
    a.acc_rows = acc_rows;
    const size_t tab = (size_t)rows * (cp + 1) * 4;                       // pitch cp + 1
    const size_t frag = (size_t)nt * (3 + n_out) * 64 * 32;               // static fragments
    const size_t stage = want1 ? (size_t)kFuWaves * 32 * kStagePitch * 4 : 0;
    const size_t red = (size_t)std::max(4 * nt, 2 * nt) * 4 * 64 * sizeof(double);  // end-of-kernel wave sums
    a.frag_off = (int)((tab + 15) / 16 * 16);
    a.stage_off = (int)(a.frag_off + frag);
    a.acc_off = (int)(a.stage_off + (std::max(stage, red) + 15) / 16 * 16);
    return (size_t)a.acc_off + (size_t)kFuWaves * acc_rows * cp * 4;
  };
  FusedArgs a{};
  size_t lds = layout(a);
  while (lds > kFuLdsMax) {
    if (!halve_largest()) break;
    a = FusedArgs{};
    lds = layout(a);
  }
  if (lds > kFuLdsMax || steps() < 64) return fp;
  a.n0 = p0.dims[0];
  a.n1 = p0.dims[1];
  a.n_out = n_out;
  int64_t stride = p0.dims[0] * p0.dims[1];
  for (int k = 0; k < n_out; ++k) {
    a.o_size[k] = o_size[k];
    a.o_stride[k] = stride;
    stride *= o_size[k];
    a.box[k] = box[k];
    a.nbox[k] = (int)((o_size[k] + box[k] - 1) / box[k]);
  }
  a.f_blocks = f_blocks;
  a.row_blocks = row_blocks;
  a.want = want;
  for (int m = 0; m < d; ++m) a.ell[m] = ell[m];
  a.seed = p0.seed;
  a.draw = p0.draw;
  a.memo = p0.sketch_id == kMemoSketch ? 1 : 0;
  // the outer modes reuse the mode-0 product when every mode is sketched
  // with the shared factors and mode 0 has the widest column range
  a.reuse = (a.memo && want == (1 << d) - 1 && ell[0] == lmax) ? 1 : 0;
  fp.args_bytes = sizeof(FusedArgs);
  static_assert(sizeof(FusedArgs) <= sizeof(fp.args), "FusedPlan::args holds FusedArgs");
  std::memcpy(fp.args, &a, sizeof(FusedArgs));
  fp.nt = nt;
  fp.lds = lds;
  const int64_t nb = nboxes();
  fp.grid_x = (int64_t)f_blocks * nb;
  fp.grid_y = row_blocks;
  // partial blocks per mode and the reduction's workspace
  size_t off = 0;
  for (int m = 0; m < d; ++m) {
    fp.nparts[m] = 0;
    if (!((want >> m) & 1)) continue;
    int64_t np;
    if (m == 0) np = (int64_t)f_blocks * nb;
    else if (m == 1) np = (int64_t)row_blocks * nb;
    else np = (int64_t)row_blocks * f_blocks * (nb / a.nbox[m - 2]);
    fp.nparts[m] = np;
    fp.part_off[m] = off;
    off = round256(off + (size_t)np * p0.dims[m] * ell[m] * sizeof(float));
    fp.lvl_off[m] = off;
    off = round256(off + partial_reduce_lvl_bytes((int)np, p0.dims[m], cp, 1));
  }
  fp.ws_bytes = off;
  fp.ok = true;
  return fp;
}

hipError_t launch_fused(const FusedPlan& fp, const SketchProblem* pbs, int nmodes, void* ws,
                        double* const* y64, void* const* y_out, int out_is_double, hipStream_t st) {
  if (!fp.ok || nmodes < 1) return hipErrorInvalidValue;
  FusedArgs a;
  std::memcpy(&a, fp.args, sizeof(FusedArgs));
  a.x = reinterpret_cast<const float*>(pbs[0].x);
  if ((reinterpret_cast<uintptr_t>(a.x) & 15) != 0) return hipErrorInvalidValue;
  char* w = reinterpret_cast<char*>(ws);
  for (int j = 0; j < nmodes; ++j) {
    const int m = pbs[j].mode;
    a.part[m] = reinterpret_cast<float*>(w + fp.part_off[m]);
  }
  const dim3 grid((unsigned)fp.grid_x, (unsigned)fp.grid_y);
  hipError_t e;
  switch (pbs[0].prec) {
    case kFP32: e = fused_go<kFP32>(fp.nt, a, grid, fp.lds, st); break;
    case kBF16: e = fused_go<kBF16>(fp.nt, a, grid, fp.lds, st); break;
    case kBF16X3: e = fused_go<kBF16X3>(fp.nt, a, grid, fp.lds, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  for (int j = 0; j < nmodes; ++j) {
    const int m = pbs[j].mode;
    e = launch_partial_reduce(w + fp.part_off[m], false, (int)fp.nparts[m], pbs[j].dims[m], pbs[j].ell,
                              16 * fp.nt, 1, w + fp.lvl_off[m], y64 ? y64[j] : nullptr,
                              y_out ? y_out[j] : nullptr, out_is_double, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace krp
