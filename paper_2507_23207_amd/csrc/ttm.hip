// Tensor-times-matrix G_new = G x_i Q^T (Algorithm 7, step 6; Algorithm 8,
// step 6): G_new_(i) = Q^T G_(i) for a tensor in Kolda order and an n x l
// orthonormal Q.  The tensor is viewed as g[p, a, q] (p = modes before i,
// a = i_i, q = modes after i); G_new[p, c, q] = sum_a g[p, a, q] Q[a, c].
//
// Mode 0 (p empty): MFMA tile D[q][c] = sum_a G[a, q] Q[a, c]; the reduction
// runs along the contiguous index a (vector loads), results are written row
// by row of the l x (rest) output.
// Other modes: D[c][(p, q)] = sum_a Q[a, c] g[p, a, q]; 16 columns (p, q)
// form the B operand and the output columns: 16 consecutive p of one q, or,
// for a short p range (a compressed first mode, P < 64), 16 consecutive
// values of the flattened index J = p + P q (runs of P contiguous elements,
// a tile may span several q), which leaves no lanes idle.
// The workgroup walks the reduction index in 32-wide slices in lockstep; each
// slice of Q is staged once in LDS (double-buffered) for all its waves.
#include "device_common.h"
#include "kernels.h"

#include <algorithm>
#include <type_traits>

namespace krp {

namespace {

constexpr int kTtmWaves = 8;
constexpr int kSlicePitch = 36;  // 32 reduction slots + padding (elements)
constexpr int64_t kSplitMaxWaves = 8192;  // below this many one-wave items, the split kernel
constexpr int kTtmColTiles = 2;  // non-mode-0: 16-column tiles of (p, q) per wave

struct TtmArgs {
  const void* g;
  void* out;
  const double* q;
  int64_t P, n, Q;  // g[p, a, q] sizes
  int ell;
  int64_t ldc;      // extent of the output mode (ell, or more for a column chunk)
  int cw;           // output columns written: ell, or ldc when the padding is zero-filled
  int64_t items;
  int p_groups;     // non-mode-0: p groups per q (0: flattened (p, q) columns)
};

// Reduction slot -> k offset inside a 32-wide slice.  With vector loads of VW
// elements along the contiguous index, lane group g reads VW-element pieces so
// that the four groups of a row cover 4 VW contiguous elements per load.
template <int VW>
__device__ __forceinline__ int tkmap(int g, int j) {
  if constexpr (VW > 1) {
    return VW * g + 4 * VW * (j / VW) + (j % VW);
  } else {
    return 8 * g + j;
  }
}

// VW consecutive elements at p (aligned to VW elements).
template <typename Tin, int VW>
__device__ __forceinline__ void load_vec(const Tin* p, Tin (&q)[VW]) {
  if constexpr (VW == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    q[0] = t.x;
    q[1] = t.y;
    q[2] = t.z;
    q[3] = t.w;
  } else if constexpr (VW == 2 && sizeof(Tin) == 8) {
    const double2 t = *reinterpret_cast<const double2*>(p);
    q[0] = t.x;
    q[1] = t.y;
  } else if constexpr (VW == 2) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    q[0] = t.x;
    q[1] = t.y;
  } else {
    q[0] = p[0];
  }
}

// VW: elements per load along the reduction index of mode 0 (1, 2 or 4 for
// fp32 storage; 1 or 2 for fp64), chosen from n and the alignment of G.
template <typename Tin, int P, bool MODE0, int VW, int MT, int NT>
__global__ __launch_bounds__(64 * kTtmWaves) void ttm_kernel(TtmArgs a) {
  using Pol = Policy<P>;
  using T = typename Pol::T;
  using Tout = typename std::conditional<P == kFP64, double, float>::type;
  constexpr int CQ = 16 * (MODE0 ? NT : MT);  // padded columns of Q
  __shared__ __align__(16) T slice[2][CQ * kSlicePitch];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = lane & 15, g = lane >> 4;
  const int64_t item = (int64_t)blockIdx.x * kTtmWaves + wave;
  const bool active = item < a.items;
  int64_t q0 = 0;
  // non-mode-0: element (p, a = 0, q) of the tile-t column J = 16 (NT item + t) + n
  int64_t jb[NT], jo[NT];
  bool jv[NT];
  if constexpr (MODE0) {
    q0 = item * (16 * MT);
  } else if (a.p_groups == 0) {  // flattened (p, q) columns
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t J = (item * NT + t) * 16 + n;
      jv[t] = J < a.P * a.Q;
      const int64_t qi = J / a.P, pi = J - qi * a.P;
      jb[t] = pi + a.P * a.n * qi;
      jo[t] = pi + a.P * a.ldc * qi;
    }
  } else {  // groups of 16 NT consecutive p of one q
    const int64_t qi = item / a.p_groups;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t pi = (item % a.p_groups) * (16 * NT) + 16 * t + n;
      jv[t] = pi < a.P;
      jb[t] = pi + a.P * a.n * qi;
      jo[t] = pi + a.P * a.ldc * qi;
    }
  }
  const Tin* G = reinterpret_cast<const Tin*>(a.g);

  typename Pol::Acc acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = Pol::zero();

  auto stage = [&](int buf, int64_t k0) {
    constexpr int kPer = (CQ * 32 + 64 * kTtmWaves - 1) / (64 * kTtmWaves);
    T qv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + u * 64 * kTtmWaves;
      const int c = e / 32, k = e % 32;
      qv[u] = (e < CQ * 32 && c < a.ell && k0 + k < a.n) ? (T)a.q[(k0 + k) + a.n * c] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + u * 64 * kTtmWaves;
      if (e < CQ * 32) slice[buf][(e / 32) * kSlicePitch + e % 32] = qv[u];
    }
  };

  const int nslices = (int)((a.n + 31) / 32);
  stage(0, 0);
  __syncthreads();
  for (int s = 0; s < nslices; ++s) {
    const int buf = s & 1;
    const int64_t k0 = (int64_t)s * 32;
    if (s + 1 < nslices) stage(buf ^ 1, k0 + 32);
    if (active) {
      const T* sl = slice[buf];
      if constexpr (MODE0) {
        typename Pol::Frag bf[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          T v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = sl[(16 * t + n) * kSlicePitch + tkmap<VW>(g, j)];
          bf[t] = Pol::make(v);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          // branch-free: the row is clamped to Q - 1 and the piece to the
          // last one (n is a multiple of VW), out-of-range values zeroed by a
          // select after unconditional loads, so the loads stay in flight
          const int64_t qi = q0 + 16 * m + n;
          const bool qv = qi < a.Q;
          const int64_t base = a.n * (qv ? qi : a.Q - 1);
          T v[8];
#pragma unroll
          for (int h = 0; h < 8 / VW; ++h) {
            const int64_t kk = k0 + (VW > 1 ? VW * g + 4 * VW * h : 8 * g + h);
            const bool kv = qv && kk < a.n;
            Tin q[VW];
            load_vec<Tin, VW>(G + base + (kk < a.n ? kk : a.n - VW), q);
#pragma unroll
            for (int u = 0; u < VW; ++u) v[VW * h + u] = kv ? (T)q[u] : (T)0;
          }
          const typename Pol::Frag af = Pol::make(v);
#pragma unroll
          for (int t = 0; t < NT; ++t) Pol::mma(acc[m][t], af, bf[t]);
        }
      } else {
        typename Pol::Frag af[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          T v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = sl[(16 * m + n) * kSlicePitch + 8 * g + j];
          af[m] = Pol::make(v);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          T v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int64_t ai = k0 + 8 * g + j;
            Tin x = (Tin)0;
            if (jv[t] && ai < a.n) x = G[jb[t] + a.P * ai];
            v[j] = (T)x;
          }
          const typename Pol::Frag bfr = Pol::make(v);
#pragma unroll
          for (int m = 0; m < MT; ++m) Pol::mma(acc[m][t], af[m], bfr);
        }
      }
    }
    __syncthreads();
  }

  if (!active) return;
  Tout* out = reinterpret_cast<Tout*>(a.out);
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (MODE0) {
          const int64_t qi = q0 + 16 * m + Pol::out_row(g, r);
          const int c = 16 * t + n;
          if (qi < a.Q && c < a.cw) out[c + a.ldc * qi] = (Tout)acc[m][t][r];
        } else {
          const int c = 16 * m + Pol::out_row(g, r);
          if (jv[t] && c < a.ell) out[jo[t] + a.P * c] = (Tout)acc[m][t][r];
        }
      }
}

// Other modes with few items (small cores): one workgroup per (q, p group)
// and the reduction index split over the waves.  Wave w takes the 32-row
// slices w, w + 8, ...; it loads a slice's G and Q together and stages Q in
// a private LDS region.
// The eight partial accumulators are summed in wave order through LDS.
template <typename Tin, int P, int MT, int NT>
__global__ __launch_bounds__(64 * kTtmWaves) void ttm_split_kernel(TtmArgs a) {
  using Pol = Policy<P>;
  using T = typename Pol::T;
  using AccT = typename Pol::AccT;
  using Tout = typename std::conditional<P == kFP64, double, float>::type;
  constexpr int CQ = 16 * MT;
  constexpr int kStage = CQ * kSlicePitch;
  extern __shared__ __align__(16) unsigned char ttm_smem[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = lane & 15, g = lane >> 4;
  T* st = reinterpret_cast<T*>(ttm_smem) + wave * kStage;
  const int64_t qq = blockIdx.x / a.p_groups;
  const int64_t p0 = (int64_t)(blockIdx.x % a.p_groups) * (16 * NT);
  const Tin* G = reinterpret_cast<const Tin*>(a.g);
  const int nslices = (int)((a.n + 31) / 32);

  typename Pol::Acc acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = Pol::zero();

  auto load_b = [&](Tin (&x)[NT][8], int s) {
    const int64_t k0 = (int64_t)s * 32;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t pi = p0 + 16 * t + n;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t ai = k0 + 8 * g + j;
        x[t][j] = (pi < a.P && ai < a.n) ? G[pi + a.P * (ai + a.n * qq)] : (Tin)0;
      }
    }
  };
  // One slice: its loads of G and of Q are issued together (one memory
  // latency per slice), then Q goes through the wave's LDS region.
  auto step = [&](int s) {
    Tin x[NT][8];
    load_b(x, s);
    const int64_t k0 = (int64_t)s * 32;
    T qv[CQ / 2];
#pragma unroll
    for (int u = 0; u < CQ / 2; ++u) {
      const int e = lane + 64 * u;
      const int c = e / 32, k = e % 32;
      qv[u] = (c < a.ell && k0 + k < a.n) ? (T)a.q[(k0 + k) + a.n * c] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < CQ / 2; ++u) {
      const int e = lane + 64 * u;
      st[(e / 32) * kSlicePitch + e % 32] = qv[u];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    typename Pol::Frag af[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      T v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = st[(16 * m + n) * kSlicePitch + 8 * g + j];
      af[m] = Pol::make(v);
    }
    // the next slice's staging must not overtake these reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      T v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (T)x[t][j];
      const typename Pol::Frag bfr = Pol::make(v);
#pragma unroll
      for (int m = 0; m < MT; ++m) Pol::mma(acc[m][t], af[m], bfr);
    }
  };
  for (int s = wave; s < nslices; s += kTtmWaves) step(s);

  // sum of the eight partial accumulators, in wave order
  __syncthreads();
  AccT* red = reinterpret_cast<AccT*>(ttm_smem);
  constexpr int E = MT * NT * 4 * 64;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave * E + ((m * NT + t) * 4 + r) * 64 + lane] = acc[m][t][r];
  __syncthreads();
  Tout* out = reinterpret_cast<Tout*>(a.out);
  for (int e = threadIdx.x; e < E; e += 64 * kTtmWaves) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kTtmWaves; ++w) sum += (double)red[w * E + e];
    const int ln = e % 64, mtr = e / 64;
    const int r = mtr % 4, mt = mtr / 4;
    const int t = mt % NT, m = mt / NT;
    const int c = 16 * m + Pol::out_row(ln >> 4, r);
    const int64_t pi = p0 + 16 * t + (ln & 15);
    if (pi < a.P && c < a.ell) out[pi + a.P * (c + a.ldc * qq)] = (Tout)sum;
  }
}

template <typename Tin, int P, int MT, int NT>
hipError_t ttm_split_go(const TtmArgs& a, hipStream_t st) {
  using T = typename Policy<P>::T;
  using AccT = typename Policy<P>::AccT;
  constexpr size_t stage = (size_t)kTtmWaves * 16 * MT * kSlicePitch * sizeof(T);
  constexpr size_t red = (size_t)kTtmWaves * MT * NT * 4 * 64 * sizeof(AccT);
  constexpr size_t lds = stage > red ? stage : red;
  auto kern = ttm_split_kernel<Tin, P, MT, NT>;
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)a.items), dim3(64 * kTtmWaves), lds, st, a);
  return hipGetLastError();
}

template <typename Tin, int P, int MT>
hipError_t ttm_split_nt(int nt, const TtmArgs& a, hipStream_t st) {
  // fp64 arithmetic: at most two p tiles (the double-buffered fp64 loads and
  // accumulators of wider groups do not fit in registers)
  // (four Q tiles: one p tile in fp64, three otherwise)
  if constexpr (P == kFP64 && MT == 4) {
    return ttm_split_go<Tin, P, MT, 1>(a, st);
  } else if constexpr (P == kFP64) {
    return nt == 1 ? ttm_split_go<Tin, P, MT, 1>(a, st) : ttm_split_go<Tin, P, MT, 2>(a, st);
  } else if constexpr (MT == 4) {
    switch (nt) {
      case 1: return ttm_split_go<Tin, P, MT, 1>(a, st);
      case 2: return ttm_split_go<Tin, P, MT, 2>(a, st);
      default: return ttm_split_go<Tin, P, MT, 3>(a, st);
    }
  } else {
    switch (nt) {
      case 1: return ttm_split_go<Tin, P, MT, 1>(a, st);
      case 2: return ttm_split_go<Tin, P, MT, 2>(a, st);
      case 3: return ttm_split_go<Tin, P, MT, 3>(a, st);
      default: return ttm_split_go<Tin, P, MT, 4>(a, st);
    }
  }
}

template <typename Tin, int P>
hipError_t ttm_split_dispatch(int tiles_c, int nt, const TtmArgs& a, hipStream_t st) {
  switch (tiles_c) {
    case 1: return ttm_split_nt<Tin, P, 1>(nt, a, st);
    case 2: return ttm_split_nt<Tin, P, 2>(nt, a, st);
    case 3: return ttm_split_nt<Tin, P, 3>(nt, a, st);
    default: return ttm_split_nt<Tin, P, 4>(nt, a, st);
  }
}

template <typename Tin, int P, bool MODE0, int VW, int MT, int NT>
hipError_t ttm_go(const TtmArgs& a, hipStream_t st) {
  const unsigned grid = (unsigned)((a.items + kTtmWaves - 1) / kTtmWaves);
  hipLaunchKernelGGL((ttm_kernel<Tin, P, MODE0, VW, MT, NT>), dim3(grid), dim3(64 * kTtmWaves), 0,
                     st, a);
  return hipGetLastError();
}

template <typename Tin, int P, int VW>
hipError_t ttm_mode0(int tiles_c, const TtmArgs& a, hipStream_t st) {
  switch (tiles_c) {
    case 1: return ttm_go<Tin, P, true, VW, 4, 1>(a, st);
    case 2: return ttm_go<Tin, P, true, VW, 4, 2>(a, st);
    case 3: return ttm_go<Tin, P, true, VW, 4, 3>(a, st);
    default: return ttm_go<Tin, P, true, VW, 4, 4>(a, st);
  }
}

template <typename Tin, int P>
hipError_t ttm_dispatch(bool mode0, int vw, int tiles_c, const TtmArgs& a, hipStream_t st) {
  if (mode0) {
    if constexpr (sizeof(Tin) == 4) {
      if (vw == 4) return ttm_mode0<Tin, P, 4>(tiles_c, a, st);
    }
    if (vw == 2) return ttm_mode0<Tin, P, 2>(tiles_c, a, st);
    return ttm_mode0<Tin, P, 1>(tiles_c, a, st);
  }
  switch (tiles_c) {
    case 1: return ttm_go<Tin, P, false, 1, 1, kTtmColTiles>(a, st);
    case 2: return ttm_go<Tin, P, false, 1, 2, kTtmColTiles>(a, st);
    case 3: return ttm_go<Tin, P, false, 1, 3, kTtmColTiles>(a, st);
    default: return ttm_go<Tin, P, false, 1, 4, kTtmColTiles>(a, st);
  }
}

}  // namespace

hipError_t launch_ttm(const TtmProblem& pb, hipStream_t st) {
  if (pb.ell < 1 || pb.ell > 64) return hipErrorInvalidValue;
  if (pb.out_ld != 0 && pb.out_ld < pb.ell) return hipErrorInvalidValue;
  TtmArgs a{};
  a.g = pb.g;
  a.out = pb.out;
  a.q = pb.q64;
  int64_t P = 1, Q = 1;
  for (int k = 0; k < pb.mode; ++k) P *= pb.dims[k];
  for (int k = pb.mode + 1; k < pb.d; ++k) Q *= pb.dims[k];
  a.P = P;
  a.n = pb.dims[pb.mode];
  a.Q = Q;
  a.ell = pb.ell;
  a.ldc = pb.out_ld > 0 ? pb.out_ld : pb.ell;
  a.cw = pb.zero_pad ? (int)a.ldc : pb.ell;  // the accumulators of columns past ell are zero
  if (pb.zero_pad && (P != 1 || a.ldc > 64)) return hipErrorInvalidValue;
  const int tiles_c = (a.cw + 15) / 16;
  const bool mode0 = (P == 1);
  // widest aligned load along the reduction index of mode 0
  const uintptr_t gaddr = reinterpret_cast<uintptr_t>(pb.g);
  const size_t esz = pb.g_is_double ? 8 : 4;
  int vw = 1;
  if (mode0) {
    if (!pb.g_is_double && a.n % 4 == 0 && (gaddr & 15) == 0) vw = 4;
    else if (a.n % 2 == 0 && (gaddr & (2 * esz - 1)) == 0) vw = 2;
  }
  // Few items (small cores): the split kernel, one workgroup per (q, group of
  // up to 64 p) with the reduction index spread over its waves.
  bool split = false;
  int split_nt = 4;
  const int nt_max = pb.prec == kFP64 ? (tiles_c >= 4 ? 1 : 2) : (tiles_c >= 4 ? 3 : 4);
  const bool want_split = pb.tile.split >= 0 ? pb.tile.split == 1 : Q * ((P + 31) / 32) < kSplitMaxWaves;
  if (mode0) {
    a.items = (Q + 63) / 64;
    a.p_groups = 1;
  } else if (want_split) {
    split = true;
    const int nt = pb.tile.nt > 0 ? std::min(pb.tile.nt, nt_max) : nt_max;
    split_nt = (int)std::min<int64_t>(nt, (P + 15) / 16);
    a.p_groups = (int)((P + 16 * split_nt - 1) / (16 * split_nt));
    a.items = Q * a.p_groups;
  } else {
    constexpr int cw = 16 * kTtmColTiles;  // (p, q) columns of a wave
    if (P < 64) {
      a.p_groups = 0;
      a.items = (P * Q + cw - 1) / cw;
    } else {
      a.p_groups = (int)((P + cw - 1) / cw);
      a.items = Q * a.p_groups;
    }
  }
  if (a.items == 0) return hipSuccess;
  const bool wants_double_out = pb.prec == kFP64;
  if (wants_double_out != (pb.out_is_double != 0)) return hipErrorInvalidValue;
  if (split) {
    if (pb.g_is_double) {
      if (pb.prec != kFP64) return hipErrorInvalidValue;
      return ttm_split_dispatch<double, kFP64>(tiles_c, split_nt, a, st);
    }
    switch (pb.prec) {
      case kFP64: return ttm_split_dispatch<float, kFP64>(tiles_c, split_nt, a, st);
      case kFP32: return ttm_split_dispatch<float, kFP32>(tiles_c, split_nt, a, st);
      case kBF16: return ttm_split_dispatch<float, kBF16>(tiles_c, split_nt, a, st);
      default: return ttm_split_dispatch<float, kBF16X3>(tiles_c, split_nt, a, st);
    }
  }
  if (pb.g_is_double) {
    if (pb.prec != kFP64) return hipErrorInvalidValue;
    return ttm_dispatch<double, kFP64>(mode0, vw, tiles_c, a, st);
  }
  switch (pb.prec) {
    case kFP64: return ttm_dispatch<float, kFP64>(mode0, vw, tiles_c, a, st);
    case kFP32: return ttm_dispatch<float, kFP32>(mode0, vw, tiles_c, a, st);
    case kBF16: return ttm_dispatch<float, kBF16>(mode0, vw, tiles_c, a, st);
    default: return ttm_dispatch<float, kBF16X3>(mode0, vw, tiles_c, a, st);
  }
}


int ttm_tile_candidates(const TtmProblem& pb, TtmTile* out, int max) {
  int n = 0;
  if (max < 1) return 0;
  out[n++] = TtmTile{};  // the planner's choice
  int64_t P = 1;
  for (int k = 0; k < pb.mode; ++k) P *= pb.dims[k];
  if (P == 1) return n;  // mode 1: one tiling
  const int tiles_c = (pb.ell + 15) / 16;
  const int nt_max = pb.prec == kFP64 ? (tiles_c >= 4 ? 1 : 2) : (tiles_c >= 4 ? 3 : 4);
  if (n < max) out[n++] = TtmTile{0, 0};
  for (int nt = 1; nt <= nt_max && n < max; ++nt)
    if (16 * (nt - 1) < P) out[n++] = TtmTile{1, nt};
  return n;
}

}  // namespace krp
