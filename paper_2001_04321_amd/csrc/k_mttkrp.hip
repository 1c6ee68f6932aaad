// Dense MTTKRP on gfx950 matrix cores.
//
// P[i, p] = sum_{(a, b)} T[a, i, b] * K[(a, b), p],   K[(a,b), p] = prod_{l != n} A_l[j_l, p]
//
// (paper Sec. 2, eqs. def:B and def:grad: the data term T_[n] B^(n)). T is viewed from
// mode n as a C-order (L, I_n, R) array, L = prod_{l<n} I_l, R = prod_{l>n} I_l. The
// reduction index (a, b) is split into chunks of KC consecutive values:
//   layout 0 (R > 1): a chunk is one a and KC consecutive b, so each output row reads a
//                     contiguous KC-element segment of T;
//   layout 1 (R = 1): a chunk is KC consecutive a; rows i are contiguous in memory and the
//                     tile is transposed while it is stored to LDS.
// A workgroup (4 waves) owns MT = 32*WM output rows and a contiguous range of chunks
// (one reduction split); WK waves share a chunk along the reduction. Per chunk it streams
// the T tile from HBM into registers one chunk ahead, forms the Khatri-Rao rows of the
// chunk in LDS from factor rows (never in HBM), and runs 32x32 MFMAs: float32 tensors on
// v_mfma_f32_32x32x2_f32, bfloat16 tensors on v_mfma_f32_32x32x16_bf16, accumulating in
// float32. Splits write partial tiles that a second kernel sums in a fixed order, so the
// result is deterministic.
#include "ntf_internal.h"

namespace ntf {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;

// Magic-number division for 0 <= x < 2^31 (Granlund-Montgomery round-up method):
// q = (x * m) >> (31 + l) with l = ceil(log2 d), m = ceil(2^(31+l) / d) < 2^32.
struct FastDiv {
  uint32_t d;
  uint32_t m;
  uint32_t sh;  // l - 1 (shift applied to the high product word), or 0xffffffff for d == 1
};

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  if (d == 1) {
    f.m = 0;
    f.sh = 0xffffffffu;
    return f;
  }
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  __uint128_t num = (__uint128_t(1) << (31 + l));
  uint64_t m = uint64_t((num + d - 1) / d);
  f.m = uint32_t(m);
  f.sh = l - 1;
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv& f) {
  if (f.sh == 0xffffffffu) return x;
  return __umulhi(x, f.m) >> f.sh;
}

struct KArgs {
  const void* T;
  float* out;               // P (splits == 1) or partials
  FactorPtrs A;
  int64_t L, I, R;          // mode view
  int64_t chunks;           // total reduction chunks
  int64_t nb;               // chunks per a (layout 0)
  int64_t chunks_per_split; // floor
  int64_t extra;            // first `extra` splits take one more chunk
  int order, mode, r;
  FastDiv fd[kMaxOrder];    // per-mode divisors
  FastDiv fd_nb;            // divisor nb (chunk -> (a, b-chunk), layout 0)
  int32_t dims[kMaxOrder];
  int vec_ok;               // 16-byte vector loads allowed along the contiguous index
};

template <bool BF16>
struct Cfg {
  static constexpr int S = BF16 ? 2 : 4;       // bytes per element
  static constexpr int KCW = BF16 ? 64 : 32;   // reduction elements per wave per chunk
  static constexpr int VEC = 16 / S;           // elements per 16-byte vector
  static constexpr int PAD = BF16 ? 8 : 1;     // LDS row padding (elements)
};

__device__ __forceinline__ float bf16_to_float(uint16_t h) {
  return __uint_as_float(uint32_t(h) << 16);
}

__device__ __forceinline__ uint16_t float_to_bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  if ((b & 0x7fffffffu) > 0x7f800000u) return uint16_t((b >> 16) | 0x40u);
  return uint16_t((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

// Mixed-radix digits of x over modes [lo, hi] (C order: mode hi fastest).
__device__ __forceinline__ void digits_of(uint32_t x, int lo, int hi, const KArgs& k,
                                          uint32_t* d) {
  for (int l = hi; l >= lo; --l) {
    uint32_t q = fdiv(x, k.fd[l]);
    d[l] = x - q * k.fd[l].d;
    x = q;
  }
}

// E consecutive Khatri-Rao values  v[e] = scale * prod_{l in [lo,hi]} A_l[digit_l(x0+e), p]
// (zero when x0 + e >= xmax or p >= r). Digits advance by one per element with carries.
template <int E>
__device__ __forceinline__ void kr_run(float (&v)[E], const KArgs& k, int lo, int hi,
                                       uint32_t x0, int64_t xmax, int p, float scale) {
  if (int64_t(x0) >= xmax) {  // whole run past the end: digits of x0 may be out of range
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = 0.f;
    return;
  }
  if (p >= k.r || lo > hi) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = (p < k.r && int64_t(x0) + e < xmax) ? scale : 0.f;
    return;
  }
  uint32_t d[kMaxOrder];
  digits_of(x0, lo, hi, k, d);
  const int r = k.r;
  float head = scale;
  for (int l = lo; l < hi; ++l) head *= k.A.p[l][int64_t(d[l]) * r + p];
  const float* last = k.A.p[hi];
  const uint32_t dim_last = uint32_t(k.dims[hi]);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool ok = int64_t(x0) + e < xmax;
    v[e] = ok ? head * last[int64_t(d[hi]) * r + p] : 0.f;
    if (e + 1 < E) {
      d[hi] += 1;
      if (d[hi] == dim_last) {  // carry into the slower modes (rare)
        d[hi] = 0;
        int l = hi - 1;
        while (l >= lo) {
          d[l] += 1;
          if (d[l] < uint32_t(k.dims[l])) break;
          d[l] = 0;
          --l;
        }
        head = scale;
        for (int m = lo; m < hi; ++m) head *= k.A.p[m][int64_t(d[m]) * r + p];
      }
    }
  }
}

template <bool BF16, int NT, int WM, int WK, int LAYOUT>
__global__ __launch_bounds__(kThreads) void mttkrp_kernel(KArgs k) {
  using C = Cfg<BF16>;
  constexpr int MT = 32 * WM;
  constexpr int KC = C::KCW * WK;
  constexpr int RP = 32 * NT;
  constexpr int LDT = KC + C::PAD;                 // T tile row stride ([m][k])
  constexpr int LDK = BF16 ? (KC + C::PAD) : RP;   // KR tile stride: bf16 [p][k], f32 [k][p]
  constexpr int T_ELEMS = MT * LDT;
  constexpr int K_ELEMS = BF16 ? RP * LDK : KC * LDK;
  constexpr int NV = (MT * KC * C::S) / (16 * kThreads);   // 16-byte vectors per thread
  static_assert(NV >= 1, "tile too small");
  using TE = typename std::conditional<BF16, uint16_t, float>::type;

  __shared__ __attribute__((aligned(16))) TE s_t[2][T_ELEMS];
  __shared__ __attribute__((aligned(16))) TE s_k[2][K_ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM;
  const int wk = wave / WM;
  const int64_t i0 = int64_t(blockIdx.x) * MT;
  const int64_t split = blockIdx.y;
  const int64_t c_beg = split * k.chunks_per_split + (split < k.extra ? split : k.extra);
  const int64_t c_end = c_beg + k.chunks_per_split + (split < k.extra ? 1 : 0);
  const TE* __restrict__ T = static_cast<const TE*>(k.T);

  f32x16 acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[nt][v] = 0.f;

  // ---- T tile loads (one chunk ahead, in registers) ----
  uint4 reg[NV];

  auto load_tile = [&](int64_t c) {
    if (LAYOUT == 0) {
      const int64_t a = fdiv(uint32_t(c), k.fd_nb);
      const int64_t b0 = (c - a * k.nb) * KC;
      constexpr int VPR = KC / C::VEC;  // vectors per tile row
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int q = v * kThreads + tid;
        const int m = q / VPR;
        const int kk = (q % VPR) * C::VEC;
        const int64_t i = i0 + m;
        const int64_t b = b0 + kk;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (i < k.I) {
          const int64_t off = (a * k.I + i) * k.R + b;
          if (k.vec_ok && b + C::VEC <= k.R) {
            val = *reinterpret_cast<const uint4*>(T + off);
          } else {
            TE tmp[C::VEC];
#pragma unroll
            for (int e = 0; e < C::VEC; ++e) tmp[e] = (b + e < k.R) ? T[off + e] : TE(0);
            val = *reinterpret_cast<uint4*>(tmp);
          }
        }
        reg[v] = val;
      }
    } else {
      const int64_t a0 = c * KC;
      constexpr int VPR = MT / C::VEC;  // vectors per a-row of the tile
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int q = v * kThreads + tid;
        const int kr = q / VPR;
        const int ii = (q % VPR) * C::VEC;
        const int64_t a = a0 + kr;
        const int64_t i = i0 + ii;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (a < k.L) {
          const int64_t off = a * k.I + i;
          if (k.vec_ok && i + C::VEC <= k.I) {
            val = *reinterpret_cast<const uint4*>(T + off);
          } else {
            TE tmp[C::VEC];
#pragma unroll
            for (int e = 0; e < C::VEC; ++e) tmp[e] = (i + e < k.I) ? T[off + e] : TE(0);
            val = *reinterpret_cast<uint4*>(tmp);
          }
        }
        reg[v] = val;
      }
    }
  };

  auto store_tile = [&](int buf) {
    TE* st = s_t[buf];
    if (LAYOUT == 0) {
      constexpr int VPR = KC / C::VEC;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int q = v * kThreads + tid;
        const int m = q / VPR;
        const int kk = (q % VPR) * C::VEC;
        const TE* src = reinterpret_cast<const TE*>(&reg[v]);
        if (BF16) {
          *reinterpret_cast<uint4*>(&st[m * LDT + kk]) = reg[v];  // LDT*2 bytes is 16-aligned
        } else {
#pragma unroll
          for (int e = 0; e < C::VEC; ++e) st[m * LDT + kk + e] = src[e];
        }
      }
    } else {
      constexpr int VPR = MT / C::VEC;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int q = v * kThreads + tid;
        const int kr = q / VPR;
        const int ii = (q % VPR) * C::VEC;
        const TE* src = reinterpret_cast<const TE*>(&reg[v]);
#pragma unroll
        for (int e = 0; e < C::VEC; ++e) st[(ii + e) * LDT + kr] = src[e];
      }
    }
  };

  // ---- Khatri-Rao rows of a chunk into LDS ----
  // Thread t owns column p = t % RP and E consecutive reduction positions.
  constexpr int E = (KC * RP) / kThreads;
  static_assert(E >= 1 && (KC * RP) % kThreads == 0, "KR split");
  auto form_kr = [&](int64_t c, int buf) {
    TE* sk = s_k[buf];
    const int p = tid % RP;
    const int kg = tid / RP;
    const int kk0 = kg * E;
    float v[E];
    if (LAYOUT == 0) {
      const int64_t a = fdiv(uint32_t(c), k.fd_nb);
      const int64_t b0 = (c - a * k.nb) * KC + kk0;
      // left product over modes [0, n-1] at a, right run over modes [n+1, N-1]
      float left = 1.f;
      if (p < k.r && k.mode > 0) {
        uint32_t d[kMaxOrder];
        digits_of(uint32_t(a), 0, k.mode - 1, k, d);
        for (int l = 0; l < k.mode; ++l) left *= k.A.p[l][int64_t(d[l]) * k.r + p];
      }
      kr_run<E>(v, k, k.mode + 1, k.order - 1, uint32_t(b0), k.R, p, left);
    } else {
      const int64_t a0 = c * KC + kk0;
      kr_run<E>(v, k, 0, k.order - 2, uint32_t(a0), k.L, p, 1.f);
    }
    if (BF16) {
      // [p][k]: E consecutive k, 8 per 16-byte store
#pragma unroll
      for (int e0 = 0; e0 < E; e0 += 8) {
        uint16_t h[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = (e0 + e < E) ? float_to_bf16_rne(v[e0 + e]) : 0;
        *reinterpret_cast<uint4*>(&sk[p * LDK + kk0 + e0]) = *reinterpret_cast<uint4*>(h);
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) reinterpret_cast<float*>(sk)[(kk0 + e) * LDK + p] = v[e];
    }
  };

  // ---- MFMA over one chunk ----
  auto compute = [&](int buf) {
    const TE* st = s_t[buf];
    const TE* sk = s_k[buf];
    const int row = wm * 32 + (lane & 31);
    const int half = lane >> 5;
    const int kb = wk * C::KCW;
    if (BF16) {
#pragma unroll
      for (int s = 0; s < C::KCW / 16; ++s) {
        const int kk = kb + s * 16 + half * 8;
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&st[row * LDT + kk]);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const bf16x8 b =
              *reinterpret_cast<const bf16x8*>(&sk[(nt * 32 + (lane & 31)) * LDK + kk]);
          acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[nt], 0, 0, 0);
        }
      }
    } else {
      const float* stf = reinterpret_cast<const float*>(st);
      const float* skf = reinterpret_cast<const float*>(sk);
#pragma unroll
      for (int s = 0; s < C::KCW / 2; ++s) {
        const int kk = kb + s * 2 + half;
        const float a = stf[row * LDT + kk];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const float b = skf[kk * LDK + nt * 32 + (lane & 31)];
          acc[nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[nt], 0, 0, 0);
        }
      }
    }
  };

  if (c_beg < c_end) {
    load_tile(c_beg);
    int buf = 0;
    for (int64_t c = c_beg; c < c_end; ++c) {
      store_tile(buf);
      form_kr(c, buf);
      __syncthreads();
      if (c + 1 < c_end) load_tile(c + 1);
      compute(buf);
      buf ^= 1;
    }
  }

  // ---- reduce the WK waves that share rows, then write ----
  if (WK > 1) {
    __syncthreads();
    float* red = reinterpret_cast<float*>(&s_t[0][0]);  // reuse LDS
    static_assert((WK - 1) * WM * 64 * 16 * NT * 4 <= 2 * T_ELEMS * (int)sizeof(TE) +
                                                          2 * K_ELEMS * (int)sizeof(TE),
                  "reduction scratch");
    if (wk > 0) {
      float* dst = red + ((wk - 1) * WM + wm) * (64 * 16 * NT);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 16; ++v) dst[(nt * 16 + v) * 64 + lane] = acc[nt][v];
    }
    __syncthreads();
    if (wk == 0) {
      for (int w = 1; w < WK; ++w) {
        const float* src = red + ((w - 1) * WM + wm) * (64 * 16 * NT);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[nt][v] += src[(nt * 16 + v) * 64 + lane];
      }
    }
  }
  if (wk == 0) {
    float* out = k.out + split * k.I * k.r;
    const int col0 = lane & 31;
    const int hi4 = (lane >> 5) * 4;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int p = nt * 32 + col0;
      if (p >= k.r) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t i = i0 + wm * 32 + 8 * (v >> 2) + hi4 + (v & 3);
        if (i < k.I) out[i * k.r + p] = acc[nt][v];
      }
    }
  }
}

// Fixed-order sum of split partials; optionally resets inner-solver slots.
__global__ __launch_bounds__(256) void mttkrp_reduce_kernel(const float* __restrict__ part,
                                                            int64_t splits, int64_t n,
                                                            float* __restrict__ P,
                                                            double* slots, int64_t nslots) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = tid; e < n; e += stride) {
    double s = 0.0;
    for (int64_t q = 0; q < splits; ++q) s += double(part[q * n + e]);
    P[e] = float(s);
  }
  for (int64_t e = tid; e < nslots; e += stride)
    slots[e] = __longlong_as_double(-1ll);
}

using KernelFn = void (*)(KArgs);

template <bool BF16, int NT, int WM, int WK, int LAYOUT>
KernelFn pick() {
  return mttkrp_kernel<BF16, NT, WM, WK, LAYOUT>;
}

// Instantiated shapes keep LDS <= ~65 KB (two or more workgroups per CU): the Khatri-Rao
// tile grows with NT * WK, so wide ranks use WK = 1.
template <bool BF16, int LAYOUT>
KernelFn pick_w(int wm, int nt) {
  if (nt == 1) {
    if (wm == 1) return pick<BF16, 1, 1, 4, LAYOUT>();
    if (wm == 2) return pick<BF16, 1, 2, 2, LAYOUT>();
    return pick<BF16, 1, 4, 1, LAYOUT>();
  }
  if (nt == 2) {
    if (wm == 2) return pick<BF16, 2, 2, 2, LAYOUT>();
    return pick<BF16, 2, 4, 1, LAYOUT>();
  }
  if (nt == 4) return pick<BF16, 4, 4, 1, LAYOUT>();
  return pick<BF16, 8, 4, 1, LAYOUT>();
}

KernelFn select_kernel(bool bf16, int layout, int wm, int nt) {
  if (bf16) return layout ? pick_w<true, 1>(wm, nt) : pick_w<true, 0>(wm, nt);
  return layout ? pick_w<false, 1>(wm, nt) : pick_w<false, 0>(wm, nt);
}

int n_tiles(int r) {
  int nt = (r + 31) / 32;
  if (nt <= 1) return 1;
  if (nt <= 2) return 2;
  if (nt <= 4) return 4;
  return 8;
}

}  // namespace

ModeView make_mode_view(const ntf_tensor& T, int mode) {
  ModeView v;
  v.order = T.order;
  v.mode = mode;
  v.L = 1;
  v.R = 1;
  for (int l = 0; l < kMaxOrder; ++l) v.dims[l] = l < T.order ? T.dims[l] : 1;
  for (int l = 0; l < mode; ++l) v.L *= T.dims[l];
  for (int l = mode + 1; l < T.order; ++l) v.R *= T.dims[l];
  v.I = T.dims[mode];
  return v;
}

MttkrpPlan plan_mttkrp(const ntf_tensor& T, int mode, int r, int num_cus) {
  MttkrpPlan pl;
  pl.v = make_mode_view(T, mode);
  pl.dtype = T.dtype;
  pl.r = r;
  const int nt = n_tiles(r);
  pl.rpad = 32 * nt;
  pl.layout = pl.v.R == 1 ? 1 : 0;
  // rows per workgroup: the largest of 128 / 64 / 32 whose padding wastes <= 12.5%
  // Allowed shapes: NT = 1 any WM; NT = 2 WM in {2, 4}; NT >= 4 WM = 4 (LDS budget).
  const int64_t I = pl.v.I;
  const int wm_min = nt == 1 ? 1 : (nt == 2 ? 2 : 4);
  pl.wm = 0;
  for (int wm : {4, 2, 1}) {
    if (wm < wm_min) break;
    const int64_t mt = 32 * wm;
    const int64_t padded = ceil_div(I, mt) * mt;
    if (padded * 8 <= I * 9) {
      pl.wm = wm;
      break;
    }
  }
  if (pl.wm == 0) {  // no shape within 12.5% padding: take the least padded allowed one
    int64_t best = -1;
    for (int wm : {4, 2, 1}) {
      if (wm < wm_min) break;
      const int64_t padded = ceil_div(I, 32 * wm) * 32 * wm;
      if (best < 0 || padded < best) {
        best = padded;
        pl.wm = wm;
      }
    }
  }
  pl.wk = 4 / pl.wm;
  const int kcw = T.dtype == NTF_BF16 ? 64 : 32;
  const int64_t kc = int64_t(kcw) * pl.wk;
  pl.mtiles = ceil_div(I, 32 * pl.wm);
  if (pl.layout == 0) {
    const int64_t nb = ceil_div(pl.v.R, kc);
    pl.chunks = pl.v.L * nb;
  } else {
    pl.chunks = ceil_div(pl.v.L, kc);
  }
  const int64_t target = int64_t(num_cus) * 4;
  int64_t splits = ceil_div(target, pl.mtiles);
  splits = std::max<int64_t>(1, std::min<int64_t>(splits, pl.chunks));
  splits = std::min<int64_t>(splits, 65535);
  pl.splits = splits;
  pl.variant = nt;
  return pl;
}

hipError_t launch_mttkrp(const MttkrpPlan& pl, const void* T, const FactorPtrs& A, float* P,
                         float* partials, double* slots, int64_t nslots, hipStream_t s) {
  KArgs k;
  k.T = T;
  k.A = A;
  k.L = pl.v.L;
  k.I = pl.v.I;
  k.R = pl.v.R;
  k.order = pl.v.order;
  k.mode = pl.v.mode;
  k.r = pl.r;
  const bool bf16 = pl.dtype == NTF_BF16;
  const int kcw = bf16 ? 64 : 32;
  const int64_t kc = int64_t(kcw) * pl.wk;
  k.nb = pl.layout == 0 ? ceil_div(pl.v.R, kc) : 1;
  k.fd_nb = make_fastdiv(uint32_t(k.nb));
  k.chunks = pl.chunks;
  k.chunks_per_split = pl.chunks / pl.splits;
  k.extra = pl.chunks % pl.splits;
  for (int l = 0; l < kMaxOrder; ++l) {
    const int64_t d = l < pl.v.order ? pl.v.dims[l] : 1;
    k.dims[l] = int32_t(d);
    k.fd[l] = make_fastdiv(uint32_t(d));
  }
  const int vec = bf16 ? 8 : 4;
  k.vec_ok = pl.layout == 0 ? (pl.v.R % vec == 0) : (pl.v.I % vec == 0);
  const bool split = pl.splits > 1;
  k.out = split ? partials : P;
  KernelFn fn = select_kernel(bf16, pl.layout, pl.wm, pl.variant);
  dim3 grid(unsigned(pl.mtiles), unsigned(pl.splits));
  hipLaunchKernelGGL(fn, grid, dim3(kThreads), 0, s, k);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (split || nslots > 0) {
    const int64_t n = split ? pl.v.I * pl.r : 0;
    const int64_t work = std::max<int64_t>(n, nslots);
    const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(ceil_div(work, 256), 2048)));
    hipLaunchKernelGGL(mttkrp_reduce_kernel, dim3(blocks), dim3(256), 0, s, partials,
                       pl.splits, n, P, slots, nslots);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace ntf
