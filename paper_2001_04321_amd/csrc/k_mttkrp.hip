// Dense MTTKRP on gfx950 matrix cores, in factored form.
//
//   P[i, p] = sum over all j_{-n} of T[j] * prod_{l != n} A_l[j_l, p]
//
// (paper Sec. 2, eqs. def:B and def:grad: the data term T_[n] B^(n)). Let v be the
// fastest-varying mode other than n (the last mode, or mode N-2 when n is the last mode)
// and let u enumerate the remaining modes in C order. The Khatri-Rao row of (u, v) is the
// Hadamard product X[u] (*) A_v[v] with X[u][p] = prod_{l != n, v} A_l[u_l, p], so
//
//   P[i, p] = sum_u X[u][p] * Y_u[i, p],      Y_u[i, p] = sum_v T(u, i, v) A_v[v, p].
//
// Y_u is a plain matrix product whose right operand A_v is the same for every u: a
// workgroup keeps a block of A_v in LDS as the MFMA B operand for its whole run, streams
// T once from HBM as the A operand, and folds each Y_u into the float32 accumulators
// with one FMA per accumulator register (X[u][p] is a per-lane scalar because the
// accumulator column is the lane's column). The Khatri-Rao product is never formed,
// neither in HBM nor in LDS.
//
// Layouts: case A (n < N-1): v is the last mode, so every output row reads a contiguous
// run of T along v; lanes load their MFMA A fragments straight from global memory.
// Case B (n = N-1): i is the contiguous index. float32: one element per lane per
// v_mfma_f32_32x32x2_f32 step, already in MFMA layout (32 lanes cover 32 consecutive i).
// bfloat16: the wave stages a 64 x 32 tile in LDS in memory order and reads it back with
// ds_read_b64_tr_b16, which returns 4 consecutive v of one i per lane.
//
// Precision of the bfloat16 form: only the stored tensor is bfloat16. The float32 factor
// block A_v is kept in LDS as two bfloat16 halves (hi + lo, 16 significant bits) and each
// fragment takes two matrix-core products, so P carries the rounding of T and float32
// accumulation, not a second rounding of the factors. The kernel is bound by the tensor
// stream, with the matrix cores mostly idle, so the second product costs no time.
//
// Work split: grid = (row tiles of 32*WM rows, splits of the (v-block, u) sequence). WK
// waves share a row tile and take interleaved 64-element (bf16) / 32-element (f32) chunks
// of v; their accumulators are summed once at the end. Splits write partial tiles that
// a second pass sums in a fixed order: the result is deterministic.
#include "gram_chunk.h"
#include "ntf_internal.h"

namespace ntf {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) i16x4 lds_i16x4;

constexpr int kThreads = 256;
constexpr int kStageLd = 40;  // bf16 case-B staging row stride (32 columns + 8 pad)

// Magic-number division for 0 <= x < 2^31 (round-up method of Granlund and Montgomery):
// q = floor(x * m / 2^(31 + l)), l = ceil(log2 d), m = ceil(2^(31 + l) / d) < 2^32.
struct FastDiv {
  uint32_t d;
  uint32_t m;
  uint32_t sh;  // l - 1, or 0xffffffff for d == 1
};

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  if (d <= 1) {
    f.d = 1;
    f.m = 0;
    f.sh = 0xffffffffu;
    return f;
  }
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  const unsigned __int128 num = (unsigned __int128)1 << (31 + l);
  f.m = uint32_t((num + d - 1) / d);
  f.sh = l - 1;
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv& f) {
  if (f.sh == 0xffffffffu) return x;
  return __umulhi(x, f.m) >> f.sh;
}

struct KArgs {
  const void* T;
  float* out;                  // P (one split) or partials [split][I][r]
  const float* Av;             // I_v x r
  const float* Ao[kMaxOrder];  // factors of the u modes, slowest first
  FastDiv fd_o[kMaxOrder];
  int n_o;
  int64_t I, Iv, U;
  int64_t R;                   // case A: row stride of T (prod of modes after n)
  int64_t a_stride;            // case A: T offset of one step of the modes before n
  FastDiv fd_Rp;               // case A: u = a * Rp + b_hi, Rp = R / I_v
  int64_t Rp;
  int64_t per_split, extra;
  int64_t mtiles;              // row tiles (the grid is mtiles x splits workgroups)
  int av_vec;                  // A_v rows are RP floats (r == RP) and 16-byte aligned
  int64_t tbytes;              // tensor size in bytes (< 2^31: buffer-resource offsets)
  float* ystore;               // case A, one wave per row tile: store Y[i][u][:] = T_u A_v
                               // rows instead of folding them (null: fold into P)
  int r;
  int vb;                      // v-block length (multiple of the chunk)
  int ub;                      // u values per X batch
  int uk;                      // 1: the WK waves of a row tile take interleaved u values
                               // (each covers every v chunk); 0: interleaved v chunks
  int nh;                      // leading workgroups that compute a Hadamard product instead
  HadamardLaunch had;
};

// Tensor loads go through a buffer resource: an offset at or past the resource's size
// (kOOB) reads zeros in hardware, so tails and padding need neither branches nor selects on
// the loaded value (either would make the compiler drain the load queue at every join).
// Resource word 3 (data format 32, the CDNA setting for raw buffer loads).
constexpr int kBufWord3 = 0x00020000;
constexpr uint32_t kOOB = 0x80000000u;
typedef int i32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 bload16(__amdgpu_buffer_rsrc_t rs, uint32_t byte_off) {
  const i32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, byte_off, 0, 0);
  return make_uint4(uint32_t(v.x), uint32_t(v.y), uint32_t(v.z), uint32_t(v.w));
}

// float32 -> bfloat16 bits, round to nearest even (NaN stays a quiet NaN); branch-free
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t b = __float_as_uint(f);
  const uint32_t rne = (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
  const uint32_t nan = (b >> 16) | 0x40u;
  return uint16_t((b & 0x7fffffffu) > 0x7f800000u ? nan : rne);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __uint_as_float(uint32_t(b) << 16);
}

// Stage rows [v0, v0 + vb) of a float32 factor A (I_v x r, row-major) into LDS as the sum
// of two bf16 values, hi = RNE(x) and lo = RNE(x - hi) (x - hi is exact in float32; hi + lo
// carries 16 significant bits), transposed: hi[p * ldb + kk], lo at element offset lo_off
// (zero beyond I_v and r). A thread takes groups of 8 consecutive kk by 4 consecutive p:
// the group's loads are all issued before any is used (addresses clamped into A, values
// selected; no branch per load), then it is written as eight 16-byte stores. vb and ldb are
// multiples of 8; kThreads threads take part. vec: r == RP and A 16-byte aligned (one
// 16-byte load per row of a group).
__device__ __forceinline__ void stage_av_hilo(uint16_t* s, int lo_off, int ldb,
                                              const float* __restrict__ A, int r, int RP,
                                              int64_t v0, int vb, int64_t Iv, int tid,
                                              bool vec) {
  const int np4 = RP / 4;
  const int n = (vb / 8) * np4;
  for (int e = tid; e < n; e += kThreads) {
    const int g8 = e / np4;
    const int p = (e - g8 * np4) * 4;
    float x[8][4];
    if (vec) {
      float4 t[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t v = v0 + g8 * 8 + j;
        t[j] = *reinterpret_cast<const float4*>(A + (v < Iv ? v : 0) * r + p);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bool ok = v0 + g8 * 8 + j < Iv;
        x[j][0] = ok ? t[j].x : 0.f;
        x[j][1] = ok ? t[j].y : 0.f;
        x[j][2] = ok ? t[j].z : 0.f;
        x[j][3] = ok ? t[j].w : 0.f;
      }
    } else {
      float t[8][4];
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t v = v0 + g8 * 8 + j;
          const bool ok = v < Iv && p + q < r;
          t[j][q] = A[(ok ? v * r + p + q : 0)];
        }
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool ok = v0 + g8 * 8 + j < Iv && p + q < r;
          x[j][q] = ok ? t[j][q] : 0.f;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      union {
        uint16_t h[8];
        uint4 v;
      } hi, lo;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        hi.h[j] = f2bf(x[j][q]);
        lo.h[j] = f2bf(x[j][q] - bf16_bits_to_f32(hi.h[j]));
      }
      *reinterpret_cast<uint4*>(&s[(p + q) * ldb + g8 * 8]) = hi.v;
      *reinterpret_cast<uint4*>(&s[lo_off + (p + q) * ldb + g8 * 8]) = lo.v;
    }
  }
}

// One work item of a bf16 tensor against an A_v block staged as hi and lo halves:
// y[nt] += T_frag(t) * (B_hi + B_lo)(t, nt) for the four 8-element K steps t of the item
// (the lane's T fragment reg[t], B rows col + 32 nt, K offset kk0 + 8 t). NT <= 2: the
// B fragments are read from LDS in batches of eight, then their products issue back to back
// (one LDS round trip per batch, not one per product); wider tiles have NT independent
// products per fragment of T to cover the reads.
template <int NT>
__device__ __forceinline__ void mfma_hilo_item(f32x16 (&y)[NT], const uint4 (&reg)[4],
                                               const uint16_t* s_av, int lo_off, int ldb,
                                               int kk0, int col) {
  constexpr int TB = NT >= 4 ? 1 : 4 / NT;
#pragma unroll
  for (int t0 = 0; t0 < 4; t0 += TB) {
    bf16x8 bh[TB][NT], bl[TB][NT];
#pragma unroll
    for (int tt = 0; tt < TB; ++tt) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int bo = (nt * 32 + col) * ldb + kk0 + (t0 + tt) * 8;
        bh[tt][nt] = *reinterpret_cast<const bf16x8*>(&s_av[bo]);
        bl[tt][nt] = *reinterpret_cast<const bf16x8*>(&s_av[lo_off + bo]);
      }
    }
    if constexpr (NT <= 2) __builtin_amdgcn_sched_barrier(0);  // reads ahead of products
#pragma unroll
    for (int tt = 0; tt < TB; ++tt) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&reg[t0 + tt]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        y[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bh[tt][nt], y[nt], 0, 0, 0);
        y[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bl[tt][nt], y[nt], 0, 0, 0);
      }
    }
  }
}

// X[u][p] = prod over the u modes of A_l[u_l, p].
__device__ __forceinline__ float x_value(const KArgs& k, uint32_t u, int p) {
  float x = 1.f;
  for (int q = k.n_o - 1; q >= 0; --q) {
    const uint32_t qq = fdiv(u, k.fd_o[q]);
    const uint32_t d = u - qq * k.fd_o[q].d;
    u = qq;
    x *= k.Ao[q][int64_t(d) * k.r + p];
  }
  return x;
}

template <bool LAST>
__device__ __forceinline__ int64_t t_base(const KArgs& k, uint32_t u) {
  if (LAST) return int64_t(u) * k.Iv * k.I;
  const uint32_t a = fdiv(u, k.fd_Rp);
  const int64_t bhi = int64_t(u) - int64_t(a) * k.Rp;
  return int64_t(a) * k.a_stride + bhi * k.Iv;
}

// Workgroup barrier that orders LDS accesses only: tensor loads issued before it stay in
// flight (__syncthreads would wait for them too).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <bool BF16, int NT, int WM, int WK, bool LAST, bool VEC>
__global__ __launch_bounds__(kThreads, 2) void mttkrp_kernel(KArgs k) {
  if (int(blockIdx.x) < k.nh) {  // the Hadamard product of the next A-HALS launch
    hadamard_work(k.had.job, k.had.r, k.had.G32, k.had.G64, k.had.slots, k.had.nslots,
                  blockIdx.x, k.nh);
    return;
  }
  constexpr int RP = 32 * NT;
  constexpr int KCH = BF16 ? 64 : 32;
  constexpr int MT = 32 * WM;
  using TE = typename std::conditional<BF16, uint16_t, float>::type;
  extern __shared__ __attribute__((aligned(16))) char smem[];

  const int vb = k.vb;
  const int ldb = BF16 ? vb + 8 : RP;
  // bf16: the A_v block as hi and lo halves, s_av[p][kk] and s_av[RP * ldb + p * ldb + kk]
  const size_t av_bytes = align_up(size_t(BF16 ? 2 * RP * ldb * 2 : vb * RP * 4), 16);
  TE* s_av = reinterpret_cast<TE*>(smem);
  const int lo_off = RP * ldb;  // bf16: element offset of the lo half
  float* s_x = reinterpret_cast<float*>(smem + av_bytes);
  uint16_t* s_stage =
      reinterpret_cast<uint16_t*>(smem + av_bytes + align_up(size_t(k.ub) * RP * 4, 16));

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM;
  const int wk = wave / WM;
  const int col = lane & 31;
  const int half = lane >> 5;
  // XCD-aware numbering: workgroups are dealt to the 8 XCDs round-robin by launch index;
  // logical workgroups are renumbered so that consecutive row tiles of a split (which
  // share cache lines at their edges) run on the same XCD and hit the same L2
  uint32_t lw = blockIdx.x - uint32_t(k.nh);  // (nh is a multiple of 8)
  {
    const uint32_t per = (gridDim.x - uint32_t(k.nh)) / 8;
    if (lw < per * 8) lw = (lw % 8) * per + lw / 8;
  }
  const int64_t tile = lw % uint32_t(k.mtiles);
  const int64_t i0 = tile * MT;
  const int64_t row = i0 + wm * 32 + col;  // case A / f32 case B: the lane's output row
  const bool row_ok = row < k.I;
  const int64_t split = lw / uint32_t(k.mtiles);
  const int64_t w_beg = split * k.per_split + (split < k.extra ? split : k.extra);
  const int64_t w_end = w_beg + k.per_split + (split < k.extra ? 1 : 0);
  const TE* __restrict__ T = static_cast<const TE*>(k.T);
  uint16_t* stage = s_stage + wave * 64 * kStageLd;

  f32x16 acc[NT], y[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      acc[nt][e] = 0.f;
      y[nt][e] = 0.f;
    }

  // One work item = (u, chunk kc of the current v-block) for this wave. Registers of one
  // item: bf16 case A: 32 elements along v (4 x 16 B); f32 case A: 16 floats; f32 case B:
  // 16 floats; bf16 case B: 4 x 16 B of the wave's 64 x 32 tile. PD items are in flight
  // per wave (a ring of register buffers, indexed at compile time).
  constexpr int PD = NT <= 2 ? 4 : 2;
  uint4 buf[PD][4];
#pragma unroll
  for (int d = 0; d < PD; ++d)
#pragma unroll
    for (int q = 0; q < 4; ++q) buf[d][q] = make_uint4(0, 0, 0, 0);

  // Loads are predicated by address, not by branches: an element outside the tensor (or an
  // item past the end) loads from T[0] and is replaced by zero. Branch-free item code lets
  // the compiler keep all prefetched items in flight instead of draining the load queue at
  // every control-flow join.
  const uint4 zero4 = make_uint4(0, 0, 0, 0);
  (void)zero4;
  const __amdgpu_buffer_rsrc_t trs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(k.T), short(0), int(k.tbytes), kBufWord3);
  auto load_item = [&](uint4 (&reg)[4], int64_t base, int64_t v0c, bool valid) {
    if (!LAST) {
      // lane (row, half): elements v0c + half*KCH/2 + [0, KCH/2) of its row
      constexpr int EPL = KCH / 2;
      constexpr int SLOT = EPL / 4;  // elements per 16 bytes
      const int64_t v = v0c + half * EPL;
      const int64_t off = base + row * k.R + v;
      if constexpr (VEC) {
        // rows 16-byte aligned and I_v a multiple of 16 bytes: whole slots in or out
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool ok = valid && row_ok && v + (q + 1) * SLOT <= k.Iv;
          reg[q] = bload16(trs, ok ? uint32_t((off + q * SLOT) * sizeof(TE)) : kOOB);
        }
      } else {
        TE tmp[EPL];
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const bool ok = valid && row_ok && v + e < k.Iv;
          const uint32_t bo = ok ? uint32_t((off + e) * sizeof(TE)) : kOOB;
          if constexpr (BF16)
            tmp[e] = TE(__builtin_amdgcn_raw_buffer_load_b16(trs, bo, 0, 0));
          else
            tmp[e] = __builtin_bit_cast(TE, __builtin_amdgcn_raw_buffer_load_b32(trs, bo, 0, 0));
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) reg[q] = reinterpret_cast<uint4*>(tmp)[q];
      }
    } else if (!BF16) {
      // lane (row, half): v = v0c + 2t + half, t = 0..15
      float tmp[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int64_t v = v0c + 2 * t + half;
        const bool ok = valid && row_ok && v < k.Iv;
        tmp[t] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(
                       trs, ok ? uint32_t((base + v * k.I + row) * 4) : kOOB, 0, 0));
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) reg[q] = reinterpret_cast<uint4*>(tmp)[q];
    } else {
      // wave tile: 64 v rows x 32 i columns; lane loads rows q*16 + lane/4, columns
      // (lane%4)*8 .. +8 (16 bytes), q = 0..3
      const int c8 = (lane & 3) * 8;
      const int64_t ic = i0 + wm * 32 + c8;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t v = v0c + q * 16 + (lane >> 2);
        const int64_t off = base + v * k.I + ic;
        if constexpr (VEC) {
          // I is a multiple of 8: a 16-byte group is wholly inside or outside
          const bool ok = valid && v < k.Iv && ic + 8 <= k.I;
          reg[q] = bload16(trs, ok ? uint32_t(off * 2) : kOOB);
        } else {
          uint16_t tmp[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const bool ok = valid && v < k.Iv && ic + e < k.I;
            tmp[e] = uint16_t(
                __builtin_amdgcn_raw_buffer_load_b16(trs, ok ? uint32_t((off + e) * 2) : kOOB, 0, 0));
          }
          reg[q] = *reinterpret_cast<uint4*>(tmp);
        }
      }
    }
  };

  auto compute_item = [&](const uint4 (&reg)[4], int kc) {
    if (BF16 && !LAST) {
      mfma_hilo_item<NT>(y, reg, reinterpret_cast<const uint16_t*>(s_av), lo_off, ldb,
                         kc * KCH + half * 32, col);
    } else if (BF16 && LAST) {
      // stage the tile in memory order; transposing reads give K-contiguous fragments
      const int c8 = (lane & 3) * 8;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<uint4*>(&stage[(q * 16 + (lane >> 2)) * kStageLd + c8]) = reg[q];
      const int g = lane >> 4;
      const int m0 = 16 * (g & 1);
      const int src = lane & 15;
      const int jj = src >> 2;
      const int s4 = (src & 3) * 4;
      // NT <= 2: the fragments of TB K steps (T from the stage, B hi and lo) are read
      // together, then their products issue back to back
      constexpr int TB = NT >= 4 ? 1 : 4 / NT;
#pragma unroll
      for (int t0 = 0; t0 < 4; t0 += TB) {
        union {
          i16x4 h[2];
          bf16x8 v;
        } a[TB];
        bf16x8 bh[TB][NT], bl[TB][NT];
#pragma unroll
        for (int tt = 0; tt < TB; ++tt) {
          const int t = t0 + tt;
          const int kq = 16 * t + 8 * (g >> 1);
          a[tt].h[0] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
              (lds_i16x4*)(&stage[(kq + jj) * kStageLd + m0 + s4]));
          a[tt].h[1] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
              (lds_i16x4*)(&stage[(kq + 4 + jj) * kStageLd + m0 + s4]));
          const int kk = kc * KCH + 16 * t + 8 * half;
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int bo = (nt * 32 + col) * ldb + kk;
            bh[tt][nt] = *reinterpret_cast<const bf16x8*>(&s_av[bo]);
            bl[tt][nt] = *reinterpret_cast<const bf16x8*>(&s_av[lo_off + bo]);
          }
        }
        if constexpr (NT <= 2) __builtin_amdgcn_sched_barrier(0);  // reads ahead of products
#pragma unroll
        for (int tt = 0; tt < TB; ++tt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            y[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[tt].v, bh[tt][nt], y[nt], 0, 0, 0);
            y[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[tt].v, bl[tt][nt], y[nt], 0, 0, 0);
          }
      }
    } else {
      const float* rf = reinterpret_cast<const float*>(reg);
      const float* sf = reinterpret_cast<const float*>(s_av);
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int kk = LAST ? kc * KCH + 2 * t + half : kc * KCH + half * 16 + t;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const float b = sf[kk * RP + nt * 32 + col];
          y[nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(rf[t], b, y[nt], 0, 0, 0);
        }
      }
    }
  };

  int cur_vb = -1;
  int64_t w = w_beg;
  while (w < w_end) {
    const int vbi = int(w / k.U);
    const int64_t v0 = int64_t(vbi) * vb;
    const int nkc = int(ceil_div(std::min<int64_t>(vb, k.Iv - v0), KCH));  // chunks with data
    // items per u (this wave): every chunk when the waves split u, else every WK-th chunk
    const int ipu = k.uk ? nkc : (nkc + WK - 1) / WK;
    // ---- a batch of u values within this v-block; the first items' tensor loads go out
    // before the A_v block and X are staged, so their latency overlaps the staging ----
    const int64_t u0 = w - int64_t(vbi) * k.U;
    const int64_t w_stop = std::min<int64_t>(w_end, int64_t(vbi + 1) * k.U);
    const int nu = int(std::min<int64_t>(k.ub, w_stop - w));
    // this wave's u values: all of the batch (waves split v chunks) or every WK-th from wk
    const int nuw = k.uk ? (nu > wk ? (nu - wk + WK - 1) / WK : 0) : nu;
    const int nitems = nuw * ipu;
    auto u_of = [&](int m) { return k.uk ? wk + m * WK : m; };   // batch index of u number m
    auto kc_of = [&](int j) { return k.uk ? j : wk + j * WK; };  // chunk of item number j
    // prefetch cursor (pu, pj) and compute cursor (cu, cj) over (u, chunk) items; items past
    // the end load zeros (see load_item), so the loop body has no data-dependent branches
    int pu = 0, pj = 0, pit = 0;
    auto prefetch = [&](uint4 (&reg)[4]) {
      const int kc = kc_of(pj);
      const bool valid = pit < nitems && kc < nkc;
      const uint32_t uq = uint32_t(u0 + (pit < nitems ? u_of(pu) : 0));
      load_item(reg, t_base<LAST>(k, uq), v0 + int64_t(kc) * KCH, valid);
      ++pit;
      if (++pj == ipu) {
        pj = 0;
        ++pu;
      }
    };
#pragma unroll
    for (int d = 0; d < PD - 1; ++d) prefetch(buf[d]);

    // ---- A_v block into LDS (zero beyond I_v and r) ----
    if (vbi != cur_vb) {
      lds_barrier();
      const int nv = int(std::min<int64_t>(vb, k.Iv - v0));
      if (BF16) {
        stage_av_hilo(reinterpret_cast<uint16_t*>(s_av), lo_off, ldb, k.Av, k.r, RP, v0, vb,
                      k.Iv, tid, k.av_vec != 0);
      } else if (k.av_vec) {
        // r == RP and A_v 16-byte aligned: the block is contiguous; 16-byte loads, eight
        // in flight per thread
        const int n4 = vb * RP / 4;
        const float4* src = reinterpret_cast<const float4*>(k.Av + v0 * RP);
        for (int b0 = tid; b0 < n4; b0 += kThreads * 8) {
          float4 t[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int e4 = b0 + j * kThreads;
            t[j] = (e4 < n4 && (e4 * 4) / RP < nv) ? src[e4] : make_float4(0.f, 0.f, 0.f, 0.f);
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int e4 = b0 + j * kThreads;
            if (e4 >= n4) continue;
            const int kk = (e4 * 4) / RP;
            const int p = e4 * 4 - kk * RP;
            *reinterpret_cast<float4*>(&reinterpret_cast<float*>(s_av)[kk * RP + p]) = t[j];
          }
        }
      } else {
        for (int e = tid; e < vb * RP; e += kThreads) {
          const int kk = e / RP;
          const int p = e - kk * RP;
          const int64_t v = v0 + kk;
          reinterpret_cast<float*>(s_av)[kk * RP + p] =
              (p < k.r && v < k.Iv) ? k.Av[v * k.r + p] : 0.f;
        }
      }
      cur_vb = vbi;
    }
    lds_barrier();
    for (int e = tid; e < nu * RP; e += kThreads) {
      const int uu = e / RP;
      const int p = e - uu * RP;
      s_x[e] = p < k.r ? x_value(k, uint32_t(u0 + uu), p) : 0.f;
    }
    lds_barrier();

    int cu = 0, cj = 0;
    for (int base = 0; base < nitems; base += PD) {
#pragma unroll
      for (int d = 0; d < PD; ++d) {
        prefetch(buf[(d + PD - 1) % PD]);
        if (base + d < nitems) {
          if (cj == 0) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
              for (int e = 0; e < 16; ++e) y[nt][e] = 0.f;
          }
          const int kc = kc_of(cj);
          if (kc < nkc) compute_item(buf[d], kc);
          if (cj == ipu - 1) {
            if (k.ystore) {
              // Y[i][u][p] (the wave covers every v chunk of u: WK == 1 or waves split u)
              const int64_t uu = u0 + u_of(cu);
#pragma unroll
              for (int nt = 0; nt < NT; ++nt) {
                const int p = nt * 32 + col;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                  // out-of-range entries go to the padding past Y (no branches)
                  const int64_t i = i0 + wm * 32 + 8 * (e >> 2) + half * 4 + (e & 3);
                  const bool ok = p < k.r && i < k.I;
                  k.ystore[ok ? (i * k.U + uu) * k.r + p : k.I * k.U * k.r + col] = y[nt][e];
                }
              }
            } else {
              const float* xs = s_x + u_of(cu) * RP;
#pragma unroll
              for (int nt = 0; nt < NT; ++nt) {
                const float x = xs[nt * 32 + col];
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[nt][e] = fmaf(x, y[nt][e], acc[nt][e]);
              }
            }
          }
          if (++cj == ipu) {
            cj = 0;
            ++cu;
          }
        }
      }
    }
    w += nu;
  }

  // ---- sum the WK waves of each row tile (fixed order), write rows < I, cols < r ----
  __syncthreads();
  float* red = reinterpret_cast<float*>(smem);
  if (WK > 1 && wk > 0) {
    float* dst = red + ((wk - 1) * WM + wm) * (64 * 16 * NT);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int e = 0; e < 16; ++e) dst[(nt * 16 + e) * 64 + lane] = acc[nt][e];
  }
  __syncthreads();
  if (wk == 0 && !k.ystore) {
    for (int ww = 1; ww < WK; ++ww) {
      const float* src = red + ((ww - 1) * WM + wm) * (64 * 16 * NT);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[nt][e] += src[(nt * 16 + e) * 64 + lane];
    }
    float* out = k.out + split * k.I * k.r;
    const int hi4 = half * 4;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int p = nt * 32 + col;
      if (p >= k.r) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t i = i0 + wm * 32 + 8 * (e >> 2) + hi4 + (e & 3);
        if (i < k.I) out[i * k.r + p] = acc[nt][e];
      }
    }
  }
}

// ---- Row-slab variant (bfloat16, n < N-1) ----
// The kernel above puts 32 rows i of the output in the MFMA M dimension, so every load
// instruction touches 32 rows of T at the row stride. When that stride is a multiple of a
// large power of two (e.g. 4 MiB for the first mode of a 128^4 tensor) all 32 rows fall in the
// same DRAM bank and channel and the stream slows down by a third. This variant keeps one
// output row i per workgroup and puts 32 consecutive values of the innermost u mode in M:
//
//   Z[u, p] = sum_v T(u, i, v) A_v[v, p]   (MFMA, A operand = 32 u rows of T),
//   P[i, p] += sum_u X[u][p] Z[u, p],       X[u][p] = C[p] * A_in[j_in(u), p],
//
// where A_in is the factor of the innermost u mode and C[p] the product of the other u
// modes' factor rows (one value per batch of 32 u). Consecutive u are adjacent runs of T
// for modes before N-2, so a workgroup streams long contiguous ranges. Batches (32 values
// of the innermost u mode, the other u modes fixed) are split over `S` workgroups per row
// and interleaved over the 4 waves; the waves' sums are combined in a fixed order and
// written as split partials [split][I][r] (P itself when S == 1).
struct SArgs {
  const void* T;
  int64_t tbytes;
  float* out;
  const float* Av;             // I_v x r
  const float* Ain;            // I_in x r (innermost u mode)
  const float* Ao[kMaxOrder];  // the other u modes, slowest first
  FastDiv fd_o[kMaxOrder];
  int n_o;
  int64_t I, Iv, R, a_stride, Rp;
  FastDiv fd_Rp;
  int64_t I_in, nb_in, nbatch, S;
  int r, vb;
  int av_vec;                  // A_v rows are RP floats (r == RP) and 16-byte aligned
  int nh;
  HadamardLaunch had;
};

template <int NT>
__global__ __launch_bounds__(kThreads, 2) void mttkrp_slab_kernel(SArgs k) {
  if (int(blockIdx.x) < k.nh) {
    hadamard_work(k.had.job, k.had.r, k.had.G32, k.had.G64, k.had.slots, k.had.nslots,
                  blockIdx.x, k.nh);
    return;
  }
  constexpr int RP = 32 * NT;
  constexpr int KCH = 64;
  constexpr int PD = 4;
  constexpr int NW = kThreads / 64;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int ldb = k.vb + 8;
  uint16_t* s_av = reinterpret_cast<uint16_t*>(smem);  // A_v hi half; the lo half follows
  const int lo_off = RP * ldb;
  float* s_ain = reinterpret_cast<float*>(smem + align_up(size_t(2) * RP * ldb * 2, 16));
  float* s_red = s_ain + k.I_in * RP;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int col = lane & 31;
  const int half = lane >> 5;
  const int64_t lw = int64_t(blockIdx.x) - k.nh;
  const int64_t i = lw % k.I;
  const int64_t split = lw / k.I;
  const int64_t per = k.nbatch / k.S, extra = k.nbatch % k.S;
  const int64_t b_beg = split * per + (split < extra ? split : extra);
  const int64_t b_end = b_beg + per + (split < extra ? 1 : 0);
  // this wave's batches: b_beg + wave + NW * m
  const int64_t nbw = b_end - b_beg > wave ? (b_end - b_beg - wave + NW - 1) / NW : 0;
  const int nkc = int(ceil_div(k.Iv, int64_t(KCH)));
  const int64_t nitems = nbw * nkc;

  const __amdgpu_buffer_rsrc_t trs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(k.T), short(0), int(k.tbytes), kBufWord3);
  // item (batch m of this wave, chunk c): lane (row, half) loads 32 elements of v along its
  // u row; rows past I_in and items past the end load zeros (buffer out-of-range reads)
  auto load_item = [&](uint4 (&reg)[4], int64_t m, int c) {
    const bool valid = m < nbw;
    const int64_t b = b_beg + wave + NW * (valid ? m : 0);
    const int64_t uo = b / k.nb_in;
    const int64_t j = (b - uo * k.nb_in) * 32 + col;
    const bool ok_row = valid && j < k.I_in;
    const uint32_t u = uint32_t(uo * k.I_in + (ok_row ? j : 0));
    const uint32_t a = fdiv(u, k.fd_Rp);
    const int64_t bhi = int64_t(u) - int64_t(a) * k.Rp;
    const int64_t v = int64_t(c) * KCH + half * 32;
    const int64_t off = int64_t(a) * k.a_stride + i * k.R + bhi * k.Iv + v;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = ok_row && v + (q + 1) * 8 <= k.Iv;
      reg[q] = bload16(trs, ok ? uint32_t((off + q * 8) * 2) : kOOB);
    }
  };

  uint4 buf[PD][4];
  int64_t pm = 0;
  int pc = 0;
  auto prefetch = [&](uint4 (&reg)[4]) {
    load_item(reg, pm, pc);
    if (++pc == nkc) {
      pc = 0;
      ++pm;
    }
  };
#pragma unroll
  for (int d = 0; d < PD - 1; ++d) prefetch(buf[d]);

  // A_v (bf16 hi and lo halves, s_av[p][v]) and A_in (float32, s_ain[j][p]) into LDS,
  // zero-padded
  stage_av_hilo(s_av, lo_off, ldb, k.Av, k.r, RP, 0, k.vb, k.Iv, tid, k.av_vec != 0);
  for (int64_t e = tid; e < k.I_in * RP; e += kThreads) {
    const int64_t j = e / RP;
    const int p = int(e - j * RP);
    s_ain[e] = p < k.r ? k.Ain[j * k.r + p] : 0.f;
  }
  lds_barrier();

  f32x16 acc[NT], y[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[nt][e] = 0.f;

  int64_t cm = 0;
  int cc = 0;
  for (int64_t base = 0; base < nitems; base += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      prefetch(buf[(d + PD - 1) % PD]);
      if (base + d < nitems) {
        if (cc == 0) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int e = 0; e < 16; ++e) y[nt][e] = 0.f;
        }
        mfma_hilo_item<NT>(y, buf[d], s_av, lo_off, ldb, cc * KCH + half * 32, col);
        if (cc == nkc - 1) {
          // fold the batch: acc[u, p] += C[p] * A_in[j(u), p] * Z[u, p]
          const int64_t b = b_beg + wave + NW * cm;
          const int64_t uo = b / k.nb_in;
          const int64_t j0 = (b - uo * k.nb_in) * 32;
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int p = nt * 32 + col;
            float c = 1.f;
            uint32_t rest = uint32_t(uo);
            for (int q = k.n_o - 1; q >= 0; --q) {
              const uint32_t qq = fdiv(rest, k.fd_o[q]);
              const uint32_t dd = rest - qq * k.fd_o[q].d;
              rest = qq;
              c *= p < k.r ? k.Ao[q][int64_t(dd) * k.r + p] : 0.f;
            }
#pragma unroll
            for (int e = 0; e < 16; ++e) {
              const int64_t j = std::min<int64_t>(j0 + 8 * (e >> 2) + half * 4 + (e & 3),
                                                  k.I_in - 1);
              acc[nt][e] = fmaf(c * s_ain[j * RP + p], y[nt][e], acc[nt][e]);
            }
          }
        }
        if (++cc == nkc) {
          cc = 0;
          ++cm;
        }
      }
    }
  }

  // sum over the 32 u rows (registers, then the two lane halves), then over the waves in
  // order; lanes < 32 of each wave hold the column sums
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    float s = 0.f;
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[nt][e];
    const float o = __shfl_xor(s, 32);
    s = half ? o + s : s + o;
    if (half == 0) s_red[wave * RP + nt * 32 + col] = s;
  }
  __syncthreads();
  if (tid < RP && tid < k.r) {
    float s = s_red[tid];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += s_red[w * RP + tid];
    k.out[(split * k.I + i) * k.r + tid] = s;
  }
}

// ---- Fused all-mode MTTKRP of a 4-way bfloat16 tensor (modes 3 and 4 of size 128) ----
// Every mode's MTTKRP with the same factors A_1..A_4 in one pass over T (the gradient of the
// objective at one point, Sec. 2, eq. def:grad). T is a sequence of slabs M_ij = T(i, j, :, :)
// (128 x 128, 32 KB). Per slab, on matrix cores:
//   Z = M_ij A_4      (rows k of M, K = l),   U = M_ij^T A_3   (rows l, K = k),
// and in float32 registers, with ab[p] = A_1[i, p] A_2[j, p]:
//   P_3[k, p] += ab[p] Z[k, p],   P_4[l, p] += ab[p] U[l, p],
//   W[i, j, p] = sum_k A_3[k, p] Z[k, p],
// after which P_1 = sum_j A_2[j, p] W[i, j, p] and P_2 = sum_i A_1[i, p] W[i, j, p] are the
// two folds of W used by the 3-way solver. 4r flops of MFMA per tensor element instead of
// 8r for four MTTKRPs; T is read once. A workgroup takes slabs gridDim.x apart, holds the
// slab in LDS (rows padded to 136 elements), keeps the next two in flight into registers,
// and writes its P_3 and P_4 sums as split partials that the fixed-order reduction adds.
struct F4Args {
  const uint16_t* T;
  const float* A1;
  const float* A2;
  const float* A3;
  const float* A4;
  float* W;      // I_1 x I_2 x r
  float* part3;  // [nwg][128][r]
  float* part4;  // [nwg][128][r]
  int64_t I2, nslab;
  FastDiv fd_I2;
  int r;
};

constexpr int kF4Ld = 136;  // LDS row stride (elements) of the slab and the factor blocks

template <int NT>
__global__ __launch_bounds__(kThreads, 2) void mttkrp_fused4_kernel(F4Args k) {
  constexpr int RP = 32 * NT;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  uint16_t* s_m = reinterpret_cast<uint16_t*>(smem);       // [128][kF4Ld]
  uint16_t* s_d = s_m + 128 * kF4Ld;                        // A_4 as [p][l]
  uint16_t* s_c = s_d + RP * kF4Ld;                         // A_3 as [p][k]
  float* s_w = reinterpret_cast<float*>(s_c + RP * kF4Ld);  // [2][4][RP]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int col = lane & 31;
  const int half = lane >> 5;
  const int64_t stride = gridDim.x;

  for (int e = tid; e < 128 * RP; e += kThreads) {
    const int x = e / RP;
    const int p = e - x * RP;
    s_d[p * kF4Ld + x] = f2bf(p < k.r ? k.A4[x * k.r + p] : 0.f);
    s_c[p * kF4Ld + x] = f2bf(p < k.r ? k.A3[x * k.r + p] : 0.f);
  }

  // slab s: thread tid loads 16-byte chunks q = tid + 256 t (row q / 16, 8 elements each);
  // two slabs are in flight per workgroup (two register buffers, used alternately)
  auto load_slab = [&](uint4 (&pf)[8], int64_t s) {
    const bool ok = s < k.nslab;
    const uint4* src = reinterpret_cast<const uint4*>(k.T + (ok ? s : 0) * 16384);
#pragma unroll
    for (int t = 0; t < 8; ++t) pf[t] = ok ? src[tid + 256 * t] : make_uint4(0, 0, 0, 0);
  };

  f32x16 acc3[NT], acc4[NT], z[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      acc3[nt][e] = 0.f;
      acc4[nt][e] = 0.f;
    }

  int64_t prev = -1;
  int par = 0;
  auto step = [&](uint4 (&pf)[8], int64_t s) {
    lds_barrier();  // every wave is done with the previous slab in LDS
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int q = tid + 256 * t;
      *reinterpret_cast<uint4*>(&s_m[(q >> 4) * kF4Ld + (q & 15) * 8]) = pf[t];
    }
    lds_barrier();
    // W of the previous slab: the four waves' sums in order
    if (prev >= 0 && tid < k.r) {
      const float* w = s_w + (par ^ 1) * 4 * RP;
      k.W[prev * k.r + tid] = ((w[tid] + w[RP + tid]) + w[2 * RP + tid]) + w[3 * RP + tid];
    }
    load_slab(pf, s + 2 * stride);
    const uint32_t i = fdiv(uint32_t(s), k.fd_I2);
    const uint32_t j = uint32_t(s) - i * uint32_t(k.I2);
    float ab[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int p = nt * 32 + col;
      ab[nt] = p < k.r ? k.A1[i * k.r + p] * k.A2[j * k.r + p] : 0.f;
    }
    // Z = M A_4 for this wave's rows k = 32 wave + [0, 32) (the first product starts from a
    // zero accumulator operand)
    const f32x16 zero16 = {};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const bf16x8 a =
          *reinterpret_cast<const bf16x8*>(&s_m[(32 * wave + col) * kF4Ld + c * 16 + half * 8]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const bf16x8 b =
            *reinterpret_cast<const bf16x8*>(&s_d[(nt * 32 + col) * kF4Ld + c * 16 + half * 8]);
        z[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c == 0 ? zero16 : z[nt], 0, 0, 0);
      }
    }
    // P_3 += ab Z; this wave's share of W = sum_k A_3[k, p] Z[k, p]
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int p = nt * 32 + col;
      float w = 0.f;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int kk = 32 * wave + 8 * (e >> 2) + half * 4 + (e & 3);
        w = fmaf(bf16_bits_to_f32(s_c[p * kF4Ld + kk]), z[nt][e], w);
        acc3[nt][e] = fmaf(ab[nt], z[nt][e], acc3[nt][e]);
      }
      const float o = __shfl_xor(w, 32);
      if (half == 0) s_w[(par * 4 + wave) * RP + p] = w + o;
    }
    // U = M^T A_3 for this wave's rows l = 32 wave + [0, 32): transposing LDS reads of the
    // slab give each lane 8 consecutive k of its column l
    {
      const int g = lane >> 4;
      const int m0 = 16 * (g & 1);
      const int src = lane & 15;
      const int jj = src >> 2;
      const int s4 = (src & 3) * 4;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int kq = 16 * c + 8 * (g >> 1);
        union {
          i16x4 h[2];
          bf16x8 v;
        } a;
        a.h[0] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (lds_i16x4*)(&s_m[(kq + jj) * kF4Ld + 32 * wave + m0 + s4]));
        a.h[1] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (lds_i16x4*)(&s_m[(kq + 4 + jj) * kF4Ld + 32 * wave + m0 + s4]));
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const bf16x8 b = *reinterpret_cast<const bf16x8*>(
              &s_c[(nt * 32 + col) * kF4Ld + 16 * c + 8 * half]);
          z[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, b, c == 0 ? zero16 : z[nt], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc4[nt][e] = fmaf(ab[nt], z[nt][e], acc4[nt][e]);
    prev = s;
    par ^= 1;
  };

  uint4 pf0[8], pf1[8];
  int64_t s = blockIdx.x;
  load_slab(pf0, s);
  load_slab(pf1, s + stride);
  for (; s < k.nslab; s += 2 * stride) {
    step(pf0, s);
    if (s + stride < k.nslab) step(pf1, s + stride);
  }
  __syncthreads();
  if (prev >= 0 && tid < k.r) {
    const float* w = s_w + (par ^ 1) * 4 * RP;
    k.W[prev * k.r + tid] = ((w[tid] + w[RP + tid]) + w[2 * RP + tid]) + w[3 * RP + tid];
  }
  // this workgroup's P_3 and P_4 sums (rows 32 wave + row of the accumulator register)
  float* o3 = k.part3 + int64_t(blockIdx.x) * 128 * k.r;
  float* o4 = k.part4 + int64_t(blockIdx.x) * 128 * k.r;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int p = nt * 32 + col;
    if (p >= k.r) continue;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = 32 * wave + 8 * (e >> 2) + half * 4 + (e & 3);
      o3[row * k.r + p] = acc3[nt][e];
      o4[row * k.r + p] = acc4[nt][e];
    }
  }
}

// Fixed-order sum of split partials: each output element is summed by 4 threads over
// interleaved splits (float64), then combined in thread order.
__global__ __launch_bounds__(256) void mttkrp_reduce_kernel(const float* __restrict__ part,
                                                            int64_t splits, int64_t n,
                                                            float* __restrict__ P) {
  __shared__ double s[4][64];
  const int o = threadIdx.x & 63;
  const int g = threadIdx.x >> 6;
  for (int64_t e0 = int64_t(blockIdx.x) * 64; e0 < n; e0 += int64_t(gridDim.x) * 64) {
    const int64_t e = e0 + o;
    double acc = 0.0;
    if (e < n) {
      // splits g, g + 4, ... in order: sixteen loads in flight (clamped, no branch per load)
      // while at least sixteen remain, then the rest one by one (few splits: no repeated
      // loads of the last one)
      int64_t q0 = g;
      for (; q0 + 60 < splits; q0 += 64) {
        float v[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] = part[(q0 + 4 * t) * n + e];
#pragma unroll
        for (int t = 0; t < 16; ++t) acc += double(v[t]);
      }
      for (; q0 < splits; q0 += 4) acc += double(part[q0 * n + e]);
    }
    s[g][o] = acc;
    __syncthreads();
    if (g == 0 && e < n) P[e] = float(((s[0][o] + s[1][o]) + s[2][o]) + s[3][o]);
    __syncthreads();
  }
}

// The same sums for at most four splits, four elements per thread with 16-byte loads: for
// splits <= 4 the fixed order above is ((s0 + s1) + s2) + s3 with s_g = 0 + part[g] (and
// +0 for a missing split), which this computes in the same float64 steps.
__global__ __launch_bounds__(256) void mttkrp_reduce4_kernel(const float4* __restrict__ part,
                                                             int splits, int64_t n4,
                                                             float4* __restrict__ P) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n4; e += stride) {
    float4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      v[q] = q < splits ? part[int64_t(q) * n4 + e] : make_float4(0.f, 0.f, 0.f, 0.f);
    double sx[4], sy[4], sz[4], sw[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool in = q < splits;
      sx[q] = in ? 0.0 + double(v[q].x) : 0.0;
      sy[q] = in ? 0.0 + double(v[q].y) : 0.0;
      sz[q] = in ? 0.0 + double(v[q].z) : 0.0;
      sw[q] = in ? 0.0 + double(v[q].w) : 0.0;
    }
    P[e] = make_float4(float(((sx[0] + sx[1]) + sx[2]) + sx[3]),
                       float(((sy[0] + sy[1]) + sy[2]) + sy[3]),
                       float(((sz[0] + sz[1]) + sz[2]) + sz[3]),
                       float(((sw[0] + sw[1]) + sw[2]) + sw[3]));
  }
}

// P[e] = the fixed-order sum over the splits of part[split][e], e < n
hipError_t launch_reduce(const float* part, int64_t splits, int64_t n, float* P,
                         hipStream_t s) {
  if (splits <= 4 && n % 4 == 0 &&
      ((reinterpret_cast<uintptr_t>(part) | reinterpret_cast<uintptr_t>(P)) & 15) == 0) {
    const int64_t n4 = n / 4;
    const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(ceil_div(n4, 256), 4096)));
    hipLaunchKernelGGL(mttkrp_reduce4_kernel, dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(part), int(splits), n4,
                       reinterpret_cast<float4*>(P));
    return hipGetLastError();
  }
  const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 64), 4096)));
  hipLaunchKernelGGL(mttkrp_reduce_kernel, dim3(blocks), dim3(256), 0, s, part, splits, n, P);
  return hipGetLastError();
}

// Folds of a stored Y[I][U][r] (3-way tensors: Y = T x_3 A_3, u = mode 2):
//   fold_u: P[i, p] = sum_u X[u, p] Y[i, u, p]   (the mode-1 MTTKRP, X = A_2)
//   fold_i: P[u, p] = sum_i X[i, p] Y[i, u, p]   (the mode-2 MTTKRP, X = A_1), as partial
//           sums over i ranges that mttkrp_reduce_kernel adds in order.
// fold_u: one workgroup per i; 8 groups of u summed in fixed order.
__global__ __launch_bounds__(256) void fold_u_kernel(const float* __restrict__ Y,
                                                     const float* __restrict__ X, int64_t U,
                                                     int r, float* __restrict__ P) {
  __shared__ float s[8][256];
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  const float* yi = Y + i * U * r;
  for (int p0 = 0; p0 < r; p0 += 32) {
    const int p = p0 + (tid & 31);
    const int g = tid >> 5;
    // four independent partial sums (u = g + 8 (4 t + j)), combined in a fixed order: a
    // step t adds u, u + 8, u + 16, u + 24 into a0..a3 while u + 24 < U, then the rest
    // (at most three) go into a0. The loads of four steps (and of the rest) are issued
    // together at clamped in-range u; steps past the bound add nothing.
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    if (p < r) {
      int64_t u = g;
      while (u + 24 < U) {
        float xv[16], yv[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int64_t uu = std::min<int64_t>(u + 8 * k, U - 1);
          xv[k] = X[uu * r + p];
          yv[k] = yi[uu * r + p];
        }
        int nv = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const bool ok = u + 32 * t + 24 < U;
          nv += ok ? 1 : 0;
          a0 = ok ? fmaf(xv[4 * t], yv[4 * t], a0) : a0;
          a1 = ok ? fmaf(xv[4 * t + 1], yv[4 * t + 1], a1) : a1;
          a2 = ok ? fmaf(xv[4 * t + 2], yv[4 * t + 2], a2) : a2;
          a3 = ok ? fmaf(xv[4 * t + 3], yv[4 * t + 3], a3) : a3;
        }
        u += 32 * nv;
      }
      float xt[3], yt[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int64_t uu = std::min<int64_t>(u + 8 * k, U - 1);
        xt[k] = X[uu * r + p];
        yt[k] = yi[uu * r + p];
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) a0 = u + 8 * k < U ? fmaf(xt[k], yt[k], a0) : a0;
    }
    s[g][tid & 31] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (tid < 32 && p0 + tid < r) {
      float t = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) t += s[q][tid];
      P[i * r + p0 + tid] = t;
    }
    __syncthreads();
  }
}

// fold_i: workgroup (u tile of 256 / r' outputs, i range); partial[split][u][p].
// With a Hadamard job, the first `has_had` rows of blocks compute it instead (enough
// blocks for four threads per entry of G).
__global__ __launch_bounds__(256) void fold_i_kernel(const float* __restrict__ Y,
                                                     const float* __restrict__ X, int64_t I,
                                                     int64_t U, int r, int64_t per,
                                                     float* __restrict__ part, int has_had,
                                                     HadamardLaunch had) {
  if (int(blockIdx.y) < has_had) {
    hadamard_work(had.job, had.r, had.G32, had.G64, had.slots, had.nslots,
                  int64_t(blockIdx.y) * gridDim.x + blockIdx.x, int64_t(has_had) * gridDim.x);
    return;
  }
  const int64_t n = U * r;
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;  // (u, p) flattened
  const int64_t split = blockIdx.y - has_had;
  const int64_t i_lo = split * per, i_hi = std::min<int64_t>(I, i_lo + per);
  if (e >= n) return;
  const int p = int(e % r);
  float a0 = 0.f, a1 = 0.f;
  int64_t i = i_lo;
  for (; i + 1 < i_hi; i += 2) {
    a0 = fmaf(X[i * r + p], Y[i * n + e], a0);
    a1 = fmaf(X[(i + 1) * r + p], Y[(i + 1) * n + e], a1);
  }
  if (i < i_hi) a0 = fmaf(X[i * r + p], Y[i * n + e], a0);
  part[split * n + e] = a0 + a1;
}

using KernelFn = void (*)(KArgs);

template <bool BF16, int NT, int WM, int WK, bool LAST, bool VEC>
KernelFn pick() {
  return mttkrp_kernel<BF16, NT, WM, WK, LAST, VEC>;
}

// WM x WK = 4 waves. Ranks above 64 use row tiles of at least 64 rows.
template <bool BF16, bool LAST, bool VEC>
KernelFn pick_shape(int wm, int nt) {
  if (nt == 1) {
    if (wm == 1) return pick<BF16, 1, 1, 4, LAST, VEC>();
    if (wm == 2) return pick<BF16, 1, 2, 2, LAST, VEC>();
    return pick<BF16, 1, 4, 1, LAST, VEC>();
  }
  if (nt == 2) {
    if (wm == 1) return pick<BF16, 2, 1, 4, LAST, VEC>();
    if (wm == 2) return pick<BF16, 2, 2, 2, LAST, VEC>();
    return pick<BF16, 2, 4, 1, LAST, VEC>();
  }
  if (nt == 4) {
    if (wm == 4) return pick<BF16, 4, 4, 1, LAST, VEC>();
    return pick<BF16, 4, 2, 2, LAST, VEC>();
  }
  if (wm == 4) return pick<BF16, 8, 4, 1, LAST, VEC>();
  return pick<BF16, 8, 2, 2, LAST, VEC>();
}

using SlabFn = void (*)(SArgs);
SlabFn select_slab(int nt) {
  return nt == 1 ? mttkrp_slab_kernel<1> : mttkrp_slab_kernel<2>;
}

KernelFn select_kernel(bool bf16, bool last, int wm, int nt, bool vec) {
  if (vec) {
    if (bf16)
      return last ? pick_shape<true, true, true>(wm, nt) : pick_shape<true, false, true>(wm, nt);
    return last ? pick_shape<false, true, true>(wm, nt) : pick_shape<false, false, true>(wm, nt);
  }
  if (bf16)
    return last ? pick_shape<true, true, false>(wm, nt) : pick_shape<true, false, false>(wm, nt);
  return last ? pick_shape<false, true, false>(wm, nt) : pick_shape<false, false, false>(wm, nt);
}

// 16-byte loads apply: every row start is 16-byte aligned and the contiguous extent is a
// multiple of 16 bytes (the tensor base is 16-byte aligned)
bool vec_loads(const MttkrpPlan& pl) {
  const int vec = pl.dtype == NTF_BF16 ? 8 : 4;
  return pl.layout == 1 ? (pl.v.I % vec == 0) : (pl.v.R % vec == 0 && pl.Iv % vec == 0);
}

int n_tiles(int r) {
  const int nt = (r + 31) / 32;
  return nt <= 1 ? 1 : nt <= 2 ? 2 : nt <= 4 ? 4 : 8;
}

size_t lds_bytes(bool bf16, bool last, int rp, int vb, int ub) {
  const size_t av = bf16 ? size_t(2) * rp * (vb + 8) * 2 : size_t(vb) * rp * 4;
  size_t b = align_up(av, 16) + align_up(size_t(ub) * rp * 4, 16);
  if (bf16 && last) b += size_t(4) * 64 * kStageLd * 2;
  return b;
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

// The row-slab kernel applies to bfloat16 modes before the last (order >= 3, r <= 64: two N
// tiles keep the accumulators, the batch and its prefetch in 256 registers) when the
// tensor's rows and runs are 16-byte aligned, the innermost u mode has at least 16 values
// and the LDS blocks fit; returns the LDS bytes, or 0 where it does not apply.
static size_t slab_lds(const MttkrpPlan& pl, const ntf_tensor& T) {
  const int N = T.order;
  const int n = pl.v.mode;
  if (pl.dtype != NTF_BF16 || pl.layout != 0 || pl.store_y || pl.variant > 2 || N < 3) return 0;
  if (!vec_loads(pl)) return 0;
  const int inner = n < N - 2 ? N - 2 : N - 3;
  const int64_t I_in = T.dims[inner];
  if (I_in < 16) return 0;
  const int64_t vb = ceil_div(pl.Iv, int64_t(64)) * 64;
  const size_t lds = align_up(size_t(2) * pl.rpad * (vb + 8) * 2, 16) + size_t(I_in) * pl.rpad * 4 +
                     size_t(kThreads / 64) * pl.rpad * 4;
  return lds > 72 * 1024 ? 0 : lds;
}

// Switch a plan to the row-slab kernel. By default the planner does so when the row stride
// is a multiple of 1 MiB (rows that share DRAM banks); a tuned choice decides otherwise.
static void plan_slab(MttkrpPlan& pl, const ntf_tensor& T, int num_cus,
                      const MttkrpChoice* choice) {
  if (choice && choice->kernel == 1) return;
  const size_t lds = slab_lds(pl, T);
  if (lds == 0) return;
  const bool forced = choice && choice->kernel == 2;
  if (!forced && (pl.v.R * 2) % (int64_t(1) << 20) != 0) return;
  const int N = T.order;
  const int inner = pl.v.mode < N - 2 ? N - 2 : N - 3;
  const int64_t I_in = T.dims[inner];
  const int64_t vb = ceil_div(pl.Iv, int64_t(64)) * 64;
  SlabFn fn = select_slab(pl.variant);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn),
                                                   kThreads, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int64_t nb_in = ceil_div(I_in, int64_t(32));
  const int64_t nbatch = pl.U / I_in * nb_in;
  const int64_t slots = int64_t(per_cu) * num_cus;
  int64_t S = std::max<int64_t>(1, slots / pl.v.I);
  S = std::min<int64_t>({S, std::max<int64_t>(1, nbatch / 4), int64_t(65535)});
  pl.slab = true;
  pl.slab_inner = inner;
  pl.vb = int(vb);
  pl.nvb = 1;
  pl.splits = S;
  pl.lds = lds;
}

MttkrpPlan plan_mttkrp(const ntf_tensor& T, int mode, int r, int num_cus, bool store_y,
                       const MttkrpChoice* choice) {
  MttkrpPlan pl;
  pl.store_y = store_y;
  pl.v = make_mode_view(T, mode);
  pl.dtype = T.dtype;
  pl.r = r;
  const int nt = n_tiles(r);
  pl.rpad = 32 * nt;
  pl.variant = nt;
  const bool bf16 = T.dtype == NTF_BF16;
  const bool last = mode == T.order - 1;
  pl.layout = last ? 1 : 0;
  pl.vmode = last ? T.order - 2 : T.order - 1;
  pl.Iv = T.dims[pl.vmode];
  pl.U = 1;
  for (int l = 0; l < T.order; ++l)
    if (l != mode && l != pl.vmode) pl.U *= T.dims[l];
  // row tile: least padding among the instantiated shapes (ties: the taller tile)
  const int64_t I = pl.v.I;
  // bf16 last mode: a wave's tile spans 32 contiguous elements (64 B); two waves side by
  // side make whole 128-byte lines per workgroup
  const int wm_min = (nt >= 4 || (bf16 && last)) ? 2 : 1;
  int64_t best = -1;
  pl.wm = 4;
  for (int wm : {4, 2, 1}) {
    if (wm < wm_min) continue;
    const int64_t padded = ceil_div(I, 32 * wm) * 32 * wm;
    if (best < 0 || padded < best) {
      best = padded;
      pl.wm = wm;
    }
  }
  if (choice && choice->kernel == 1 && !store_y &&
      (choice->wm == 1 || choice->wm == 2 || choice->wm == 4) && choice->wm >= wm_min)
    pl.wm = choice->wm;
  // Y rows are whole only when one wave covers every v chunk of its u: the WK waves of a
  // row tile take interleaved u values instead of interleaved v chunks
  pl.uk = store_y;
  pl.wk = 4 / pl.wm;
  // v-block: all of I_v when its A_v block fits 64 KB of LDS
  const int kch = bf16 ? 64 : 32;
  const int64_t per_k = int64_t(pl.rpad) * 4;  // bf16: hi and lo halves
  int64_t vbmax = (64 * 1024) / per_k - (bf16 ? 8 : 0);
  vbmax = std::max<int64_t>(kch, vbmax / kch * kch);
  const int64_t iv_pad = ceil_div(pl.Iv, kch) * kch;
  pl.vb = int(std::min(iv_pad, vbmax));
  pl.nvb = int(ceil_div(pl.Iv, pl.vb));
  pl.mtiles = ceil_div(I, 32 * pl.wm);
  pl.chunks = pl.U * pl.nvb;  // work items (v-block, u)
  // the end-of-kernel reduction of the WK waves reuses the same LDS
  const size_t red = size_t(pl.wk - 1) * pl.wm * 64 * 16 * nt * sizeof(float);
  // One residency wave: grid = resident workgroups per CU x CUs (a partial second wave
  // would double the time of the tail). The X batch (and so LDS and occupancy) depends on
  // the split count; two refinement passes settle it (LDS only shrinks between passes).
  KernelFn fn = select_kernel(bf16, last, pl.wm, nt, vec_loads(pl));
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  pl.ub = int(std::max<int64_t>(1, std::min<int64_t>(int64_t(8192 / pl.rpad), pl.U)));
  for (int pass = 0; pass < 3; ++pass) {
    pl.lds = std::max(lds_bytes(bf16, last, pl.rpad, pl.vb, pl.ub), red);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn),
                                                     kThreads, pl.lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    const int64_t slots = int64_t(per_cu) * num_cus;
    int64_t splits = std::max<int64_t>(1, slots / pl.mtiles);
    splits = std::min<int64_t>({splits, pl.chunks, int64_t(65535)});
    pl.splits = splits;
    const int64_t per = ceil_div(pl.chunks, splits);
    pl.ub = int(std::max<int64_t>(1, std::min<int64_t>({per, int64_t(8192 / pl.rpad), pl.U})));
  }
  pl.lds = std::max(lds_bytes(bf16, last, pl.rpad, pl.vb, pl.ub), red);
  if (!store_y) plan_slab(pl, T, num_cus, choice);
  return pl;
}

int mttkrp_candidates(const ntf_tensor& T, int mode, int r, MttkrpChoice* out, int cap) {
  // the planner's default first (as an explicit choice), then the other shapes; same rules
  // as plan_mttkrp: rank above 64 or a bf16 last mode needs tiles of 2+ waves
  const MttkrpPlan def = plan_mttkrp(T, mode, r, 1);
  const MttkrpChoice d = def.slab ? MttkrpChoice{2, 0} : MttkrpChoice{1, def.wm};
  int n = 0;
  if (n < cap) out[n++] = d;
  const bool last = mode == T.order - 1;
  const int wm_min = (n_tiles(r) >= 4 || (T.dtype == NTF_BF16 && last)) ? 2 : 1;
  for (int wm : {4, 2, 1})
    if (wm >= wm_min && n < cap && !(d.kernel == 1 && d.wm == wm)) out[n++] = MttkrpChoice{1, wm};
  if (d.kernel != 2 && slab_lds(def, T) > 0 && n < cap) out[n++] = MttkrpChoice{2, 0};
  return n;
}

std::string tune_key(const ntf_tensor& T, int mode, int r) {
  std::string k = T.dtype == NTF_BF16 ? "bf16" : "f32";
  for (int l = 0; l < T.order; ++l) k += (l ? "x" : ":") + std::to_string(T.dims[l]);
  k += ":mode" + std::to_string(mode) + ":r" + std::to_string(r);
  return k;
}

const MttkrpChoice* tuned_choice(const ntf_handle* h, const ntf_tensor& T, int mode, int r) {
  if (h->tune.empty()) return nullptr;
  const auto it = h->tune.find(tune_key(T, mode, r));
  return it == h->tune.end() ? nullptr : &it->second;
}

static hipError_t launch_slab(const MttkrpPlan& pl, const void* T, const FactorPtrs& A, float* P,
                              float* partials, bool reduce, hipStream_t s,
                              const HadamardLaunch* had) {
  SArgs k{};
  if (had) {
    k.nh = hadamard_blocks(had->r);
    k.had = *had;
  }
  const int N = pl.v.order;
  const int n = pl.v.mode;
  k.T = T;
  k.tbytes = pl.v.L * pl.v.I * pl.v.R * 2;
  k.Av = A.p[pl.vmode];
  k.Ain = A.p[pl.slab_inner];
  k.n_o = 0;
  for (int l = 0; l < N; ++l) {
    if (l == n || l == pl.vmode || l == pl.slab_inner) continue;
    k.Ao[k.n_o] = A.p[l];
    k.fd_o[k.n_o] = make_fastdiv(uint32_t(pl.v.dims[l]));
    k.n_o++;
  }
  k.I = pl.v.I;
  k.Iv = pl.Iv;
  k.R = pl.v.R;
  k.a_stride = pl.v.I * pl.v.R;
  k.Rp = pl.v.R / pl.Iv;
  k.fd_Rp = make_fastdiv(uint32_t(k.Rp));
  k.I_in = pl.v.dims[pl.slab_inner];
  k.nb_in = ceil_div(k.I_in, int64_t(32));
  k.nbatch = pl.U / k.I_in * k.nb_in;
  k.S = pl.splits;
  k.r = pl.r;
  k.vb = pl.vb;
  k.av_vec = (pl.r == pl.rpad && (reinterpret_cast<uintptr_t>(k.Av) & 15) == 0) ? 1 : 0;
  const bool split = pl.splits > 1;
  k.out = split ? partials : P;
  SlabFn fn = select_slab(pl.variant);
  dim3 grid(unsigned(pl.v.I * pl.splits + k.nh));
  hipLaunchKernelGGL(fn, grid, dim3(kThreads), pl.lds, s, k);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (split && reduce) e = launch_reduce(partials, pl.splits, pl.v.I * pl.r, P, s);
  return e;
}

hipError_t launch_mttkrp(const MttkrpPlan& pl, const void* T, const FactorPtrs& A, float* P,
                         float* partials, bool reduce, hipStream_t s, float* ystore,
                         const HadamardLaunch* had) {
  KArgs k{};
  if (pl.slab) return launch_slab(pl, T, A, P, partials, reduce, s, had);
  if (had) {
    k.nh = hadamard_blocks(had->r);
    k.had = *had;
  }
  k.ystore = pl.store_y ? ystore : nullptr;
  k.T = T;
  const int N = pl.v.order;
  const int n = pl.v.mode;
  const bool last = pl.layout == 1;
  k.Av = A.p[pl.vmode];
  k.av_vec = (pl.r == pl.rpad && (reinterpret_cast<uintptr_t>(k.Av) & 15) == 0) ? 1 : 0;
  k.n_o = 0;
  for (int l = 0; l < N; ++l) {
    if (l == n || l == pl.vmode) continue;
    k.Ao[k.n_o] = A.p[l];
    k.fd_o[k.n_o] = make_fastdiv(uint32_t(pl.v.dims[l]));
    k.n_o++;
  }
  k.I = pl.v.I;
  k.Iv = pl.Iv;
  k.U = pl.U;
  k.R = pl.v.R;
  k.a_stride = pl.v.I * pl.v.R;
  k.Rp = last ? 1 : pl.v.R / pl.Iv;
  k.fd_Rp = make_fastdiv(uint32_t(k.Rp));
  k.per_split = pl.chunks / pl.splits;
  k.mtiles = pl.mtiles;
  k.extra = pl.chunks % pl.splits;
  k.r = pl.r;
  k.vb = pl.vb;
  k.ub = pl.ub;
  k.uk = pl.uk ? 1 : 0;
  const bool bf16 = pl.dtype == NTF_BF16;
  const bool vec = vec_loads(pl);
  k.tbytes = pl.v.L * pl.v.I * pl.v.R * (bf16 ? 2 : 4);
  const bool split = pl.splits > 1;
  k.out = split ? partials : P;
  KernelFn fn = select_kernel(bf16, last, pl.wm, pl.variant, vec);
  static bool attr_done[2][2][2][4][8] = {};
  bool& done = attr_done[vec][bf16][last][pl.wm - 1][pl.variant - 1];
  if (!done) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    done = true;
  }
  dim3 grid(unsigned(pl.mtiles * pl.splits + k.nh));
  hipLaunchKernelGGL(fn, grid, dim3(kThreads), pl.lds, s, k);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (k.ystore) return e;
  if (split && reduce) e = launch_reduce(partials, pl.splits, pl.v.I * pl.r, P, s);
  return e;
}

bool fused4_applies(const ntf_tensor& T, int r) {
  return T.order == 4 && T.dtype == NTF_BF16 && T.dims[2] == 128 && T.dims[3] == 128 &&
         r <= 64 && (reinterpret_cast<uintptr_t>(T.data) & 15) == 0 &&
         T.dims[0] * T.dims[1] < (int64_t(1) << 31);
}

static int fused4_grid(const ntf_tensor& T, int r, int num_cus, size_t* lds_out) {
  const int rp = r <= 32 ? 32 : 64;
  const size_t lds = size_t(128) * kF4Ld * 2 + size_t(2) * rp * kF4Ld * 2 + size_t(8) * rp * 4;
  const void* fn = rp == 32 ? reinterpret_cast<const void*>(mttkrp_fused4_kernel<1>)
                            : reinterpret_cast<const void*>(mttkrp_fused4_kernel<2>);
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (lds_out) *lds_out = lds;
  return int(std::max<int64_t>(1, std::min<int64_t>(int64_t(per_cu) * num_cus,
                                                    T.dims[0] * T.dims[1])));
}

size_t fused4_workspace_floats(const ntf_tensor& T, int r, int num_cus) {
  const int64_t nwg = fused4_grid(T, r, num_cus, nullptr);
  const int64_t I1 = T.dims[0], I2 = T.dims[1];
  return size_t(align_up(size_t(I1 * I2 * r), 64) + 2 * align_up(size_t(nwg * 128 * r), 64) +
                align_up(size_t(fold_i_splits(I1, I2, r) * I2 * r), 64));
}

hipError_t launch_fused4(const ntf_tensor& T, const float* const* A, int r, int num_cus,
                         float* const* P, float* ws, hipStream_t s) {
  size_t lds = 0;
  const int nwg = fused4_grid(T, r, num_cus, &lds);
  const int64_t I1 = T.dims[0], I2 = T.dims[1];
  F4Args k{};
  k.T = static_cast<const uint16_t*>(T.data);
  k.A1 = A[0];
  k.A2 = A[1];
  k.A3 = A[2];
  k.A4 = A[3];
  k.W = ws;
  k.part3 = ws + align_up(size_t(I1 * I2 * r), 64);
  k.part4 = k.part3 + align_up(size_t(int64_t(nwg) * 128 * r), 64);
  float* fpart = k.part4 + align_up(size_t(int64_t(nwg) * 128 * r), 64);
  k.I2 = I2;
  k.fd_I2 = make_fastdiv(uint32_t(I2));
  k.nslab = I1 * I2;
  k.r = r;
  if (r <= 32)
    hipLaunchKernelGGL(mttkrp_fused4_kernel<1>, dim3(nwg), dim3(kThreads), lds, s, k);
  else
    hipLaunchKernelGGL(mttkrp_fused4_kernel<2>, dim3(nwg), dim3(kThreads), lds, s, k);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n34 = int64_t(128) * r;
  const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(ceil_div(n34, 64), 4096)));
  if (P[2]) {
    hipLaunchKernelGGL(mttkrp_reduce_kernel, dim3(blocks), dim3(256), 0, s, k.part3,
                       int64_t(nwg), n34, P[2]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (P[3]) {
    hipLaunchKernelGGL(mttkrp_reduce_kernel, dim3(blocks), dim3(256), 0, s, k.part4,
                       int64_t(nwg), n34, P[3]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (P[0] && (e = launch_fold_u(k.W, A[1], I1, I2, r, P[0], s)) != hipSuccess) return e;
  if (P[1] && (e = launch_fold_i(k.W, A[0], I1, I2, r, fpart, P[1], s)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_fold_u(const float* Y, const float* X, int64_t I, int64_t U, int r, float* P,
                         hipStream_t s) {
  hipLaunchKernelGGL(fold_u_kernel, dim3(unsigned(I)), dim3(256), 0, s, Y, X, U, r, P);
  return hipGetLastError();
}

int64_t fold_i_splits(int64_t I, int64_t U, int r) {
  // enough workgroups to stream Y: about 1024 in total, at least 4 rows of i each
  const int64_t tiles = ceil_div(U * r, 256);
  return std::max<int64_t>(1, std::min<int64_t>(ceil_div(1024, tiles), ceil_div(I, 4)));
}

hipError_t launch_fold_i(const float* Y, const float* X, int64_t I, int64_t U, int r,
                         float* partials, float* P, hipStream_t s, const HadamardLaunch* had) {
  const int64_t splits = fold_i_splits(I, U, r);
  const int64_t per = ceil_div(I, splits);
  const int64_t n = U * r;
  const int64_t gx = ceil_div(n, 256);
  // rows of Hadamard blocks: four threads per entry of the r x r product
  const int has_had =
      had ? int(ceil_div(ceil_div(4 * int64_t(had->r) * had->r, int64_t(256)), gx)) : 0;
  HadamardLaunch h{};
  if (had) h = *had;
  hipLaunchKernelGGL(fold_i_kernel, dim3(unsigned(gx), unsigned(splits + has_had)), dim3(256),
                     0, s, Y, X, I, U, r, per, partials, has_had, h);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 64), 4096)));
  hipLaunchKernelGGL(mttkrp_reduce_kernel, dim3(blocks), dim3(256), 0, s, partials, splits, n,
                     P);
  return hipGetLastError();
}

}  // namespace ntf
