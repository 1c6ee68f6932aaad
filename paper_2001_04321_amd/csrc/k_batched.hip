// Batched HER-A-HALS (Algorithm 2 with A-HALS blocks, Sec. 2.1.4 and 3.1) for many
// independent small 3-way problems. One outer iteration of every problem is a sequence of
// grouped launches, each covering all problems at once:
//
//   by_kernel      Y = T x_3 Â^(3) (I_1 I_2 x r), from the previous iteration's Â^(3)
//   bfold (mode 0) P^(1)[i, p] = sum_j Â^(2)[j, p] Y[(i, j), p]
//   bhals (block 1)
//   bfold (mode 1) P^(2)[j, p] = sum_i Â^(1)[i, p] Y[(i, j), p]     (Â^(3) has not changed,
//   bhals (block 2)                                                  so Y serves both blocks)
//   blast          P^(3)[k, p] = sum_i Â^(1)[i, p] sum_j Â^(2)[j, p] T[i, j, k], as partial
//                  sums over chunks of four i, added in chunk order by bsum
//   bhals (block 3, then F-hat by the Gram trick of Sec. 3.1.3 and the restart decision)
//
// The set-up (once per call) sums ||T||^2 over the same Y tiles (bnorm), then per problem
// stages A_0 and its Grams (bsetup) and forms F-hat_0 from a last-mode pass.
//
// The tensor passes (Y, the last mode) and the folds give each problem many workgroups
// (tiles of rows), so the large problems of a batch no longer set the pace on one compute
// unit; the A-HALS blocks take one workgroup per problem (one lane per row, stopping rule
// of Sec. 4.1 on the workgroup-wide ||W_s - W_{s-1}||). The HER scalars and the survivor
// buffer of each block live in device memory between launches. Extrapolation (eq.
// extproj_her), Grams, F-hat and the decision are float64; every reduction has a fixed
// order. Ranks are padded to a multiple of 4 (RB) with zero columns.
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kBT = 256;            // threads of a per-problem (A-HALS) workgroup
constexpr int kBW = kBT / 64;
constexpr int kGT = 256;            // threads of a grouped (tile) workgroup
constexpr int kTileLd = 33;         // row stride of a wave's 64 x 32 tensor tile in LDS
constexpr int kYRows = 256;         // Y rows (i, j) per workgroup: 64 per wave
constexpr int kFoldRows = 4;        // fold outputs per workgroup: one per wave
constexpr int kLastChunk = 4;       // i values per last-mode workgroup (one partial sum)

// HER scalars and survivor buffers of one problem, kept in device memory between launches
struct BScal {
  double beta, beta_bar, fhat_prev, normT2;
  double k, nrestarts;
  int32_t s_id[3];  // survivor buffer (0..2) of each block
  int32_t it;       // outer iterations done in this call (trace index)
};

struct BProb {
  const float* T;
  int I[3];
  int r, rb;
  float* A_user[3];
  float* buf[3][3];    // per mode, three I_n x rb buffers
  double* gram[3][3];  // their Grams, rb x rb
  float* Y;            // I_1 I_2 x rb
  float* P;            // I_max x rb
  float* part;         // ceil(I_1 / 4) x I_3 x rb: last-mode partial sums
  double* normp;       // ||T||^2 over each Y tile's rows (set-up)
  BScal* sc;
  ntf_her_state* st;
  double* tr_fhat;
  int32_t* tr_restart;
  int32_t* tr_sweeps;
};

struct BArgs {
  const BProb* probs;
  const int32_t* order;   // per-problem launches: problem of workgroup x
  const uint32_t* items;  // grouped launches: (problem << 16) | tile
  int nprob;
  int resume;
  int max_inner;
  double beta0, gamma, gamma_bar, eta, tol;
  uint32_t* flags;
};

template <int CTRL>
__device__ __forceinline__ double dpp64(double x) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((int64_t(hi) << 32) | uint32_t(lo));
}

__device__ __forceinline__ double readlane64(double x, int l) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), l);
  return __longlong_as_double((int64_t(hi) << 32) | uint32_t(lo));
}

// fixed-order wave sum (rows of 16 by DPP, then the four rows)
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp64<0xB1>(x);
  x += dpp64<0x4E>(x);
  x += dpp64<0x141>(x);
  x += dpp64<0x140>(x);
  return (readlane64(x, 0) + readlane64(x, 16)) + (readlane64(x, 32) + readlane64(x, 48));
}

// fixed-order workgroup sum (kBT threads); every thread gets the result. s_red: kBW + 1.
__device__ double block_sum(double x, double* s_red) {
  const double w = wave_sum(x);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kBW; ++k) t += s_red[k];
    s_red[kBW] = t;
  }
  __syncthreads();
  const double r = s_red[kBW];
  __syncthreads();
  return r;
}

// The same sum with one barrier, for the A-HALS sweeps: each wave's sum goes to buffer
// `parity` of buf (2 x kBW; alternate the parity every call: a wave can only write the
// same buffer again after the next call's barrier, which every wave reaches after its reads
// of this one), then every thread adds the waves' sums in order: the bits of block_sum.
__device__ double sweep_sum(double x, double* buf, int parity) {
  const double w = wave_sum(x);
  double* b = buf + parity * kBW;
  if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = w;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < kBW; ++k) t += b[k];
  return t;
}

// Gram of a rows x RB buffer (float64, rows in order); out: rb x rb global.
template <int RB>
__device__ void gram_of(const float* X, int rows, double* out) {
  for (int e = threadIdx.x; e < RB * RB; e += kBT) {
    const int p = e / RB, q = e - (e / RB) * RB;
    double acc = 0.0;
    for (int i = 0; i < rows; ++i) acc = fma(double(X[i * RB + p]), double(X[i * RB + q]), acc);
    out[e] = acc;
  }
}

__device__ __forceinline__ void item_of(const BArgs& a, int& b, int& t) {
  const uint32_t it = a.items[blockIdx.x];
  b = int(it >> 16);
  t = int(it & 0xffff);
}

// ---- grouped launches ----

// Y[(i, j), :] = sum_k T[i, j, k] A3[k, :] for rows t * 256 .. +256 of problem b. Lanes
// own rows; each wave stages 64 rows x 32 k of T in LDS with row-contiguous loads and
// reads them back per lane (one multiply-add per element and column, in k order).
template <int RB>
__device__ void y_tile(const BProb& pb, int t, float* lds) {
  const int I2 = pb.I[2];
  const int R = pb.I[0] * pb.I[1];
  const float* __restrict__ A3 = pb.buf[2][pb.sc->s_id[2]];
  float* A3s = lds;  // I2 x RB
  float* tiles = lds + align_up(size_t(I2) * RB, 4);
  for (int e = threadIdx.x; e < I2 * RB; e += kGT) A3s[e] = A3[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* tile = tiles + wave * 64 * kTileLd;
  const int row0 = t * kYRows + wave * 64;
  if (row0 >= R) return;  // no barrier follows
  const float* __restrict__ T = pb.T;
  float acc[RB];
#pragma unroll
  for (int p = 0; p < RB; ++p) acc[p] = 0.f;
  const int cc = lane & 31;
  // chunk c0 (32 values of k for 64 rows): lane (rr = 2 q + lane / 32, cc) loads
  // T[row0 + rr, c0 + cc]; entries outside the problem load T[0] and become 0 (no branch,
  // so all 32 loads stay in flight)
  float v[32];
  auto load_chunk = [&](int c0) {
    const int nc = min(32, I2 - c0);
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const int row = row0 + 2 * q + (lane >> 5);
      const bool ok = row < R && cc < nc;
      const float x = T[ok ? int64_t(row) * I2 + c0 + cc : 0];
      v[q] = ok ? x : 0.f;
    }
  };
  load_chunk(0);
  for (int c0 = 0; c0 < I2; c0 += 32) {
    const int nc = min(32, I2 - c0);
#pragma unroll
    for (int q = 0; q < 32; ++q) tile[(2 * q + (lane >> 5)) * kTileLd + cc] = v[q];
    // the next chunk's loads are in flight while this one is used
    if (c0 + 32 < I2) load_chunk(c0 + 32);
    // the tile is written and read by this wave only; LDS operations of a wave complete
    // in order
    for (int c = 0; c < nc; ++c) {
      const float tv = tile[lane * kTileLd + c];
      const float* av = A3s + (c0 + c) * RB;
#pragma unroll
      for (int p = 0; p < RB; ++p) acc[p] = fmaf(tv, av[p], acc[p]);
    }
  }
  const int row = row0 + lane;
  if (row < R) {
    float4* y = reinterpret_cast<float4*>(pb.Y + int64_t(row) * RB);
#pragma unroll
    for (int p = 0; p < RB; p += 4) y[p / 4] = make_float4(acc[p], acc[p + 1], acc[p + 2], acc[p + 3]);
  }
}

__global__ __launch_bounds__(kGT) void by_kernel(BArgs a) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  int b, t;
  item_of(a, b, t);
  const BProb& pb = a.probs[b];
  switch (pb.rb) {
    case 4: y_tile<4>(pb, t, lds); break;
    case 8: y_tile<8>(pb, t, lds); break;
    case 12: y_tile<12>(pb, t, lds); break;
    case 16: y_tile<16>(pb, t, lds); break;
    case 20: y_tile<20>(pb, t, lds); break;
    case 24: y_tile<24>(pb, t, lds); break;
    case 28: y_tile<28>(pb, t, lds); break;
    default: y_tile<32>(pb, t, lds); break;
  }
}

// Folds of Y, one output row per wave:
//   mode 0: P[i, p] = sum_j W[j, p] Y[(i, j), p]   (W = Â^(2), the survivor of block 2)
//   mode 1: P[j, p] = sum_i W[i, p] Y[(i, j), p]   (W = Â^(1) of this iteration)
// Lane (p, g), p < 32, g < 2, sums the terms with index = g mod 2 in order; the two sums
// are added in a fixed order.
__global__ __launch_bounds__(kGT) void bfold_kernel(BArgs a, int mode) {
  int b, t;
  item_of(a, b, t);
  const BProb& pb = a.probs[b];
  const int RB = pb.rb;
  const int I0 = pb.I[0], I1 = pb.I[1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int o = t * kFoldRows + wave;  // output row
  const int Iout = mode == 0 ? I0 : I1;
  const int Isum = mode == 0 ? I1 : I0;
  if (o >= Iout) return;
  const int p = lane & 31, g = lane >> 5;
  const bool act = p < RB;
  const int pp = act ? p : 0;
  const int32_t* sid = pb.sc->s_id;
  const float* __restrict__ W = mode == 0 ? pb.buf[1][sid[1]] : pb.buf[0][(sid[0] + 2) % 3];
  const float* __restrict__ Y = pb.Y;
  const int64_t ystep = mode == 0 ? int64_t(RB) : int64_t(I1) * RB;
  const float* y = Y + (mode == 0 ? int64_t(o) * I1 * RB : int64_t(o) * RB) + pp;
  // a step adds k into acc0 and k + 2 into acc1 while k + 2 < Isum (k += 4), then the
  // last k (if any) into acc0; eight steps' loads are issued together at clamped in-range
  // k, and steps past the bound add nothing
  float acc0 = 0.f, acc1 = 0.f;
  int k = g;
  while (k + 2 < Isum) {
    float wv[16], yv[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int kk = min(k + 2 * m, Isum - 1);
      wv[m] = W[kk * RB + pp];
      yv[m] = y[kk * ystep];
    }
    int nv = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const bool ok = k + 4 * t + 2 < Isum;
      nv += ok ? 1 : 0;
      acc0 = ok ? fmaf(wv[2 * t], yv[2 * t], acc0) : acc0;
      acc1 = ok ? fmaf(wv[2 * t + 1], yv[2 * t + 1], acc1) : acc1;
    }
    k += 4 * nv;
  }
  if (k < Isum) acc0 = fmaf(W[k * RB + pp], y[k * ystep], acc0);
  float s = acc0 + acc1;
  const float other = __shfl_xor(s, 32);
  s = g == 0 ? s + other : other + s;  // (group 0) + (group 1)
  if (g == 0 && act) pb.P[o * RB + p] = s;
}

// Last-mode partial sums for chunk t (i = 4t .. 4t+3) of problem b:
//   part[t][k, p] = sum_{i in chunk} A1[i, p] sum_j A2[j, p] T[i, j, k].
// Lanes own k (64-wide chunks of the contiguous mode); with fewer than four k chunks the
// waves also split the chunk's i values, and their sums are added in wave order.
template <int RB>
__device__ void last_tile(const BArgs& a, const BProb& pb, int t, int init, float* lds) {
  const int I0 = pb.I[0], I1 = pb.I[1], I2 = pb.I[2];
  const int32_t* sid = pb.sc->s_id;
  const float* __restrict__ A1 = init ? pb.buf[0][0] : pb.buf[0][(sid[0] + 2) % 3];
  const float* __restrict__ A2 = init ? pb.buf[1][0] : pb.buf[1][(sid[1] + 2) % 3];
  float* A2s = lds;                                      // I1 x RB
  float* comb = lds + align_up(size_t(I1) * RB, 4);      // [4 waves][64][RB]
  for (int e = threadIdx.x; e < I1 * RB; e += kGT) A2s[e] = A2[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nkc = (I2 + 63) / 64;
  const int nig = max(1, 4 / nkc);
  const int i_lo = t * kLastChunk, i_hi = min(I0, i_lo + kLastChunk);
  float acc[RB];
#pragma unroll
  for (int p = 0; p < RB; ++p) acc[p] = 0.f;
  const bool wact = wave < nkc * nig;
  const int kc = wave % nkc, ig = wave / nkc;
  const int k = kc * 64 + lane;
  if (wact) {
    for (int i = i_lo + ig; i < i_hi; i += nig) {
      float z[RB];
#pragma unroll
      for (int p = 0; p < RB; ++p) z[p] = 0.f;
      // lanes past I_3 read column 0 (their sums are never written)
      const float* trow = pb.T + int64_t(i) * I1 * I2 + (k < I2 ? k : 0);
      for (int j0 = 0; j0 < I1; j0 += 16) {
        float tv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) tv[u] = trow[int64_t(min(j0 + u, I1 - 1)) * I2];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          if (j0 + u < I1) {
            const float* av = A2s + (j0 + u) * RB;
#pragma unroll
            for (int p = 0; p < RB; ++p) z[p] = fmaf(tv[u], av[p], z[p]);
          }
        }
      }
      const float* a1 = A1 + i * RB;
#pragma unroll
      for (int p = 0; p < RB; ++p) acc[p] = fmaf(a1[p], z[p], acc[p]);
    }
  }
  if (nig > 1) {
    // waves with ig > 0 hand their sums to the wave with ig = 0 of the same k chunk
    if (wact && ig > 0) {
      float* c = comb + (int64_t(wave) * 64 + lane) * RB;
#pragma unroll
      for (int p = 0; p < RB; ++p) c[p] = acc[p];
    }
    __syncthreads();
    if (wact && ig == 0) {
      for (int g2 = 1; g2 < nig; ++g2) {
        const float* c = comb + (int64_t(g2 * nkc + kc) * 64 + lane) * RB;
#pragma unroll
        for (int p = 0; p < RB; ++p) acc[p] += c[p];
      }
    }
  }
  if (wact && ig == 0 && k < I2) {
    float4* o = reinterpret_cast<float4*>(pb.part + (int64_t(t) * I2 + k) * RB);
#pragma unroll
    for (int p = 0; p < RB; p += 4) o[p / 4] = make_float4(acc[p], acc[p + 1], acc[p + 2], acc[p + 3]);
  }
}

__global__ __launch_bounds__(kGT) void blast_kernel(BArgs a, int init) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  int b, t;
  item_of(a, b, t);
  const BProb& pb = a.probs[b];
  switch (pb.rb) {
    case 4: last_tile<4>(a, pb, t, init, lds); break;
    case 8: last_tile<8>(a, pb, t, init, lds); break;
    case 12: last_tile<12>(a, pb, t, init, lds); break;
    case 16: last_tile<16>(a, pb, t, init, lds); break;
    case 20: last_tile<20>(a, pb, t, init, lds); break;
    case 24: last_tile<24>(a, pb, t, init, lds); break;
    case 28: last_tile<28>(a, pb, t, init, lds); break;
    default: last_tile<32>(a, pb, t, init, lds); break;
  }
}

// P[k, p] = sum over chunks (in order) of part[chunk][k, p], elements t * 256 .. +256 of
// problem b's I_3 x rb output; sixteen partials in flight per thread
__global__ __launch_bounds__(kGT) void bsum_kernel(BArgs a) {
  int b, t;
  item_of(a, b, t);
  const BProb& pb = a.probs[b];
  const int64_t n = int64_t(pb.I[2]) * pb.rb;
  const int64_t e = int64_t(t) * kGT + threadIdx.x;
  if (e >= n) return;
  const int nch = (pb.I[0] + kLastChunk - 1) / kLastChunk;
  const float* __restrict__ part = pb.part + e;
  float s = 0.f;
  for (int c0 = 0; c0 < nch; c0 += 16) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = part[int64_t(min(c0 + u, nch - 1)) * n];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (c0 + u < nch) s += v[u];
  }
  pb.P[e] = s;
}

// ---- per-problem launches (one workgroup of kBT threads per problem) ----


// A-HALS on the rows of one block, one lane per row. Gt: scaled G, transposed and with a
// zero diagonal, RB x RB in LDS, 16-byte aligned: Gt[j][l] = G_lj / G_jj (0 for l = j or a
// dead j), so column j's update is W_j = max(0, P_j / G_jj - sum_l W_l Gt[j][l]).
// ginv: 1 / G_jj or 0. Returns the sweeps done; w holds the lane's new row.
template <int RB>
__device__ int hals_rows(const float* __restrict__ W0, float* __restrict__ Wn,
                         const float* __restrict__ P, const float* Gt, const float* ginv,
                         int rows, int max_inner, double tol, double* s_red, float (&w)[RB]) {
  const int i = threadIdx.x;
  const bool act = i < rows;
  const int ri = act ? i : 0;  // inactive lanes read row 0 and keep zeros (no branches)
  const float4* W04 = reinterpret_cast<const float4*>(W0 + ri * RB);
  const float4* P4 = reinterpret_cast<const float4*>(P + ri * RB);
  const float4* gi4 = reinterpret_cast<const float4*>(ginv);
  float pinv[RB];
#pragma unroll
  for (int k4 = 0; k4 < RB / 4; ++k4) {
    const float4 v = W04[k4];
    const float4 pv = P4[k4];
    const float4 gv = gi4[k4];
    w[4 * k4 + 0] = act ? v.x : 0.f;
    w[4 * k4 + 1] = act ? v.y : 0.f;
    w[4 * k4 + 2] = act ? v.z : 0.f;
    w[4 * k4 + 3] = act ? v.w : 0.f;
    pinv[4 * k4 + 0] = act ? pv.x * gv.x : 0.f;
    pinv[4 * k4 + 1] = act ? pv.y * gv.y : 0.f;
    pinv[4 * k4 + 2] = act ? pv.z * gv.z : 0.f;
    pinv[4 * k4 + 3] = act ? pv.w * gv.w : 0.f;
  }
  const double tol2 = tol * tol;
  double lim = 0.0;
  int done = max_inner;
  for (int s = 1; s <= max_inner; ++s) {
    // an opaque (zero) offset per sweep keeps G in LDS, read where it is used, instead of
    // being hoisted out of the loop into RB * RB registers
    int zero = 0;
    asm volatile("" : "+v"(zero));
    const float4* G4 = reinterpret_cast<const float4*>(Gt) + zero;
    double d2 = 0.0;
    // row j of Gt is read (RB / 4 broadcast loads) while column j - 1 is updated
    float4 gb[2][RB / 4];
#pragma unroll
    for (int l4 = 0; l4 < RB / 4; ++l4) gb[0][l4] = G4[l4];
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      if (j + 1 < RB) {
#pragma unroll
        for (int l4 = 0; l4 < RB / 4; ++l4) gb[(j + 1) & 1][l4] = G4[(j + 1) * (RB / 4) + l4];
      }
      // four partial sums; the terms are taken in the order l = j + 1, ..., j - 1
      // (cyclically; the l = j term of Gt is zero and adds nothing), so the column updated
      // last enters last and the chain from it to W_j is one multiply-add, the two adds and
      // the max
      float acc[4] = {pinv[j], 0.f, 0.f, 0.f};
#pragma unroll
      for (int m = 1; m < RB; ++m) {
        const int l = (j + m) % RB;
        const float4 g4 = gb[j & 1][l / 4];
        const float g = (l & 3) == 0 ? g4.x : (l & 3) == 1 ? g4.y : (l & 3) == 2 ? g4.z : g4.w;
        acc[m & 3] = fmaf(-w[l], g, acc[m & 3]);
      }
      const float wn = fmaxf((acc[0] + acc[1]) + (acc[2] + acc[3]), 0.f);
      const double dd = double(wn) - double(w[j]);
      d2 = fma(dd, dd, d2);
      w[j] = wn;
    }
    const double D = sweep_sum(d2, s_red + kBW + 1, s & 1);
    if (s == 1) lim = tol2 * D;
    if (D <= lim) {
      done = s;
      break;
    }
  }
  if (act) {
    float4* Wn4 = reinterpret_cast<float4*>(Wn + i * RB);
#pragma unroll
    for (int k4 = 0; k4 < RB / 4; ++k4)
      Wn4[k4] = make_float4(w[4 * k4], w[4 * k4 + 1], w[4 * k4 + 2], w[4 * k4 + 3]);
  }
  return done;
}

// Block n of this iteration for one problem: G^(n) from the cached Grams (Â of this
// iteration for l < n, the survivors for l > n), A-HALS from the survivor, extrapolation,
// Grams of the new and extrapolated rows; after block 3, F-hat and the restart decision.
// G32s, ginv: LDS, 16-byte aligned, RB x RB and RB floats; G64s: LDS, RB x RB doubles;
// s_rows: LDS, 2 I_n x RB floats (the new and the extrapolated rows, for their Grams).
template <int RB>
__device__ void block_update(const BArgs& a, const BProb& pb, int n, double* s_red,
                             float* G32s, float* ginv, double* G64s, float* s_rows) {
  const int tid = threadIdx.x;
  BScal* sc = pb.sc;
  int sid[3], nw[3], ht[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    sid[l] = sc->s_id[l];
    nw[l] = (sid[l] + 1) % 3;
    ht[l] = (sid[l] + 2) % 3;
  }
  const double beta = sc->beta;
  const int In = pb.I[n];
  const int la = n == 0 ? 1 : 0, lb = n == 2 ? 1 : 2;
  const double* g1 = pb.gram[la][la < n ? ht[la] : sid[la]];
  const double* g2 = pb.gram[lb][lb < n ? ht[lb] : sid[lb]];
  for (int e = tid; e < RB * RB; e += kBT) G64s[e] = g1[e] * g2[e];
  __syncthreads();
  for (int e = tid; e < RB * RB; e += kBT) {
    const int j = e / RB, l = e - (e / RB) * RB;
    const float gjj = float(G64s[j * RB + j]);
    G32s[e] = (j != l && gjj != 0.f) ? float(G64s[l * RB + j]) * (1.f / gjj) : 0.f;
  }
  if (tid < RB) {
    const float gjj = float(G64s[tid * RB + tid]);
    ginv[tid] = gjj != 0.f ? 1.f / gjj : 0.f;
  }
  __syncthreads();
  float w[RB];
  const int sweeps = hals_rows<RB>(pb.buf[n][sid[n]], pb.buf[n][nw[n]], pb.P, G32s, ginv, In,
                                   a.max_inner, a.tol, s_red, w);
  // extrapolation A_hat = max(0, A_new + beta (A_new - A_old)), float64; the new and
  // extrapolated rows are also staged in LDS for their Grams
  double ip = 0.0;
  float* s_new = s_rows;
  float* s_hat = s_rows + In * RB;
  if (tid < In) {
    const float* w0 = pb.buf[n][sid[n]] + tid * RB;
    float* hh = pb.buf[n][ht[n]] + tid * RB;
#pragma unroll
    for (int p = 0; p < RB; ++p) {
      const double x = w[p];
      const double y = x + beta * (x - double(w0[p]));
      const float yh = float(y > 0.0 ? y : 0.0);
      hh[p] = yh;
      s_new[tid * RB + p] = w[p];
      s_hat[tid * RB + p] = yh;
    }
    if (n == 2) {
#pragma unroll
      for (int p = 0; p < RB; ++p) ip = fma(double(pb.P[tid * RB + p]), double(w[p]), ip);
    }
  }
  __syncthreads();
  // Grams of the new and extrapolated rows (float64, rows in order)
  {
    double* gn = pb.gram[n][nw[n]];
    double* gh = pb.gram[n][ht[n]];
    for (int e = tid; e < RB * RB; e += kBT) {
      const int p = e / RB, q = e - (e / RB) * RB;
      double an = 0.0, ah = 0.0;
      for (int i = 0; i < In; ++i) {
        an = fma(double(s_new[i * RB + p]), double(s_new[i * RB + q]), an);
        ah = fma(double(s_hat[i * RB + p]), double(s_hat[i * RB + q]), ah);
      }
      gn[e] = an;
      gh[e] = ah;
    }
  }
  const int it = sc->it;
  if (tid == 0 && pb.tr_sweeps) pb.tr_sweeps[int64_t(it) * 3 + n] = sweeps;
  if (n != 2) return;
  __syncthreads();
  // ---- F-hat_k (Gram trick with G^(3) and A_new^(3)) and the restart decision ----
  double gg = 0.0;
  for (int e = tid; e < RB * RB; e += kBT) gg = fma(G64s[e], pb.gram[2][nw[2]][e], gg);
  const double IP = block_sum(ip, s_red);
  const double GG = block_sum(gg, s_red);
  if (tid == 0) {
    const double fh = 0.5 * (sc->normT2 - 2.0 * IP + GG);
    const bool finite = isfinite(fh);
    const bool restart = !finite || fh > sc->fhat_prev;
    if (!finite && a.flags)
      __hip_atomic_fetch_or(a.flags, NTF_FLAG_NONFINITE, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
    double bt = sc->beta, bb = sc->beta_bar;
    if (restart) {
      bb = bt;
      bt = bt / a.eta;
    } else {
      const double bn = fmin(bb, a.gamma * bt);
      bb = fmin(1.0, a.gamma_bar * bb);
      bt = bn;
    }
    sc->beta = bt;
    sc->beta_bar = bb;
    if (finite) sc->fhat_prev = fh;  // a non-finite F-hat is no reference for the next test
    sc->k += 1.0;
    if (restart) sc->nrestarts += 1.0;
    for (int l = 0; l < 3; ++l) sc->s_id[l] = restart ? nw[l] : ht[l];
    sc->it = it + 1;
    if (pb.tr_fhat) pb.tr_fhat[it] = fh;
    if (pb.tr_restart) pb.tr_restart[it] = restart ? 1 : 0;
  }
}

__global__ __launch_bounds__(kBT) void bhals_kernel(BArgs a, int n) {
  extern __shared__ __attribute__((aligned(16))) float s_rows[];  // 2 I_n x RB
  __shared__ double s_red[3 * kBW + 1];  // block_sum's, then the sweep sums' two buffers
  __shared__ __attribute__((aligned(16))) float G32s[kBatchedMaxRank * kBatchedMaxRank];
  __shared__ __attribute__((aligned(16))) float ginv[kBatchedMaxRank];
  __shared__ double G64s[kBatchedMaxRank * kBatchedMaxRank];
  const BProb& pb = a.probs[a.order[blockIdx.x]];
  switch (pb.rb) {
    case 4: block_update<4>(a, pb, n, s_red, G32s, ginv, G64s, s_rows); break;
    case 8: block_update<8>(a, pb, n, s_red, G32s, ginv, G64s, s_rows); break;
    case 12: block_update<12>(a, pb, n, s_red, G32s, ginv, G64s, s_rows); break;
    case 16: block_update<16>(a, pb, n, s_red, G32s, ginv, G64s, s_rows); break;
    case 20: block_update<20>(a, pb, n, s_red, G32s, ginv, G64s, s_rows); break;
    case 24: block_update<24>(a, pb, n, s_red, G32s, ginv, G64s, s_rows); break;
    case 28: block_update<28>(a, pb, n, s_red, G32s, ginv, G64s, s_rows); break;
    default: block_update<32>(a, pb, n, s_red, G32s, ginv, G64s, s_rows); break;
  }
}

// Set-up of one problem: A_0 into buffer 0 of each block (zero padded), their Grams,
// ||T||^2, and the HER scalars (from the caller's state when resuming).
template <int RB>
__device__ void setup_problem(const BArgs& a, const BProb& pb, double* s_red) {
  const int tid = threadIdx.x;
  const int r = pb.r;
  for (int n = 0; n < 3; ++n) {
    const int In = pb.I[n];
    for (int e = tid; e < In * RB; e += kBT) {
      const int i = e / RB, p = e - (e / RB) * RB;
      pb.buf[n][0][e] = p < r ? pb.A_user[n][i * r + p] : 0.f;
    }
  }
  __syncthreads();
  for (int n = 0; n < 3; ++n) gram_of<RB>(pb.buf[n][0], pb.I[n], pb.gram[n][0]);
  // ||T||^2: the Y tiles' sums (bnorm_kernel), thread k adding tiles k, k + kBT, ... in order
  const int ntiles = int((int64_t(pb.I[0]) * pb.I[1] + kYRows - 1) / kYRows);
  double acc = 0.0;
  for (int t = tid; t < ntiles; t += kBT) acc += pb.normp[t];
  const double nt2 = block_sum(acc, s_red);
  if (tid == 0) {
    BScal* sc = pb.sc;
    sc->normT2 = nt2;
    for (int l = 0; l < 3; ++l) sc->s_id[l] = 0;
    sc->it = 0;
    if (a.resume) {
      sc->beta = pb.st->beta;
      sc->beta_bar = pb.st->beta_bar;
      sc->fhat_prev = pb.st->fhat_prev;
      sc->k = double(pb.st->k);
      sc->nrestarts = double(pb.st->nrestarts);
    } else {
      sc->beta = a.beta0;
      sc->beta_bar = 1.0;
      sc->fhat_prev = 0.0;  // F-hat_0, set by bfhat0_kernel
      sc->k = 0.0;
      sc->nrestarts = 0.0;
    }
  }
}

// Sum of T^2 over the rows of one Y tile (rows t * kYRows .. +kYRows of I_1 I_2, each I_3
// contiguous elements): eight loads in flight per thread at clamped in-range offsets, four
// float64 chains, then the fixed-order block sum. Many workgroups per problem, so the
// set-up reads the tensors at streaming rate.
__global__ __launch_bounds__(kGT) void bnorm_kernel(BArgs a) {
  __shared__ double s_red[kBW + 1];
  int b, t;
  item_of(a, b, t);
  const BProb& pb = a.probs[b];
  const int64_t I2 = pb.I[2];
  const int64_t R = int64_t(pb.I[0]) * pb.I[1];
  const int64_t lo = int64_t(t) * kYRows * I2;
  const int64_t hi = std::min<int64_t>(R, int64_t(t + 1) * kYRows) * I2;
  const float* __restrict__ T = pb.T;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t e0 = lo + threadIdx.x; e0 < hi; e0 += 8 * kGT) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t e = e0 + int64_t(u) * kGT;
      v[u] = T[e < hi ? e : lo];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double x = fma(double(v[u]), double(v[u]), acc[u & 3]);
      acc[u & 3] = e0 + int64_t(u) * kGT < hi ? x : acc[u & 3];
    }
  }
  const double sum = block_sum((acc[0] + acc[1]) + (acc[2] + acc[3]), s_red);
  if (threadIdx.x == 0) pb.normp[t] = sum;
}

__global__ __launch_bounds__(kBT) void bsetup_kernel(BArgs a) {
  __shared__ double s_red[kBW + 1];
  const BProb& pb = a.probs[a.order[blockIdx.x]];
  switch (pb.rb) {
    case 4: setup_problem<4>(a, pb, s_red); break;
    case 8: setup_problem<8>(a, pb, s_red); break;
    case 12: setup_problem<12>(a, pb, s_red); break;
    case 16: setup_problem<16>(a, pb, s_red); break;
    case 20: setup_problem<20>(a, pb, s_red); break;
    case 24: setup_problem<24>(a, pb, s_red); break;
    case 28: setup_problem<28>(a, pb, s_red); break;
    default: setup_problem<32>(a, pb, s_red); break;
  }
}

// F-hat_0 = F(A_0) by the Gram trick from the last mode's MTTKRP (blast_kernel with
// init = 1, then bsum_kernel).
template <int RB>
__device__ void fhat0_problem(const BProb& pb, double* s_red) {
  const int tid = threadIdx.x;
  double ip = 0.0, gg = 0.0;
  const int I2 = pb.I[2];
  for (int e = tid; e < I2 * RB; e += kBT) ip = fma(double(pb.P[e]), double(pb.buf[2][0][e]), ip);
  for (int e = tid; e < RB * RB; e += kBT)
    gg = fma(pb.gram[0][0][e] * pb.gram[1][0][e], pb.gram[2][0][e], gg);
  const double IP = block_sum(ip, s_red);
  const double GG = block_sum(gg, s_red);
  if (tid == 0) pb.sc->fhat_prev = 0.5 * (pb.sc->normT2 - 2.0 * IP + GG);
}

__global__ __launch_bounds__(kBT) void bfhat0_kernel(BArgs a) {
  __shared__ double s_red[kBW + 1];
  const BProb& pb = a.probs[a.order[blockIdx.x]];
  switch (pb.rb) {
    case 4: fhat0_problem<4>(pb, s_red); break;
    case 8: fhat0_problem<8>(pb, s_red); break;
    case 12: fhat0_problem<12>(pb, s_red); break;
    case 16: fhat0_problem<16>(pb, s_red); break;
    case 20: fhat0_problem<20>(pb, s_red); break;
    case 24: fhat0_problem<24>(pb, s_red); break;
    case 28: fhat0_problem<28>(pb, s_red); break;
    default: fhat0_problem<32>(pb, s_red); break;
  }
}

// Results: the survivors to the caller's factors, and the state.
__global__ __launch_bounds__(kBT) void bfinal_kernel(BArgs a) {
  const BProb& pb = a.probs[a.order[blockIdx.x]];
  const BScal* sc = pb.sc;
  const int r = pb.r, RB = pb.rb;
  for (int n = 0; n < 3; ++n) {
    const float* src = pb.buf[n][sc->s_id[n]];
    for (int e = threadIdx.x; e < pb.I[n] * r; e += kBT) {
      const int i = e / r, p = e - (e / r) * r;
      pb.A_user[n][e] = src[i * RB + p];
    }
  }
  if (threadIdx.x == 0 && pb.st) {
    pb.st->beta = sc->beta;
    pb.st->beta_bar = sc->beta_bar;
    pb.st->fhat_prev = sc->fhat_prev;
    pb.st->fhat = sc->fhat_prev;
    pb.st->k = int64_t(sc->k);
    pb.st->restart = 0;
    pb.st->nrestarts = int32_t(sc->nrestarts);
    pb.st->it = sc->it;
  }
}

// ---- host side ----

int y_tiles(const int I[3]) { return int(ceil_div(int64_t(I[0]) * I[1], kYRows)); }
int last_chunks(const int I[3]) { return int(ceil_div(I[0], kLastChunk)); }

// Per-problem device workspace layout (bytes), shared by sizing and carving.
struct BatchedLayout {
  size_t buf[3], gram, Y, P, part, normp, sc, st, total;
};

BatchedLayout batched_layout(const int I[3], int rb) {
  BatchedLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, 256);
    const size_t o = off;
    off += bytes;
    return o;
  };
  for (int n = 0; n < 3; ++n) L.buf[n] = take(3 * size_t(I[n]) * rb * sizeof(float));
  L.gram = take(9 * size_t(rb) * rb * sizeof(double));
  L.Y = take(size_t(I[0]) * I[1] * rb * sizeof(float));
  L.P = take(size_t(std::max({I[0], I[1], I[2]})) * rb * sizeof(float));
  L.part = take(size_t(last_chunks(I)) * I[2] * rb * sizeof(float));
  L.normp = take(size_t(y_tiles(I)) * sizeof(double));
  L.sc = take(sizeof(BScal));
  L.st = take(sizeof(ntf_her_state));
  L.total = align_up(off, 256);
  return L;
}

// dynamic LDS limits of the launches that stage tiles or rows (bhals_kernel also has
// about 13 KB of static LDS)
hipError_t launch_attrs() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(by_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024)) !=
      hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(blast_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024)) !=
      hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(bhals_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024)) !=
      hipSuccess)
    return e;
  done = true;
  return hipSuccess;
}

BArgs make_args(const BatchedJob& job, const BatchedPlan& pl, const uint32_t* items) {
  BArgs a{};
  a.probs = reinterpret_cast<const BProb*>(job.dev_desc);
  a.order = reinterpret_cast<const int32_t*>(static_cast<char*>(job.dev_desc) + pl.off_order);
  a.items = items;
  a.nprob = job.nprob;
  a.resume = job.resume;
  a.max_inner = job.params.max_inner;
  a.beta0 = job.params.beta0;
  a.gamma = job.params.gamma;
  a.gamma_bar = job.params.gamma_bar;
  a.eta = job.params.eta;
  a.tol = job.params.inner_tol;
  a.flags = job.flags;
  return a;
}

const uint32_t* list_ptr(const BatchedJob& job, size_t off) {
  return reinterpret_cast<const uint32_t*>(static_cast<char*>(job.dev_desc) + off);
}

}  // namespace

size_t batched_problem_bytes(const int I[3], int rb) { return batched_layout(I, rb).total; }

// Descriptor area: descriptors, the per-problem order, and the five item lists.
BatchedPlan batched_plan(const BatchedJob& job) {
  static_assert(sizeof(BProb) <= kBatchedDescBytes, "descriptor slot too small");
  BatchedPlan pl{};
  size_t off = size_t(job.nprob) * sizeof(BProb);
  pl.off_order = off;
  off += size_t(job.nprob) * sizeof(int32_t);
  int64_t ny = 0, nfu = 0, nfi = 0, nl = 0, ns = 0;
  size_t lds_y = 0, lds_l = 0, lds_h = 0;
  for (int b = 0; b < job.nprob; ++b) {
    const BatchedProblem& q = job.probs[b];
    ny += y_tiles(q.I);
    nfu += ceil_div(q.I[0], kFoldRows);
    nfi += ceil_div(q.I[1], kFoldRows);
    nl += last_chunks(q.I);
    ns += ceil_div(int64_t(q.I[2]) * q.rb, kGT);
    lds_y = std::max(lds_y, (align_up(size_t(q.I[2]) * q.rb, 4) + size_t(4) * 64 * kTileLd) * 4);
    lds_l = std::max(lds_l, (align_up(size_t(q.I[1]) * q.rb, 4) + size_t(4) * 64 * q.rb) * 4);
    lds_h = std::max(lds_h, size_t(2) * std::max({q.I[0], q.I[1], q.I[2]}) * q.rb * 4);
  }
  pl.n_y = ny;
  pl.n_fu = nfu;
  pl.n_fi = nfi;
  pl.n_last = nl;
  pl.n_sum = ns;
  off = align_up(off, 16);
  pl.off_y = off;
  off += size_t(ny) * 4;
  pl.off_fu = off;
  off += size_t(nfu) * 4;
  pl.off_fi = off;
  off += size_t(nfi) * 4;
  pl.off_last = off;
  off += size_t(nl) * 4;
  pl.off_sum = off;
  off += size_t(ns) * 4;
  pl.bytes = align_up(off, 256);
  pl.lds_y = lds_y;
  pl.lds_last = lds_l;
  pl.lds_hals = lds_h;
  return pl;
}

// Build the device descriptors and item lists in the pinned staging area and enqueue their
// upload.
hipError_t batched_upload(const BatchedJob& job, const BatchedPlan& pl, hipStream_t s) {
  char* host = static_cast<char*>(job.host_desc);
  BProb* hd = reinterpret_cast<BProb*>(host);
  for (int b = 0; b < job.nprob; ++b) {
    const BatchedProblem& q = job.probs[b];
    BProb& d = hd[b];
    d = BProb{};
    d.T = q.T;
    d.r = q.r;
    d.rb = q.rb;
    for (int n = 0; n < 3; ++n) {
      d.I[n] = q.I[n];
      d.A_user[n] = q.A[n];
    }
    const BatchedLayout L = batched_layout(q.I, q.rb);
    char* base = q.ws;
    for (int n = 0; n < 3; ++n)
      for (int k = 0; k < 3; ++k)
        d.buf[n][k] = reinterpret_cast<float*>(base + L.buf[n]) + size_t(k) * q.I[n] * q.rb;
    for (int n = 0; n < 3; ++n)
      for (int k = 0; k < 3; ++k)
        d.gram[n][k] = reinterpret_cast<double*>(base + L.gram) + size_t(n * 3 + k) * q.rb * q.rb;
    d.Y = reinterpret_cast<float*>(base + L.Y);
    d.P = reinterpret_cast<float*>(base + L.P);
    d.part = reinterpret_cast<float*>(base + L.part);
    d.normp = reinterpret_cast<double*>(base + L.normp);
    d.sc = reinterpret_cast<BScal*>(base + L.sc);
    d.st = q.state ? q.state : reinterpret_cast<ntf_her_state*>(base + L.st);
    d.tr_fhat = q.tr_fhat;
    d.tr_restart = q.tr_restart;
    d.tr_sweeps = q.tr_sweeps;
  }
  int32_t* ho = reinterpret_cast<int32_t*>(host + pl.off_order);
  for (int b = 0; b < job.nprob; ++b) ho[b] = job.order[b];
  // item lists in the processing order (largest problems first)
  uint32_t* ly = reinterpret_cast<uint32_t*>(host + pl.off_y);
  uint32_t* lfu = reinterpret_cast<uint32_t*>(host + pl.off_fu);
  uint32_t* lfi = reinterpret_cast<uint32_t*>(host + pl.off_fi);
  uint32_t* ll = reinterpret_cast<uint32_t*>(host + pl.off_last);
  uint32_t* lsu = reinterpret_cast<uint32_t*>(host + pl.off_sum);
  for (int x = 0; x < job.nprob; ++x) {
    const int b = job.order[x];
    const BatchedProblem& q = job.probs[b];
    const uint32_t hb = uint32_t(b) << 16;
    for (int t = 0; t < y_tiles(q.I); ++t) *ly++ = hb | uint32_t(t);
    for (int t = 0; t < int(ceil_div(q.I[0], kFoldRows)); ++t) *lfu++ = hb | uint32_t(t);
    for (int t = 0; t < int(ceil_div(q.I[1], kFoldRows)); ++t) *lfi++ = hb | uint32_t(t);
    for (int t = 0; t < last_chunks(q.I); ++t) *ll++ = hb | uint32_t(t);
    for (int t = 0; t < int(ceil_div(int64_t(q.I[2]) * q.rb, kGT)); ++t) *lsu++ = hb | uint32_t(t);
  }
  return hipMemcpyAsync(job.dev_desc, job.host_desc, pl.bytes, hipMemcpyHostToDevice, s);
}

// Set-up of every problem (and F-hat_0 unless resuming).
hipError_t batched_setup(const BatchedJob& job, const BatchedPlan& pl, hipStream_t s) {
  hipError_t e = launch_attrs();
  if (e != hipSuccess) return e;
  const BArgs a = make_args(job, pl, nullptr);
  hipLaunchKernelGGL(bnorm_kernel, dim3(unsigned(pl.n_y)), dim3(kGT), 0, s,
                     make_args(job, pl, list_ptr(job, pl.off_y)));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bsetup_kernel, dim3(job.nprob), dim3(kBT), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess || job.resume) return e;
  hipLaunchKernelGGL(blast_kernel, dim3(unsigned(pl.n_last)), dim3(kGT), pl.lds_last, s,
                     make_args(job, pl, list_ptr(job, pl.off_last)), 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bsum_kernel, dim3(unsigned(pl.n_sum)), dim3(kGT), 0, s,
                     make_args(job, pl, list_ptr(job, pl.off_sum)));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bfhat0_kernel, dim3(job.nprob), dim3(kBT), 0, s, a);
  return hipGetLastError();
}

// One outer iteration of every problem (eight grouped or per-problem launches).
hipError_t batched_iteration(const BatchedJob& job, const BatchedPlan& pl, hipStream_t s) {
  hipError_t e = launch_attrs();
  if (e != hipSuccess) return e;
  const BArgs per = make_args(job, pl, nullptr);
  hipLaunchKernelGGL(by_kernel, dim3(unsigned(pl.n_y)), dim3(kGT), pl.lds_y, s,
                     make_args(job, pl, list_ptr(job, pl.off_y)));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bfold_kernel, dim3(unsigned(pl.n_fu)), dim3(kGT), 0, s,
                     make_args(job, pl, list_ptr(job, pl.off_fu)), 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bhals_kernel, dim3(job.nprob), dim3(kBT), pl.lds_hals, s, per, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bfold_kernel, dim3(unsigned(pl.n_fi)), dim3(kGT), 0, s,
                     make_args(job, pl, list_ptr(job, pl.off_fi)), 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bhals_kernel, dim3(job.nprob), dim3(kBT), pl.lds_hals, s, per, 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(blast_kernel, dim3(unsigned(pl.n_last)), dim3(kGT), pl.lds_last, s,
                     make_args(job, pl, list_ptr(job, pl.off_last)), 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bsum_kernel, dim3(unsigned(pl.n_sum)), dim3(kGT), 0, s,
                     make_args(job, pl, list_ptr(job, pl.off_sum)));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bhals_kernel, dim3(job.nprob), dim3(kBT), pl.lds_hals, s, per, 2);
  return hipGetLastError();
}

hipError_t batched_final(const BatchedJob& job, const BatchedPlan& pl, hipStream_t s) {
  hipLaunchKernelGGL(bfinal_kernel, dim3(job.nprob), dim3(kBT), 0, s, make_args(job, pl, nullptr));
  return hipGetLastError();
}

}  // namespace ntf
