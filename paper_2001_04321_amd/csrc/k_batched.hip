// Batched HER-A-HALS (Algorithm 2 with A-HALS blocks, Sec. 2.1.4 and 3.1) for many
// independent small 3-way problems in one persistent launch: one workgroup owns one
// problem for all outer iterations, so no synchronization beyond workgroup barriers is
// needed and problems of any shape mix run side by side.
//
// Per outer iteration and problem the tensor is read twice:
//  - Y = T x_3 Â^(3) (I_1 I_2 x r) from the previous iteration's Â^(3). Both mode-1 and
//    mode-2 MTTKRPs are contractions of Y (Â^(3) does not change before the mode-3 update):
//      P^(1)[i, p] = sum_j Â^(2)[j, p] Y[(i, j), p],  P^(2)[j, p] = sum_i Â^(1)[i, p] Y[(i, j), p]
//  - P^(3)[k, p] = sum_i Â^(1)[i, p] sum_j Â^(2)[j, p] T[i, j, k].
// A-HALS: one lane per row, W_j = max(0, P_j / G_jj - sum_{l != j} W_l G_lj / G_jj) column
// by column, stopping rule of Sec. 4.1 on the workgroup-wide ||W_s - W_{s-1}||. Extrapolation (eq. extproj_her), Grams, F-hat (Gram
// trick, Sec. 3.1.3) and the restart decision are float64; every reduction has a fixed order.
// Ranks are padded to a multiple of 8 (RB) with zero columns.
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kBT = 512;       // threads per workgroup
constexpr int kBW = kBT / 64;  // waves per workgroup
constexpr int kTileLd = 33;    // row stride of a wave's 64 x 32 tensor tile in LDS

struct BProb {
  const float* T;
  int I[3];
  int r, rb;
  float* A_user[3];
  float* buf[3][3];    // per mode, three I_n x rb buffers
  double* gram[3][3];  // their Grams, rb x rb
  float* Y;            // I_1 I_2 x rb
  float* P;            // I_max x rb
  double* normT2;
  ntf_her_state* st;
  double* tr_fhat;
  int32_t* tr_restart;
  int32_t* tr_sweeps;
};

struct BArgs {
  const BProb* probs;
  const int32_t* order;
  int nprob;
  int iters;
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

// fixed-order workgroup sum; every thread gets the result. s_red: kBW + 1 doubles.
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

// Y[(i, j), :] = sum_k T[i, j, k] A3[k, :]. Lanes own rows (i, j); the wave stages 64 rows
// x 32 k of T in LDS with row-contiguous loads and reads them back per lane.
template <int RB>
__device__ void y_pass(const float* __restrict__ T, int I0, int I1, int I2,
                       const float* __restrict__ A3, float* __restrict__ Y, float* lds) {
  float* A3s = lds;                          // I2 x RB
  float* tiles = lds + align_up(size_t(I2) * RB, 4);
  for (int e = threadIdx.x; e < I2 * RB; e += kBT) A3s[e] = A3[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* tile = tiles + wave * 64 * kTileLd;
  const int R = I0 * I1;
  const int ntile = int(ceil_div(R, 64));
  for (int tt = wave; tt < ntile; tt += kBW) {
    const int row0 = tt * 64;
    float acc[RB];
#pragma unroll
    for (int p = 0; p < RB; ++p) acc[p] = 0.f;
    for (int c0 = 0; c0 < I2; c0 += 32) {
      const int nc = min(32, I2 - c0);
      const int cc = lane & 31;
#pragma unroll 8
      for (int k = 0; k < 32; ++k) {
        const int rr = 2 * k + (lane >> 5);
        const int row = row0 + rr;
        float v = 0.f;
        if (row < R && cc < nc) v = T[int64_t(row) * I2 + c0 + cc];
        tile[rr * kTileLd + cc] = v;
      }
      // the tile is written and read by this wave only; LDS operations of a wave complete
      // in order
      for (int c = 0; c < nc; ++c) {
        const float t = tile[lane * kTileLd + c];
        const float* a = A3s + (c0 + c) * RB;
#pragma unroll
        for (int p = 0; p < RB; ++p) acc[p] = fmaf(t, a[p], acc[p]);
      }
    }
    const int row = row0 + lane;
    if (row < R) {
      float4* y = reinterpret_cast<float4*>(Y + int64_t(row) * RB);
#pragma unroll
      for (int p = 0; p < RB; p += 4) y[p / 4] = make_float4(acc[p], acc[p + 1], acc[p + 2], acc[p + 3]);
    }
  }
  __syncthreads();
}

// mode 0: P[i, p] = sum_j W[j, p] Y[(i, j), p];  mode 1: P[j, p] = sum_i W[i, p] Y[(i, j), p]
template <int RB>
__device__ void fold(const float* __restrict__ Y, const float* __restrict__ W, int I0, int I1,
                     int mode, float* __restrict__ P) {
  const int Iout = mode == 0 ? I0 : I1;
  const int Isum = mode == 0 ? I1 : I0;
  for (int e = threadIdx.x; e < Iout * RB; e += kBT) {
    const int i = e / RB, p = e - (e / RB) * RB;
    float acc = 0.f;
    if (mode == 0) {
      const float* y = Y + int64_t(i) * I1 * RB + p;
      for (int k = 0; k < Isum; ++k) acc = fmaf(W[k * RB + p], y[int64_t(k) * RB], acc);
    } else {
      const float* y = Y + int64_t(i) * RB + p;
      for (int k = 0; k < Isum; ++k) acc = fmaf(W[k * RB + p], y[int64_t(k) * I1 * RB], acc);
    }
    P[e] = acc;
  }
  __syncthreads();
}

// P[k, p] = sum_i A1[i, p] sum_j A2[j, p] T[i, j, k]: lanes own k (64-wide chunks of the
// contiguous mode), waves split the i range; partial sums are combined in split order.
template <int RB>
__device__ void last_pass(const float* __restrict__ T, int I0, int I1, int I2,
                          const float* __restrict__ A1, const float* __restrict__ A2,
                          float* __restrict__ P, float* lds) {
  float* A1s = lds;                               // I0 x RB
  float* A2s = A1s + I0 * RB;                     // I1 x RB
  float* part = A2s + I1 * RB;                    // [nsplit][nchunk * 64][RB]
  for (int e = threadIdx.x; e < I0 * RB; e += kBT) A1s[e] = A1[e];
  for (int e = threadIdx.x; e < I1 * RB; e += kBT) A2s[e] = A2[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nchunk = int(ceil_div(I2, 64));
  const int nsplit = max(1, kBW / nchunk);
  if (wave < nchunk * nsplit) {
    const int chunk = wave % nchunk, split = wave / nchunk;
    const int k = chunk * 64 + lane;
    const int i_lo = split * I0 / nsplit, i_hi = (split + 1) * I0 / nsplit;
    float acc[RB];
#pragma unroll
    for (int p = 0; p < RB; ++p) acc[p] = 0.f;
    for (int i = i_lo; i < i_hi; ++i) {
      float z[RB];
#pragma unroll
      for (int p = 0; p < RB; ++p) z[p] = 0.f;
      const float* trow = T + int64_t(i) * I1 * I2 + k;
#pragma unroll 4
      for (int j = 0; j < I1; ++j) {
        const float t = k < I2 ? trow[int64_t(j) * I2] : 0.f;
        const float* a = A2s + j * RB;
#pragma unroll
        for (int p = 0; p < RB; ++p) z[p] = fmaf(t, a[p], z[p]);
      }
      const float* a = A1s + i * RB;
#pragma unroll
      for (int p = 0; p < RB; ++p) acc[p] = fmaf(a[p], z[p], acc[p]);
    }
    float* pt = part + (int64_t(split) * nchunk * 64 + k) * RB;
#pragma unroll
    for (int p = 0; p < RB; ++p) pt[p] = acc[p];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < I2 * RB; e += kBT) {
    const int k = e / RB, p = e - (e / RB) * RB;
    float s = 0.f;
    for (int sp = 0; sp < nsplit; ++sp) s += part[(int64_t(sp) * nchunk * 64 + k) * RB + p];
    P[e] = s;
  }
  __syncthreads();
}

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
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      // four partial sums in a fixed pattern shorten the dependency chain
      float acc[4] = {pinv[j], 0.f, 0.f, 0.f};
#pragma unroll
      for (int l4 = 0; l4 < RB / 4; ++l4) {
        const float4 g = G4[j * (RB / 4) + l4];
        acc[0] = fmaf(-w[4 * l4 + 0], g.x, acc[0]);
        acc[1] = fmaf(-w[4 * l4 + 1], g.y, acc[1]);
        acc[2] = fmaf(-w[4 * l4 + 2], g.z, acc[2]);
        acc[3] = fmaf(-w[4 * l4 + 3], g.w, acc[3]);
      }
      const float wn = fmaxf((acc[0] + acc[1]) + (acc[2] + acc[3]), 0.f);
      const double dd = double(wn) - double(w[j]);
      d2 = fma(dd, dd, d2);
      w[j] = wn;
    }
    const double D = block_sum(d2, s_red);
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

template <int RB>
__device__ void solve_problem(const BArgs& a, const BProb& pb, float* lds, double* s_red,
                              double* s_sc, int* s_id) {
  const int tid = threadIdx.x;
  const int I0 = pb.I[0], I1 = pb.I[1], I2 = pb.I[2];
  const int r = pb.r;
  float* G32s = lds;                           // RB x RB scaled G (HALS)
  float* ginv = G32s + RB * RB;                // RB
  double* G64s = reinterpret_cast<double*>(ginv + RB);  // RB x RB (8-byte aligned: RB % 8 == 0)
  float* work = reinterpret_cast<float*>(G64s + RB * RB);

  // ---- set-up: A_0 into buffer 0 of each mode (zero padded), Grams, ||T||^2 ----
  for (int n = 0; n < 3; ++n) {
    const int In = pb.I[n];
    for (int e = tid; e < In * RB; e += kBT) {
      const int i = e / RB, p = e - (e / RB) * RB;
      pb.buf[n][0][e] = p < r ? pb.A_user[n][i * r + p] : 0.f;
    }
  }
  if (tid < 3) s_id[tid] = 0;  // survivor buffer per mode
  __syncthreads();
  for (int n = 0; n < 3; ++n) gram_of<RB>(pb.buf[n][0], pb.I[n], pb.gram[n][0]);
  {
    const int64_t tot = int64_t(I0) * I1 * I2;
    double acc = 0.0;
    for (int64_t e = tid; e < tot; e += kBT) acc = fma(double(pb.T[e]), double(pb.T[e]), acc);
    const double nt2 = block_sum(acc, s_red);
    if (tid == 0) *pb.normT2 = nt2;
  }
  __syncthreads();
  const double normT2 = *pb.normT2;

  // HER scalars in LDS: [0] beta, [1] beta_bar, [2] fhat_prev, [3] k, [4] nrestarts
  if (a.resume) {
    if (tid == 0) {
      s_sc[0] = pb.st->beta;
      s_sc[1] = pb.st->beta_bar;
      s_sc[2] = pb.st->fhat_prev;
      s_sc[3] = double(pb.st->k);
      s_sc[4] = double(pb.st->nrestarts);
    }
  } else {
    // F-hat_0 = F(A_0) by the Gram trick from the last mode's MTTKRP
    last_pass<RB>(pb.T, I0, I1, I2, pb.buf[0][0], pb.buf[1][0], pb.P, work);
    double ip = 0.0, gg = 0.0;
    for (int e = tid; e < I2 * RB; e += kBT) ip = fma(double(pb.P[e]), double(pb.buf[2][0][e]), ip);
    for (int e = tid; e < RB * RB; e += kBT)
      gg = fma(pb.gram[0][0][e] * pb.gram[1][0][e], pb.gram[2][0][e], gg);
    const double IP = block_sum(ip, s_red);
    const double GG = block_sum(gg, s_red);
    if (tid == 0) {
      s_sc[0] = a.beta0;
      s_sc[1] = 1.0;
      s_sc[2] = 0.5 * (normT2 - 2.0 * IP + GG);
      s_sc[3] = 0.0;
      s_sc[4] = 0.0;
    }
  }
  __syncthreads();

  for (int it = 0; it < a.iters; ++it) {
    const double beta = s_sc[0];
    int nw[3], ht[3];
    double ip = 0.0;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int In = pb.I[n];
      const int sv = s_id[n];
      nw[n] = (sv + 1) % 3;
      ht[n] = (sv + 2) % 3;
      // factors seen by mode n: Â of this iteration for l < n, of the last one for l > n
      auto hat_id = [&](int l) { return l < n ? ht[l] : s_id[l]; };
      // G^(n) (float64) and its scaled float32 form
      const int la = n == 0 ? 1 : 0, lb = n == 2 ? 1 : 2;
      const double* g1 = pb.gram[la][hat_id(la)];
      const double* g2 = pb.gram[lb][hat_id(lb)];
      // MTTKRP of mode n into pb.P
      if (n == 0) {
        y_pass<RB>(pb.T, I0, I1, I2, pb.buf[2][s_id[2]], pb.Y, work);
        fold<RB>(pb.Y, pb.buf[1][s_id[1]], I0, I1, 0, pb.P);
      } else if (n == 1) {
        fold<RB>(pb.Y, pb.buf[0][ht[0]], I0, I1, 1, pb.P);
      } else {
        last_pass<RB>(pb.T, I0, I1, I2, pb.buf[0][ht[0]], pb.buf[1][ht[1]], pb.P, work);
      }
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
      const int sweeps = hals_rows<RB>(pb.buf[n][sv], pb.buf[n][nw[n]], pb.P, G32s, ginv, In,
                                       a.max_inner, a.tol, s_red, w);
      // extrapolation A_hat = max(0, A_new + beta (A_new - A_old)), float64
      if (tid < In) {
        const float* w0 = pb.buf[n][sv] + tid * RB;
        float* hh = pb.buf[n][ht[n]] + tid * RB;
#pragma unroll
        for (int p = 0; p < RB; ++p) {
          const double x = w[p];
          const double y = x + beta * (x - double(w0[p]));
          hh[p] = float(y > 0.0 ? y : 0.0);
        }
        if (n == 2) {
#pragma unroll
          for (int p = 0; p < RB; ++p) ip = fma(double(pb.P[tid * RB + p]), double(w[p]), ip);
        }
      }
      __syncthreads();
      gram_of<RB>(pb.buf[n][nw[n]], In, pb.gram[n][nw[n]]);
      gram_of<RB>(pb.buf[n][ht[n]], In, pb.gram[n][ht[n]]);
      if (tid == 0 && pb.tr_sweeps) pb.tr_sweeps[int64_t(it) * 3 + n] = sweeps;
      __syncthreads();
    }
    // ---- F-hat_k (Gram trick with G^(3) and A_new^(3)) and the restart decision ----
    double gg = 0.0;
    for (int e = tid; e < RB * RB; e += kBT) gg = fma(G64s[e], pb.gram[2][nw[2]][e], gg);
    const double IP = block_sum(ip, s_red);
    const double GG = block_sum(gg, s_red);
    if (tid == 0) {
      const double fh = 0.5 * (normT2 - 2.0 * IP + GG);
      const double fprev = s_sc[2];
      const bool finite = isfinite(fh);
      const bool restart = !finite || fh > fprev;
      if (!finite && a.flags)
        __hip_atomic_fetch_or(a.flags, NTF_FLAG_NONFINITE, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      double b = s_sc[0], bb = s_sc[1];
      if (restart) {
        bb = b;
        b = b / a.eta;
      } else {
        const double bn = fmin(bb, a.gamma * b);
        bb = fmin(1.0, a.gamma_bar * bb);
        b = bn;
      }
      s_sc[0] = b;
      s_sc[1] = bb;
      if (finite) s_sc[2] = fh;  // a non-finite F-hat is no reference for the next test
      s_sc[3] += 1.0;
      if (restart) s_sc[4] += 1.0;
      for (int n = 0; n < 3; ++n) s_id[n] = restart ? nw[n] : ht[n];
      if (pb.tr_fhat) pb.tr_fhat[it] = fh;
      if (pb.tr_restart) pb.tr_restart[it] = restart ? 1 : 0;
    }
    __syncthreads();
  }

  // ---- results: survivors to the caller's factors, state ----
  for (int n = 0; n < 3; ++n) {
    const float* src = pb.buf[n][s_id[n]];
    for (int e = tid; e < pb.I[n] * r; e += kBT) {
      const int i = e / r, p = e - (e / r) * r;
      pb.A_user[n][e] = src[i * RB + p];
    }
  }
  if (tid == 0 && pb.st) {
    pb.st->beta = s_sc[0];
    pb.st->beta_bar = s_sc[1];
    pb.st->fhat_prev = s_sc[2];
    pb.st->fhat = s_sc[2];
    pb.st->k = int64_t(s_sc[3]);
    pb.st->restart = 0;
    pb.st->nrestarts = int32_t(s_sc[4]);
    pb.st->it = a.iters;
  }
}

__global__ __launch_bounds__(kBT) void batched_solve_kernel(BArgs a) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  __shared__ double s_red[kBW + 1];
  __shared__ double s_sc[8];
  __shared__ int s_id[4];
  const BProb& pb = a.probs[a.order[blockIdx.x]];
  switch (pb.rb) {
    case 8: solve_problem<8>(a, pb, lds, s_red, s_sc, s_id); break;
    case 16: solve_problem<16>(a, pb, lds, s_red, s_sc, s_id); break;
    case 24: solve_problem<24>(a, pb, lds, s_red, s_sc, s_id); break;
    default: solve_problem<32>(a, pb, lds, s_red, s_sc, s_id); break;
  }
}

}  // namespace

// LDS bytes a problem needs (largest phase plus the G area).
size_t batched_lds_bytes(int I0, int I1, int I2, int rb) {
  const size_t g = size_t(rb) * rb * 4 + size_t(rb) * 4 + size_t(rb) * rb * 8;
  const size_t ypass = (align_up(size_t(I2) * rb, 4) + size_t(kBW) * 64 * kTileLd) * 4;
  const int nchunk = int(ceil_div(I2, 64));
  const int nsplit = std::max(1, kBW / nchunk);
  const size_t lpass = (size_t(I0 + I1) * rb + size_t(nsplit) * nchunk * 64 * rb) * 4;
  return align_up(g, 16) + std::max(ypass, lpass);
}

// Per-problem device workspace layout (bytes), shared by sizing and carving.
struct BatchedLayout {
  size_t buf[3], gram, Y, P, misc, total;
};

static BatchedLayout batched_layout(const int I[3], int rb) {
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
  L.misc = take(sizeof(double) + sizeof(ntf_her_state));
  L.total = align_up(off, 256);
  return L;
}

size_t batched_problem_bytes(const int I[3], int rb) { return batched_layout(I, rb).total; }

// Build the device descriptors in the pinned staging area and enqueue their upload.
hipError_t batched_upload(const BatchedJob& job, size_t* lds_out, hipStream_t s) {
  static_assert(sizeof(BProb) <= kBatchedDescBytes, "descriptor slot too small");
  BProb* hd = reinterpret_cast<BProb*>(job.host_desc);
  size_t maxlds = 0;
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
    d.normT2 = reinterpret_cast<double*>(base + L.misc);
    d.st = q.state ? q.state
                   : reinterpret_cast<ntf_her_state*>(base + L.misc + sizeof(double));
    d.tr_fhat = q.tr_fhat;
    d.tr_restart = q.tr_restart;
    d.tr_sweeps = q.tr_sweeps;
    maxlds = std::max(maxlds, batched_lds_bytes(q.I[0], q.I[1], q.I[2], q.rb));
  }
  int32_t* ho = reinterpret_cast<int32_t*>(static_cast<char*>(job.host_desc) +
                                           size_t(job.nprob) * sizeof(BProb));
  for (int b = 0; b < job.nprob; ++b) ho[b] = job.order[b];
  *lds_out = maxlds;
  return hipMemcpyAsync(job.dev_desc, job.host_desc,
                        size_t(job.nprob) * (sizeof(BProb) + sizeof(int32_t)),
                        hipMemcpyHostToDevice, s);
}

size_t batched_desc_bytes(int nprob) { return size_t(nprob) * (sizeof(BProb) + sizeof(int32_t)); }

// The persistent launch (one workgroup per problem, all outer iterations).
hipError_t batched_launch(const BatchedJob& job, size_t lds, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(batched_solve_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  BArgs a{};
  a.probs = reinterpret_cast<const BProb*>(job.dev_desc);
  a.order = reinterpret_cast<const int32_t*>(static_cast<char*>(job.dev_desc) +
                                             size_t(job.nprob) * sizeof(BProb));
  a.nprob = job.nprob;
  a.iters = job.iters;
  a.resume = job.resume;
  a.max_inner = job.params.max_inner;
  a.beta0 = job.params.beta0;
  a.gamma = job.params.gamma;
  a.gamma_bar = job.params.gamma_bar;
  a.eta = job.params.eta;
  a.tol = job.params.inner_tol;
  a.flags = job.flags;
  hipLaunchKernelGGL(batched_solve_kernel, dim3(job.nprob), dim3(kBT), lds, s, a);
  return hipGetLastError();
}

}  // namespace ntf
