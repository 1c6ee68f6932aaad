// Projected-gradient block solvers (Sec. 2.2): for one block with data P = T_[n] B^(n)
// (I x r) and G = B^T B (r x r), repeated steps
//
//   W <- max(0, Y - (Y G - P) / L),   L = ||G||_2,
//
// with Y = W (plain projected gradient, HER-PGD of Sec. 3.1.4) or Y the Nesterov point
// W_s + ((t_{s-1} - 1) / t_s) (W_s - W_{s-1}), t_0 = 1, t_s = (1 + sqrt(1 + 4 t_{s-1}^2)) / 2
// (accelerated projected gradient, HER-Nesterov). Rows are independent given G and P, so
// a workgroup owns a few rows for all steps: thread (row, p) holds W[row, p], its previous
// value and column p of G in registers, and the row of Y in LDS (read as a broadcast by the
// threads of the row). A fixed number of steps is run (the paper's HER-PGD50 and
// HER-Nesterov50); a step that changes nothing leaves every later step unchanged, so this
// equals stopping at the first unchanged step.
//
// L is the largest eigenvalue of the symmetric G. G is entrywise nonnegative (a Hadamard
// product of Grams of nonnegative factors), so its largest eigenvalue is its Perron root:
// power iteration from the all-ones vector (float64, Rayleigh quotient, until it moves by
// less than 1e-12 relative or after 100 iterations).
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kPgdThreads = 256;
constexpr int kPowerIters = 100;

// One wave: G in LDS (G is symmetric, so lane t reads column t, conflict-free), lanes own
// rows t and t + 64; sums over the wave by DPP (the same value on every lane). The Rayleigh quotient is formed every fourth iteration; the iteration
// stops when it moves by less than 1e-12 relative, at most kPowerIters. Lane 0 then
// writes the Nesterov weights of every step.
// Sum over the 64 lanes with DPP moves (shuffles through LDS would cost a round trip per
// step): inclusive sums within each row of 16 lanes (row_shr 1, 2, 4, 8), then the row
// totals carried by row_bcast 15 and 31, so lane 63 ends with the total, in a fixed order.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_d<0x111, 0xF>(x);  // row_shr:1
  x += dpp_d<0x112, 0xF>(x);  // row_shr:2
  x += dpp_d<0x114, 0xF>(x);  // row_shr:4
  x += dpp_d<0x118, 0xF>(x);  // row_shr:8
  x += dpp_d<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_d<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), 63);
  return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(64) void lipschitz_kernel(const float* __restrict__ G, int r,
                                                       double* __restrict__ L, int steps,
                                                       float* __restrict__ coef) {
  extern __shared__ float s_g[];  // r x r
  __shared__ double s_v[128];
  const int t = threadIdx.x;
  // G into LDS, eight loads in flight per lane (clamped indices, no branch per load)
  const int rr = r * r;
  for (int e0 = t; e0 < rr; e0 += 64 * 8) {
    float gv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) gv[u] = G[min(e0 + 64 * u, rr - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (e0 + 64 * u < rr) s_g[e0 + 64 * u] = gv[u];
  }
  for (int q = t; q < r; q += 64) s_v[q] = 1.0;
  __syncthreads();
  const bool a0 = t < r, a1 = t + 64 < r;
  double lambda = 0.0, prev = -1.0;
  for (int it = 1; it <= kPowerIters; ++it) {
    // (G v)[t] and (G v)[t + 64]: four interleaved partial sums so that the LDS reads of
    // several q are in flight together (rows past r read row 0 and are not used)
    const int t1 = a1 ? t + 64 : 0;
    double p0[4] = {0.0, 0.0, 0.0, 0.0}, p1[4] = {0.0, 0.0, 0.0, 0.0};
    int q = 0;
    const int t0 = a0 ? t : 0;
    for (; q + 4 <= r; q += 4) {
      // all eight LDS reads of G first, so that they are in flight together
      float g0[4], g1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        g0[u] = s_g[(q + u) * r + t0];
        g1[u] = s_g[(q + u) * r + t1];
      }
      double vq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) vq[u] = s_v[q + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        p0[u] = fma(double(g0[u]), vq[u], p0[u]);
        p1[u] = fma(double(g1[u]), vq[u], p1[u]);
      }
    }
    for (; q < r; ++q) {
      const double vq = s_v[q];
      p0[0] = fma(double(s_g[q * r + t0]), vq, p0[0]);
      p1[0] = fma(double(s_g[q * r + t1]), vq, p1[0]);
    }
    const double w0 = a0 ? (p0[0] + p0[1]) + (p0[2] + p0[3]) : 0.0;
    const double w1 = a1 ? (p1[0] + p1[1]) + (p1[2] + p1[3]) : 0.0;
    // the Rayleigh quotient (two more sums) every fourth iteration and at the last
    const bool check = (it & 3) == 0 || it == kPowerIters;
    if (check) {
      const double v0 = a0 ? s_v[t] : 0.0, v1 = a1 ? s_v[t + 64] : 0.0;
      const double vw = wave_sum(v0 * w0 + v1 * w1);
      const double vv = wave_sum(v0 * v0 + v1 * v1);
      lambda = vv > 0.0 ? vw / vv : 0.0;
    }
    const double ww = wave_sum(w0 * w0 + w1 * w1);
    const double inv = ww > 0.0 ? 1.0 / sqrt(ww) : 0.0;
    __syncthreads();
    if (a0) s_v[t] = w0 * inv;
    if (a1) s_v[t + 64] = w1 * inv;
    __syncthreads();
    if (check) {
      // converged when the quotient moves by less than 1e-12 relative in four iterations
      // (far below the float32 rounding of the steps it scales)
      if (fabs(lambda - prev) <= 1e-12 * fabs(lambda)) break;
      prev = lambda;
    }
  }
  if (t == 0) {
    *L = lambda;
    // Nesterov weights (t_{s-1} - 1) / t_s of steps s = 1..steps (float64 recurrence)
    if (coef) {
      double tk = 1.0;
      for (int st = 0; st < steps; ++st) {
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tk * tk));
        coef[st] = float((tk - 1.0) / tn);
        tk = tn;
      }
    }
  }
}

template <int RP, bool ACCEL>
__global__ __launch_bounds__(kPgdThreads) void pgd_kernel(PgdArgs a) {
  constexpr int RB = kPgdThreads / RP;  // rows per workgroup
  __shared__ __attribute__((aligned(16))) float s_y[RB][RP];
  const int t = threadIdx.x;
  const int rl = t / RP;
  const int p = t - rl * RP;
  const int64_t row = int64_t(blockIdx.x) * RB + rl;
  const bool live = row < a.rows && p < a.r;
  const int r = a.r;
  // column p of G: loads at clamped indices, then a select (a conditional load per entry
  // would become a branch that waits for each load in turn)
  float g[RP];
#pragma unroll
  for (int q = 0; q < RP; ++q) g[q] = a.G[min(q, r - 1) * r + min(p, r - 1)];
#pragma unroll
  for (int q = 0; q < RP; ++q) g[q] = (q < r && p < r) ? g[q] : 0.f;
  const double L = *a.L;
  const float inv_l = L > 0.0 ? float(1.0 / L) : 0.f;
  const int64_t ix = live ? row * r + p : 0;
  const float pv0 = a.P[ix], w00 = a.W0[ix];
  const float pv = live ? pv0 : 0.f;
  float w = live ? w00 : 0.f;
  float y = w;
  for (int s = 0; s < a.steps; ++s) {
    s_y[rl][p] = y;
    __syncthreads();
    // (Y G)[row, p]: four interleaved partial sums over 16-byte broadcast reads of the row
    float acc4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < RP; q += 4) {
      const float4 yq = *reinterpret_cast<const float4*>(&s_y[rl][q]);
      acc4[0] = fmaf(yq.x, g[q], acc4[0]);
      acc4[1] = fmaf(yq.y, g[q + 1], acc4[1]);
      acc4[2] = fmaf(yq.z, g[q + 2], acc4[2]);
      acc4[3] = fmaf(yq.w, g[q + 3], acc4[3]);
    }
    const float acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
    __syncthreads();
    const float wn = L > 0.0 ? fmaxf(0.f, y - (acc - pv) * inv_l) : 0.f;
    if (ACCEL) {
      y = wn + a.coef[s] * (wn - w);
    } else {
      y = wn;
    }
    w = wn;
  }
  if (live) a.W[row * r + p] = w;
  if (blockIdx.x == 0 && t == 0 && a.steps_out) *a.steps_out = a.steps;
}

template <int RP>
hipError_t launch_rp(const PgdArgs& a, hipStream_t s) {
  const int64_t rb = kPgdThreads / RP;
  const dim3 grid(unsigned(ceil_div(a.rows, rb)));
  if (a.accel)
    hipLaunchKernelGGL((pgd_kernel<RP, true>), grid, dim3(kPgdThreads), 0, s, a);
  else
    hipLaunchKernelGGL((pgd_kernel<RP, false>), grid, dim3(kPgdThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lipschitz(const float* G, int r, double* L, int steps, float* coef,
                            hipStream_t s) {
  static bool attr_done = false;  // r = 128: 64 KB of G plus the vector exceed the default
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(lipschitz_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  hipLaunchKernelGGL(lipschitz_kernel, dim3(1), dim3(64), size_t(r) * r * sizeof(float), s, G, r,
                     L, steps, coef);
  return hipGetLastError();
}

hipError_t launch_pgd_steps(const PgdArgs& a, hipStream_t s) {
  if (a.r <= 32) return launch_rp<32>(a, s);
  if (a.r <= 64) return launch_rp<64>(a, s);
  return launch_rp<128>(a, s);
}

hipError_t launch_pgd(const PgdArgs& a, hipStream_t s) {
  hipError_t e = launch_lipschitz(a.G, a.r, a.L, a.steps, a.accel ? a.coef : nullptr, s);
  if (e != hipSuccess) return e;
  return launch_pgd_steps(a, s);
}

}  // namespace ntf
