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
// power iteration from the all-ones vector (float64, fixed count, Rayleigh quotient).
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kPgdThreads = 256;
constexpr int kPowerIters = 100;

__global__ __launch_bounds__(256) void lipschitz_kernel(const float* __restrict__ G, int r,
                                                        double* __restrict__ L) {
  __shared__ double v[kMaxRank], w[kMaxRank], red[256];
  const int t = threadIdx.x;
  if (t < r) v[t] = 1.0;
  __syncthreads();
  double lambda = 0.0;
  for (int it = 0; it < kPowerIters; ++it) {
    double acc = 0.0;
    if (t < r)
      for (int q = 0; q < r; ++q) acc += double(G[t * r + q]) * v[q];
    if (t < r) w[t] = acc;
    // Rayleigh quotient v.w / v.v and the norm of w (fixed-order sums by thread 0)
    __syncthreads();
    if (t == 0) {
      double vw = 0.0, vv = 0.0, ww = 0.0;
      for (int q = 0; q < r; ++q) {
        vw += v[q] * w[q];
        vv += v[q] * v[q];
        ww += w[q] * w[q];
      }
      red[0] = vv > 0.0 ? vw / vv : 0.0;
      red[1] = ww > 0.0 ? 1.0 / sqrt(ww) : 0.0;
    }
    __syncthreads();
    lambda = red[0];
    if (t < r) v[t] = w[t] * red[1];
    __syncthreads();
  }
  if (t == 0) *L = lambda;
}

template <int RP, bool ACCEL>
__global__ __launch_bounds__(kPgdThreads) void pgd_kernel(PgdArgs a) {
  constexpr int RB = kPgdThreads / RP;  // rows per workgroup
  __shared__ float s_y[RB][RP];
  const int t = threadIdx.x;
  const int rl = t / RP;
  const int p = t - rl * RP;
  const int64_t row = int64_t(blockIdx.x) * RB + rl;
  const bool live = row < a.rows && p < a.r;
  const int r = a.r;
  float g[RP];
#pragma unroll
  for (int q = 0; q < RP; ++q) g[q] = (q < r && p < r) ? a.G[q * r + p] : 0.f;
  const double L = *a.L;
  const float inv_l = L > 0.0 ? float(1.0 / L) : 0.f;
  const float pv = live ? a.P[row * r + p] : 0.f;
  float w = live ? a.W0[row * r + p] : 0.f;
  float y = w;
  double tk = 1.0;
  for (int s = 0; s < a.steps; ++s) {
    s_y[rl][p] = y;
    __syncthreads();
    float acc = 0.f;
#pragma unroll
    for (int q = 0; q < RP; ++q) acc = fmaf(s_y[rl][q], g[q], acc);
    __syncthreads();
    const float wn = L > 0.0 ? fmaxf(0.f, y - (acc - pv) * inv_l) : 0.f;
    if (ACCEL) {
      const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tk * tk));
      y = wn + float((tk - 1.0) / tn) * (wn - w);
      tk = tn;
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

hipError_t launch_pgd(const PgdArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(lipschitz_kernel, dim3(1), dim3(256), 0, s, a.G, a.r, a.L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.r <= 32) return launch_rp<32>(a, s);
  if (a.r <= 64) return launch_rp<64>(a, s);
  return launch_rp<128>(a, s);
}

}  // namespace ntf
