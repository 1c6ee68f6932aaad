// ADMM block solver (Sec. 2.1.2: AO-ADMM solves each NNLS block with a few ADMM steps;
// HER-ADMM is Algorithm 2 with it). For one block with P = T_[n] B^(n) (I x r) and
// G = B^T B (r x r), scaled ADMM on the splitting W = Z of f(W) = 1/2 ||T_[n] - W B^T||^2
// and the nonnegativity of Z:
//
//   W_s = (P + rho (Z_{s-1} - U_{s-1})) (G + rho I)^-1,
//   Z_s = max(0, W_s + U_{s-1}),   U_s = U_{s-1} + W_s - Z_s,
//
// rho = trace(G) / r, Z_0 the warm start, U_0 = 0, and the block's result the nonnegative
// Z_s. The inner stopping rule of Sec. 4.1 (||Z_s - Z_{s-1}|| <= tol ||Z_1 - Z_0||, at most
// max_steps) couples all rows, while the steps themselves do not: the rows are independent
// given P, G and rho. So the solver runs in four launches: one workgroup forms
// K = (G + rho I)^-1 in float64 (Gauss-Jordan sweeps of the symmetric positive definite
// matrix, no pivoting needed) and rounds it to float32; a row-parallel pass runs every
// step and records each workgroup's share of ||Z_s - Z_{s-1}||^2 per step; one workgroup
// sums the shares in a fixed order and finds the step the rule stops at; a second
// row-parallel pass repeats the same arithmetic up to that step and writes Z. Both passes
// compute the same bits, so the result is the iterate the sequential rule returns.
// G + rho I has eigenvalues in [rho, lambda_max + rho] with lambda_max <= trace(G) = r rho,
// so its condition number is at most r + 1: the explicit float32 inverse is accurate.
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kAdmmThreads = 256;

// G (float32) -> K = (G + rho I)^-1 (float32) and rho, by r Gauss-Jordan sweeps in float64.
// Sweeping pivot k of a symmetric matrix A: A_ij -= A_ik A_kj / A_kk (i, j != k), then
// A_ik /= A_kk, A_kj /= A_kk, A_kk = -1 / A_kk; after every pivot A = -(G + rho I)^-1.
__global__ __launch_bounds__(kAdmmThreads) void admm_prep_kernel(const float* __restrict__ G,
                                                                 int r, float* __restrict__ K,
                                                                 float* __restrict__ rho_out) {
  extern __shared__ double s_a[];  // r x r
  __shared__ double s_red[kAdmmThreads];
  __shared__ double s_rho;
  const int t = threadIdx.x;
  const int rr = r * r;
  double tr = 0.0;
  for (int e = t; e < rr; e += kAdmmThreads) {
    const double v = double(G[e]);
    s_a[e] = v;
    const int i = e / r;
    if (e == i * r + i) tr += v;
  }
  s_red[t] = tr;
  __syncthreads();
  if (t == 0) {
    double sum = 0.0;
    for (int k = 0; k < kAdmmThreads; ++k) sum += s_red[k];  // fixed order
    s_rho = sum / r;
  }
  __syncthreads();
  const double rho = s_rho;
  if (!(rho > 0.0)) {  // every component dead: the block solution is 0
    for (int e = t; e < rr; e += kAdmmThreads) K[e] = 0.f;
    if (t == 0) *rho_out = 0.f;
    return;
  }
  for (int i = t; i < r; i += kAdmmThreads) s_a[i * r + i] += rho;
  __syncthreads();
  for (int k = 0; k < r; ++k) {
    const double d = s_a[k * r + k];
    const double inv = 1.0 / d;
    for (int e = t; e < rr; e += kAdmmThreads) {
      const int i = e / r;
      const int j = e - i * r;
      if (i != k && j != k) s_a[e] -= s_a[i * r + k] * s_a[k * r + j] * inv;
    }
    __syncthreads();
    for (int e = t; e < r; e += kAdmmThreads) {
      if (e == k) continue;
      s_a[e * r + k] *= inv;
      s_a[k * r + e] *= inv;
    }
    if (t == 0) s_a[k * r + k] = -inv;
    __syncthreads();
  }
  for (int e = t; e < rr; e += kAdmmThreads) K[e] = float(-s_a[e]);
  if (t == 0) *rho_out = float(rho);
}

// PASS 1: every step, per-workgroup shares of ||Z_s - Z_{s-1}||^2 into part[s][wg];
// PASS 2: *steps_dev steps, then Z into W. Thread (row, p) holds Z[row, p], U[row, p],
// P[row, p] and column p of K in registers; the row of P + rho (Z - U) is shared in LDS.
template <int RP, int PASS>
__global__ __launch_bounds__(kAdmmThreads) void admm_kernel(AdmmArgs a) {
  constexpr int RB = kAdmmThreads / RP;  // rows per workgroup
  __shared__ __attribute__((aligned(16))) float s_y[RB][RP];
  __shared__ double s_w[kAdmmMaxSteps][kAdmmThreads / 64];
  const int t = threadIdx.x;
  const int rl = t / RP;
  const int p = t - rl * RP;
  const int64_t row = int64_t(blockIdx.x) * RB + rl;
  const bool live = row < a.rows && p < a.r;
  const int r = a.r;
  float kc[RP];
#pragma unroll
  for (int q = 0; q < RP; ++q) kc[q] = a.K[min(q, r - 1) * r + min(p, r - 1)];
#pragma unroll
  for (int q = 0; q < RP; ++q) kc[q] = (q < r && p < r) ? kc[q] : 0.f;
  const float rho = *a.rho;
  const int64_t ix = live ? row * r + p : 0;
  const float pv0 = a.P[ix], z00 = a.W0[ix];
  const float pv = live ? pv0 : 0.f;
  float z = live ? z00 : 0.f;
  float u = 0.f;
  const int steps = PASS == 1 ? a.max_steps : *a.steps_dev;
  for (int s = 0; s < steps; ++s) {
    s_y[rl][p] = pv + rho * (z - u);
    __syncthreads();
    float acc4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < RP; q += 4) {
      const float4 yq = *reinterpret_cast<const float4*>(&s_y[rl][q]);
      acc4[0] = fmaf(yq.x, kc[q], acc4[0]);
      acc4[1] = fmaf(yq.y, kc[q + 1], acc4[1]);
      acc4[2] = fmaf(yq.z, kc[q + 2], acc4[2]);
      acc4[3] = fmaf(yq.w, kc[q + 3], acc4[3]);
    }
    const float w = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
    __syncthreads();
    const float zn = fmaxf(0.f, w + u);
    u = u + (w - zn);
    if (PASS == 1) {
      const double df = live ? double(zn) - double(z) : 0.0;
      double x = df * df;
      // sum over the wave in a fixed order (xor butterfly), one slot per wave and step
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
      if ((t & 63) == 0) s_w[s][t >> 6] = x;
    }
    z = zn;
  }
  if (PASS == 1) {
    __syncthreads();
    for (int s = t; s < a.max_steps; s += kAdmmThreads) {
      double x = 0.0;
#pragma unroll
      for (int k = 0; k < kAdmmThreads / 64; ++k) x += s_w[s][k];
      a.part[int64_t(s) * gridDim.x + blockIdx.x] = x;
    }
  } else if (live) {
    a.W[row * r + p] = z;
  }
}

// The stopping rule: D_s = sum over workgroups of part[s][wg] (fixed order); stop at
// s = 1 if D_1 = 0 (or the block is dead), else at the first s >= 2 with
// sqrt(D_s) <= tol sqrt(D_1), else at max_steps.
__global__ __launch_bounds__(64) void admm_decide_kernel(AdmmArgs a, int nwg) {
  __shared__ double s_d[kAdmmMaxSteps];
  const int t = threadIdx.x;
  if (t < a.max_steps) {
    // workgroups in order, sixteen loads in flight
    double x = 0.0;
    const double* pt = a.part + int64_t(t) * nwg;
    for (int k0 = 0; k0 < nwg; k0 += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = pt[min(k0 + u, nwg - 1)];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (k0 + u < nwg) x += v[u];
    }
    s_d[t] = x;
  }
  __syncthreads();
  if (t == 0) {
    int stop = a.max_steps;
    const double d1 = sqrt(s_d[0]);
    if (!(*a.rho > 0.f) || d1 == 0.0) {
      stop = 1;
    } else {
      for (int s = 2; s <= a.max_steps; ++s)
        if (sqrt(s_d[s - 1]) <= a.tol * d1) {
          stop = s;
          break;
        }
    }
    *a.steps_dev = stop;
    if (a.steps_out) *a.steps_out = stop;
  }
}

template <int RP>
hipError_t launch_passes(const AdmmArgs& a, hipStream_t s) {
  constexpr int64_t RB = kAdmmThreads / RP;
  const int nwg = int(ceil_div(a.rows, RB));
  hipLaunchKernelGGL((admm_kernel<RP, 1>), dim3(nwg), dim3(kAdmmThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(admm_decide_kernel, dim3(1), dim3(64), 0, s, a, nwg);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((admm_kernel<RP, 2>), dim3(nwg), dim3(kAdmmThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

int64_t admm_workgroups(int64_t rows, int r) {
  const int rp = r <= 32 ? 32 : r <= 64 ? 64 : 128;
  return ceil_div(rows, kAdmmThreads / rp);
}

hipError_t launch_admm(const AdmmArgs& a, hipStream_t s) {
  static bool attr_done = false;  // r = 128: 128 KB of float64 G exceeds the default
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(admm_prep_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 136 * 1024);
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  hipLaunchKernelGGL(admm_prep_kernel, dim3(1), dim3(kAdmmThreads),
                     size_t(a.r) * a.r * sizeof(double), s, a.G, a.r, a.K, a.rho);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.r <= 32) return launch_passes<32>(a, s);
  if (a.r <= 64) return launch_passes<64>(a, s);
  return launch_passes<128>(a, s);
}

}  // namespace ntf
