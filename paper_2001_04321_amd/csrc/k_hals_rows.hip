// A-HALS for blocks of any number of rows (Sec. 2.1.4; stopping rule of Sec. 4.1). The
// column updates of A-HALS touch one row at a time:
//
//   W[i, j] <- max(0, P[i, j] - sum_{l != j} W[i, l] G[l, j]) / G[j, j]   (j = 1..r in order)
//
// (a dead component, G[j, j] = 0, gives 0), so rows are independent given P and G; only the
// stopping rule couples them. The resident A-HALS kernel (k_hals.hip) decides the rule
// across workgroups while they run, which bounds a block to the rows that stay resident at
// once. This variant has no such bound (r <= 32): one thread owns one row (W and P rows in
// registers, G in LDS, read as broadcasts), a first pass runs every sweep and records
// each workgroup's share of ||W_s - W_{s-1}||^2 per sweep, one workgroup sums the shares in
// a fixed order and finds the sweep the rule stops at, and a second pass repeats the same
// arithmetic up to that sweep and writes W. Both passes compute the same bits, so the
// result is the iterate the sequential rule returns.
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kRowThreads = 256;

template <int RMAX, int PASS>
__global__ __launch_bounds__(kRowThreads) void hals_rows_kernel(HalsRowsArgs a) {
  extern __shared__ float s_g[];  // r x r
  __shared__ double s_w[kHalsRowsMaxSweeps][kRowThreads / 64];
  const int t = threadIdx.x;
  const int r = a.r;
  for (int e = t; e < r * r; e += kRowThreads) s_g[e] = a.G[e];
  __syncthreads();
  const int64_t row = int64_t(blockIdx.x) * kRowThreads + t;
  const bool live = row < a.rows;
  const int64_t base = (live ? row : 0) * r;
  float w[RMAX], pv[RMAX];
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    const int jj = j < r ? j : 0;
    const float pw = a.P[base + jj], ww = a.W0[base + jj];
    pv[j] = (live && j < r) ? pw : 0.f;
    w[j] = (live && j < r) ? ww : 0.f;
  }
  const int sweeps = PASS == 1 ? a.max_sweeps : *a.sweeps_dev;
  for (int s = 0; s < sweeps; ++s) {
    double d2 = 0.0;
    // columns past r hold zeros in w and are skipped (predicated, so the loops unroll and
    // w stays in registers)
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
      if (j < r) {
        float num = pv[j];
#pragma unroll
        for (int l = 0; l < RMAX; ++l)
          if (l < r && l != j) num = fmaf(-w[l], s_g[l * r + j], num);
        const float gjj = s_g[j * r + j];
        const float nw = gjj > 0.f ? fmaxf(0.f, num) / gjj : 0.f;
        const double df = double(nw) - double(w[j]);
        d2 = fma(df, df, d2);
        w[j] = nw;
      }
    }
    if (PASS == 1) {
      double x = live ? d2 : 0.0;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
      if ((t & 63) == 0) s_w[s][t >> 6] = x;
    }
  }
  if (PASS == 1) {
    __syncthreads();
    for (int s = t; s < a.max_sweeps; s += kRowThreads) {
      double x = 0.0;
#pragma unroll
      for (int k = 0; k < kRowThreads / 64; ++k) x += s_w[s][k];
      a.part[int64_t(s) * gridDim.x + blockIdx.x] = x;
    }
  } else if (live) {
#pragma unroll
    for (int j = 0; j < RMAX; ++j)
      if (j < r) a.W[base + j] = w[j];
  }
}

// The stopping rule from the per-sweep shares: the first sweep s with
// ||W_s - W_{s-1}|| <= tol ||W_1 - W_0|| (at s = 1: only a sweep that changed nothing, for
// tol < 1), else max_sweeps.
__global__ __launch_bounds__(64) void hals_rows_decide_kernel(HalsRowsArgs a, int nwg) {
  __shared__ double s_d[kHalsRowsMaxSweeps];
  const int t = threadIdx.x;
  if (t < a.max_sweeps) {
    double x = 0.0;
    for (int k = 0; k < nwg; ++k) x += a.part[int64_t(t) * nwg + k];
    s_d[t] = x;
  }
  __syncthreads();
  if (t == 0) {
    int stop = a.max_sweeps;
    const double d1 = sqrt(s_d[0]);
    for (int s = 1; s <= a.max_sweeps; ++s)
      if (sqrt(s_d[s - 1]) <= a.tol * d1) {
        stop = s;
        break;
      }
    *a.sweeps_dev = stop;
    if (a.sweeps_out) *a.sweeps_out = stop;
  }
}

template <int RMAX>
hipError_t launch_passes(const HalsRowsArgs& a, hipStream_t s) {
  const int nwg = int(hals_rows_workgroups(a.rows));
  const size_t lds = size_t(a.r) * a.r * sizeof(float);
  hipLaunchKernelGGL((hals_rows_kernel<RMAX, 1>), dim3(nwg), dim3(kRowThreads), lds, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hals_rows_decide_kernel, dim3(1), dim3(64), 0, s, a, nwg);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((hals_rows_kernel<RMAX, 2>), dim3(nwg), dim3(kRowThreads), lds, s, a);
  return hipGetLastError();
}

}  // namespace

int64_t hals_rows_workgroups(int64_t rows) { return ceil_div(rows, kRowThreads); }

hipError_t launch_hals_rows(const HalsRowsArgs& a, hipStream_t s) {
  if (a.r > kHalsRowsMaxRank) return hipErrorInvalidValue;
  if (a.r <= 16) return launch_passes<16>(a, s);
  return launch_passes<32>(a, s);
}

}  // namespace ntf
