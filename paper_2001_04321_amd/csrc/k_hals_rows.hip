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

// RM columns per row in registers: RM = r (EXACT) or the next of 24, 32 (columns past r hold
// zeros and are skipped; predicated, so the loops unroll and w stays in registers). G is in
// LDS transposed, s_gt[j * RM + l] = G[l][j]; column j's terms are taken in the order
// l = j + 1, ..., j - 1 (cyclically) over four partial sums, so the column updated last
// enters last, and row j + 1 of s_gt is read while column j is updated. The division by
// G[j][j] is a product with its reciprocal, formed once per launch (a dead component,
// G[j][j] <= 0, keeps the reciprocal 0 and its column 0).
template <int RM, bool EXACT, int PASS>
__global__ __launch_bounds__(kRowThreads) void hals_rows_kernel(HalsRowsArgs a) {
  __shared__ float s_gt[RM * RM];
  __shared__ double s_w[kHalsRowsMaxSweeps][kRowThreads / 64];
  const int t = threadIdx.x;
  const int r = EXACT ? RM : a.r;
  for (int e = t; e < RM * RM; e += kRowThreads) {
    const int j = e / RM, l = e - (e / RM) * RM;
    s_gt[e] = (j < r && l < r) ? a.G[l * r + j] : 0.f;
  }
  __syncthreads();
  const int64_t row = int64_t(blockIdx.x) * kRowThreads + t;
  const bool live = row < a.rows;
  const int64_t base = (live ? row : 0) * r;
  float w[RM], pv[RM];
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const bool in = EXACT || j < r;
    const int jj = in ? j : 0;
    const float pw = a.P[base + jj], ww = a.W0[base + jj];
    pv[j] = (live && in) ? pw : 0.f;
    w[j] = (live && in) ? ww : 0.f;
  }
  float ginv[RM];
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const float gjj = s_gt[j * RM + j];
    ginv[j] = gjj > 0.f ? 1.f / gjj : 0.f;
  }
  const int sweeps = PASS == 1 ? a.max_sweeps : *a.sweeps_dev;
  for (int s = 0; s < sweeps; ++s) {
    // an opaque (zero) offset per sweep keeps G in LDS, read where it is used, instead of
    // being hoisted out of the loop into RM * RM registers
    int zero = 0;
    asm volatile("" : "+v"(zero));
    const float* gt = s_gt + zero;
    double d2 = 0.0;
    float gb[2][RM];
#pragma unroll
    for (int l = 0; l < RM; ++l) gb[0][l] = gt[l];
#pragma unroll
    for (int j = 0; j < RM; ++j) {
      if (j + 1 < RM) {
#pragma unroll
        for (int l = 0; l < RM; ++l) gb[(j + 1) & 1][l] = gt[(j + 1) * RM + l];
      }
      if (EXACT || j < r) {
        float acc[4] = {pv[j], 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 1; m < RM; ++m) {
          const int l = (j + m) % RM;
          if (EXACT || l < r) acc[m & 3] = fmaf(-w[l], gb[j & 1][l], acc[m & 3]);
        }
        const float num = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        const float nw = ginv[j] != 0.f ? fmaxf(0.f, num) * ginv[j] : 0.f;
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
    for (int j = 0; j < RM; ++j)
      if (EXACT || j < r) a.W[base + j] = w[j];
  }
}

// The stopping rule from the per-sweep shares: the first sweep s with
// ||W_s - W_{s-1}|| <= tol ||W_1 - W_0|| (at s = 1: only a sweep that changed nothing, for
// tol < 1), else max_sweeps.
__global__ __launch_bounds__(64) void hals_rows_decide_kernel(HalsRowsArgs a, int nwg) {
  __shared__ double s_d[kHalsRowsMaxSweeps];
  const int t = threadIdx.x;
  if (t < a.max_sweeps) {
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

template <int RM, bool EXACT>
hipError_t launch_passes(const HalsRowsArgs& a, hipStream_t s) {
  const int nwg = int(hals_rows_workgroups(a.rows));
  hipLaunchKernelGGL((hals_rows_kernel<RM, EXACT, 1>), dim3(nwg), dim3(kRowThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hals_rows_decide_kernel, dim3(1), dim3(64), 0, s, a, nwg);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((hals_rows_kernel<RM, EXACT, 2>), dim3(nwg), dim3(kRowThreads), 0, s, a);
  return hipGetLastError();
}

template <int R>
hipError_t launch_exact(const HalsRowsArgs& a, hipStream_t s) {
  if constexpr (R > 16) {
    return hipErrorInvalidValue;
  } else {
    if (a.r == R) return launch_passes<R, true>(a, s);
    return launch_exact<R + 1>(a, s);
  }
}

}  // namespace

int64_t hals_rows_workgroups(int64_t rows) { return ceil_div(rows, kRowThreads); }

hipError_t launch_hals_rows(const HalsRowsArgs& a, hipStream_t s) {
  if (a.r < 1 || a.r > kHalsRowsMaxRank) return hipErrorInvalidValue;
  if (a.r <= 16) return launch_exact<1>(a, s);
  if (a.r <= 24) return launch_passes<24, false>(a, s);
  return launch_passes<32, false>(a, s);
}

}  // namespace ntf
