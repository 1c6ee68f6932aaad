// Data given in Tucker format (Appendix A): T = (U^(1) (x) ... (x) U^(N)) G with a small
// core G (r_1 x ... x r_N) and bases U^(p) (n_p x r_p). The MTTKRP of mode i is
//
//   P = U^(i) G_[i] [KR_{p != i} (U^(p))^T A^(p)]  =  U^(i) MTTKRP_i(G; Q^(p)),  Q^(p) = (U^(p))^T A^(p),
//
// so the full tensor is never formed: projections Q^(p) (r_p x r, a reduction over the long
// mode n_p, float64 accumulation), the core's MTTKRP with the projected factors (the
// library's matrix-core MTTKRP on the float32 core), and the expansion U^(i) P_core. Its
// squared norm is <G x_1 (U^(1)T U^(1)) ... x_N (U^(N)T U^(N)), G> (||G||^2 for orthonormal
// bases), in float64 by mode products on the core.
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kTThreads = 256;

// Q = U^T A for small outputs (rp r <= kProjOut): workgroup g takes row chunks g, g + G, ...
// of cr rows, stages each chunk's U and A rows in LDS and accumulates its outputs (thread
// t: outputs t, t + 256, ...) over the rows in order (float64); partial[g] holds its sums,
// which tucker_proj_sum_kernel adds in workgroup order.
constexpr int kProjOut = 8 * kTThreads;
constexpr int kProjWgs = 1024;

// rows per chunk: what fits 64 KB of LDS, at most 256, and few enough that the rows spread
// over about 128 workgroups, but at least 8 (a short block gets few partials to sum)
int proj_chunk_rows(int64_t n, int rp, int r) {
  const int64_t spread = std::max<int64_t>(8, ceil_div(n, int64_t(128)));
  return int(std::max<int64_t>(1, std::min<int64_t>({256, 16384 / (rp + r), spread})));
}

int64_t proj_wgs(int64_t n, int rp, int r) {
  return std::min<int64_t>(kProjWgs, ceil_div(n, proj_chunk_rows(n, rp, r)));
}

__global__ __launch_bounds__(kTThreads) void tucker_proj_part_kernel(
    const float* __restrict__ U, const float* __restrict__ A, int64_t n, int rp, int r, int cr,
    double* __restrict__ part) {
  extern __shared__ float sm[];
  float* Us = sm;            // cr x rp
  float* As = sm + cr * rp;  // cr x r
  const int t = threadIdx.x;
  const int no = rp * r;
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  for (int64_t c = blockIdx.x; c * cr < n; c += gridDim.x) {
    const int64_t m0 = c * cr;
    const int rows = int(std::min<int64_t>(cr, n - m0));
    for (int e = t; e < rows * rp; e += kTThreads) Us[e] = U[m0 * rp + e];
    for (int e = t; e < rows * r; e += kTThreads) As[e] = A[m0 * r + e];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int o = t + q * kTThreads;
      if (o < no) {
        const int i = o / r, p = o - (o / r) * r;
        double a = acc[q];
        for (int m = 0; m < rows; ++m) a = fma(double(Us[m * rp + i]), double(As[m * r + p]), a);
        acc[q] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int o = t + q * kTThreads;
    if (o < no) part[int64_t(blockIdx.x) * no + o] = acc[q];
  }
}

// Q[o] = sum over workgroups g (in order) of part[g][o]; thirty-two loads in flight per thread
__global__ __launch_bounds__(kTThreads) void tucker_proj_sum_kernel(
    const double* __restrict__ part, int nwg, int no, float* __restrict__ Q32,
    double* __restrict__ Q64) {
  const int o = blockIdx.x * kTThreads + threadIdx.x;
  if (o >= no) return;
  double s = 0.0;
  for (int g0 = 0; g0 < nwg; g0 += 32) {
    double v[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) v[u] = part[int64_t(min(g0 + u, nwg - 1)) * no + o];
#pragma unroll
    for (int u = 0; u < 32; ++u)
      if (g0 + u < nwg) s += v[u];
  }
  if (Q32) Q32[o] = float(s);
  if (Q64) Q64[o] = s;
}

// Q[i][p] = sum_n U[n][i] A[n][p] (U: n x rp, A: n x r), for outputs too large for the
// kernels above. Workgroup i; its threads are 8 lanes along n by 32 along p, summed over
// the lanes in a fixed order (float64).
__global__ __launch_bounds__(kTThreads) void tucker_proj_kernel(const float* __restrict__ U,
                                                                const float* __restrict__ A,
                                                                int64_t n, int rp, int r,
                                                                float* __restrict__ Q32,
                                                                double* __restrict__ Q64) {
  __shared__ double s_red[8][32];
  const int i = blockIdx.x;
  const int t = threadIdx.x;
  const int pl = t & 31;
  const int nl = t >> 5;
  for (int p0 = 0; p0 < r; p0 += 32) {
    const int p = p0 + pl;
    double acc = 0.0;
    if (p < r)
      for (int64_t m = nl; m < n; m += 8) acc = fma(double(U[m * rp + i]), double(A[m * r + p]), acc);
    s_red[nl][pl] = acc;
    __syncthreads();
    if (nl == 0 && p < r) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) s += s_red[k][pl];
      if (Q32) Q32[i * r + p] = float(s);
      if (Q64) Q64[i * r + p] = s;
    }
    __syncthreads();
  }
}

// P[m][p] = sum_i U[m][i] Pc[i][p] (U: n x rp, Pc: rp x r), float64 accumulation
__global__ __launch_bounds__(kTThreads) void tucker_expand_kernel(const float* __restrict__ U,
                                                                  const float* __restrict__ Pc,
                                                                  int64_t n, int rp, int r,
                                                                  float* __restrict__ P) {
  const int64_t e = int64_t(blockIdx.x) * kTThreads + threadIdx.x;
  if (e >= n * r) return;
  const int64_t m = e / r;
  const int p = int(e - m * r);
  // the chain over i = 0 .. rp - 1 in order; sixteen terms' loads issued together (clamped
  // in range, the ones past rp add nothing)
  double acc = 0.0;
  for (int i0 = 0; i0 < rp; i0 += 16) {
    float u[16], c[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int i = min(i0 + t, rp - 1);
      u[t] = U[m * rp + i];
      c[t] = Pc[i * r + p];
    }
#pragma unroll
    for (int t = 0; t < 16; ++t)
      if (i0 + t < rp) acc = fma(double(u[t]), double(c[t]), acc);
  }
  P[e] = float(acc);
}

// Y = X x_mode M for a small float64 tensor X (dims d, C order) and an r_mode x r_mode M:
// Y[.., a, ..] = sum_b M[a][b] X[.., b, ..]. One thread per output element.
__global__ __launch_bounds__(kTThreads) void mode_product_kernel(const double* __restrict__ X,
                                                                 const double* __restrict__ M,
                                                                 int64_t total, int64_t inner,
                                                                 int dm, double* __restrict__ Y) {
  const int64_t e = int64_t(blockIdx.x) * kTThreads + threadIdx.x;
  if (e >= total) return;
  const int64_t hi = e / (inner * dm);
  const int64_t rem = e - hi * inner * dm;
  const int a = int(rem / inner);
  const int64_t lo = rem - int64_t(a) * inner;
  const double* xb = X + hi * inner * dm + lo;
  double acc = 0.0;
  for (int b = 0; b < dm; ++b) acc = fma(M[a * dm + b], xb[int64_t(b) * inner], acc);
  Y[e] = acc;
}

__global__ __launch_bounds__(kTThreads) void f32_to_f64_kernel(const float* __restrict__ x,
                                                               double* __restrict__ y,
                                                               int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * kTThreads;
  for (int64_t e = int64_t(blockIdx.x) * kTThreads + threadIdx.x; e < n; e += stride)
    y[e] = double(x[e]);
}

// out = <X, G> (float64, one workgroup, fixed order)
__global__ __launch_bounds__(kTThreads) void dot_core_kernel(const double* __restrict__ X,
                                                             const float* __restrict__ G,
                                                             int64_t n, double* out) {
  __shared__ double s[kTThreads];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int64_t e = t; e < n; e += kTThreads) acc = fma(X[e], double(G[e]), acc);
  s[t] = acc;
  __syncthreads();
  if (t == 0) {
    double sum = 0.0;
    for (int k = 0; k < kTThreads; ++k) sum += s[k];
    *out = sum;
  }
}

int blocks_for(int64_t n) { return int(std::max<int64_t>(1, ceil_div(n, kTThreads))); }

}  // namespace

size_t tucker_proj_part_doubles(int64_t n, int rp, int r) {
  if (int64_t(rp) * r > kProjOut) return 0;
  return size_t(proj_wgs(n, rp, r)) * rp * r;
}

hipError_t launch_tucker_proj(const float* U, const float* A, int64_t n, int rp, int r,
                              float* Q32, double* Q64, double* part, hipStream_t s) {
  if (int64_t(rp) * r > kProjOut) {
    hipLaunchKernelGGL(tucker_proj_kernel, dim3(rp), dim3(kTThreads), 0, s, U, A, n, rp, r,
                       Q32, Q64);
    return hipGetLastError();
  }
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(tucker_proj_part_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int cr = proj_chunk_rows(n, rp, r);
  const int nwg = int(proj_wgs(n, rp, r));
  hipLaunchKernelGGL(tucker_proj_part_kernel, dim3(nwg), dim3(kTThreads),
                     size_t(cr) * (rp + r) * sizeof(float), s, U, A, n, rp, r, cr, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int no = rp * r;
  hipLaunchKernelGGL(tucker_proj_sum_kernel, dim3(unsigned(ceil_div(no, kTThreads))),
                     dim3(kTThreads), 0, s, part, nwg, no, Q32, Q64);
  return hipGetLastError();
}

hipError_t launch_tucker_expand(const float* U, const float* Pc, int64_t n, int rp, int r,
                                float* P, hipStream_t s) {
  hipLaunchKernelGGL(tucker_expand_kernel, dim3(blocks_for(n * r)), dim3(kTThreads), 0, s, U,
                     Pc, n, rp, r, P);
  return hipGetLastError();
}

size_t tucker_norm_workspace_doubles(const TuckerDesc& X) {
  int64_t core = 1;
  size_t grams = 0, part = 0;
  for (int p = 0; p < X.core.order; ++p) {
    core *= X.core.dims[p];
    grams = std::max(grams, size_t(X.core.dims[p]) * X.core.dims[p]);
    part = std::max(part, tucker_proj_part_doubles(X.dims[p], int(X.core.dims[p]),
                                                   int(X.core.dims[p])));
  }
  return size_t(2 * core) + grams + part;
}

hipError_t launch_tucker_norm2(const TuckerDesc& X, double* ws, double* out, hipStream_t s) {
  const int N = X.core.order;
  int64_t total = 1;
  for (int p = 0; p < N; ++p) total *= X.core.dims[p];
  double* buf[2] = {ws, ws + total};
  double* gram = ws + 2 * total;
  size_t gmax = 0;
  for (int p = 0; p < N; ++p) gmax = std::max(gmax, size_t(X.core.dims[p]) * X.core.dims[p]);
  double* part = gram + gmax;
  const float* core = static_cast<const float*>(X.core.data);
  hipLaunchKernelGGL(f32_to_f64_kernel, dim3(std::min(blocks_for(total), 4096)), dim3(kTThreads),
                     0, s, core, buf[0], total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int cur = 0;
  int64_t inner = total;
  for (int p = 0; p < N; ++p) {
    const int dm = int(X.core.dims[p]);
    inner /= dm;
    // M = U^(p)T U^(p) (float64)
    if ((e = launch_tucker_proj(X.U[p], X.U[p], X.dims[p], dm, dm, nullptr, gram, part, s)) !=
        hipSuccess)
      return e;
    hipLaunchKernelGGL(mode_product_kernel, dim3(blocks_for(total)), dim3(kTThreads), 0, s,
                       buf[cur], gram, total, inner, dm, buf[cur ^ 1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    cur ^= 1;
  }
  hipLaunchKernelGGL(dot_core_kernel, dim3(1), dim3(kTThreads), 0, s, buf[cur], core, total, out);
  return hipGetLastError();
}

}  // namespace ntf
