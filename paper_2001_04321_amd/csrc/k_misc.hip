// Streaming and scalar kernels of the HER / A-HALS path:
//  - ||T||^2 in float64 (restart surrogate needs it, paper Sec. 3.1.3),
//  - float32 -> bfloat16 copy of the tensor (stored-tensor form),
//  - extrapolate-project (eq. extproj_her),
//  - the restart surrogate F-hat from the last block's MTTKRP and Grams (Sec. 3.1.3),
//  - HER state init / restart decision with the beta schedule (Algorithm 2, eqs.
//    HER_eq:beta_update and HER_eq:beta_bar_update) and the post-decision selection,
//  - || T - [[A]] ||^2 from the explicit residual (eq. err_true_def).
// Every reduction has a fixed order (per-block tree, then an ordered sum of partials).
#include "her_update.h"
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kNormBlocks = 1024;
constexpr int kResidBlocks = 1024;

// Sum of a double over a 256-thread block; result valid in thread 0.
__device__ double block_sum(double v) { return block_sum256(v); }

__device__ __forceinline__ float bf16_bits_to_float(uint32_t h) { return __uint_as_float(h << 16); }

__global__ __launch_bounds__(256) void norm2_f32_kernel(const float* __restrict__ x, int64_t n,
                                                        double* partials) {
  double acc = 0.0;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t n4 = n / 4;
  const float4* x4 = reinterpret_cast<const float4*>(x);
  for (int64_t i = tid; i < n4; i += stride) {
    const float4 v = x4[i];
    acc += double(v.x) * v.x + double(v.y) * v.y + double(v.z) * v.z + double(v.w) * v.w;
  }
  for (int64_t i = n4 * 4 + tid; i < n; i += stride) acc += double(x[i]) * x[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void norm2_bf16_kernel(const uint16_t* __restrict__ x,
                                                         int64_t n, double* partials) {
  double acc = 0.0;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t n8 = n / 8;
  const uint4* x8 = reinterpret_cast<const uint4*>(x);
  for (int64_t i = tid; i < n8; i += stride) {
    const uint4 v = x8[i];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double lo = bf16_bits_to_float(w[q] & 0xffffu);
      const double hi = bf16_bits_to_float(w[q] >> 16);
      acc += lo * lo + hi * hi;
    }
  }
  for (int64_t i = n8 * 8 + tid; i < n; i += stride) {
    const double v = bf16_bits_to_float(x[i]);
    acc += v * v;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Ordered sum of `n` partials by one block: thread t sums t, t+256, ...; then a tree.
__device__ double ordered_sum(const double* partials, int64_t n) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += partials[i];
  return block_sum(s);
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* partials, int64_t n,
                                                           double* out) {
  const double s = ordered_sum(partials, n);
  if (threadIdx.x == 0) *out = s;
}

__device__ __forceinline__ uint16_t to_bf16_rne(float f) {
  const uint32_t b = __float_as_uint(f);
  if ((b & 0x7fffffffu) > 0x7f800000u) return uint16_t((b >> 16) | 0x40u);
  return uint16_t((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

__global__ __launch_bounds__(256) void cast_bf16_kernel(const float* __restrict__ src,
                                                        uint16_t* __restrict__ dst, int64_t n) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t n4 = n / 4;
  for (int64_t i = tid; i < n4; i += stride) {
    const float4 v = reinterpret_cast<const float4*>(src)[i];
    uint2 o;
    o.x = uint32_t(to_bf16_rne(v.x)) | (uint32_t(to_bf16_rne(v.y)) << 16);
    o.y = uint32_t(to_bf16_rne(v.z)) | (uint32_t(to_bf16_rne(v.w)) << 16);
    reinterpret_cast<uint2*>(dst)[i] = o;
  }
  for (int64_t i = n4 * 4 + tid; i < n; i += stride) dst[i] = to_bf16_rne(src[i]);
}

__global__ __launch_bounds__(256) void extrapolate_kernel(const float* __restrict__ a_new,
                                                          const float* __restrict__ a_old,
                                                          float* __restrict__ out, int64_t n,
                                                          const double* beta_src, int project) {
  const double beta = *beta_src;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = tid; i < n; i += stride) {
    const double x = a_new[i];
    const double y = x + beta * (x - double(a_old[i]));
    out[i] = float((y > 0.0 || !project) ? y : 0.0);
  }
}

__global__ __launch_bounds__(256) void fill_sentinel_kernel(double* p, int64_t n) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = tid; i < n; i += stride) p[i] = __longlong_as_double(-1ll);
}

__global__ __launch_bounds__(256) void copy_f32_kernel(const float* __restrict__ src,
                                                       float* __restrict__ dst, int64_t n) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = tid; i < n; i += stride) dst[i] = src[i];
}

// Per block: sum over its (row, p) entries of a_ip (2 p_ip - (G a_i)_p), in float64.
// Summed over all entries this is 2 <P, A> - <G, A^T A>.
__global__ __launch_bounds__(256) void error_partials_kernel(const float* __restrict__ P,
                                                             const float* __restrict__ A,
                                                             const double* __restrict__ G,
                                                             int64_t rows, int r,
                                                             double* partials) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double t = 0.0;
  if (e < rows * r) {
    const int64_t i = e / r;
    const int p = int(e - i * r);
    const float* ai = A + i * r;
    double g = 0.0;
    for (int q = 0; q < r; ++q) g += G[int64_t(p) * r + q] * double(ai[q]);
    t = double(ai[p]) * (2.0 * double(P[e]) - g);
  }
  const double s = block_sum(t);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void error_finalize_kernel(const double* normT2,
                                                             const double* partials,
                                                             int64_t nparts, double* fhat,
                                                             uint32_t* flags, double scale) {
  const double s = ordered_sum(partials, nparts);
  if (threadIdx.x == 0) {
    const double f = scale * (*normT2 - s);
    if (!isfinite(f)) flag_set(flags, NTF_FLAG_NONFINITE);
    *fhat = f;
  }
}

// Gradient of the squared-error loss with respect to one factor (Sec. 2, eq. def:grad):
// out[i, p] = alpha * scale * (sum_l A[i, l] G[l, p] - P[i, p]), with G the Hadamard product
// of the other factors' Grams and P the MTTKRP of the factor's mode; float64 accumulation.
__global__ __launch_bounds__(256) void cp_grad_kernel(const float* __restrict__ A,
                                                      const float* __restrict__ P,
                                                      const double* __restrict__ G,
                                                      int64_t rows, int r,
                                                      const double* __restrict__ scale,
                                                      float alpha, float* __restrict__ out) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= rows * r) return;
  const int64_t i = e / r;
  const int p = int(e - i * r);
  const float* ai = A + i * r;
  double g = 0.0;
  for (int l = 0; l < r; ++l) g += double(ai[l]) * G[int64_t(l) * r + p];
  const double f = double(alpha) * (scale ? *scale : 1.0);
  out[e] = float(f * (g - double(P[e])));
}

__global__ void her_init_kernel(ntf_her_state* st, double beta0, int scheme,
                                const double* fhat0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    // scheme 1 keeps omega_1 in beta and h in beta_bar
    st->beta = scheme == 1 ? bro_omega(1, bro_h(0)) : beta0;
    st->beta_bar = scheme == 1 ? bro_h(0) : 1.0;
    st->fhat_prev = *fhat0;
    st->fhat = *fhat0;
    st->k = 0;
    st->restart = 0;
    st->nrestarts = 0;
    st->it = 0;
  }
}

__global__ void reset_call_kernel(ntf_her_state* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->it = 0;
}

__global__ __launch_bounds__(256) void her_decide_kernel(DecideArgs a) {
  double f;
  if (a.partials) {
    const double s = ordered_sum(a.partials, a.nparts);
    f = 0.5 * (*a.normT2 - s);
  } else {
    f = *a.fhat;
  }
  if (threadIdx.x != 0) return;
  her_update(a.st, a.p, f, a.st->fhat_prev, a.trace, a.order, a.sweeps_src, a.fhat_out,
             a.flags);
}

__global__ __launch_bounds__(256) void select_kernel(SelectJob j, const ntf_her_state* st) {
  const bool restart = st->restart != 0;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int b = 0; b < j.nblocks; ++b) {
    const float* src = restart ? j.a_new[b] : j.a_hat[b];
    for (int64_t i = tid; i < j.n[b]; i += stride) j.dst[b][i] = src[i];
    if (j.ddst[b]) {
      const double* dsrc = restart ? j.dnew[b] : j.dhat[b];
      for (int64_t i = tid; i < j.dn[b]; i += stride) j.ddst[b][i] = dsrc[i];
    }
  }
}

// Residual: thread block handles prefixes (all modes but the last) in a fixed pattern.
struct ResidArgs {
  const void* T;
  int dtype;
  FactorPtrs A;
  int order;
  int r;
  int64_t dims[kMaxOrder];
  int64_t nprefix;  // prod of all dims but the last
  int64_t ilast;
  double* partials;
};

__global__ __launch_bounds__(256) void residual_kernel(ResidArgs a) {
  __shared__ double w[kMaxRank];
  double acc = 0.0;
  for (int64_t pre = blockIdx.x; pre < a.nprefix; pre += gridDim.x) {
    // w[p] = prod_{l < N-1} A_l[j_l, p] for this prefix
    for (int p = threadIdx.x; p < a.r; p += blockDim.x) {
      int64_t x = pre;
      double prod = 1.0;
      for (int l = a.order - 2; l >= 0; --l) {
        const int64_t j = x % a.dims[l];
        x /= a.dims[l];
        prod *= double(a.A.p[l][j * a.r + p]);
      }
      w[p] = prod;
    }
    __syncthreads();
    const float* last = a.A.p[a.order - 1];
    for (int64_t j = threadIdx.x; j < a.ilast; j += blockDim.x) {
      double m = 0.0;
      for (int p = 0; p < a.r; ++p) m += w[p] * double(last[j * a.r + p]);
      const int64_t idx = pre * a.ilast + j;
      const double t = a.dtype == NTF_BF16
                           ? double(bf16_bits_to_float(static_cast<const uint16_t*>(a.T)[idx]))
                           : double(static_cast<const float*>(a.T)[idx]);
      const double d = t - m;
      acc += d * d;
    }
    __syncthreads();
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) a.partials[blockIdx.x] = s;
}

int grid_for(int64_t n, int cap = 4096) {
  return int(std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), cap)));
}

}  // namespace

int norm2_partials() { return kNormBlocks; }

hipError_t launch_norm2(const void* data, int dtype, int64_t n, double* partials, double* out,
                        hipStream_t s) {
  if (dtype == NTF_BF16)
    hipLaunchKernelGGL(norm2_bf16_kernel, dim3(kNormBlocks), dim3(256), 0, s,
                       static_cast<const uint16_t*>(data), n, partials);
  else
    hipLaunchKernelGGL(norm2_f32_kernel, dim3(kNormBlocks), dim3(256), 0, s,
                       static_cast<const float*>(data), n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partials,
                     int64_t(kNormBlocks), out);
  return hipGetLastError();
}

hipError_t launch_cast_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(cast_bf16_kernel, dim3(grid_for(n / 4 + 1, 8192)), dim3(256), 0, s, src,
                     dst, n);
  return hipGetLastError();
}

hipError_t launch_extrapolate(const float* a_new, const float* a_old, float* out, int64_t n,
                              const double* beta_src, hipStream_t s, bool project) {
  hipLaunchKernelGGL(extrapolate_kernel, dim3(grid_for(n)), dim3(256), 0, s, a_new, a_old, out,
                     n, beta_src, project ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_fill_sentinel(double* slots, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_sentinel_kernel, dim3(grid_for(n)), dim3(256), 0, s, slots, n);
  return hipGetLastError();
}

hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

int64_t error_partial_count(int64_t rows, int r) { return ceil_div(rows * r, 256); }

hipError_t launch_error_partials(const float* P, const float* A, const double* G, int64_t rows,
                                 int r, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(error_partials_kernel, dim3(unsigned(error_partial_count(rows, r))),
                     dim3(256), 0, s, P, A, G, rows, r, partials);
  return hipGetLastError();
}

hipError_t launch_error_finalize(const double* normT2, const double* partials, int64_t nparts,
                                 double* fhat, uint32_t* flags, hipStream_t s, double scale) {
  hipLaunchKernelGGL(error_finalize_kernel, dim3(1), dim3(256), 0, s, normT2, partials, nparts,
                     fhat, flags, scale);
  return hipGetLastError();
}

hipError_t launch_cp_grad(const float* A, const float* P, const double* G, int64_t rows, int r,
                          const double* scale, float alpha, float* out, hipStream_t s) {
  const int64_t n = rows * r;
  hipLaunchKernelGGL(cp_grad_kernel, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, s, A, P, G,
                     rows, r, scale, alpha, out);
  return hipGetLastError();
}

hipError_t launch_her_init(ntf_her_state* st, const ntf_her_params& p, const double* fhat0,
                           hipStream_t s) {
  hipLaunchKernelGGL(her_init_kernel, dim3(1), dim3(64), 0, s, st, p.beta0, int(p.scheme),
                     fhat0);
  return hipGetLastError();
}

hipError_t launch_reset_call(ntf_her_state* st, hipStream_t s) {
  hipLaunchKernelGGL(reset_call_kernel, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_her_decide(const DecideArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(her_decide_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_select(const SelectJob& j, const ntf_her_state* st, hipStream_t s) {
  int64_t n = 0;
  for (int b = 0; b < j.nblocks; ++b) n = std::max(n, std::max(j.n[b], j.dn[b]));
  hipLaunchKernelGGL(select_kernel, dim3(grid_for(n, 1024)), dim3(256), 0, s, j, st);
  return hipGetLastError();
}

int residual_partials() { return kResidBlocks; }

hipError_t launch_residual(const ntf_tensor& T, const FactorPtrs& A, int r, double* partials,
                           double* out, hipStream_t s) {
  ResidArgs a;
  a.T = T.data;
  a.dtype = T.dtype;
  a.A = A;
  a.order = T.order;
  a.r = r;
  a.nprefix = 1;
  for (int l = 0; l < kMaxOrder; ++l) a.dims[l] = l < T.order ? T.dims[l] : 1;
  for (int l = 0; l < T.order - 1; ++l) a.nprefix *= T.dims[l];
  a.ilast = T.dims[T.order - 1];
  a.partials = partials;
  hipLaunchKernelGGL(residual_kernel, dim3(kResidBlocks), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partials,
                     int64_t(kResidBlocks), out);
  return hipGetLastError();
}

}  // namespace ntf
