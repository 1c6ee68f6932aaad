// The paper's comparison algorithms on the GPU, on the same kernels as the HER solver:
//
// * APG (Sec. 2.2.1; Appendix, algorithm APG): outer iteration k, block i with the other
//   blocks' latest values: w = min(w_hat_{k-1}, delta_w sqrt(L_{k-2} / L_{k-1})),
//   A-hat = A_{k-1} + w (A_{k-1} - A_{k-2}), one projected gradient step
//   A_k = max(0, A-hat - (A-hat G - P) / L); when F(A_k) > F(A_{k-1}) the iteration is
//   redone from A_{k-1} without extrapolation.
// * iBPG (Sec. 2.2.2; Appendix, algorithm iBPG): per block a gradient point
//   Y1 = A_cur + w (A_cur - A_prev) and an inertial point Y2 = A_cur + beta w (A_cur - A_prev),
//   A_prev <- A_cur, A_cur <- max(0, Y2 - (Y1 G - P) / L), `inner_steps` times; no restart.
//
// w_hat_{k-1} = (t_{k-1} - 1) / t_k with t_0 = 1, t_k = (1 + sqrt(1 + 4 t_{k-1}^2)) / 2, the
// same for every block of iteration k; L = ||G||_2 of the block's problem (power iteration
// on the device); at k = 1 the ratio L_{k-2} / L_{k-1} is 1; A_{-1} = A_0. The host runs the
// iterations (APG reads F(A_k) back once per iteration to decide its restart); every
// arithmetic step runs in the kernels below or in the MTTKRP, Gram, Lipschitz, gradient
// step and F-hat kernels of the library.
#include <cmath>
#include <vector>

#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kCThreads = 256;

// w = min(w_hat, delta_w sqrt(L_prev / L_cur)); ratio 1 without a previous L
__global__ void comp_weight_kernel(double w_hat, double delta_w, const double* L_prev,
                                   const double* L_cur, double* w) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double lc = *L_cur;
  const double ratio = (L_prev && lc > 0.0) ? *L_prev / lc : 1.0;
  *w = fmin(w_hat, delta_w * sqrt(ratio));
}

// out = a + w (a - a_prev), w = *w_src; no projection (APG's extrapolation point)
__global__ __launch_bounds__(kCThreads) void extrap_dev_kernel(const float* __restrict__ a,
                                                               const float* __restrict__ a_prev,
                                                               float* __restrict__ out,
                                                               int64_t n, const double* w_src) {
  const double w = *w_src;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double x = a[i];
    out[i] = float(x + w * (x - double(a_prev[i])));
  }
}

// iBPG's updates of one block in place on (A_cur, A_prev): thread (row, p) holds both
// values, P[row, p] and column p of G in registers; the row of Y1 is shared in LDS.
template <int RP>
__global__ __launch_bounds__(kCThreads) void ibpg_kernel(float* __restrict__ Acur,
                                                         float* __restrict__ Aprev,
                                                         const float* __restrict__ P,
                                                         const float* __restrict__ G,
                                                         const double* L_src,
                                                         const double* w_src, double beta,
                                                         int64_t rows, int r, int steps) {
  constexpr int RB = kCThreads / RP;
  __shared__ __attribute__((aligned(16))) float s_y[RB][RP];
  const int t = threadIdx.x;
  const int rl = t / RP;
  const int p = t - rl * RP;
  const int64_t row = int64_t(blockIdx.x) * RB + rl;
  const bool live = row < rows && p < r;
  float g[RP];
#pragma unroll
  for (int q = 0; q < RP; ++q) g[q] = G[min(q, r - 1) * r + min(p, r - 1)];
#pragma unroll
  for (int q = 0; q < RP; ++q) g[q] = (q < r && p < r) ? g[q] : 0.f;
  const double L = *L_src;
  const double wd = *w_src;
  const float inv_l = L > 0.0 ? float(1.0 / L) : 0.f;
  const float w = float(wd), bw = float(beta * wd);
  const int64_t ix = live ? row * r + p : 0;
  const float pv0 = P[ix], c0 = Acur[ix], q0 = Aprev[ix];
  const float pv = live ? pv0 : 0.f;
  float ac = live ? c0 : 0.f, ap = live ? q0 : 0.f;
  for (int s = 0; s < steps; ++s) {
    const float d = ac - ap;
    const float y1 = ac + w * d;
    const float y2 = ac + bw * d;
    s_y[rl][p] = y1;
    __syncthreads();
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
    ap = ac;
    ac = L > 0.0 ? fmaxf(0.f, y2 - (acc - pv) * inv_l) : 0.f;
  }
  if (live) {
    Acur[row * r + p] = ac;
    Aprev[row * r + p] = ap;
  }
}

int grid_for(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 4096))); }

hipError_t launch_ibpg(float* Acur, float* Aprev, const float* P, const float* G,
                       const double* L, const double* w, double beta, int64_t rows, int r,
                       int steps, hipStream_t s) {
  const int rp = r <= 32 ? 32 : r <= 64 ? 64 : 128;
  const dim3 grid(unsigned(ceil_div(rows, kCThreads / rp)));
  if (rp == 32)
    hipLaunchKernelGGL(ibpg_kernel<32>, grid, dim3(kCThreads), 0, s, Acur, Aprev, P, G, L, w,
                       beta, rows, r, steps);
  else if (rp == 64)
    hipLaunchKernelGGL(ibpg_kernel<64>, grid, dim3(kCThreads), 0, s, Acur, Aprev, P, G, L, w,
                       beta, rows, r, steps);
  else
    hipLaunchKernelGGL(ibpg_kernel<128>, grid, dim3(kCThreads), 0, s, Acur, Aprev, P, G, L, w,
                       beta, rows, r, steps);
  return hipGetLastError();
}

// Device buffers of one comparator solve, carved from the handle's workspace.
struct CompBufs {
  double* norm_part;
  double* normT2;
  float* A_prev[kMaxOrder];
  float* A_new[kMaxOrder];
  double* gp[kMaxOrder];  // Gram partials of each block's current value
  float* A_hat;
  float* G32;
  double* G64;
  float* P;
  float* mt_part;
  double* L_cur;  // [N]
  double* L_prev; // [N]
  double* w;
  double* err_part;
  double* F;      // [iters + 1]
};

void carve(Arena& ar, CompBufs& b, const ntf_tensor& T, int r, const MttkrpPlan* plans,
           int iters) {
  const int N = T.order;
  const size_t rr = size_t(r) * r;
  b.norm_part = ar.take<double>(norm2_partials());
  b.normT2 = ar.take<double>(1);
  int64_t maxI = 0;
  size_t maxpart = 1;
  for (int n = 0; n < N; ++n) {
    const int64_t I = T.dims[n];
    maxI = std::max(maxI, I);
    b.A_prev[n] = ar.take<float>(size_t(I) * r);
    b.A_new[n] = ar.take<float>(size_t(I) * r);
    b.gp[n] = ar.take<double>(size_t(gram_chunks(I, r)) * rr);
    maxpart = std::max(maxpart, plans[n].partial_floats());
  }
  b.A_hat = ar.take<float>(size_t(maxI) * r);
  b.G32 = ar.take<float>(rr);
  b.G64 = ar.take<double>(rr);
  b.P = ar.take<float>(size_t(maxI) * r);
  b.mt_part = ar.take<float>(maxpart);
  b.L_cur = ar.take<double>(kMaxOrder);
  b.L_prev = ar.take<double>(kMaxOrder);
  b.w = ar.take<double>(1);
  b.err_part = ar.take<double>(size_t(error_partial_count(T.dims[N - 1], r)));
  b.F = ar.take<double>(size_t(iters) + 1);
}

struct Comp {
  const ntf_tensor& T;
  int r;
  int N;
  const MttkrpPlan* plans;
  CompBufs& b;
  hipStream_t s;
  uint32_t* flags;

  // G^(i) (float32 and float64) from the cached Gram partials of the other blocks
  hipError_t gram_of_others(int i) const {
    HadamardJob hj{};
    for (int l = 0; l < N; ++l) {
      if (l == i) continue;
      hj.part[hj.nfac] = b.gp[l];
      hj.nchunks[hj.nfac] = gram_chunks(T.dims[l], r);
      hj.nfac++;
    }
    return launch_hadamard(hj, r, b.G32, b.G64, nullptr, 0, s);
  }
  hipError_t gram_partials(const float* const* A, int first, int count) const {
    GramJob gj{};
    for (int l = first; l < first + count; ++l) {
      gj.A[gj.nfac] = A[l];
      gj.out[gj.nfac] = b.gp[l];
      gj.rows[gj.nfac] = T.dims[l];
      gj.nfac++;
    }
    return launch_gram_partials(gj, r, s);
  }
  hipError_t mttkrp(int i, const float* const* cur) const {
    FactorPtrs fp{};
    for (int l = 0; l < N; ++l) fp.p[l] = cur[l];
    return launch_mttkrp(plans[i], T.data, fp, b.P, b.mt_part, true, s);
  }
  // F of the blocks `cur` from the last block's P and G (the Gram trick of Sec. 3.1.3)
  hipError_t objective(const float* last, double* out) const {
    const int64_t I = T.dims[N - 1];
    hipError_t e = launch_error_partials(b.P, last, b.G64, I, r, b.err_part, s);
    if (e != hipSuccess) return e;
    return launch_error_finalize(b.normT2, b.err_part, error_partial_count(I, r), out, flags, s);
  }
  // one projected gradient step of block i from `from` into `to` with L = L_cur[i]
  hipError_t pg_step(int i, const float* from, float* to) const {
    PgdArgs pa{};
    pa.W0 = from;
    pa.W = to;
    pa.P = b.P;
    pa.G = b.G32;
    pa.L = b.L_cur + i;
    pa.rows = T.dims[i];
    pa.r = r;
    pa.steps = 1;
    return launch_pgd_steps(pa, s);
  }
};

ntf_status prepare(ntf_handle* h, const ntf_tensor* T, int32_t r, float* const* A,
                   int32_t iters, MttkrpPlan* plans, CompBufs& b) {
  ntf_status st = check_tensor(T);
  if (st) return st;
  if ((st = check_rank(r))) return st;
  NTF_RETURN_IF(!A, NTF_EINVAL, "factor array is NULL");
  NTF_RETURN_IF(iters < 0, NTF_EINVAL, "iters < 0");
  NTF_RETURN_IF(r > 128, NTF_EUNSUPPORTED, "gradient kernels support r <= 128");
  for (int n = 0; n < T->order; ++n) NTF_RETURN_IF(!A[n], NTF_EINVAL, "factor %d is NULL", n);
  for (int n = 0; n < T->order; ++n) {
    plans[n] = plan_mttkrp(*T, n, r, h->num_cus, false, tuned_choice(h, *T, n, r));
    NTF_RETURN_IF(plans[n].chunks >= (int64_t(1) << 31), NTF_EUNSUPPORTED, "reduction too long");
  }
  Arena dry;
  carve(dry, b, *T, r, plans, iters);
  if ((st = ensure_workspace(h, dry.off + 256))) return st;
  Arena ar{h->ws, 0};
  carve(ar, b, *T, r, plans, iters);
  return NTF_OK;
}

double t_next(double t) { return 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t)); }

}  // namespace
}  // namespace ntf

using namespace ntf;

#define CK(expr) NTF_HIP(expr)

extern "C" ntf_status ntf_solve_apg(ntf_handle* h, const ntf_tensor* T, int32_t r,
                                    float* const* A, int32_t iters, double delta_w,
                                    double* objective, int32_t* restarts, void* stream) {
  clear_error();
  NTF_RETURN_IF(!h, NTF_EINVAL, "handle is NULL");
  DeviceGuard guard(h->device);
  NTF_RETURN_IF(!guard.ok, NTF_EDEVICE, "cannot select device %d", h->device);
  NTF_RETURN_IF(!(delta_w >= 0.0 && delta_w < 1.0), NTF_EINVAL, "delta_w must lie in [0, 1)");
  MttkrpPlan plans[kMaxOrder];
  CompBufs b{};
  ntf_status st = prepare(h, T, r, A, iters, plans, b);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int N = T->order;
  Comp c{*T, r, N, plans, b, s, h->dev_flags};
  int64_t n_all = 1;
  for (int l = 0; l < N; ++l) n_all *= T->dims[l];
  CK(launch_norm2(T->data, T->dtype, n_all, b.norm_part, b.normT2, s));
  for (int l = 0; l < N; ++l) CK(launch_copy_f32(A[l], b.A_prev[l], T->dims[l] * r, s));
  CK(c.gram_partials(A, 0, N));
  // F(A_0)
  CK(c.gram_of_others(N - 1));
  CK(c.mttkrp(N - 1, A));
  CK(c.objective(A[N - 1], b.F));
  double f_prev = 0.0;
  CK(hipMemcpyAsync(&f_prev, b.F, sizeof(double), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  double t = 1.0;
  bool have_prev = false;
  const float* cur[kMaxOrder];
  for (int k = 0; k < iters; ++k) {
    const double tn = t_next(t);
    const double w_hat = (t - 1.0) / tn;
    for (int l = 0; l < N; ++l) cur[l] = A[l];
    for (int i = 0; i < N; ++i) {
      const int64_t n = T->dims[i] * r;
      CK(c.gram_of_others(i));
      CK(c.mttkrp(i, cur));
      CK(launch_lipschitz(b.G32, r, b.L_cur + i, 0, nullptr, s));
      hipLaunchKernelGGL(comp_weight_kernel, dim3(1), dim3(64), 0, s, w_hat, delta_w,
                         have_prev ? b.L_prev + i : nullptr, b.L_cur + i, b.w);
      CK(hipGetLastError());
      hipLaunchKernelGGL(extrap_dev_kernel, dim3(grid_for(n)), dim3(kCThreads), 0, s, A[i],
                         b.A_prev[i], b.A_hat, n, b.w);
      CK(hipGetLastError());
      CK(c.pg_step(i, b.A_hat, b.A_new[i]));
      CK(c.gram_partials(b.A_new, i, 1));
      cur[i] = b.A_new[i];
    }
    CK(c.objective(b.A_new[N - 1], b.F + k + 1));
    double f = 0.0;
    CK(hipMemcpyAsync(&f, b.F + k + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    const bool restart = f > f_prev;
    if (restart) {
      // redo the iteration from A_{k-1} without extrapolation
      for (int l = 0; l < N; ++l) cur[l] = A[l];
      CK(c.gram_partials(A, 0, N));
      for (int i = 0; i < N; ++i) {
        CK(c.gram_of_others(i));
        CK(c.mttkrp(i, cur));
        CK(launch_lipschitz(b.G32, r, b.L_cur + i, 0, nullptr, s));
        CK(c.pg_step(i, A[i], b.A_new[i]));
        CK(c.gram_partials(b.A_new, i, 1));
        cur[i] = b.A_new[i];
      }
      CK(c.objective(b.A_new[N - 1], b.F + k + 1));
      CK(hipMemcpyAsync(&f, b.F + k + 1, sizeof(double), hipMemcpyDeviceToHost, s));
      CK(hipStreamSynchronize(s));
    }
    // A_{k-2} <- A_{k-1}, A_{k-1} <- A_k (the Gram partials already describe A_k)
    for (int l = 0; l < N; ++l) {
      CK(launch_copy_f32(A[l], b.A_prev[l], T->dims[l] * r, s));
      CK(launch_copy_f32(b.A_new[l], A[l], T->dims[l] * r, s));
    }
    CK(hipMemcpyAsync(b.L_prev, b.L_cur, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    have_prev = true;
    t = tn;
    f_prev = f;
    if (objective) objective[k] = f;
    if (restarts) restarts[k] = restart ? 1 : 0;
  }
  CK(hipStreamSynchronize(s));
  return NTF_OK;
}

extern "C" ntf_status ntf_solve_ibpg(ntf_handle* h, const ntf_tensor* T, int32_t r,
                                     float* const* A, int32_t iters, int32_t inner_steps,
                                     double delta_w, double beta, double* objective,
                                     void* stream) {
  clear_error();
  NTF_RETURN_IF(!h, NTF_EINVAL, "handle is NULL");
  DeviceGuard guard(h->device);
  NTF_RETURN_IF(!guard.ok, NTF_EDEVICE, "cannot select device %d", h->device);
  NTF_RETURN_IF(!(delta_w >= 0.0 && delta_w < 1.0), NTF_EINVAL, "delta_w must lie in [0, 1)");
  NTF_RETURN_IF(!(beta >= 0.0 && std::isfinite(beta)), NTF_EINVAL, "beta must be >= 0");
  NTF_RETURN_IF(inner_steps < 1 || inner_steps > kMaxSweeps, NTF_EINVAL,
                "inner_steps outside [1, %d]", kMaxSweeps);
  MttkrpPlan plans[kMaxOrder];
  CompBufs b{};
  ntf_status st = prepare(h, T, r, A, iters, plans, b);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int N = T->order;
  Comp c{*T, r, N, plans, b, s, h->dev_flags};
  int64_t n_all = 1;
  for (int l = 0; l < N; ++l) n_all *= T->dims[l];
  CK(launch_norm2(T->data, T->dtype, n_all, b.norm_part, b.normT2, s));
  for (int l = 0; l < N; ++l) CK(launch_copy_f32(A[l], b.A_prev[l], T->dims[l] * r, s));
  CK(c.gram_partials(A, 0, N));
  double t = 1.0;
  for (int k = 0; k < iters; ++k) {
    const double tn = t_next(t);
    const double w_hat = (t - 1.0) / tn;
    for (int i = 0; i < N; ++i) {
      CK(c.gram_of_others(i));
      CK(c.mttkrp(i, A));
      CK(launch_lipschitz(b.G32, r, b.L_cur + i, 0, nullptr, s));
      hipLaunchKernelGGL(comp_weight_kernel, dim3(1), dim3(64), 0, s, w_hat, delta_w,
                         k > 0 ? b.L_prev + i : nullptr, b.L_cur + i, b.w);
      CK(hipGetLastError());
      CK(launch_ibpg(A[i], b.A_prev[i], b.P, b.G32, b.L_cur + i, b.w, beta, T->dims[i], r,
                     inner_steps, s));
      CK(c.gram_partials(A, i, 1));
    }
    CK(c.objective(A[N - 1], b.F + k + 1));
    CK(hipMemcpyAsync(b.L_prev, b.L_cur, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    t = tn;
  }
  if (objective && iters > 0)
    CK(hipMemcpyAsync(objective, b.F + 1, sizeof(double) * iters, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  return NTF_OK;
}
