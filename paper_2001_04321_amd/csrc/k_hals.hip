// A-HALS block solver (paper Sec. 2.1.4) with the inner stopping rule of Sec. 4.1.
//
// Rows of the block are independent NNLS problems coupled only through the stopping rule.
// A group of L lanes owns one row and C columns per lane (blocked: lane g holds columns
// g*C .. g*C+C-1), W and P of the row live in registers, G in LDS. Column j of a sweep:
//   each lane forms its share of sum_{l != j} W[l] G[l, j], a DPP butterfly sums the
//   group (all lanes end with the same value), and the owner lane sets
//   W[j] = max(0, P[j] - sum) / G[j, j]   (0 if G[j, j] = 0: a dead component).
// Stopping rule: after sweep s every workgroup publishes its share of ||W_s - W_{s-1}||^2
// (float64) in slot (s, wg); the rule for sweep s-1 is evaluated after sweep s has been
// computed, so the cross-workgroup wait overlaps a sweep of work. Every workgroup sums the
// slots in the same order and takes the same decision; when sweep s-1 met the rule the
// workgroup restores its snapshot of W_{s-1}. Waits are bounded by a wall-clock deadline
// (a timeout sets NTF_FLAG_WAIT_TIMEOUT and ends the kernel). The grid never exceeds the
// CU count, so every workgroup can be resident at once.
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kThreads = 256;
constexpr uint64_t kSentinel = ~uint64_t(0);

struct HKArgs {
  const float* W0;
  float* W;
  const float* P;
  const float* G;
  int64_t rows;
  int r;
  int max_sweeps;
  double tol;
  int32_t* sweeps_out;
  uint64_t* slots;
  uint32_t* flags;
  float* A_hat;
  const double* beta_src;
  int nwg;
  uint64_t timeout_ticks;
};

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Sum over aligned groups of L lanes (L <= 16); every lane of a group gets the same bits.
template <int L>
__device__ __forceinline__ float group_sum(float x) {
  if (L >= 2) x += dpp<0xB1>(x);    // quad_perm [1,0,3,2]: partner lane ^ 1
  if (L >= 4) x += dpp<0x4E>(x);    // quad_perm [2,3,0,1]: partner lane ^ 2
  if (L >= 8) x += dpp<0x141>(x);   // row_half_mirror: other quad of the 8
  if (L >= 16) x += dpp<0x140>(x);  // row_mirror: other half of the 16
  return x;
}

// Block-wide float64 sum with a fixed tree; result returned to every thread.
__device__ double block_sum_all(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

template <int L, int C>
__global__ __launch_bounds__(kThreads) void hals_kernel(HKArgs a) {
  constexpr int RPW = kThreads / L;  // rows per workgroup
  constexpr int RP = L * C;          // padded rank
  extern __shared__ float s_g[];     // r rows of RP floats, then r reciprocals
  __shared__ double s_red[4];
  __shared__ int s_timeout;

  const int tid = threadIdx.x;
  const int grp = tid / L;
  const int li = tid % L;
  const int64_t i = int64_t(blockIdx.x) * RPW + grp;
  const bool row_ok = i < a.rows;
  const int r = a.r;
  float* s_inv = s_g + r * RP;

  for (int e = tid; e < r * RP; e += kThreads) {
    const int j = e / RP;
    const int l = e - j * RP;
    s_g[e] = l < r ? a.G[j * r + l] : 0.f;
  }
  for (int j = tid; j < r; j += kThreads) {
    const float g = a.G[j * r + j];
    s_inv[j] = g != 0.f ? 1.f / g : 0.f;
  }
  if (tid == 0) s_timeout = 0;
  __syncthreads();

  float w[C], p[C], w0[C], prev[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int j = li * C + c;
    const bool ok = row_ok && j < r;
    w[c] = ok ? a.W0[i * r + j] : 0.f;
    p[c] = ok ? a.P[i * r + j] : 0.f;
    w0[c] = w[c];
  }

  const int nown = (r + C - 1) / C;  // lanes that own at least one column
  int done = a.max_sweeps;
  double d1 = 0.0;
  const uint64_t t_start = wall_clock64();

  for (int s = 1; s <= a.max_sweeps; ++s) {
#pragma unroll
    for (int c = 0; c < C; ++c) prev[c] = w[c];

#pragma unroll 1
    for (int jo = 0; jo < nown; ++jo) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int j = jo * C + c;
        if (j >= r) break;
        const float* grow = s_g + j * RP + li * C;
        float part = 0.f;
#pragma unroll
        for (int c2 = 0; c2 < C; ++c2) {
          const float wv = (li == jo && c2 == c) ? 0.f : w[c2];
          part = fmaf(wv, grow[c2], part);
        }
        part = group_sum<L>(part);
        if (li == jo) w[c] = fmaxf(p[c] - part, 0.f) * s_inv[j];
      }
    }

    // this workgroup's share of ||W_s - W_{s-1}||_F^2
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const double df = double(w[c]) - double(prev[c]);
      d2 += df * df;
    }
    const double wg_d2 = block_sum_all(d2, s_red);
    if (tid == 0)
      __hip_atomic_store(&a.slots[int64_t(s - 1) * a.nwg + blockIdx.x],
                         uint64_t(__double_as_longlong(wg_d2)), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);

    if (s >= 2) {
      // stopping rule for sweep s-1: wait for every workgroup's slot, sum in wg order
      double v = 0.0;
      if (tid < a.nwg) {
        const uint64_t* slot = &a.slots[int64_t(s - 2) * a.nwg + tid];
        uint64_t bits;
        for (;;) {
          bits = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (bits != kSentinel) break;
          if (wall_clock64() - t_start > a.timeout_ticks) {
            s_timeout = 1;
            bits = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        v = __longlong_as_double(int64_t(bits));
      }
      const double D = block_sum_all(v, s_red);  // includes the barrier for s_timeout
      if (s_timeout) {
        if (tid == 0)
          __hip_atomic_fetch_or(a.flags, NTF_FLAG_WAIT_TIMEOUT, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
        done = s;
        break;
      }
      const double delta = sqrt(D);
      if (s - 1 == 1) d1 = delta;
      if (delta <= a.tol * d1) {
#pragma unroll
        for (int c = 0; c < C; ++c) w[c] = prev[c];
        done = s - 1;
        break;
      }
    }
  }

  if (row_ok) {
    double beta = 0.0;
    if (a.A_hat) beta = *a.beta_src;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = li * C + c;
      if (j < r) {
        a.W[i * r + j] = w[c];
        if (a.A_hat) {
          const double x = w[c];
          const double y = x + beta * (x - double(w0[c]));
          a.A_hat[i * r + j] = float(y > 0.0 ? y : 0.0);
        }
      }
    }
  }
  if (blockIdx.x == 0 && tid == 0 && a.sweeps_out) *a.sweeps_out = done;
}

struct Shape {
  int L, C;
};

Shape hals_shape(int r) {
  if (r <= 64) {
    int L = 1;
    while (L * 4 < r) L *= 2;
    return {L, 4};
  }
  return {16, 8};  // r <= 128
}

using HFn = void (*)(HKArgs);

HFn hals_fn(Shape sh) {
  if (sh.C == 8) return hals_kernel<16, 8>;
  switch (sh.L) {
    case 1: return hals_kernel<1, 4>;
    case 2: return hals_kernel<2, 4>;
    case 4: return hals_kernel<4, 4>;
    case 8: return hals_kernel<8, 4>;
    default: return hals_kernel<16, 4>;
  }
}

int hals_wgs(int64_t rows, int r) {
  const Shape sh = hals_shape(r);
  return int(ceil_div(rows, kThreads / sh.L));
}

}  // namespace

bool hals_supported(int64_t rows, int r, int num_cus) {
  if (r < 1 || r > 128) return false;
  return hals_wgs(rows, r) <= std::min(256, num_cus);
}

int64_t hals_slot_count(int64_t rows, int r, int max_sweeps) {
  return int64_t(hals_wgs(rows, r)) * max_sweeps;
}

hipError_t launch_hals(const HalsArgs& h, int num_cus, hipStream_t s) {
  const Shape sh = hals_shape(h.r);
  HKArgs a;
  a.W0 = h.W0;
  a.W = h.W;
  a.P = h.P;
  a.G = h.G;
  a.rows = h.rows;
  a.r = h.r;
  a.max_sweeps = h.max_sweeps;
  a.tol = h.tol;
  a.sweeps_out = h.sweeps_out;
  a.slots = reinterpret_cast<uint64_t*>(h.slots);
  a.flags = h.flags;
  a.A_hat = h.A_hat;
  a.beta_src = h.beta_src;
  a.nwg = hals_wgs(h.rows, h.r);
  // wall_clock64 runs at the device's wall-clock rate (100 MHz on MI300-class parts);
  // 2 s is far above any legitimate wait.
  static const int rate_khz = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) != hipSuccess || v <= 0)
      v = 100000;
    return v;
  }();
  a.timeout_ticks = uint64_t(rate_khz) * 1000ull * 2ull;
  (void)num_cus;
  const size_t lds = (size_t(h.r) * sh.L * sh.C + h.r) * sizeof(float);
  hipLaunchKernelGGL(hals_fn(sh), dim3(a.nwg), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

}  // namespace ntf
