// HER restart decision and extrapolation-weight schedule (Algorithm 2; eqs.
// HER_eq:beta_update and HER_eq:beta_bar_update), and Bro's sequence in the block-wise form
// of Sec. 3.3. Shared by the decision kernel and by the A-HALS launch of the last block,
// which takes the decision in its own epilogue: both sum the F-hat shares with the same
// 256-thread fixed-order reduction, so both give the same bits.
#pragma once

#include "ntf_internal.h"

namespace ntf {

// Bro's sequence: omega for outer iteration k after `nrestarts` increases of the error;
// h = 3 grows by one every fifth increase, and no extrapolation happens before iteration 5.
__device__ inline double bro_h(int nrestarts) { return 3.0 + double(nrestarts / 5); }
__device__ inline double bro_omega(int64_t k, double h) {
  return k < 5 ? 0.0 : pow(double(k), 1.0 / h) - 1.0;
}

__device__ inline void flag_set(uint32_t* flags, uint32_t bit) {
  if (flags) __hip_atomic_fetch_or(flags, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of a double over a 256-thread block in a fixed order (each wave by shuffles, then the
// four waves in order); the result is valid in thread 0. Every thread must call it.
__device__ inline double block_sum256(double v) {
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return s;
}

// Algorithm 2: restart when F-hat_k > F-hat_{k-1}; a non-finite F-hat also discards the
// extrapolated sequence.
__device__ inline bool her_restart(double f, double fhat_prev) {
  return !isfinite(f) || f > fhat_prev;
}

// The state update after the test (one thread): beta schedule, restart count, the reference
// F-hat of the next test, the trace record of this iteration. `fhat_prev` is the value the
// test used (read before any thread could have written the state).
__device__ inline void her_update(ntf_her_state* st, const ntf_her_params& p, double f,
                                  double fhat_prev, const ntf_trace& trace, int order,
                                  const int32_t* sweeps_src, double* fhat_out,
                                  uint32_t* flags) {
  const bool finite = isfinite(f);
  if (!finite) flag_set(flags, NTF_FLAG_NONFINITE);
  const bool restart = her_restart(f, fhat_prev);
  const double beta = st->beta;
  const double beta_bar = st->beta_bar;
  if (p.scheme == 1) {
    // Bro: the next iteration's omega from its index and the increases so far
    const int nr = st->nrestarts + (restart ? 1 : 0);
    const double h = bro_h(nr);
    st->beta = bro_omega(st->k + 2, h);
    st->beta_bar = h;
  } else if (restart) {
    st->beta_bar = beta;
    st->beta = beta / p.eta;
  } else {
    st->beta = fmin(beta_bar, p.gamma * beta);
    st->beta_bar = fmin(1.0, p.gamma_bar * beta_bar);
  }
  st->restart = restart ? 1 : 0;
  st->nrestarts += restart ? 1 : 0;
  // a non-finite F-hat is not a reference for the next test (f > NaN is false, which
  // would accept the next extrapolation unconditionally): the last finite value stays
  if (finite) st->fhat_prev = f;
  st->fhat = f;
  st->k += 1;
  const int64_t it = st->it;
  if (trace.fhat) trace.fhat[it] = f;
  if (trace.beta) trace.beta[it] = st->beta;
  if (trace.beta_bar) trace.beta_bar[it] = st->beta_bar;
  if (trace.restart) trace.restart[it] = restart ? 1 : 0;
  if (trace.sweeps && sweeps_src)
    for (int n = 0; n < order; ++n) trace.sweeps[it * order + n] = sweeps_src[n];
  if (fhat_out) *fhat_out = f;
  st->it = it + 1;
}

}  // namespace ntf
