// A-HALS block solver (paper Sec. 2.1.4) with the inner stopping rule of Sec. 4.1, fused
// with what surrounds it in an outer iteration of Algorithm 2.
//
// Rows of the block are independent NNLS problems coupled only through the stopping rule.
// A group of RPAD lanes (16 or 64) owns one row; lane g holds columns g, g + RPAD, ... The
// column update W_j = max(0, P_j - sum_{l != j} W_l G_lj) / G_jj is computed from
//   q_k = P_k / G_kk - sum_{l != k} W_l (G_lk / G_kk)   (W_j <- max(0, q_j))
// kept as the step z_k = q_k - W_k: the change of column j is delta = max(z_j, -W_j), and
// then z_k -= delta G_jk / G_kk for k != j and z_j -= delta. With the scaled table
// S_jk = -G_jk / G_kk (k != j), S_jj = -1, both are one multiply-add z_k += delta S_jk, so a
// column costs a max and a broadcast multiply-add on its critical path. z is kept current
// across sweeps and formed from scratch (z = P / diag(G) + W S) every kRefresh sweeps. A
// dead component (G_jj = 0) has an all-zero column in S and z_j = W_j = 0, so it stays 0,
// as the method prescribes. The rank is padded to a compile-time multiple of 8 with zero
// columns, whose updates are 0.
//
// Stopping rule: a fourth wave of each workgroup runs it while three waves sweep (so it has
// a SIMD of its own and takes no issue cycles from a row wave). It sums the row waves'
// shares of ||W_s - W_{s-1}||^2 (float64, fixed order), publishes the workgroup's share,
// sums every workgroup's shares in a fixed order (so every workgroup takes the same
// decision) and posts the decisions in LDS. Row waves run up to `lag` sweeps past the last
// decision, keeping those iterates in an LDS ring, and restore the iterate of the sweep
// the rule stops at. Waits are bounded by a wall-clock deadline
// (timeout: NTF_FLAG_WAIT_TIMEOUT). The grid never exceeds the CU count, so all
// workgroups are resident together.
//
// Fused around the sweeps (each optional):
//  - epilogue: extrapolation A_hat = max(0, W + beta (W - W_0)) (eq. extproj_her), the
//    float64 partial Grams of the new and extrapolated rows (Gram cache of the solver), and
//    the workgroup's share of 2 <P, W> - <G, W^T W> for the restart surrogate F-hat;
//  - the outer iteration's HER decision (Algorithm 2, last block): every workgroup reads
//    every share, forms F-hat in the decision kernel's order, applies the restart test and
//    writes its part of the survivor selection; workgroup 0 updates the state.
#include "gram_chunk.h"
#include "her_update.h"
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kWaves = kHalsRowWaves;      // waves that own rows
constexpr int kCT = 64 * kWaves;           // their threads
constexpr int kThreads = kCT + 64;         // plus one wave that runs the stopping rule
constexpr int kMaxLag = 16;                // sweeps the row waves may run ahead of a decision
constexpr int kRefresh = 4;  // sweeps between exact recomputations of q
constexpr uint64_t kSentinel = ~uint64_t(0);

struct HKArgs {
  const float* W0;
  float* W;
  const float* P;        // rows x r
  const float* G;        // r x r float32
  const double* G64;     // r x r float64 (for the F-hat share)
  int64_t rows;
  int r;
  int max_sweeps;
  double tol;
  int32_t* sweeps_out;
  uint64_t* slots;
  uint32_t* flags;
  float* A_hat;
  const double* beta_src;
  int project;
  double* gp_new;
  double* gp_hat;
  double* err_part;
  int nwg;
  int lag;                 // sweeps the row waves may run ahead of the last decision
  uint64_t timeout_ticks;
  // fused decision of the outer iteration (null st: none)
  ntf_her_state* st;
  ntf_her_params hp;
  const double* normT2;
  ntf_trace trace;
  int order;
  const int32_t* sweeps_src;
  SelectJob sel;
};

// dst[i] = src[i] for i = t0, t0 + stride, ... < n, eight loads in flight per thread
template <typename T>
__device__ __forceinline__ void copy_strided(T* dst, const T* src, int64_t n, int64_t t0,
                                             int64_t stride) {
  for (int64_t i0 = t0; i0 < n; i0 += 8 * stride) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = i0 + u * stride;
      v[u] = i < n ? src[i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n) dst[i] = v[u];
    }
  }
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp64(double x) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((int64_t(hi) << 32) | uint32_t(lo));
}

__device__ __forceinline__ double readlane64(double x, int lane) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffff), lane);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
  return __longlong_as_double((int64_t(hi) << 32) | uint32_t(lo));
}

// Sum over aligned groups of L lanes (L <= 16); every lane of a group gets the same bits.
template <int L>
__device__ __forceinline__ float group_sum(float x) {
  if (L >= 2) x += dpp<0xB1>(x);    // quad_perm [1,0,3,2]: partner lane ^ 1
  if (L >= 4) x += dpp<0x4E>(x);    // quad_perm [2,3,0,1]: partner lane ^ 2
  if (L >= 8) x += dpp<0x141>(x);   // row_half_mirror: the other quad of the 8
  if (L >= 16) x += dpp<0x140>(x);  // row_mirror: the other 8 of the 16
  return x;
}

// Wave-wide float64 sum in a fixed order (rows of 16 by DPP, then the 4 rows).
__device__ __forceinline__ double wave_sum64(double x) {
  x += dpp64<0xB1>(x);
  x += dpp64<0x4E>(x);
  x += dpp64<0x141>(x);
  x += dpp64<0x140>(x);
  return (readlane64(x, 0) + readlane64(x, 16)) + (readlane64(x, 32) + readlane64(x, 48));
}

// Broadcast lane `o` of each aligned group of G lanes (G = 16: DPP row_newbcast; G = 64:
// readlane) to the whole group; `o` must be a compile-time constant after unrolling.
template <int G>
__device__ __forceinline__ float bcast(float x, int o) {
  if (G == 16) {
    int v = 0;
    switch (o) {
#define NTF_BC(n) \
  case n: v = __builtin_amdgcn_mov_dpp(__float_as_int(x), 0x150 + n, 0xF, 0xF, true); break;
      NTF_BC(0) NTF_BC(1) NTF_BC(2) NTF_BC(3) NTF_BC(4) NTF_BC(5) NTF_BC(6) NTF_BC(7)
      NTF_BC(8) NTF_BC(9) NTF_BC(10) NTF_BC(11) NTF_BC(12) NTF_BC(13) NTF_BC(14) NTF_BC(15)
#undef NTF_BC
    }
    return __int_as_float(v);
  }
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), o));
}

// Workgroup barrier that orders LDS accesses only: global stores issued before it may still
// be in flight (__syncthreads would wait for them too).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Column steps for 16-lane row groups, in the step form described at the top:
//   d = max(z_cs, -w); w += f_o d; z_c += bcast_o(d) g_c for each slot c,
// where slot cs holds the column, bcast_o is lane o of each 16-lane row (a DPP operand of
// v_fmac_f32) and f_o is 1 on the lanes that hold column o, else 0. Written out because the
// compiler neither folds a DPP broadcast into a multiply-add nor keeps the owner select off
// the scalar unit. With two slots (C = 2) the update of the slot that the next column does
// not read is deferred into the next column's step, so a column is four VALU instructions
// and the critical path is the max and one multiply-add: the deferred update and the w
// update fill the two wait states a DPP read of the freshly written d needs. Per element
// the updates keep the column order, so the results do not depend on the deferral.
// Eight columns (one block of G) form one asm statement: between two statements where the
// second reads what the first wrote, the compiler inserts a wait state of its own.
//
// Operands of a block starting at column J0 (t = 0..7, column j = J0 + t, o = j mod 16):
// zc / zo the slot of the block's columns and the other one, w that slot's iterate entries,
// d0 / d1 the changes of even / odd t, dp and gp the previous column's change and the
// coefficient of its deferred update, gi_t the coefficient of column t's immediate update,
// gd_t that of its deferred one, f_t its owner flag, n_t = o and p_t = (j - 1) mod 16.
#define NTF_BC(x) " row_newbcast:%[" #x "] row_mask:0xf bank_mask:0xf bound_ctrl:1"
// first column of a sweep, and every column of a one-slot sweep: nothing deferred; the w
// update and an s_nop fill the two wait states
#define NTF_C16F(t, dc)                                   \
  "v_max_f32_e64 %[" #dc "], %[zc], -%[w]\n\t"            \
  "v_fmac_f32_e32 %[w], %[" #dc "], %[f" #t "]\n\t"       \
  "s_nop 0\n\t"                                           \
  "v_fmac_f32_dpp %[zc], %[" #dc "], %[gi" #t "]" NTF_BC(n##t) "\n\t"
// next column in the same slot (deferred update of the previous column into zo)
#define NTF_C16S(t, dc, dpr, gpr)                                        \
  "v_max_f32_e64 %[" #dc "], %[zc], -%[w]\n\t"                           \
  "v_fmac_f32_dpp %[zo], %[" #dpr "], %[" #gpr "]" NTF_BC(p##t) "\n\t"   \
  "v_fmac_f32_e32 %[w], %[" #dc "], %[f" #t "]\n\t"                      \
  "v_fmac_f32_dpp %[zc], %[" #dc "], %[gi" #t "]" NTF_BC(n##t) "\n\t"
// next column in the other slot: the immediate update goes to zo, the deferred one (of zc)
// to the next block
#define NTF_C16X(t, dc, dpr, gpr)                                        \
  "v_max_f32_e64 %[" #dc "], %[zc], -%[w]\n\t"                           \
  "v_fmac_f32_dpp %[zo], %[" #dpr "], %[" #gpr "]" NTF_BC(p##t) "\n\t"   \
  "v_fmac_f32_e32 %[w], %[" #dc "], %[f" #t "]\n\t"                      \
  "v_fmac_f32_dpp %[zo], %[" #dc "], %[gi" #t "]" NTF_BC(n##t) "\n\t"
#define NTF_GI(g) [gi0] "v"(g[0]), [gi1] "v"(g[1]), [gi2] "v"(g[2]), [gi3] "v"(g[3]), \
                  [gi4] "v"(g[4]), [gi5] "v"(g[5]), [gi6] "v"(g[6]), [gi7] "v"(g[7])
#define NTF_GD(g) [gd0] "v"(g[0]), [gd1] "v"(g[1]), [gd2] "v"(g[2]), [gd3] "v"(g[3]), \
                  [gd4] "v"(g[4]), [gd5] "v"(g[5]), [gd6] "v"(g[6])
#define NTF_FL(f) [f0] "v"(f[0]), [f1] "v"(f[1]), [f2] "v"(f[2]), [f3] "v"(f[3]), \
                  [f4] "v"(f[4]), [f5] "v"(f[5]), [f6] "v"(f[6]), [f7] "v"(f[7])
#define NTF_IMM(c, J, k)                                                            \
  [c##0] "i"((J + 0 - k) & 15), [c##1] "i"((J + 1 - k) & 15), [c##2] "i"((J + 2 - k) & 15), \
  [c##3] "i"((J + 3 - k) & 15), [c##4] "i"((J + 4 - k) & 15), [c##5] "i"((J + 5 - k) & 15), \
  [c##6] "i"((J + 6 - k) & 15), [c##7] "i"((J + 7 - k) & 15)

// One-slot block (C = 1): columns J0 .. J0 + 7 of zc / w.
template <int J0>
__device__ __forceinline__ void blk16_one(float& zc, float& w, const float (&gi)[8],
                                          const float (&f)[8]) {
  float d0, d1;
  asm volatile(NTF_C16F(0, d0) NTF_C16F(1, d1) NTF_C16F(2, d0) NTF_C16F(3, d1)
               NTF_C16F(4, d0) NTF_C16F(5, d1) NTF_C16F(6, d0) NTF_C16F(7, d1)
               : [zc] "+v"(zc), [w] "+v"(w), [d0] "=&v"(d0), [d1] "=&v"(d1)
               : NTF_GI(gi), NTF_FL(f), NTF_IMM(n, J0, 0));
}
// Two-slot block (C = 2): columns J0 .. J0 + 7 (all in slot zc); SW: the column after the
// block is in the other slot. dp / gp carry the deferred update in and out.
template <int J0, bool SW>
__device__ __forceinline__ void blk16_two(float& zc, float& zo, float& w, float& dp, float& gp,
                                          const float (&gi)[8], const float (&gd)[8],
                                          const float (&f)[8]) {
  float d0, d1;
  if constexpr (J0 == 0) {
    static_assert(!SW, "a block of eight starts every slot");
    asm volatile(NTF_C16F(0, d0) NTF_C16S(1, d1, d0, gd0) NTF_C16S(2, d0, d1, gd1)
                 NTF_C16S(3, d1, d0, gd2) NTF_C16S(4, d0, d1, gd3) NTF_C16S(5, d1, d0, gd4)
                 NTF_C16S(6, d0, d1, gd5) NTF_C16S(7, d1, d0, gd6)
                 : [zc] "+v"(zc), [zo] "+v"(zo), [w] "+v"(w), [d0] "=&v"(d0), [d1] "=&v"(d1)
                 : NTF_GI(gi), NTF_GD(gd), NTF_FL(f), NTF_IMM(n, J0, 0), NTF_IMM(p, J0, 1));
  } else if constexpr (!SW) {
    asm volatile(NTF_C16S(0, d0, dp, gp) NTF_C16S(1, d1, d0, gd0) NTF_C16S(2, d0, d1, gd1)
                 NTF_C16S(3, d1, d0, gd2) NTF_C16S(4, d0, d1, gd3) NTF_C16S(5, d1, d0, gd4)
                 NTF_C16S(6, d0, d1, gd5) NTF_C16S(7, d1, d0, gd6)
                 : [zc] "+v"(zc), [zo] "+v"(zo), [w] "+v"(w), [d0] "=&v"(d0), [d1] "=&v"(d1)
                 : [dp] "v"(dp), [gp] "v"(gp), NTF_GI(gi), NTF_GD(gd), NTF_FL(f),
                   NTF_IMM(n, J0, 0), NTF_IMM(p, J0, 1));
  } else {
    asm volatile(NTF_C16S(0, d0, dp, gp) NTF_C16S(1, d1, d0, gd0) NTF_C16S(2, d0, d1, gd1)
                 NTF_C16S(3, d1, d0, gd2) NTF_C16S(4, d0, d1, gd3) NTF_C16S(5, d1, d0, gd4)
                 NTF_C16S(6, d0, d1, gd5) NTF_C16X(7, d1, d0, gd6)
                 : [zc] "+v"(zc), [zo] "+v"(zo), [w] "+v"(w), [d0] "=&v"(d0), [d1] "=&v"(d1)
                 : [dp] "v"(dp), [gp] "v"(gp), NTF_GI(gi), NTF_GD(gd), NTF_FL(f),
                   NTF_IMM(n, J0, 0), NTF_IMM(p, J0, 1));
  }
  dp = d1;
  gp = gd[7];
}
// the update deferred from the last column of a sweep
template <int P>
__device__ __forceinline__ void col_flush(float& zo, float dp, float gp) {
  asm volatile("v_fmac_f32_dpp %[zo], %[dp], %[gp]" NTF_BC(p)
               : [zo] "+v"(zo)
               : [dp] "v"(dp), [gp] "v"(gp), [p] "i"(P));
}

// Column steps for 64-lane row groups (one slot): the owner's change d reaches the row
// through v_readlane (a scalar operand of the multiply-add z += d_o g); the owner's own w
// takes it one column later, deferred into the next step, as a multiply-add with the 0/1
// flag of its lane within its 16-lane row, written to that row only (DPP row mask,
// identity permutation). The critical path is the max, the read-lane and one multiply-add;
// the deferred update fills the wait state between the max and the read-lane. Operands of
// a block at J0: g_t the coefficient of column t, f_t / m_t the flag and row mask of the
// previous column's owner, o_t = J0 + t.
#define NTF_ROW(x) " quad_perm:[0,1,2,3] row_mask:%[" #x "] bank_mask:0xf"
#define NTF_C64F(t, dc)                                   \
  "v_max_f32_e64 %[" #dc "], %[z], -%[w]\n\t"             \
  "s_nop 0\n\t"                                           \
  "v_readlane_b32 %[s], %[" #dc "], %[o" #t "]\n\t"       \
  "v_fmac_f32_e32 %[z], %[s], %[g" #t "]\n\t"
#define NTF_C64(t, dc, dpr)                                              \
  "v_max_f32_e64 %[" #dc "], %[z], -%[w]\n\t"                            \
  "v_fmac_f32_dpp %[w], %[" #dpr "], %[f" #t "]" NTF_ROW(m##t) "\n\t"    \
  "v_readlane_b32 %[s], %[" #dc "], %[o" #t "]\n\t"                      \
  "v_fmac_f32_e32 %[z], %[s], %[g" #t "]\n\t"
#define NTF_G64(g) [g0] "v"(g[0]), [g1] "v"(g[1]), [g2] "v"(g[2]), [g3] "v"(g[3]), \
                   [g4] "v"(g[4]), [g5] "v"(g[5]), [g6] "v"(g[6]), [g7] "v"(g[7])
#define NTF_LANES(J)                                                                     \
  [o0] "i"(J + 0), [o1] "i"(J + 1), [o2] "i"(J + 2), [o3] "i"(J + 3), [o4] "i"(J + 4), \
  [o5] "i"(J + 5), [o6] "i"(J + 6), [o7] "i"(J + 7)
#define NTF_RM(J)                                                                     \
  [m0] "i"(1 << (((J + 63) & 63) / 16)), [m1] "i"(1 << ((J + 0) / 16)),               \
  [m2] "i"(1 << ((J + 1) / 16)), [m3] "i"(1 << ((J + 2) / 16)), [m4] "i"(1 << ((J + 3) / 16)), \
  [m5] "i"(1 << ((J + 4) / 16)), [m6] "i"(1 << ((J + 5) / 16)), [m7] "i"(1 << ((J + 6) / 16))
template <int J0>
__device__ __forceinline__ void blk64(float& z, float& w, float& dp, const float (&g)[8],
                                      const float (&f)[8]) {
  float d0, d1;
  int s;
  if constexpr (J0 == 0) {
    asm volatile(NTF_C64F(0, d0) NTF_C64(1, d1, d0) NTF_C64(2, d0, d1) NTF_C64(3, d1, d0)
                 NTF_C64(4, d0, d1) NTF_C64(5, d1, d0) NTF_C64(6, d0, d1) NTF_C64(7, d1, d0)
                 : [z] "+v"(z), [w] "+v"(w), [d0] "=&v"(d0), [d1] "=&v"(d1), [s] "=&s"(s)
                 : NTF_G64(g), NTF_FL(f), NTF_LANES(J0), NTF_RM(J0));
  } else {
    asm volatile(NTF_C64(0, d0, dp) NTF_C64(1, d1, d0) NTF_C64(2, d0, d1) NTF_C64(3, d1, d0)
                 NTF_C64(4, d0, d1) NTF_C64(5, d1, d0) NTF_C64(6, d0, d1) NTF_C64(7, d1, d0)
                 : [z] "+v"(z), [w] "+v"(w), [d0] "=&v"(d0), [d1] "=&v"(d1), [s] "=&s"(s)
                 : [dp] "v"(dp), NTF_G64(g), NTF_FL(f), NTF_LANES(J0), NTF_RM(J0));
  }
  dp = d1;
}
// the owner update deferred from the last column P of a sweep (its d was written three
// instructions before the end of the block, so the DPP read needs no wait state)
template <int P>
__device__ __forceinline__ void col64_flush(float& w, float dp, float fp) {
  asm volatile("v_fmac_f32_dpp %[w], %[dp], %[fp]" NTF_ROW(pm)
               : [w] "+v"(w)
               : [dp] "v"(dp), [fp] "v"(fp), [pm] "i"(1 << (P / 16)));
}
#undef NTF_ROW
#undef NTF_C64F
#undef NTF_C64
#undef NTF_G64
#undef NTF_LANES
#undef NTF_RM
#undef NTF_C16F
#undef NTF_C16S
#undef NTF_C16X
#undef NTF_GI
#undef NTF_GD
#undef NTF_FL
#undef NTF_IMM
// refresh terms of columns J0 .. J0 + 7 (one slot of w): a_c += bcast_o(w) g_c (w is not
// written during the refresh, so its DPP reads need no wait states)
#define NTF_R1(t) "v_fmac_f32_dpp %[a0], %[w], %[g" #t "]" NTF_BC(n##t) "\n\t"
#define NTF_R2(t) NTF_R1(t) "v_fmac_f32_dpp %[a1], %[w], %[h" #t "]" NTF_BC(n##t) "\n\t"
#define NTF_G8(c, g) [c##0] "v"(g[0]), [c##1] "v"(g[1]), [c##2] "v"(g[2]), [c##3] "v"(g[3]), \
                     [c##4] "v"(g[4]), [c##5] "v"(g[5]), [c##6] "v"(g[6]), [c##7] "v"(g[7])
#define NTF_N8(J) [n0] "i"((J + 0) & 15), [n1] "i"((J + 1) & 15), [n2] "i"((J + 2) & 15), \
                  [n3] "i"((J + 3) & 15), [n4] "i"((J + 4) & 15), [n5] "i"((J + 5) & 15), \
                  [n6] "i"((J + 6) & 15), [n7] "i"((J + 7) & 15)
template <int J0>
__device__ __forceinline__ void acc_blk2(float& a0, float& a1, float w, const float (&g)[8],
                                         const float (&h)[8]) {
  asm volatile(NTF_R2(0) NTF_R2(1) NTF_R2(2) NTF_R2(3) NTF_R2(4) NTF_R2(5) NTF_R2(6) NTF_R2(7)
               : [a0] "+v"(a0), [a1] "+v"(a1)
               : [w] "v"(w), NTF_G8(g, g), NTF_G8(h, h), NTF_N8(J0));
}
template <int J0>
__device__ __forceinline__ void acc_blk1(float& a0, float w, const float (&g)[8]) {
  asm volatile(NTF_R1(0) NTF_R1(1) NTF_R1(2) NTF_R1(3) NTF_R1(4) NTF_R1(5) NTF_R1(6) NTF_R1(7)
               : [a0] "+v"(a0)
               : [w] "v"(w), NTF_G8(g, g), NTF_N8(J0));
}
#undef NTF_R1
#undef NTF_R2
#undef NTF_G8
#undef NTF_N8
#undef NTF_BC

// f(std::integral_constant<int, J>()) for J = B .. E - 1, in order
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>());
    static_for<B + 1, E>(f);
  }
}

// RPAD lanes per row group (16: four groups per wave; 64: one per wave), C columns per
// lane, NR rows per group processed in lockstep, NB blocks of 8 columns swept (8 NB >= r).
template <int RPAD, int C, int NR, int NB>
__global__ __launch_bounds__(kThreads) void hals_kernel(HKArgs a) {
  constexpr int GPW = 64 / RPAD;        // row groups per wave
  constexpr int RPWV = GPW * NR;        // rows per wave
  constexpr int WPG = kWaves;           // waves that own rows
  constexpr int RPW = WPG * RPWV;       // rows per workgroup
  constexpr int RMAX = RPAD * C;        // columns held per row group
  constexpr int RB = NB * 8;            // columns swept
  static_assert(RB <= RMAX, "column blocks exceed the row group");
  // scaled G in registers when it fits, else read from LDS in blocks of 8 columns
  constexpr bool GREG = RB * C <= 64;
  extern __shared__ __attribute__((aligned(16))) float smem[];
  __shared__ double s_part[WPG + 1];  // epilogue: per-wave F-hat shares
  // rule wave -> row waves: last sweep decided, and the sweep the rule stops at (0: none,
  // -1: a wait timed out)
  __shared__ int s_decided;
  __shared__ int s_stop;

  const int r = a.r;
  float* s_g = smem;               // scaled G, RB x RMAX: s_g[j][k] = S_jk (see above)
  float* s_rows = s_g + RB * RMAX;    // RPW x r: P block, then new rows
  float* s_rows2 = s_rows + RPW * r;  // RPW x r: extrapolated rows (ring follows)

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
  const int gl = lane % RPAD;      // lane within its row group
  const int gi = lane / RPAD;      // row group within the wave
  const int64_t row0 = int64_t(blockIdx.x) * RPW;
  const int nrows = int(std::min<int64_t>(RPW, a.rows - row0));

  if (tid == 0) {
    s_decided = 0;
    s_stop = 0;
  }
  // global loads that do not depend on LDS go out first: this lane's W0 entries and diag(G)
  int lrow[NR];
  bool rok[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    lrow[q] = wave * RPWV + q * GPW + gi;
    rok[q] = wave < WPG && lrow[q] < nrows;  // the rule wave owns no rows
  }
  float w0[NR][C], ginv[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int k = c * RPAD + gl;
    const float gkk = k < r ? a.G[k * r + k] : 0.f;
    ginv[c] = gkk != 0.f ? 1.f / gkk : 0.f;
#pragma unroll
    for (int q = 0; q < NR; ++q)
      w0[q][c] = (rok[q] && k < r) ? a.W0[(row0 + lrow[q]) * r + k] : 0.f;
  }
  // LDS beyond the two row blocks: the iterate ring and the share slots of the stopping
  // rule (see below)
  const int S = a.max_sweeps;
  const int L = a.lag;
  const int R = L + 1;  // ring slots (iterates)
  const int K = L + 2;  // share slots
  float* s_ring = s_rows2 + RPW * r;                                       // [R][NR*C][kCT]
  // [K][kCT], at the 16-byte aligned end of the float area (as the host sizes it)
  double* s_sh = reinterpret_cast<double*>(
      reinterpret_cast<char*>(smem) +
      align_up((size_t(RB) * RMAX + 2 * size_t(RPW) * r + size_t(R) * NR * C * kCT) * sizeof(float),
               16));

  // setup: the scaled G table and this workgroup's P block (rows row0 .. row0+nrows-1,
  // contiguous in memory), in batches whose loads are all in flight before any is used;
  // the first batches of both go out together
  // loads per thread and batch: the whole table in one batch up to r = 64
  constexpr int kB = RB * RMAX > 8 * kThreads ? 16 : 8;
  static_assert(kThreads % RMAX == 0, "a thread's entries share one column k");
  const int np = nrows * r;
  const float* Pb = a.P + row0 * r;
  const int kcol = tid % RMAX;  // the column of every table entry this thread writes
  // G's address in vector registers (the loads are per lane anyway): short of scalar
  // registers, the compiler would reload it from the kernel arguments before every load of
  // the batch, each reload waited for
  const float* Gv = a.G;
  asm volatile("" : "+v"(Gv));
  const float gdk = kcol < r ? Gv[kcol * r + kcol] : 0.f;
  const float ginvk = gdk != 0.f ? 1.f / gdk : 0.f;  // one division per thread
  // the batches tile the table exactly (no entry past its end) when this holds
  constexpr bool kFull = (RB * RMAX) % (kB * kThreads) == 0;
  // loads at clamped (in-range) indexes and selects instead of branches around them
  auto g_load = [&](int base, float (&gv)[kB]) {
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int e = base + i * kThreads + tid;
      const int j = e / RMAX;
      const bool ok = (kFull || e < RB * RMAX) && j < r && kcol < r;
      const float x = Gv[min(j, r - 1) * r + min(kcol, r - 1)];
      gv[i] = ok ? x : 0.f;
    }
  };
  auto g_store = [&](int base, const float (&gv)[kB]) {
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int e = base + i * kThreads + tid;
      const int j = e / RMAX;
      const bool ok = j < r && kcol < r;
      if (kFull || e < RB * RMAX)
        s_g[e] = (ok && gdk != 0.f) ? (j == kcol ? -1.f : -(gv[i] * ginvk)) : 0.f;
    }
  };
  auto p_load = [&](int base, float (&pv)[kB]) {
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int e = base + i * kThreads + tid;
      const float x = Pb[min(e, np - 1)];
      pv[i] = e < np ? x : 0.f;
    }
  };
  auto p_store = [&](int base, const float (&pv)[kB]) {
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int e = base + i * kThreads + tid;
      if (e < np) s_rows[e] = pv[i];
    }
  };
  {
    float gv[kB], pv[kB];
    g_load(0, gv);
    p_load(0, pv);
    g_store(0, gv);
    p_store(0, pv);
  }
  for (int base = kB * kThreads; base < RB * RMAX; base += kB * kThreads) {
    float gv[kB];
    g_load(base, gv);
    g_store(base, gv);
  }
  for (int base = kB * kThreads; base < np; base += kB * kThreads) {
    float pv[kB];
    p_load(base, pv);
    p_store(base, pv);
  }
  for (int e = tid; e < K * kCT; e += kThreads) s_sh[e] = -1.0;  // every share slot empty
  __syncthreads();
  // for the F-hat share: the G entries of this thread's epilogue Gram tile, loaded after
  // the last barrier before the epilogue so that the sweeps hide their latency
  constexpr int TG = gram_tile_edge(RPAD == 16 ? 32 : 128);  // chunk_gram's tile edge
  const int ntg = (r + TG - 1) / TG;
  const bool gpre = a.err_part != nullptr && ntg * ntg <= kThreads;  // one tile per thread
  double gm[TG][TG];
  gram_tile_m<TG>(gpre ? a.G64 : nullptr, r, tid, gm);
  const double beta = a.A_hat ? *a.beta_src : 0.0;  // for the epilogue
  // for the fused decision: the reference F-hat of the test and ||T||^2 (read long before
  // this workgroup publishes its share, so before any workgroup can update the state)
  const double fhat_ref = a.st ? a.st->fhat_prev : 0.0;
  const double normT2 = a.st ? *a.normT2 : 0.0;

  // local row q of this lane: wave * RPWV + q * GPW + gi
  float w[NR][C], pinv[NR][C], zv[NR][C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int k = c * RPAD + gl;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const bool ok = rok[q] && k < r;
      pinv[q][c] = ok ? s_rows[lrow[q] * r + k] * ginv[c] : 0.f;
      // a dead component (G_kk = 0) is 0 after its first update and stays 0
      w[q][c] = (ok && ginv[c] != 0.f) ? w0[q][c] : 0.f;
    }
  }
  float greg[GREG ? RB : 1][C];
  if constexpr (GREG) {
#pragma unroll
    for (int j = 0; j < RB; ++j)
#pragma unroll
      for (int c = 0; c < C; ++c) greg[j][c] = s_g[j * RMAX + c * RPAD + gl];
  }

  const uint64_t t_start = wall_clock64();

  auto load_gblk = [&](int jb, float (&gb)[8][C]) {
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int c = 0; c < C; ++c)
        gb[t][c] = GREG ? greg[GREG ? jb * 8 + t : 0][c] : s_g[(jb * 8 + t) * RMAX + c * RPAD + gl];
  };
  // 1 on the lanes that hold column offset o of their group, else 0 (16-lane groups)
  // (64-lane groups: the lane within its 16-lane row, the row taken by a DPP row mask)
  float flag[16];
#pragma unroll
  for (int o = 0; o < 16; ++o) flag[o] = (lane & 15) == o ? 1.f : 0.f;
  // lanes owning column offset o of their group, as a wave-wide constant mask
  auto owner_mask = [&](int o) {
    uint64_t m = 0;
#pragma unroll
    for (int g = 0; g < GPW; ++g) m |= uint64_t(1) << (g * RPAD + o);
    return m;
  };
  // z = P / diag(G) + W S from scratch, two interleaved accumulators (fixed order)
  auto refresh = [&]() {
    if constexpr (RPAD == 16 && GREG) {
      // z = P / diag(G) + W S, one broadcast multiply-add per column and slot (in column
      // order)
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        float a[C];
#pragma unroll
        for (int c = 0; c < C; ++c) a[c] = pinv[q][c];
        asm volatile("s_nop 1");  // w may have been written just before (DPP read below)
        static_for<0, NB>([&](auto bc) {
          constexpr int J0 = decltype(bc)::value * 8;
          float g0[8], g1[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            g0[t] = greg[J0 + t][0];
            g1[t] = greg[J0 + t][C - 1];
          }
          if constexpr (C == 2)
            acc_blk2<J0>(a[0], a[1], w[q][J0 / 16], g0, g1);
          else
            acc_blk1<J0>(a[0], w[q][0], g0);
        });
#pragma unroll
        for (int c = 0; c < C; ++c) zv[q][c] = a[c];
      }
      return;
    }
    float gb0[8][C], gb1[8][C];
    float acc[2][NR][C];
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        acc[0][q][c] = pinv[q][c];
        acc[1][q][c] = 0.f;
      }
    load_gblk(0, gb0);
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
      float (&cur)[8][C] = (jb & 1) ? gb1 : gb0;
      float (&nxt)[8][C] = (jb & 1) ? gb0 : gb1;
      if (jb + 1 < NB) load_gblk(jb + 1, nxt);
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int l = jb * 8 + t;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          const float wl = bcast<RPAD>(w[q][l / RPAD], l % RPAD);
#pragma unroll
          for (int c = 0; c < C; ++c) acc[t & 1][q][c] = fmaf(wl, cur[t][c], acc[t & 1][q][c]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
      for (int c = 0; c < C; ++c) zv[q][c] = acc[0][q][c] + acc[1][q][c];
  };
  // one Gauss-Seidel sweep over the columns; every z_k (also k < j) follows each update, so
  // z stays current across sweeps and is refreshed from scratch only every kRefresh sweeps
  // to bound the drift of the rank-one updates. The owner's change reaches its group through
  // a DPP broadcast that the compiler folds into the multiply-adds.
  auto sweep = [&]() {
    if constexpr (RPAD == 16 && GREG) {
      // 16-lane groups, scaled G in registers: one inline-asm statement per block of eight
      // columns
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        // the change of the previous column and its coefficient for the slot whose update
        // is deferred into the next column's step
        float dp = 0.f, gp = 0.f;
        static_for<0, NB>([&](auto bc) {
          constexpr int J0 = decltype(bc)::value * 8;
          constexpr int cs = J0 / 16;
          float gi[8], gd[8], f[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int j = J0 + t;
            const int ns = (j + 1 < RB ? j + 1 : 0) / 16;  // slot of the column read next
            gi[t] = greg[j][C == 1 ? 0 : ns];
            gd[t] = greg[j][C == 1 ? 0 : 1 - ns];
            f[t] = flag[j % 16];
          }
          if constexpr (C == 1) {
            blk16_one<J0>(zv[q][0], w[q][0], gi, f);
          } else {
            constexpr bool sw = ((J0 + 8 < RB ? J0 + 8 : 0) / 16) != cs;
            blk16_two<J0, sw>(zv[q][cs], zv[q][1 - cs], w[q][cs], dp, gp, gi, gd, f);
          }
        });
        // the last column's next is column 0 (slot 0): its deferred update is of slot 1
        if constexpr (C == 2) col_flush<(RB - 1) % 16>(zv[q][1], dp, gp);
      }
    } else if constexpr (RPAD == 64 && C == 1 && GREG) {
      // one 64-lane group per row, scaled G in registers: one inline-asm statement per block
      // of eight columns
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        float dp = 0.f;
        static_for<0, NB>([&](auto bc) {
          constexpr int J0 = decltype(bc)::value * 8;
          float g[8], f[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            g[t] = greg[J0 + t][0];
            f[t] = flag[(J0 + t + 15) % 16];  // the previous column's owner
          }
          blk64<J0>(zv[q][0], w[q][0], dp, g, f);
        });
        col64_flush<RB - 1>(w[q][0], dp, flag[(RB - 1) % 16]);
      }
    } else {
      float gb0[8][C], gb1[8][C];
      load_gblk(0, gb0);
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        float (&cur)[8][C] = (jb & 1) ? gb1 : gb0;
        float (&nxt)[8][C] = (jb & 1) ? gb0 : gb1;
        if (jb + 1 < NB) load_gblk(jb + 1, nxt);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int j = jb * 8 + t;
          const int cs = j / RPAD;
          const int o = j % RPAD;
#pragma unroll
          for (int q = 0; q < NR; ++q) {
            // every lane forms the change of its own column in slot cs; the owner's is used
            const float d = fmaxf(zv[q][cs], -w[q][cs]);
            const float wn = w[q][cs] + d;
            if (__builtin_amdgcn_inverse_ballot_w64(owner_mask(o))) w[q][cs] = wn;
            const float delta = bcast<RPAD>(d, o);
#pragma unroll
            for (int c = 0; c < C; ++c) zv[q][c] = fmaf(delta, cur[t][c], zv[q][c]);
          }
        }
      }
    }
  };

  // ---- stopping rule (Sec. 4.1) on a wave of its own ----
  // After sweep s each row thread stores its share of ||W_s - W_{s-1}||^2 in LDS slot
  // s mod K; a slot holds -1 while empty, so the shares themselves say when a sweep is
  // complete and the row waves need no flag or fence. The rule wave sums a complete slot
  // (fixed order), empties it, publishes the workgroup's share in global slot (s, wg),
  // reads every workgroup's slots for several published sweeps per round trip, sums them
  // in workgroup order (every workgroup gets the same bits) and posts its decisions. Row
  // waves never wait for memory: they run up to `lag` sweeps past the last decision they
  // have seen (read one sweep ahead), keeping those iterates in an LDS ring, and restore
  // the sweep the rule stops at. All waits are bounded by a wall-clock deadline.
  uint64_t* const slots = a.slots;  // [sweep][wg]
  auto lds_ld = [](const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  auto sh_ld = [](const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  auto sh_st = [](double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  auto lds_st = [](int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  auto ring_put = [&](int slot) {
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
      for (int c = 0; c < C; ++c) s_ring[(slot * NR * C + q * C + c) * kCT + tid] = w[q][c];
  };
  auto ring_get = [&](int slot) {
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
      for (int c = 0; c < C; ++c) w[q][c] = s_ring[(slot * NR * C + q * C + c) * kCT + tid];
  };
  int done = S;
  bool timed_out = false;
  if (wave == WPG) {
    // ---- the rule wave ----
    // M sweeps per round trip; the lanes form M groups of G = 64 / M: lane g of group m
    // sums the global slots of sweep t_dec + m of workgroups g, g + G, ... (at most KL), in
    // that order, then the group adds its lanes with a fixed DPP pairing, so every
    // workgroup gets the same bits. Two ballots over the group leaders find the first
    // sweep not yet published everywhere and the first that meets the rule.
    auto rule = [&](auto m_tag, auto kl_tag) {
      constexpr int M = decltype(m_tag)::value;
      constexpr int KL = decltype(kl_tag)::value;
      constexpr int G = 64 / M;
      static_assert(G >= 4 && G <= 16, "groups of 4 to 16 lanes (one DPP row)");
      const int gm = lane / G;  // this lane's sweep, relative to t_dec
      const int gg = lane % G;
      int t_pub = 1, t_dec = 1;
      double lim = 0.0;
      const double tol2 = a.tol * a.tol;
      while (true) {
        if (t_dec >= S) {  // sweeps 1 .. S-1 decided without a stop
          if (lane == 0) lds_st(&s_decided, S);
          return;
        }
        if (wall_clock64() - t_start > a.timeout_ticks) {
          if (lane == 0) lds_st(&s_stop, -1);
          return;
        }
        // publish every complete sweep (emptying its LDS slot)
        for (; t_pub < S; ++t_pub) {
          double* sh = s_sh + (t_pub % K) * kCT;
          double v[WPG];
          bool empty = false;
#pragma unroll
          for (int k = 0; k < WPG; ++k) {
            v[k] = sh_ld(sh + lane + 64 * k);
            empty = empty || v[k] < 0.0;
          }
          if (__any(empty)) break;
          double x = v[0];
#pragma unroll
          for (int k = 1; k < WPG; ++k) x += v[k];
          const double D = wave_sum64(x);
#pragma unroll
          for (int k = 0; k < WPG; ++k) sh_st(sh + lane + 64 * k, -1.0);
          if (lane == 0)
            __hip_atomic_store(&slots[int64_t(t_pub - 1) * a.nwg + blockIdx.x],
                               uint64_t(__double_as_longlong(D)), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        // decide up to M published sweeps t_dec .. t_dec + n - 1 (< S) per round trip
        const int n = min(M, min(t_pub, S) - t_dec);
        if (n <= 0) {
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        uint64_t u[KL];
        const bool live = gm < n;
        const uint64_t* srow = slots + int64_t(t_dec - 1 + (live ? gm : 0)) * a.nwg;
#pragma unroll
        for (int i = 0; i < KL; ++i) {
          const int k = gg + G * i;
          u[i] = (live && k < a.nwg)
                     ? __hip_atomic_load(&srow[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : 0;  // the bits of +0.0
        }
        bool ms = false;
        double x = 0.0;
#pragma unroll
        for (int i = 0; i < KL; ++i) {
          ms = ms || u[i] == kSentinel;
          x += __longlong_as_double(int64_t(u[i]));
        }
        // the group's sum and whether any of its workgroups has not published
        int mi = ms ? 1 : 0;
        x += dpp64<0xB1>(x);
        mi |= __builtin_amdgcn_update_dpp(0, mi, 0xB1, 0xF, 0xF, false);
        x += dpp64<0x4E>(x);
        mi |= __builtin_amdgcn_update_dpp(0, mi, 0x4E, 0xF, 0xF, false);
        if constexpr (G >= 8) {
          x += dpp64<0x141>(x);
          mi |= __builtin_amdgcn_update_dpp(0, mi, 0x141, 0xF, 0xF, false);
        }
        if constexpr (G >= 16) {
          x += dpp64<0x140>(x);
          mi |= __builtin_amdgcn_update_dpp(0, mi, 0x140, 0xF, 0xF, false);
        }
        const bool lead = gg == 0;
        const uint64_t bad = __ballot(lead && (mi != 0 || !live));
        const int nd = bad ? min(n, int(__builtin_ctzll(bad)) / G) : n;  // decidable now
        if (t_dec == 1 && nd > 0) lim = tol2 * readlane64(x, 0);  // ||W_1 - W_0||^2 tol^2
        const uint64_t hit = __ballot(lead && gm < nd && x <= lim);
        const int stop = hit ? t_dec + int(__builtin_ctzll(hit)) / G : 0;
        t_dec = stop ? stop + 1 : t_dec + nd;
        // the emptied share slots are visible before the decision that lets them refill
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (stop) {
          if (lane == 0) {
            lds_st(&s_stop, stop);
            lds_st(&s_decided, stop);
          }
          return;
        }
        if (lane == 0) lds_st(&s_decided, t_dec - 1);
        if (nd == 0) __builtin_amdgcn_s_sleep(2);
      }
    };
    // M * nwg <= 512 slots per round trip (KL = 8 loads per lane), M >= 4
    if (a.nwg <= 32)
      rule(std::integral_constant<int, 16>(), std::integral_constant<int, 8>());
    else if (a.nwg <= 64)
      rule(std::integral_constant<int, 8>(), std::integral_constant<int, 8>());
    else if (a.nwg <= 128)
      rule(std::integral_constant<int, 4>(), std::integral_constant<int, 8>());
    else
      rule(std::integral_constant<int, 4>(), std::integral_constant<int, 16>());
  } else {
    // ---- the row waves ----
    // every LDS read so far (the scaled G in registers) has arrived: without this wait the
    // first use inside the loop would wait for them, on every sweep
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    int dec = 0, stp = 0;  // the decision state as last read (at most one sweep old)
    int sr = 0, sk = 0;    // s mod R, s mod K
    for (int s = 1; s <= S; ++s) {
      sr = sr + 1 == R ? 0 : sr + 1;
      sk = sk + 1 == K ? 0 : sk + 1;
      while (stp == 0 && s - dec > L) {
        __builtin_amdgcn_s_sleep(1);
        dec = __builtin_amdgcn_readfirstlane(lds_ld(&s_decided));
        stp = __builtin_amdgcn_readfirstlane(lds_ld(&s_stop));
      }
      if (stp != 0) break;
      float prev[NR][C];
#pragma unroll
      for (int q = 0; q < NR; ++q)
#pragma unroll
        for (int c = 0; c < C; ++c) prev[q][c] = s == 1 ? w0[q][c] : w[q][c];
      if ((s - 1) % kRefresh == 0) refresh();
      // read the decision state now, use it before the next sweep (the empty asm keeps
      // the wait for the reads, and their move to scalar registers, after the sweep)
      int dec_next = lds_ld(&s_decided);
      int stp_next = lds_ld(&s_stop);
      sweep();
      asm volatile("" : "+v"(dec_next), "+v"(stp_next));
      ring_put(sr);
      double d2 = 0.0;
#pragma unroll
      for (int q = 0; q < NR; ++q)
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const double df = double(w[q][c]) - double(prev[q][c]);
          d2 = fma(df, df, d2);
        }
      sh_st(s_sh + sk * kCT + tid, d2);
      // the decision state is the same on every lane: scalar, so the loop control is too
      dec = __builtin_amdgcn_readfirstlane(dec_next);
      stp = __builtin_amdgcn_readfirstlane(stp_next);
    }
    // the decision for the sweeps still open
    while (stp == 0 && __builtin_amdgcn_readfirstlane(lds_ld(&s_decided)) < S) {
      __builtin_amdgcn_s_sleep(1);
      stp = __builtin_amdgcn_readfirstlane(lds_ld(&s_stop));
    }
    if (stp > 0) {
      ring_get(stp % R);
      done = stp;
    } else if (stp < 0) {
      timed_out = true;
    }
  }
  if (timed_out && lane == 0)
    __hip_atomic_fetch_or(a.flags, NTF_FLAG_WAIT_TIMEOUT, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);

  // ---- epilogue: write W (and A_hat); stage rows for the Gram partials ----
  float pv_keep[NR][C];  // P entries of this lane's columns, read before the rows are replaced
  float xh_keep[NR][C];  // the extrapolated entries (for the fused selection)
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int c = 0; c < C; ++c) pv_keep[q][c] = xh_keep[q][c] = 0.f;
  lds_barrier();  // every lane has its P entries in registers (pinv) by now
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = c * RPAD + gl;
      if (rok[q] && j < r) {
        const int64_t gidx = (row0 + lrow[q]) * r + j;
        a.W[gidx] = w[q][c];
        pv_keep[q][c] = s_rows[lrow[q] * r + j];
        s_rows[lrow[q] * r + j] = w[q][c];
        if (a.A_hat) {
          const double x = w[q][c];
          const double y = x + beta * (x - double(w0[q][c]));
          const float xh = float((y > 0.0 || !a.project) ? y : 0.0);
          a.A_hat[gidx] = xh;
          s_rows2[lrow[q] * r + j] = xh;
          xh_keep[q][c] = xh;
        }
      }
    }
  lds_barrier();  // the W and A_hat stores may still be in flight
  const int64_t rr = int64_t(r) * r;
  // Gram partials of the new and extrapolated rows; the first also yields this thread's
  // share of <G, W^T W> over the chunk's rows for the F-hat share
  double gdot = 0.0;
  const double no_tile[TG][TG] = {};
  double* out_new = a.gp_new ? a.gp_new + blockIdx.x * rr : nullptr;
  double* out_hat = (a.gp_hat && a.A_hat) ? a.gp_hat + blockIdx.x * rr : nullptr;
  const double* gmat = a.err_part ? a.G64 : nullptr;
  if constexpr (TG == 2) {
    if (out_hat) {
      // both partials in one pass over the two row blocks (small tiles only: with 4 x 4
      // tiles the two accumulator sets would not fit in registers)
      gdot = gpre ? chunk_gram2_tiles<TG, true, 4>(s_rows, s_rows2, nrows, r, out_new,
                                                   out_hat, a.G64, gm)
                  : chunk_gram2_tiles<TG, false, 4>(s_rows, s_rows2, nrows, r, out_new,
                                                    out_hat, gmat, no_tile);
      out_hat = nullptr;
      out_new = nullptr;
      gmat = nullptr;
    }
  }
  if (out_new || gmat) {
    gdot = gpre ? chunk_gram_tiles<TG, true, 4>(s_rows, nrows, r, out_new, a.G64, gm)
                : chunk_gram_tiles<TG, false, 4>(s_rows, nrows, r, out_new, gmat, no_tile);
  }
  if (out_hat) chunk_gram_tiles<TG, false, 4>(s_rows2, nrows, r, out_hat, nullptr, no_tile);
  double e_share = 0.0;  // thread 0: this workgroup's F-hat share
  if (a.err_part) {
    // share of 2 <P, W> - <G, W^T W> over the chunk's rows
    double t = -gdot;
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int j = c * RPAD + gl;
        if (rok[q] && j < r) t = fma(2.0 * double(w[q][c]), double(pv_keep[q][c]), t);
      }
    const double ws = wave_sum64(t);
    if (lane == 0) s_part[wave] = ws;
    __syncthreads();
    if (tid == 0) {
      double e = 0.0;
      for (int k = 0; k <= WPG; ++k) e += s_part[k];
      a.err_part[blockIdx.x] = e;
      e_share = e;
    }
  }
  if (blockIdx.x == 0 && tid == 0 && a.sweeps_out) *a.sweeps_out = done;
  if (a.st == nullptr) return;

  // ---- the decision of the outer iteration (Algorithm 2), fused ----
  // Every workgroup publishes its F-hat share in a slot after the stopping rule's (set to
  // all-ones bits by the preceding kernel), reads all of them, sums them in the fixed order
  // of the decision kernel and takes the same restart decision; workgroup 0 updates the
  // state. The selection A <- restart ? A_new : A_hat (and of the Gram chunks) is split:
  // each workgroup writes its own rows and chunk of the last block from what it holds, and a
  // slice of the other blocks.
  __shared__ double s_f;  // F-hat
  uint64_t* const es = slots + int64_t(a.max_sweeps) * a.nwg;
  if (tid == 0) {
    // release: the reads of the state are complete before any workgroup can see the share,
    // and workgroup 0 writes the state only after it has seen every share
    __hip_atomic_store(&es[blockIdx.x], uint64_t(__double_as_longlong(e_share)),
                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  double x = 0.0;
  bool late = false;
  if (tid < a.nwg) {
    const uint64_t t_poll = wall_clock64();
    uint64_t u;
    while ((u = __hip_atomic_load(&es[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ==
           kSentinel) {
      if (wall_clock64() - t_poll > a.timeout_ticks) {
        late = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    x = late ? 0.0 : __longlong_as_double(int64_t(u));
  }
  const bool any_late = __syncthreads_or(late);
  const double esum = block_sum256(x);  // ordered as the decision kernel sums the partials
  if (tid == 0) s_f = 0.5 * (normT2 - esum);
  __syncthreads();
  if (any_late) {
    if (tid == 0)
      __hip_atomic_fetch_or(a.flags, NTF_FLAG_WAIT_TIMEOUT, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const double f = s_f;
  const bool restart = her_restart(f, fhat_ref);
  if (blockIdx.x == 0 && tid == 0)
    her_update(a.st, a.hp, f, fhat_ref, a.trace, a.order, a.sweeps_src, nullptr, a.flags);
  const int last = a.order - 1;
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = c * RPAD + gl;
      if (rok[q] && j < r) a.sel.dst[last][(row0 + lrow[q]) * r + j] = restart ? w[q][c] : xh_keep[q][c];
    }
  if (a.sel.ddst[last]) {
    // this workgroup's Gram chunk, written by its own threads before the barriers above
    const double* gsrc = (restart ? a.gp_new : a.gp_hat) + blockIdx.x * rr;
    copy_strided(a.sel.ddst[last] + blockIdx.x * rr, gsrc, rr, int64_t(tid), int64_t(kThreads));
  }
  // a slice of the other blocks' rows
  const int64_t gt = int64_t(blockIdx.x) * kThreads + tid;
  const int64_t gs = int64_t(gridDim.x) * kThreads;
  for (int b = 0; b < last; ++b) {
    copy_strided(a.sel.dst[b], restart ? a.sel.a_new[b] : a.sel.a_hat[b], a.sel.n[b], gt, gs);
    if (a.sel.ddst[b])
      copy_strided(a.sel.ddst[b], restart ? a.sel.dnew[b] : a.sel.dhat[b], a.sel.dn[b], gt, gs);
  }
}

using HFn = void (*)(HKArgs);

// number of 8-column blocks swept for rank r (r <= 128)
int hals_nb(int r) {
  if (r <= 32) return (r + 7) / 8;
  if (r <= 64) return (r + 7) / 8;
  return 2 * ((r + 15) / 16);
}

template <int RPAD, int C, int NB>
HFn pick_nr(int nr) {
  if (nr == 1) return hals_kernel<RPAD, C, 1, NB>;
  if (nr == 2) return hals_kernel<RPAD, C, 2, NB>;
  return hals_kernel<RPAD, C, 4, NB>;
}

HFn hals_fn(int r, int nr) {
  switch (hals_nb(r)) {
    case 1: return pick_nr<16, 1, 1>(nr);
    case 2: return pick_nr<16, 1, 2>(nr);
    case 3: return pick_nr<16, 2, 3>(nr);
    case 4: return pick_nr<16, 2, 4>(nr);
    case 5: return pick_nr<64, 1, 5>(nr);
    case 6: return pick_nr<64, 1, 6>(nr);
    case 7: return pick_nr<64, 1, 7>(nr);
    case 8: return pick_nr<64, 1, 8>(nr);
    case 10: return pick_nr<64, 2, 10>(nr);
    case 12: return pick_nr<64, 2, 12>(nr);
    case 14: return pick_nr<64, 2, 14>(nr);
    default: return pick_nr<64, 2, 16>(nr);
  }
}

constexpr size_t kLdsBudget = 150 * 1024;  // dynamic LDS (static LDS is under 1 KB)

// Dynamic LDS of a launch with run-ahead `lag`: scaled G, two row blocks, the iterate ring
// (lag + 1 slots) and the share slots (lag + 2).
size_t hals_lds_for(int r, int64_t rows, int lag) {
  const int rpad = r <= 32 ? 16 : 64;
  const int c = r <= 16 ? 1 : (r <= 32 ? 2 : (r <= 64 ? 1 : 2));
  const int rb = 8 * hals_nb(r);
  const int nr = hals_rows_interleaved(r, rows);
  const int rpw = gram_chunk_rows(r, rows);
  const size_t fl = size_t(rb) * rpad * c + 2 * size_t(rpw) * r + size_t(lag + 1) * nr * c * kCT;
  return align_up(fl * sizeof(float), 16) + size_t(lag + 2) * kCT * sizeof(double);
}

// the longest run-ahead (at most kMaxLag, at least 2) that fits the LDS budget
int hals_lag(int r, int64_t rows) {
  int lag = kMaxLag;
  while (lag > 2 && hals_lds_for(r, rows, lag) > kLdsBudget) --lag;
  return lag;
}

}  // namespace

int64_t hals_wgs(int64_t rows, int r) { return ceil_div(rows, gram_chunk_rows(r, rows)); }

bool hals_supported(int64_t rows, int r, int num_cus) {
  if (r < 1 || r > 128 || rows < 1) return false;
  return hals_wgs(rows, r) <= std::min(256, num_cus);
}

int64_t hals_slot_count(int64_t rows, int r, int max_sweeps) {
  // one share per workgroup and sweep, and one F-hat share per workgroup (fused decision)
  return int64_t(max_sweeps + 1) * hals_wgs(rows, r);
}

hipError_t launch_hals(const HalsArgs& h, int num_cus, hipStream_t s) {
  HKArgs a{};
  a.W0 = h.W0;
  a.W = h.W;
  a.P = h.P;
  a.G = h.G;
  a.G64 = h.G64;
  a.rows = h.rows;
  a.r = h.r;
  a.max_sweeps = h.max_sweeps;
  a.tol = h.tol;
  a.sweeps_out = h.sweeps_out;
  a.slots = reinterpret_cast<uint64_t*>(h.slots);
  a.flags = h.flags;
  a.A_hat = h.A_hat;
  a.beta_src = h.beta_src;
  a.project = h.project ? 1 : 0;
  a.gp_new = h.gp_new;
  a.gp_hat = h.gp_hat;
  a.err_part = h.err_part;
  a.nwg = int(hals_wgs(h.rows, h.r));
  a.st = h.st;
  if (h.st) {
    // the fused decision needs every output of the epilogue
    if (!h.err_part || !h.A_hat || !h.gp_new || !h.gp_hat || !h.normT2 || h.order < 1 ||
        h.order > kMaxOrder || h.sel.nblocks != h.order)
      return hipErrorInvalidValue;
    a.hp = h.hp;
    a.normT2 = h.normT2;
    a.trace = h.trace;
    a.order = h.order;
    a.sweeps_src = h.sweeps_src;
    a.sel = h.sel;
  }
  // wall_clock64 runs at the device's wall-clock rate; the default 2 s is far above any
  // legitimate wait
  static const int rate_khz = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) != hipSuccess || v <= 0)
      v = 100000;
    return v;
  }();
  a.timeout_ticks = uint64_t(double(rate_khz) * 1000.0 * std::max(0.0, h.wait_limit_s));
  (void)num_cus;
  HFn fn = hals_fn(h.r, hals_rows_interleaved(h.r, h.rows));
  a.lag = hals_lag(h.r, h.rows);
  const size_t lds = hals_lds_for(h.r, h.rows, a.lag);
  if (lds > kLdsBudget) return hipErrorInvalidValue;
  static bool attr_done = false;
  if (!attr_done) {
    for (int rr : {8, 16, 24, 32, 40, 48, 56, 64, 80, 96, 112, 128})
      for (int nr : {1, 2, 4}) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(hals_fn(rr, nr)),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           int(kLdsBudget));
        if (e != hipSuccess) return e;
      }
    attr_done = true;
  }
  hipLaunchKernelGGL(fn, dim3(a.nwg), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

}  // namespace ntf
