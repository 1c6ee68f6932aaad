// Internal declarations of the NTF library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <type_traits>

#include "ntf.h"

namespace ntf {

// ------------------------------------------------------------------------- errors ---
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define NTF_RETURN_IF(cond, status, ...)  \
  do {                                    \
    if (cond) {                           \
      ::ntf::set_error(__VA_ARGS__);      \
      return (status);                    \
    }                                     \
  } while (0)

#define NTF_HIP(expr)                                                           \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::ntf::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                       __FILE__, __LINE__);                                     \
      return NTF_EDEVICE;                                                       \
    }                                                                           \
  } while (0)

// Launch-error check after a kernel launch.
#define NTF_LAUNCHED() NTF_HIP(hipGetLastError())

// ---------------------------------------------------------------------- constants ---
constexpr int kMaxOrder = NTF_MAX_ORDER;
constexpr int kMaxRank = NTF_MAX_RANK;
constexpr int kGramChunk = 64;        // rows per Gram partial (LDS: 64 x r floats)
constexpr int kMaxSweeps = 1000;      // upper bound accepted for max_inner

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline size_t align_up(size_t a, size_t b) { return (a + b - 1) / b * b; }

// Pointers to the factors of one problem, passed to kernels by value.
struct FactorPtrs {
  const float* p[kMaxOrder];
};

// Tensor geometry seen from mode n: T viewed as (L, I_n, R), C-order.
struct ModeView {
  int order;
  int mode;
  int64_t dims[kMaxOrder];
  int64_t L;   // prod_{l < n} I_l
  int64_t I;   // I_n
  int64_t R;   // prod_{l > n} I_l
};
ModeView make_mode_view(const ntf_tensor& T, int mode);

// --------------------------------------------------------------- workspace arena ---
// Bump allocator over the handle's device workspace. Sizes are computed first with a
// dry run (base == nullptr), so a call can grow the workspace once before enqueueing.
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct SolveGraph;  // defined in solve.hip

// MTTKRP shape choice, as picked by the autotuner: the kernel family (0 = the planner's
// default, 1 = row tiles, 2 = row slab) and, for row tiles, the waves along rows (tile
// height 32 * wm; 0 = the planner's default).
struct MttkrpChoice {
  int kernel = 0;
  int wm = 0;
};

}  // namespace ntf

struct ntf_handle {
  int device = 0;
  int num_cus = 256;
  size_t lds_per_block = 65536;
  char* ws = nullptr;          // general workspace
  size_t ws_size = 0;
  uint64_t ws_generation = 0;  // bumped on every reallocation
  uint32_t* dev_flags = nullptr;
  hipStream_t capture_stream = nullptr;
  double wait_limit_s = 2.0;   // A-HALS cross-workgroup waits (ntf_handle_set_wait_limit)
  ntf::SolveGraph* graph = nullptr;
  // batched solver: its own workspace, pinned descriptor staging, cached graph
  char* bws = nullptr;
  size_t bws_size = 0;
  void* bstage = nullptr;      // pinned host
  size_t bstage_size = 0;
  hipEvent_t bstage_done = nullptr;
  hipGraphExec_t bgraph = nullptr;
  unsigned char bgraph_key[160] = {};
  // MTTKRP tuning table: key (tensor shape, dtype, mode, rank) -> shape choice
  std::map<std::string, ntf::MttkrpChoice> tune;
};

namespace ntf {

// Destroy the handle's cached solver graph (if any).
void release_solve_graph(ntf_handle* h);

// Make sure the handle's workspace holds at least `bytes` (synchronizes the device when
// it has to grow, invalidating cached graphs).
ntf_status ensure_workspace(ntf_handle* h, size_t bytes);

// Makes a device current for the duration of a call, then restores the previous one.
struct DeviceGuard {
  int old = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    if (old != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
  }
};

// Resolve (once per device, with that device current) the device address of the
// scratch-free MTTKRP's static scratch array; called when a handle is created.
ntf_status noalloc_scratch_attach(int device);

// Validation helpers shared by the entry points (set the thread-local error message).
ntf_status check_tensor(const ntf_tensor* T);
ntf_status check_rank(int32_t r);
ntf_status check_params(const ntf_her_params* p);

// --------------------------------------------------------------- kernel launchers ---
// Every launcher enqueues on `s` and returns hipSuccess or the launch error.

// ||T||^2 into *out (float64). `partials` holds at least norm2_partials() doubles.
int norm2_partials();
hipError_t launch_norm2(const void* data, int dtype, int64_t n, double* partials, double* out,
                        hipStream_t s);
hipError_t launch_cast_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t s);

// MTTKRP plan: chooses the kernel variant, tile and split count for one mode.
struct MttkrpPlan {
  ModeView v;
  int dtype;
  int r;
  int rpad;        // r rounded up to the kernel's N tile
  int variant;     // number of 32-column N tiles
  int layout;      // 0: mode is not the last (v = last mode); 1: mode is the last
  int wm, wk;      // waves along rows / along v
  int vmode;       // the fastest other mode (its factor is the MFMA B operand)
  int64_t Iv;      // I_v
  int64_t U;       // product of the remaining other modes
  int vb, nvb;     // v-block length and count
  int ub;          // u values per X batch
  size_t lds;      // dynamic LDS bytes
  int64_t mtiles;  // row tiles
  int64_t chunks;  // work items (v-block, u)
  bool store_y = false;  // store Y = T_u A_v rows instead of folding (case A, 3-way solver)
  bool uk = false;       // the WK waves of a row tile split u (not v chunks)
  bool slab = false;     // row-slab kernel (one output row per workgroup, u rows in M)
  int slab_inner = -1;   // its innermost u mode
  int64_t splits;  // splits of the work items (grid.y)
  size_t partial_floats() const { return splits > 1 ? size_t(splits) * v.I * r : 0; }
};
// `choice` (may be NULL) overrides the planner's default shape where it applies.
MttkrpPlan plan_mttkrp(const ntf_tensor& T, int mode, int r, int num_cus,
                       bool store_y = false, const MttkrpChoice* choice = nullptr);
// Shapes the planner can take for this mode (what the autotuner times), at most `cap`.
int mttkrp_candidates(const ntf_tensor& T, int mode, int r, MttkrpChoice* out, int cap);
// Key of the tuning table for (T's shape and dtype, mode, r).
std::string tune_key(const ntf_tensor& T, int mode, int r);
// The handle's tuned choice for this key, or NULL.
const MttkrpChoice* tuned_choice(const ntf_handle* h, const ntf_tensor& T, int mode, int r);
// MTTKRP. With one split the kernel writes P (I x r) directly. With several it writes
// plan.partial_floats() floats of split partials; if `reduce` is set a second kernel sums
// them into P in a fixed order, otherwise the caller (A-HALS) consumes the partials.
// A plan made with store_y (case A only) writes Y[i][u][:] = T_u A_v (I x U x r floats)
// to `ystore` instead, and nothing to P.
struct HadamardLaunch;
hipError_t launch_mttkrp(const MttkrpPlan& plan, const void* T, const FactorPtrs& A, float* P,
                         float* partials, bool reduce, hipStream_t s, float* ystore = nullptr,
                         const HadamardLaunch* had = nullptr);
// 3-way tensors, from a stored Y (mode 0 plan with store_y, u = mode 1):
//   P[i, p] = sum_u X[u, p] Y[i, u, p]            (mode-0 MTTKRP, X = A_1)
//   P[u, p] = sum_i X[i, p] Y[i, u, p]            (mode-1 MTTKRP, X = A_0; `partials`
//                                                  holds fold_i_splits(I, U, r) U r floats)
hipError_t launch_fold_u(const float* Y, const float* X, int64_t I, int64_t U, int r, float* P,
                         hipStream_t s);
int64_t fold_i_splits(int64_t I, int64_t U, int r);
// Fused all-mode MTTKRP of a 4-way bf16 tensor with modes 3 and 4 of size 128 and r <= 64:
// one pass over T; P[n] (NULL: not wanted) receive the four MTTKRPs. `ws` holds
// fused4_workspace_floats() floats.
bool fused4_applies(const ntf_tensor& T, int r);
size_t fused4_workspace_floats(const ntf_tensor& T, int r, int num_cus);
hipError_t launch_fused4(const ntf_tensor& T, const float* const* A, int r, int num_cus,
                         float* const* P, float* ws, hipStream_t s);
// 3-way tensors: whether the mode-1 and mode-2 MTTKRPs share one pass through Y (Y smaller
// than the tensor and A_3 in one LDS block of the store-Y plan `plan_y`).
bool use_shared_y(const ntf_tensor& T, int r, const MttkrpPlan& plan_y);
hipError_t launch_fold_i(const float* Y, const float* X, int64_t I, int64_t U, int r,
                         float* partials, float* P, hipStream_t s,
                         const HadamardLaunch* had = nullptr);

// Gram partials: for factor f (rows[f] x r), out[f] gets gram_chunks(rows, r) partial
// r x r float64 Grams (row chunks of the A-HALS workgroup size, so the A-HALS epilogue
// produces identical partials). Up to kMaxOrder factors per launch (blockIdx.y = factor).
struct GramJob {
  const float* A[kMaxOrder];
  double* out[kMaxOrder];
  int64_t rows[kMaxOrder];
  int nfac;
};
int64_t gram_chunks(int64_t rows, int r);
hipError_t launch_gram_partials(const GramJob& job, int r, hipStream_t s);

// Hadamard of summed Gram partials: G = prod_f sum_c part[f][c]. Writes G32 and/or G64;
// also resets `nslots` inner-solver wait slots to the sentinel (may be 0).
struct HadamardJob {
  const double* part[kMaxOrder];
  // a factor whose Gram is the survivor of the last HER decision: its chunks are taken from
  // part_new[f] when st->restart is set, else from part[f] (null part_new: always part)
  const double* part_new[kMaxOrder];
  const ntf_her_state* st;
  int64_t nchunks[kMaxOrder];
  int nfac;
};
hipError_t launch_hadamard(const HadamardJob& job, int r, float* G32, double* G64,
                           double* slots, int64_t nslots, hipStream_t s);
// The same work done by hadamard_blocks(r) leading workgroups of another launch (the MTTKRP
// or fold that precedes the A-HALS launch needing G), which saves a launch per block.
struct HadamardLaunch {
  HadamardJob job;
  int r;
  float* G32;
  double* G64;
  double* slots;
  int64_t nslots;
};
// leading workgroups of a launch that compute the Hadamard product: a multiple of 8 keeps
// the XCD dealing of the rest; more for large r (r^2 entries, four threads each)
inline int hadamard_blocks(int r) { return r <= 32 ? 8 : 32; }

// A-HALS on one block. `slots` holds hals_slot_count(rows, r, max_sweeps) doubles that
// are set to the sentinel (launch_fill_sentinel or launch_hadamard) before the call.
int64_t hals_slot_count(int64_t rows, int r, int max_sweeps);
int64_t hals_wgs(int64_t rows, int r);
// Workgroups never exceed min(256, CU count) so that all of them are resident at once.
bool hals_supported(int64_t rows, int r, int num_cus);
hipError_t launch_fill_sentinel(double* slots, int64_t n, hipStream_t s);
// After DECIDE: dst[b] <- restart ? a_new[b] : a_hat[b] for every block (and the same
// selection for optional float64 side buffers).
struct SelectJob {
  float* dst[kMaxOrder];
  const float* a_new[kMaxOrder];
  const float* a_hat[kMaxOrder];
  int64_t n[kMaxOrder];
  double* ddst[kMaxOrder];
  const double* dnew[kMaxOrder];
  const double* dhat[kMaxOrder];
  int64_t dn[kMaxOrder];
  int nblocks;
};
struct HalsArgs {
  const float* W0;       // warm start (may equal W)
  float* W;              // result
  const float* P;        // MTTKRP rows x r
  const float* G;        // r x r float32
  const double* G64;     // r x r float64, needed with err_part
  int64_t rows;
  int r;
  int max_sweeps;
  double tol;
  int32_t* sweeps_out;   // may be null
  double* slots;
  uint32_t* flags;
  // optional fused epilogue:
  float* A_hat;          // A_hat = max(0, W + beta (W - W0)), beta = *beta_src
  const double* beta_src;
  double* gp_new;        // Gram partials of W, hals_wgs(rows, r) x r x r
  double* gp_hat;        // Gram partials of A_hat
  double* err_part;      // per-workgroup share of 2 <P, W> - <G64, W^T W>
  double wait_limit_s = 2.0;  // bounded cross-workgroup waits give up after this long
  bool project = true;        // A_hat projected onto the nonnegative orthant
  // optional fused decision (the last block of an outer iteration, with err_part): F-hat
  // from every workgroup's share, the restart test, the state update and the selection of
  // the next iterate, which otherwise take launch_her_decide and launch_select. The shares
  // go through hals_wgs(rows, r) slots after the stopping rule's (the same reset).
  ntf_her_state* st = nullptr;
  ntf_her_params hp{};
  const double* normT2 = nullptr;
  ntf_trace trace{};
  int order = 0;
  const int32_t* sweeps_src = nullptr;
  SelectJob sel{};
};
hipError_t launch_hals(const HalsArgs& a, int num_cus, hipStream_t s);

// Projected-gradient block solver (k_pgd.hip): L <- ||G||_2 by power iteration, then
// `steps` projected gradient steps (accel: Nesterov's point), W0 -> W (may alias).
struct PgdArgs {
  const float* W0;
  float* W;
  const float* P;
  const float* G;
  double* L;
  float* coef;  // accel: `steps` floats of workspace (the Nesterov weights)
  int64_t rows;
  int r;
  int steps;
  int accel;
  int32_t* steps_out;  // may be null
};
hipError_t launch_pgd(const PgdArgs& a, hipStream_t s);
// The two parts of launch_pgd: L (and, with coef, the Nesterov weights of `steps` steps),
// then the steps with the L already in *a.L.
hipError_t launch_lipschitz(const float* G, int r, double* L, int steps, float* coef,
                            hipStream_t s);
hipError_t launch_pgd_steps(const PgdArgs& a, hipStream_t s);

// ADMM block solver (k_admm.hip): K = (G + rho I)^-1 with rho = trace(G) / r, then ADMM
// steps from W0 with the inner stopping rule (at most max_steps <= kAdmmMaxSteps), result
// into W (may alias W0). Workspace: K (r x r floats), rho (1 float), part
// (max_steps x admm_workgroups(rows, r) doubles), steps_dev (1 int).
constexpr int kAdmmMaxSteps = 64;
struct AdmmArgs {
  const float* W0;
  float* W;
  const float* P;
  const float* G;
  float* K;
  float* rho;
  double* part;
  int32_t* steps_dev;
  int64_t rows;
  int r;
  int max_steps;
  double tol;
  int32_t* steps_out;  // may be null
};
int64_t admm_workgroups(int64_t rows, int r);
hipError_t launch_admm(const AdmmArgs& a, hipStream_t s);

// A-HALS without the residency bound (k_hals_rows.hip): one thread per row, r <= 32, the
// stopping rule decided between two passes (at most kHalsRowsMaxSweeps sweeps). Workspace:
// part (max_sweeps x hals_rows_workgroups(rows) doubles), sweeps_dev (1 int).
constexpr int kHalsRowsMaxSweeps = 64;
constexpr int kHalsRowsMaxRank = 32;
struct HalsRowsArgs {
  const float* W0;
  float* W;
  const float* P;
  const float* G;
  double* part;
  int32_t* sweeps_dev;
  int64_t rows;
  int r;
  int max_sweeps;
  double tol;
  int32_t* sweeps_out;  // may be null
};
int64_t hals_rows_workgroups(int64_t rows);
hipError_t launch_hals_rows(const HalsRowsArgs& a, hipStream_t s);

// Tucker-format data (k_tucker.hip).
using TuckerDesc = ntf_tucker;
// Q = U^T A (U: n x rp, A: n x r, float64 accumulation) into Q32 (float) and/or Q64
// (double), rp x r, either may be null; part: tucker_proj_part_doubles(n, rp, r) doubles of
// workspace (may be null when that is 0).
size_t tucker_proj_part_doubles(int64_t n, int rp, int r);
hipError_t launch_tucker_proj(const float* U, const float* A, int64_t n, int rp, int r,
                              float* Q32, double* Q64, double* part, hipStream_t s);
// P = U Pc (U: n x rp, Pc: rp x r).
hipError_t launch_tucker_expand(const float* U, const float* Pc, int64_t n, int rp, int r,
                                float* P, hipStream_t s);
size_t tucker_norm_workspace_doubles(const TuckerDesc& X);
hipError_t launch_tucker_norm2(const TuckerDesc& X, double* ws, double* out, hipStream_t s);
ntf_status check_tucker(const ntf_tucker* X);

// Extrapolate-project: out = max(0, a_new + beta (a_new - a_old)), beta = *beta_src (without
// the projection when `project` is false).
hipError_t launch_extrapolate(const float* a_new, const float* a_old, float* out, int64_t n,
                              const double* beta_src, hipStream_t s, bool project = true);

// Restart surrogate pieces: per-block partial sums of 2<p_i,a_i> - a_i^T G a_i (float64).
int64_t error_partial_count(int64_t rows, int r);
hipError_t launch_error_partials(const float* P, const float* A, const double* G, int64_t rows,
                                 int r, double* partials, hipStream_t s);
// scale * (normT2 - sum partials) into *out (scale 1/2: F-hat; 1: the squared-error loss).
hipError_t launch_error_finalize(const double* normT2, const double* partials, int64_t nparts,
                                 double* out, uint32_t* flags, hipStream_t s,
                                 double scale = 0.5);
// out = alpha * (*scale or 1) * (A G - P), rows x r (loss gradient of one factor).
hipError_t launch_cp_grad(const float* A, const float* P, const double* G, int64_t rows, int r,
                          const double* scale, float alpha, float* out, hipStream_t s);

// HER state kernels.
hipError_t launch_her_init(ntf_her_state* st, const ntf_her_params& p, const double* fhat0,
                           hipStream_t s);
// Decide: F-hat from `fhat` (or from error partials when `partials` != null), update the
// state, write the trace entry.
struct DecideArgs {
  ntf_her_state* st;
  ntf_her_params p;
  const double* fhat;         // used when partials == null
  const double* normT2;       // with partials
  const double* partials;
  int64_t nparts;
  double* fhat_out;           // may be null
  ntf_trace trace;
  int order;
  const int32_t* sweeps_src;  // per-block sweep counters of this iteration (may be null)
  uint32_t* flags;
};
hipError_t launch_her_decide(const DecideArgs& a, hipStream_t s);
hipError_t launch_select(const SelectJob& j, const ntf_her_state* st, hipStream_t s);
hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_reset_call(ntf_her_state* st, hipStream_t s);

// Batched solver (many 3-way float32 problems; each outer iteration of all problems is a
// short sequence of grouped launches, captured once into a graph).
constexpr int kBatchedMaxDim = 256;
constexpr int kBatchedMaxRank = 32;
constexpr size_t kBatchedDescBytes = 512;
struct BatchedProblem {
  const float* T;
  int I[3];
  int r, rb;            // rank and its padding to a multiple of 4
  float* A[3];
  char* ws;             // batched_problem_bytes(I, rb) bytes of device workspace
  ntf_her_state* state; // may be null
  double* tr_fhat;
  int32_t* tr_restart;
  int32_t* tr_sweeps;
};
struct BatchedJob {
  const BatchedProblem* probs;
  const int32_t* order;  // host: processing order (largest first)
  int nprob;
  int resume;
  ntf_her_params params;
  void* host_desc;       // pinned, batched_plan(job).bytes
  void* dev_desc;        // device, the same size
  uint32_t* flags;
};
// Layout of the descriptor area (descriptors, order, work-item lists) and launch sizes.
struct BatchedPlan {
  size_t off_order, off_y, off_fu, off_fi, off_last, off_sum, bytes;
  int64_t n_y, n_fu, n_fi, n_last, n_sum;  // work items of the grouped launches
  size_t lds_y, lds_last, lds_hals;
};
size_t batched_problem_bytes(const int I[3], int rb);
BatchedPlan batched_plan(const BatchedJob& job);
hipError_t batched_upload(const BatchedJob& job, const BatchedPlan& pl, hipStream_t s);
hipError_t batched_setup(const BatchedJob& job, const BatchedPlan& pl, hipStream_t s);
hipError_t batched_iteration(const BatchedJob& job, const BatchedPlan& pl, hipStream_t s);
hipError_t batched_final(const BatchedJob& job, const BatchedPlan& pl, hipStream_t s);

// || T - [[A]] ||^2 (explicit residual, float64).
int residual_partials();
hipError_t launch_residual(const ntf_tensor& T, const FactorPtrs& A, int r, double* partials,
                           double* out, hipStream_t s);

}  // namespace ntf
