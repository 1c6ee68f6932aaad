// ntf_solve: Algorithm 2 (HER) with A-HALS blocks, driven entirely on the device.
//
// One outer iteration (paper Algorithm 2; block problem eq. NNLS_her_exact, extrapolation
// eq. extproj_her, restart test on F-hat, beta schedule eqs. HER_eq:beta_update /
// HER_eq:beta_bar_update) is captured once into a HIP graph and replayed `iters` times:
//
//   for block n:  G^(n)   = Hadamard of cached Grams (A-hat_k for l < n, A_{k-1} for l > n)
//                 P       = MTTKRP_n(T; A-hat_k^(l<n), A_{k-1}^(l>n))      (the hot kernel;
//                           3-way: modes 1 and 2 fold one shared Y = T x_3 A-hat_{k-1}^(3))
//                 A_new   = A-HALS(warm start A_{k-1}^(n); P, G^(n)), fused with
//                 A_hat   = max(0, A_new + beta (A_new - A_{k-1}^(n)))
//                 Grams of A_new and A_hat (float64 partials, cached)
//   F-hat_k = 1/2 (||T||^2 - 2 <P_N, A_new^(N)> + <G^(N), A_new^T A_new>)   (Sec. 3.1.3)
//   decide (restart / accept, beta update, trace) and select A_k (and its Gram cache).
//
// A-hat_{k-1} = A_{k-1} after every decision, so the caller's factor buffers always hold
// the current iterate and every block needs only two extra buffers (A_new, A_hat). The
// restart decision lives in device memory; the host never synchronizes inside the loop.
#include <cstring>

#include "ntf_internal.h"

namespace ntf {

struct SolveKey {
  const void* T;
  int32_t dtype, order, r;
  int64_t dims[kMaxOrder];
  float* A[kMaxOrder];
  ntf_her_params p;
  ntf_her_state* state;
  ntf_trace trace;
  uint64_t ws_generation;
  const float* U[kMaxOrder];  // Tucker-format data: bases (T then names the core)
  bool operator==(const SolveKey& o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
};

// One outer iteration, and kGraphUnroll iterations back to back (consecutive graph launches
// leave a gap of several microseconds between them, which the longer graph amortizes).
constexpr int kGraphUnroll = 8;
struct SolveGraph {
  SolveKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph_u = nullptr;
  hipGraphExec_t exec_u = nullptr;
};

namespace {

// 4-way tensors: two tensor passes per outer iteration instead of four. With the block
// order of Algorithm 2 the first two blocks see A-hat^(3), A-hat^(4) of the previous
// iteration and the last two see A-hat^(1), A-hat^(2) of this one, so
//   W = T x_3 A-hat^(3) x_4 A-hat^(4)  (the mode-1 MTTKRP of the (I_1 I_2) x I_3 x I_4 view)
//   V = T x_1 A-hat^(1) x_2 A-hat^(2)  (the mode-3 MTTKRP of the I_1 x I_2 x (I_3 I_4) view)
// give every block's MTTKRP by one fold: P^(1) = sum_j W[i, j] A^(2)[j], P^(2) = sum_i
// A-hat^(1)[i] W[i, j], P^(3) = sum_l V[k, l] A^(4)[l], P^(4) = sum_k A-hat^(3)[k] V[k, l]
// (equal to the four MTTKRPs up to summation order). Used when W and V are small next to
// the tensor.
struct PairPlans {
  bool on = false;
  ntf_tensor tw{}, tv{};  // the two 3-way views of T
  MttkrpPlan pw, pv;
};

// Device buffers of one solve, carved from the handle's workspace.
struct SolveBufs {
  double* norm_part;
  double* normT2;
  double* fhat0;
  ntf_her_state* state;
  float* A_new[kMaxOrder];
  float* A_hat[kMaxOrder];
  double* gp_new[kMaxOrder];
  double* gp_hat[kMaxOrder];
  float* G32;
  double* G64;
  float* P;
  float* mt_part;
  float* Y;  // 3-way: Y = T x_3 A_3 (I_1 x I_2 x r), shared by the mode-1 and mode-2 MTTKRPs
  float* W4;  // 4-way: W (I_1 I_2 x r) and V (I_3 I_4 x r), see PairPlans
  float* V4;
  double* slots;
  int64_t nslots;
  int32_t* sweeps;
  double* err_part;
  int64_t nerr;
  double* lip;  // projected-gradient blocks: L of the current block
  float* coef;  // and the Nesterov weights of its steps
  float* admm_k;        // ADMM blocks: (G + rho I)^-1, rho, per-step shares, stop step
  float* admm_rho;
  double* admm_part;
  int32_t* admm_steps;
  double* hr_part;      // A-HALS beyond the resident kernel's rows: per-sweep shares, stop
  int32_t* hr_sweeps;
  float* Q[kMaxOrder];  // Tucker-format data: projected factors U^(p)T A^(p) (r_p x r)
  float* Pc;            // and the core's MTTKRP (r_n x r)
  double* tq_part;      // per-workgroup partial sums of the projections
  double* tnorm;        // workspace of ||T||^2 of the format
};

void carve(Arena& ar, SolveBufs& b, const ntf_tensor& T, int r, int max_inner,
           const MttkrpPlan* plans, bool own_state, bool shared_y, const TuckerDesc* tk,
           const PairPlans& pp) {
  const int N = T.order;
  const size_t rr = size_t(r) * r;
  b.norm_part = ar.take<double>(norm2_partials());
  b.normT2 = ar.take<double>(1);
  b.fhat0 = ar.take<double>(1);
  b.state = own_state ? ar.take<ntf_her_state>(1) : nullptr;
  int64_t maxI = 0;
  size_t maxpart = 0;
  int64_t maxslots = 0;
  for (int n = 0; n < N; ++n) {
    const int64_t I = T.dims[n];
    maxI = std::max(maxI, I);
    b.A_new[n] = ar.take<float>(size_t(I) * r);
    b.A_hat[n] = ar.take<float>(size_t(I) * r);
    const size_t g = size_t(gram_chunks(I, r)) * rr;
    b.gp_new[n] = ar.take<double>(g);
    b.gp_hat[n] = ar.take<double>(g);
    maxpart = std::max(maxpart, plans[n].partial_floats());
    maxslots = std::max(maxslots, hals_slot_count(I, r, max_inner));
  }
  b.G32 = ar.take<float>(rr);
  b.G64 = ar.take<double>(rr);
  b.P = ar.take<float>(size_t(maxI) * r);
  if (shared_y)
    maxpart = std::max<size_t>(
        maxpart, size_t(fold_i_splits(T.dims[0], T.dims[1], r)) * T.dims[1] * r);
  if (pp.on) {
    maxpart = std::max({maxpart, pp.pw.partial_floats(), pp.pv.partial_floats(),
                        size_t(fold_i_splits(T.dims[0], T.dims[1], r)) * T.dims[1] * r,
                        size_t(fold_i_splits(T.dims[2], T.dims[3], r)) * T.dims[3] * r});
    b.W4 = ar.take<float>(size_t(T.dims[0]) * T.dims[1] * r);
    b.V4 = ar.take<float>(size_t(T.dims[2]) * T.dims[3] * r);
  } else {
    b.W4 = b.V4 = nullptr;
  }
  b.mt_part = ar.take<float>(std::max<size_t>(maxpart, 1));
  // (+64: padding that out-of-range stores of the Y kernel write to)
  b.Y = shared_y ? ar.take<float>(size_t(T.dims[0]) * T.dims[1] * r + 64) : nullptr;
  b.nslots = maxslots;
  b.slots = ar.take<double>(size_t(maxslots));
  b.sweeps = ar.take<int32_t>(kMaxOrder);
  b.nerr = std::max(error_partial_count(T.dims[N - 1], r), hals_wgs(T.dims[N - 1], r));
  b.err_part = ar.take<double>(size_t(b.nerr));
  b.lip = ar.take<double>(1);
  b.coef = ar.take<float>(size_t(max_inner));
  b.admm_k = ar.take<float>(rr);
  b.admm_rho = ar.take<float>(1);
  b.admm_part = ar.take<double>(size_t(std::min(max_inner, kAdmmMaxSteps)) *
                                size_t(admm_workgroups(maxI, r)));
  b.admm_steps = ar.take<int32_t>(1);
  b.hr_part = ar.take<double>(size_t(std::min(max_inner, kHalsRowsMaxSweeps)) *
                              size_t(hals_rows_workgroups(maxI)));
  b.hr_sweeps = ar.take<int32_t>(1);
  if (tk) {
    int64_t maxr = 1;
    for (int n = 0; n < N; ++n) {
      b.Q[n] = ar.take<float>(size_t(tk->core.dims[n]) * r);
      maxr = std::max(maxr, tk->core.dims[n]);
    }
    b.Pc = ar.take<float>(size_t(maxr) * r);
    size_t qp = 1;
    for (int n = 0; n < N; ++n)
      qp = std::max(qp, tucker_proj_part_doubles(tk->dims[n], int(tk->core.dims[n]), r));
    b.tq_part = ar.take<double>(qp);
    b.tnorm = ar.take<double>(tucker_norm_workspace_doubles(*tk));
  }
}

FactorPtrs factors_for(int n, int N, float* const* A, const SolveBufs& b) {
  FactorPtrs fp{};
  for (int l = 0; l < N; ++l) fp.p[l] = l < n ? b.A_hat[l] : A[l];
  fp.p[n] = A[n];  // not read by the MTTKRP
  return fp;
}

// Enqueue one outer iteration on stream s: per block a Hadamard kernel (also resetting the
// A-HALS wait slots), the MTTKRP (and the fixed-order sum of its split partials), and the
// fused A-HALS kernel (sweeps, extrapolation, Gram partials, F-hat share); then decide
// and select.
// The MTTKRP of mode n of Tucker-format data into b.P (Appendix A): projections of the
// other factors, the core's MTTKRP (with the next A-HALS launch's Hadamard product as its
// leading workgroups), the expansion by U^(n).
hipError_t tucker_mttkrp_into(const TuckerDesc& tk, int n, int r, const FactorPtrs& fp,
                              const MttkrpPlan& plan, const SolveBufs& b, hipStream_t s,
                              const HadamardLaunch* had) {
  const int N = tk.core.order;
  hipError_t e;
  FactorPtrs fq{};
  for (int l = 0; l < N; ++l) {
    fq.p[l] = b.Q[l];
    if (l == n) continue;
    if ((e = launch_tucker_proj(tk.U[l], fp.p[l], tk.dims[l], int(tk.core.dims[l]), r, b.Q[l],
                                nullptr, b.tq_part, s)) != hipSuccess)
      return e;
  }
  if ((e = launch_mttkrp(plan, tk.core.data, fq, b.Pc, b.mt_part, true, s, nullptr, had)) !=
      hipSuccess)
    return e;
  return launch_tucker_expand(tk.U[n], b.Pc, tk.dims[n], int(tk.core.dims[n]), r, b.P, s);
}

// Blocks the resident A-HALS kernel covers run it (fused epilogue); larger ones run the
// row-parallel A-HALS variant followed by the same epilogue steps as the other solvers.
bool fused_hals(ntf_handle* h, const ntf_her_params& p, int64_t rows, int r) {
  return p.inner_solver == 0 && hals_supported(rows, r, h->num_cus);
}

hipError_t enqueue_iteration(ntf_handle* h, const ntf_tensor& T, int r, float* const* A,
                             const ntf_her_params& p, const SolveBufs& b,
                             const MttkrpPlan* plans, const MttkrpPlan* plan_y,
                             const ntf_trace& trace, hipStream_t s, const TuckerDesc* tk,
                             const PairPlans& pp) {
  const int N = T.order;
  hipError_t e;
  // the survivor selection after the decision: A <- restart ? A_new : A_hat. The cached Gram
  // chunks are not copied: the survivor's chunks are read from gp_new or gp_hat by the flag
  // (see the Hadamard jobs below)
  SelectJob sj{};
  sj.nblocks = N;
  for (int l = 0; l < N; ++l) {
    sj.dst[l] = A[l];
    sj.a_new[l] = b.A_new[l];
    sj.a_hat[l] = b.A_hat[l];
    sj.n[l] = T.dims[l] * r;
  }
  // with the resident A-HALS kernel on the last block, its launch takes the decision too
  const bool fuse_decide = fused_hals(h, p, T.dims[N - 1], r);
  for (int n = 0; n < N; ++n) {
    const int64_t I = T.dims[n];
    HadamardJob hj{};
    hj.st = b.state;
    for (int l = 0; l < N; ++l) {
      if (l == n) continue;
      // blocks before n: their extrapolated rows of this iteration; after n: the survivor
      // of the last decision, whose chunks (new or extrapolated) stay untouched until
      // block l is updated, after every block before it
      hj.part[hj.nfac] = b.gp_hat[l];
      hj.part_new[hj.nfac] = l < n ? nullptr : b.gp_new[l];
      hj.nchunks[hj.nfac] = gram_chunks(T.dims[l], r);
      hj.nfac++;
    }
    // G^(n) (and the reset of the A-HALS wait slots) is computed by leading workgroups of
    // the tensor pass or fold that precedes the A-HALS launch, not by a launch of its own.
    // Split partials are summed by the wide reduction kernel: the A-HALS grid is too
    // narrow (one workgroup per row chunk) to stream them quickly.
    HadamardLaunch hl{hj, r, b.G32, b.G64, b.slots, hals_slot_count(I, r, p.max_inner)};
    if (tk) {
      if ((e = tucker_mttkrp_into(*tk, n, r, factors_for(n, N, A, b), plans[n], b, s, &hl)) !=
          hipSuccess)
        return e;
    } else if (pp.on) {
      // W (before block 1) and V (before block 3), each folded twice
      float* WV = n < 2 ? b.W4 : b.V4;
      const int64_t Ia = n < 2 ? T.dims[0] : T.dims[2];
      const int64_t Ib = n < 2 ? T.dims[1] : T.dims[3];
      if (n == 0 || n == 2) {
        FactorPtrs fv{};
        if (n == 0) {
          fv.p[0] = A[2];  // not read (the row mode of the view)
          fv.p[1] = A[2];
          fv.p[2] = A[3];
        } else {
          fv.p[0] = b.A_hat[0];
          fv.p[1] = b.A_hat[1];
          fv.p[2] = b.A_hat[1];  // not read
        }
        if ((e = launch_mttkrp(n == 0 ? pp.pw : pp.pv, T.data, fv, WV, b.mt_part, true, s,
                               nullptr, &hl)) != hipSuccess)
          return e;
        if ((e = launch_fold_u(WV, A[n + 1], Ia, Ib, r, b.P, s)) != hipSuccess) return e;
      } else if ((e = launch_fold_i(WV, b.A_hat[n - 1], Ia, Ib, r, b.mt_part, b.P, s, &hl)) !=
                 hipSuccess) {
        return e;
      }
    } else if (b.Y && n == 0) {
      if ((e = launch_mttkrp(*plan_y, T.data, factors_for(0, N, A, b), b.P, b.mt_part, true, s,
                             b.Y, &hl)) != hipSuccess)
        return e;
      if ((e = launch_fold_u(b.Y, A[1], T.dims[0], T.dims[1], r, b.P, s)) != hipSuccess)
        return e;
    } else if (b.Y && n == 1) {
      if ((e = launch_fold_i(b.Y, b.A_hat[0], T.dims[0], T.dims[1], r, b.mt_part, b.P, s,
                             &hl)) != hipSuccess)
        return e;
    } else if ((e = launch_mttkrp(plans[n], T.data, factors_for(n, N, A, b), b.P, b.mt_part,
                                  true, s, nullptr, &hl)) != hipSuccess) {
      return e;
    }
    if (!fused_hals(h, p, I, r)) {
      // projected-gradient (Sec. 2.2), ADMM (Sec. 2.1.2) or row-parallel A-HALS block, then
      // the steps the resident A-HALS kernel's epilogue fuses: extrapolation, Gram partials
      // of A_new and A-hat, the F-hat share of the last block
      if (p.inner_solver == 0) {
        HalsRowsArgs ra{};
        ra.W0 = A[n];
        ra.W = b.A_new[n];
        ra.P = b.P;
        ra.G = b.G32;
        ra.part = b.hr_part;
        ra.sweeps_dev = b.hr_sweeps;
        ra.rows = I;
        ra.r = r;
        ra.max_sweeps = p.max_inner;
        ra.tol = p.inner_tol;
        ra.sweeps_out = b.sweeps + n;
        if ((e = launch_hals_rows(ra, s)) != hipSuccess) return e;
      } else if (p.inner_solver == 3) {
        AdmmArgs aa{};
        aa.W0 = A[n];
        aa.W = b.A_new[n];
        aa.P = b.P;
        aa.G = b.G32;
        aa.K = b.admm_k;
        aa.rho = b.admm_rho;
        aa.part = b.admm_part;
        aa.steps_dev = b.admm_steps;
        aa.rows = I;
        aa.r = r;
        aa.max_steps = p.max_inner;
        aa.tol = p.inner_tol;
        aa.steps_out = b.sweeps + n;
        if ((e = launch_admm(aa, s)) != hipSuccess) return e;
      } else {
        PgdArgs pa{};
        pa.W0 = A[n];
        pa.W = b.A_new[n];
        pa.P = b.P;
        pa.G = b.G32;
        pa.L = b.lip;
        pa.coef = b.coef;
        pa.rows = I;
        pa.r = r;
        pa.steps = p.max_inner;
        pa.accel = p.inner_solver == 2 ? 1 : 0;
        pa.steps_out = b.sweeps + n;
        if ((e = launch_pgd(pa, s)) != hipSuccess) return e;
      }
      if ((e = launch_extrapolate(b.A_new[n], A[n], b.A_hat[n], I * r, &b.state->beta, s,
                                  p.scheme == 0)) != hipSuccess)
        return e;
      GramJob gj{};
      gj.nfac = 2;
      gj.A[0] = b.A_new[n];
      gj.out[0] = b.gp_new[n];
      gj.rows[0] = I;
      gj.A[1] = b.A_hat[n];
      gj.out[1] = b.gp_hat[n];
      gj.rows[1] = I;
      if ((e = launch_gram_partials(gj, r, s)) != hipSuccess) return e;
      if (n == N - 1 &&
          (e = launch_error_partials(b.P, b.A_new[n], b.G64, I, r, b.err_part, s)) != hipSuccess)
        return e;
      continue;
    }
    HalsArgs ha{};
    ha.wait_limit_s = h->wait_limit_s;
    ha.project = p.scheme == 0;
    ha.W0 = A[n];
    ha.W = b.A_new[n];
    ha.P = b.P;
    ha.G = b.G32;
    ha.G64 = b.G64;
    ha.rows = I;
    ha.r = r;
    ha.max_sweeps = p.max_inner;
    ha.tol = p.inner_tol;
    ha.sweeps_out = b.sweeps + n;
    ha.slots = b.slots;
    ha.flags = h->dev_flags;
    ha.A_hat = b.A_hat[n];
    ha.beta_src = &b.state->beta;
    ha.gp_new = b.gp_new[n];
    ha.gp_hat = b.gp_hat[n];
    ha.err_part = n == N - 1 ? b.err_part : nullptr;
    if (n == N - 1 && fuse_decide) {
      ha.st = b.state;
      ha.hp = p;
      ha.normT2 = b.normT2;
      ha.trace = trace;
      ha.order = N;
      ha.sweeps_src = b.sweeps;
      ha.sel = sj;
    }
    if ((e = launch_hals(ha, h->num_cus, s)) != hipSuccess) return e;
  }
  if (fuse_decide) return hipSuccess;
  const int64_t IN = T.dims[N - 1];
  DecideArgs d{};
  d.st = b.state;
  d.p = p;
  d.normT2 = b.normT2;
  d.partials = b.err_part;
  d.nparts = error_partial_count(IN, r);
  d.trace = trace;
  d.order = N;
  d.sweeps_src = b.sweeps;
  d.flags = h->dev_flags;
  if ((e = launch_her_decide(d, s)) != hipSuccess) return e;
  return launch_select(sj, b.state, s);
}

}  // namespace

// 3-way tensors: the mode-1 and mode-2 MTTKRPs share Y = T x_3 A-hat^(3) (A-hat^(3) does not
// change before the mode-3 update), so the tensor is streamed twice per iteration instead of
// three times. Used when Y is smaller than the tensor and A_3 fits one LDS block.
// The two 3-way views of a 4-way tensor and their MTTKRP plans, when W and V are each at
// most an eighth of the tensor's bytes.
PairPlans plan_pairs(const ntf_tensor& T, int r, int num_cus) {
  PairPlans pp;
  if (T.order != 4) return pp;
  const int64_t s = T.dtype == NTF_BF16 ? 2 : 4;
  int64_t n_all = 1;
  for (int l = 0; l < 4; ++l) n_all *= T.dims[l];
  const int64_t w = T.dims[0] * T.dims[1], v = T.dims[2] * T.dims[3];
  if (8 * w * r * 4 > n_all * s || 8 * v * r * 4 > n_all * s) return pp;
  if (w > (int64_t(1) << 31) - 1 || v > (int64_t(1) << 31) - 1) return pp;
  pp.tw = T;
  pp.tw.order = 3;
  pp.tw.dims[0] = w;
  pp.tw.dims[1] = T.dims[2];
  pp.tw.dims[2] = T.dims[3];
  pp.tv = T;
  pp.tv.order = 3;
  pp.tv.dims[0] = T.dims[0];
  pp.tv.dims[1] = T.dims[1];
  pp.tv.dims[2] = v;
  for (int l = 3; l < kMaxOrder; ++l) pp.tw.dims[l] = pp.tv.dims[l] = 1;
  pp.pw = plan_mttkrp(pp.tw, 0, r, num_cus, false);
  pp.pv = plan_mttkrp(pp.tv, 2, r, num_cus, false);
  pp.on = pp.pw.chunks < (int64_t(1) << 31) && pp.pv.chunks < (int64_t(1) << 31);
  return pp;
}

bool use_shared_y(const ntf_tensor& T, int r, const MttkrpPlan& plan_y) {
  if (T.order != 3 || plan_y.nvb != 1) return false;
  const int64_t s = T.dtype == NTF_BF16 ? 2 : 4;
  const int64_t ybytes = T.dims[0] * T.dims[1] * int64_t(r) * 4;
  return ybytes < T.dims[0] * T.dims[1] * T.dims[2] * s;
}

void release_solve_graph(ntf_handle* h) {
  if (!h->graph) return;
  if (h->graph->exec) (void)hipGraphExecDestroy(h->graph->exec);
  if (h->graph->graph) (void)hipGraphDestroy(h->graph->graph);
  if (h->graph->exec_u) (void)hipGraphExecDestroy(h->graph->exec_u);
  if (h->graph->graph_u) (void)hipGraphDestroy(h->graph->graph_u);
  delete h->graph;
  h->graph = nullptr;
}

}  // namespace ntf

using namespace ntf;

// Dense tensor T, or (tk != null) Tucker-format data whose logical tensor T has the sizes
// of the full tensor (its data is the core's pointer and is never read as a tensor).
static ntf_status solve_impl(ntf_handle* h, const ntf_tensor* T, const TuckerDesc* tk, int32_t r,
                             float* const* A, const ntf_her_params* params, int32_t iters,
                             ntf_her_state* state, int32_t resume, const ntf_trace* trace,
                             void* stream) {
  NTF_RETURN_IF(!h, NTF_EINVAL, "handle is NULL");
  int old_dev = -1;
  (void)hipGetDevice(&old_dev);
  if (old_dev != h->device) NTF_HIP(hipSetDevice(h->device));
  struct Restore {
    int dev;
    ~Restore() {
      if (dev >= 0) (void)hipSetDevice(dev);
    }
  } restore{old_dev != h->device ? old_dev : -1};

  ntf_status st = tk ? NTF_OK : check_tensor(T);
  if (st) return st;
  if ((st = check_rank(r))) return st;
  if ((st = check_params(params))) return st;
  NTF_RETURN_IF(iters < 0, NTF_EINVAL, "iters < 0");
  NTF_RETURN_IF(!A, NTF_EINVAL, "factor array is NULL");
  NTF_RETURN_IF(resume && !state, NTF_EINVAL, "resume needs a state");
  const int N = T->order;
  NTF_RETURN_IF((params->inner_solver == 1 || params->inner_solver == 2) &&
                    params->inner_tol != 0.0,
                NTF_EUNSUPPORTED,
                "projected-gradient blocks run exactly max_inner steps: inner_tol must be 0");
  NTF_RETURN_IF(params->inner_solver == 3 && params->max_inner > kAdmmMaxSteps,
                NTF_EUNSUPPORTED, "ADMM blocks run at most %d steps", kAdmmMaxSteps);
  for (int n = 0; n < N; ++n) {
    NTF_RETURN_IF(!A[n], NTF_EINVAL, "factor %d is NULL", n);
    if (params->inner_solver != 0) {
      NTF_RETURN_IF(r > 128, NTF_EUNSUPPORTED, "projected-gradient and ADMM kernels support r <= 128");
      continue;
    }
    if (hals_supported(T->dims[n], r, h->num_cus)) continue;
    // beyond the resident kernel's rows: the row-parallel variant
    NTF_RETURN_IF(r > kHalsRowsMaxRank || params->max_inner > kHalsRowsMaxSweeps,
                  NTF_EUNSUPPORTED,
                  "mode %d: A-HALS covers this many rows for r <= %d and at most %d sweeps", n,
                  kHalsRowsMaxRank, kHalsRowsMaxSweeps);
  }
  // the MTTKRP plans: of the tensor, or of the core for Tucker-format data
  const ntf_tensor& MT = tk ? tk->core : *T;
  MttkrpPlan plans[kMaxOrder];
  for (int n = 0; n < N; ++n) {
    plans[n] = plan_mttkrp(MT, n, r, h->num_cus, false, tuned_choice(h, MT, n, r));
    NTF_RETURN_IF(plans[n].chunks >= (int64_t(1) << 31), NTF_EUNSUPPORTED, "reduction too long");
  }
  MttkrpPlan plan_y{};
  bool shared_y = false;
  if (N == 3 && !tk) {
    plan_y = plan_mttkrp(*T, 0, r, h->num_cus, true);
    shared_y = use_shared_y(*T, r, plan_y);
  }
  ntf_trace tr{};
  if (trace) tr = *trace;

  Arena dry;
  SolveBufs b{};
  const PairPlans pp = tk ? PairPlans{} : plan_pairs(*T, r, h->num_cus);
  carve(dry, b, *T, r, params->max_inner, plans, state == nullptr, shared_y, tk, pp);
  if ((st = ensure_workspace(h, dry.off + 256))) return st;
  Arena ar{h->ws, 0};
  carve(ar, b, *T, r, params->max_inner, plans, state == nullptr, shared_y, tk, pp);
  if (state) b.state = state;

  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t n_all = 1;
  for (int l = 0; l < N; ++l) n_all *= T->dims[l];

  // ---- set-up: ||T||^2, Gram cache of A, F-hat_0 = F(A_0) (or resume) ----
  if (tk)
    NTF_HIP(launch_tucker_norm2(*tk, b.tnorm, b.normT2, s));
  else
    NTF_HIP(launch_norm2(T->data, T->dtype, n_all, b.norm_part, b.normT2, s));
  // (into both candidate caches: whichever the restart flag selects holds the chunks of A)
  GramJob gj{};
  gj.nfac = N;
  for (int l = 0; l < N; ++l) {
    gj.A[l] = A[l];
    gj.out[l] = b.gp_hat[l];
    gj.rows[l] = T->dims[l];
  }
  NTF_HIP(launch_gram_partials(gj, r, s));
  for (int l = 0; l < N; ++l) gj.out[l] = b.gp_new[l];
  NTF_HIP(launch_gram_partials(gj, r, s));
  if (!resume) {
    HadamardJob hj{};
    for (int l = 0; l < N - 1; ++l) {
      hj.part[hj.nfac] = b.gp_hat[l];
      hj.nchunks[hj.nfac] = gram_chunks(T->dims[l], r);
      hj.nfac++;
    }
    NTF_HIP(launch_hadamard(hj, r, b.G32, b.G64, nullptr, 0, s));
    FactorPtrs fp{};
    for (int l = 0; l < N; ++l) fp.p[l] = A[l];
    if (tk)
      NTF_HIP(tucker_mttkrp_into(*tk, N - 1, r, fp, plans[N - 1], b, s, nullptr));
    else
      NTF_HIP(launch_mttkrp(plans[N - 1], T->data, fp, b.P, b.mt_part, true, s));
    const int64_t IN = T->dims[N - 1];
    NTF_HIP(launch_error_partials(b.P, A[N - 1], b.G64, IN, r, b.err_part, s));
    NTF_HIP(launch_error_finalize(b.normT2, b.err_part, error_partial_count(IN, r), b.fhat0,
                                  h->dev_flags, s));
    NTF_HIP(launch_her_init(b.state, *params, b.fhat0, s));
  } else {
    NTF_HIP(launch_reset_call(b.state, s));
  }
  if (iters == 0) return NTF_OK;

  // ---- capture (or reuse) the graph of one outer iteration ----
  SolveKey key;
  std::memset(&key, 0, sizeof(key));
  key.T = T->data;
  key.dtype = T->dtype;
  key.order = N;
  key.r = r;
  for (int l = 0; l < N; ++l) {
    key.dims[l] = T->dims[l];
    key.A[l] = A[l];
  }
  key.p = *params;
  key.state = b.state;
  key.trace = tr;
  if (tk)
    for (int l = 0; l < N; ++l) key.U[l] = tk->U[l];
  key.ws_generation = h->ws_generation;
  if (!h->graph || !(h->graph->key == key)) {
    release_solve_graph(h);
    SolveGraph* g = new SolveGraph();
    g->key = key;
    // capture n iterations into (graph, exec)
    auto capture = [&](int n, hipGraph_t* graph_out, hipGraphExec_t* exec_out) -> ntf_status {
      NTF_HIP(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeRelaxed));
      hipError_t e = hipSuccess;
      for (int k = 0; k < n && e == hipSuccess; ++k)
        e = enqueue_iteration(h, *T, r, A, *params, b, plans, &plan_y, tr, h->capture_stream,
                              tk, pp);
      hipGraph_t graph = nullptr;
      hipError_t e2 = hipStreamEndCapture(h->capture_stream, &graph);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        set_error("graph capture failed: %s / %s", hipGetErrorString(e), hipGetErrorString(e2));
        return NTF_EDEVICE;
      }
      hipError_t e3 = hipGraphInstantiate(exec_out, graph, nullptr, nullptr, 0);
      if (e3 != hipSuccess) {
        (void)hipGraphDestroy(graph);
        set_error("graph instantiate failed: %s", hipGetErrorString(e3));
        return NTF_EDEVICE;
      }
      *graph_out = graph;
      return NTF_OK;
    };
    h->graph = g;  // released (both graphs) by release_solve_graph on failure below
    ntf_status cs = capture(1, &g->graph, &g->exec);
    if (cs == NTF_OK) cs = capture(kGraphUnroll, &g->graph_u, &g->exec_u);
    if (cs != NTF_OK) {
      release_solve_graph(h);
      return cs;
    }
  }
  int k = 0;
  for (; k + kGraphUnroll <= iters; k += kGraphUnroll)
    NTF_HIP(hipGraphLaunch(h->graph->exec_u, s));
  for (; k < iters; ++k) NTF_HIP(hipGraphLaunch(h->graph->exec, s));
  return NTF_OK;
}

extern "C" ntf_status ntf_solve(ntf_handle* h, const ntf_tensor* T, int32_t r, float* const* A,
                                const ntf_her_params* params, int32_t iters,
                                ntf_her_state* state, int32_t resume, const ntf_trace* trace,
                                void* stream) {
  clear_error();
  return solve_impl(h, T, nullptr, r, A, params, iters, state, resume, trace, stream);
}

extern "C" ntf_status ntf_solve_tucker(ntf_handle* h, const ntf_tucker* X, int32_t r,
                                       float* const* A, const ntf_her_params* params,
                                       int32_t iters, ntf_her_state* state, int32_t resume,
                                       const ntf_trace* trace, void* stream) {
  clear_error();
  NTF_RETURN_IF(!h, NTF_EINVAL, "handle is NULL");
  ntf_status st = check_tucker(X);
  if (st) return st;
  ntf_tensor T{};
  T.order = X->core.order;
  T.dtype = NTF_F32;
  for (int l = 0; l < T.order; ++l) T.dims[l] = X->dims[l];
  T.data = X->core.data;
  return solve_impl(h, &T, X, r, A, params, iters, state, resume, trace, stream);
}
