// C-ABI entry points: handle lifetime, error reporting, argument validation and the
// per-step calls of the hot path. Validation happens before any HIP call, so argument
// errors leave the device and every caller buffer untouched.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include <cmath>
#include <algorithm>
#include <new>
#include <vector>

#include "ntf_internal.h"

namespace ntf {

namespace {
thread_local char g_err[1024] = "";

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

ntf_status ensure_workspace(ntf_handle* h, size_t bytes) {
  if (bytes <= h->ws_size) return NTF_OK;
  NTF_HIP(hipDeviceSynchronize());
  if (h->ws) {
    NTF_HIP(hipFree(h->ws));
    h->ws = nullptr;
    h->ws_size = 0;
  }
  const size_t want = align_up(bytes + bytes / 4, size_t(1) << 20);
  if (hipMalloc(&h->ws, want) != hipSuccess) {
    (void)hipGetLastError();
    h->ws = nullptr;
    set_error("workspace allocation of %zu bytes failed", want);
    return NTF_ENOMEM;
  }
  h->ws_size = want;
  h->ws_generation += 1;
  return NTF_OK;
}

ntf_status check_tensor(const ntf_tensor* T) {
  NTF_RETURN_IF(!T, NTF_EINVAL, "tensor descriptor is NULL");
  NTF_RETURN_IF(T->order < 2 || T->order > NTF_MAX_ORDER, NTF_EINVAL,
                "tensor order %d outside [2, %d]", T->order, NTF_MAX_ORDER);
  NTF_RETURN_IF(T->dtype != NTF_F32 && T->dtype != NTF_BF16, NTF_EINVAL,
                "unsupported tensor dtype %d", T->dtype);
  NTF_RETURN_IF(!T->data, NTF_EINVAL, "tensor data pointer is NULL");
  NTF_RETURN_IF(reinterpret_cast<uintptr_t>(T->data) % 16 != 0, NTF_EINVAL,
                "tensor data must be 16-byte aligned");
  int64_t total = 1;
  for (int l = 0; l < T->order; ++l) {
    NTF_RETURN_IF(T->dims[l] < 1, NTF_EINVAL, "tensor dim %d is %lld (< 1)", l,
                  (long long)T->dims[l]);
    NTF_RETURN_IF(T->dims[l] > (int64_t(1) << 31) - 1, NTF_EUNSUPPORTED,
                  "tensor dim %d exceeds 2^31-1", l);
    NTF_RETURN_IF(total > (int64_t(1) << 62) / T->dims[l], NTF_EUNSUPPORTED,
                  "tensor too large");
    total *= T->dims[l];
  }
  // the MTTKRP streams the tensor through buffer resources with 32-bit byte offsets
  const int64_t esize = T->dtype == NTF_BF16 ? 2 : 4;
  NTF_RETURN_IF(total * esize >= (int64_t(1) << 31), NTF_EUNSUPPORTED,
                "tensor of %lld bytes: at most 2 GiB - 1 supported",
                static_cast<long long>(total * esize));
  // every mode view (L, I, R) must keep L and R below 2^31 (32-bit index arithmetic)
  for (int n = 0; n < T->order; ++n) {
    const ModeView v = make_mode_view(*T, n);
    NTF_RETURN_IF(v.L >= (int64_t(1) << 31) || v.R >= (int64_t(1) << 31), NTF_EUNSUPPORTED,
                  "mode %d: prefix/suffix extents must stay below 2^31", n);
  }
  return NTF_OK;
}

ntf_status check_tucker(const ntf_tucker* X) {
  NTF_RETURN_IF(!X, NTF_EINVAL, "Tucker descriptor is NULL");
  ntf_status st = check_tensor(&X->core);
  if (st) return st;
  NTF_RETURN_IF(X->core.dtype != NTF_F32, NTF_EUNSUPPORTED, "the Tucker core must be float32");
  for (int p = 0; p < X->core.order; ++p) {
    NTF_RETURN_IF(!X->U[p], NTF_EINVAL, "basis %d is NULL", p);
    NTF_RETURN_IF(X->dims[p] < 1, NTF_EINVAL, "size %d of the Tucker tensor is < 1", p);
    NTF_RETURN_IF(X->core.dims[p] > 4096, NTF_EUNSUPPORTED, "Tucker rank %d above 4096", p);
    NTF_RETURN_IF(X->dims[p] > (int64_t(1) << 31) - 1, NTF_EUNSUPPORTED,
                  "size %d of the Tucker tensor too large", p);
  }
  return NTF_OK;
}

ntf_status check_rank(int32_t r) {
  NTF_RETURN_IF(r < 1 || r > NTF_MAX_RANK, NTF_EINVAL, "rank %d outside [1, %d]", r,
                NTF_MAX_RANK);
  return NTF_OK;
}

ntf_status check_params(const ntf_her_params* p) {
  NTF_RETURN_IF(!p, NTF_EINVAL, "params is NULL");
  NTF_RETURN_IF(!(p->beta0 >= 0.0 && p->beta0 < 1.0), NTF_EINVAL, "beta0 must lie in [0, 1)");
  NTF_RETURN_IF(!(1.0 <= p->gamma_bar && p->gamma_bar <= p->gamma && p->gamma <= p->eta),
                NTF_EINVAL, "need 1 <= gamma_bar <= gamma <= eta");
  NTF_RETURN_IF(p->max_inner < 1 || p->max_inner > kMaxSweeps, NTF_EINVAL,
                "max_inner must lie in [1, %d]", kMaxSweeps);
  NTF_RETURN_IF(!(p->inner_tol >= 0.0), NTF_EINVAL, "inner_tol must be >= 0");
  NTF_RETURN_IF(p->inner_solver < 0 || p->inner_solver > 3, NTF_EINVAL,
                "inner_solver %d outside [0, 3]", p->inner_solver);
  NTF_RETURN_IF(p->scheme != 0 && p->scheme != 1, NTF_EINVAL, "scheme %d outside [0, 1]",
                p->scheme);
  return NTF_OK;
}

}  // namespace ntf

using namespace ntf;

#define NTF_GUARD(h)                                                   \
  NTF_RETURN_IF(!(h), NTF_EINVAL, "handle is NULL");                   \
  DeviceGuard guard_((h)->device);                                     \
  NTF_RETURN_IF(!guard_.ok, NTF_EDEVICE, "cannot select device %d", (h)->device)

extern "C" {

const char* ntf_last_error(void) { return g_err; }

const char* ntf_status_string(ntf_status s) {
  switch (s) {
    case NTF_OK: return "NTF_OK";
    case NTF_EINVAL: return "NTF_EINVAL";
    case NTF_ENOMEM: return "NTF_ENOMEM";
    case NTF_EDEVICE: return "NTF_EDEVICE";
    case NTF_EUNSUPPORTED: return "NTF_EUNSUPPORTED";
    case NTF_ENUMERIC: return "NTF_ENUMERIC";
  }
  return "NTF_UNKNOWN";
}

const char* ntf_version(void) { return "ntf-her-gfx950 0.1"; }

ntf_status ntf_handle_create(ntf_handle** out, int device) {
  clear_error();
  NTF_RETURN_IF(!out, NTF_EINVAL, "output handle pointer is NULL");
  *out = nullptr;
  int count = 0;
  NTF_HIP(hipGetDeviceCount(&count));
  NTF_RETURN_IF(device < 0 || device >= count, NTF_EINVAL, "device %d not present (%d devices)",
                device, count);
  DeviceGuard guard(device);
  NTF_RETURN_IF(!guard.ok, NTF_EDEVICE, "cannot select device %d", device);
  hipDeviceProp_t prop;
  NTF_HIP(hipGetDeviceProperties(&prop, device));
  NTF_RETURN_IF(std::strncmp(prop.gcnArchName, "gfx950", 6) != 0, NTF_EUNSUPPORTED,
                "device %d is %s; this library is built for gfx950 only", device,
                prop.gcnArchName);
  ntf_handle* h = new ntf_handle();
  h->device = device;
  h->num_cus = prop.multiProcessorCount;
  h->lds_per_block = prop.sharedMemPerBlock;
  // the scratch-free entry point's device array: its address on this device, once
  {
    const ntf_status st = noalloc_scratch_attach(device);
    if (st != NTF_OK) {
      delete h;
      return st;
    }
  }
  if (hipMalloc(&h->dev_flags, sizeof(uint32_t)) != hipSuccess) {
    delete h;
    set_error("flag allocation failed");
    return NTF_ENOMEM;
  }
  if (hipMemset(h->dev_flags, 0, sizeof(uint32_t)) != hipSuccess ||
      hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(h->dev_flags);
    delete h;
    set_error("handle initialisation failed");
    return NTF_EDEVICE;
  }
  *out = h;
  return NTF_OK;
}

void ntf_handle_destroy(ntf_handle* h) {
  if (!h) return;
  DeviceGuard guard(h->device);
  (void)hipDeviceSynchronize();
  release_solve_graph(h);
  if (h->bgraph) (void)hipGraphExecDestroy(h->bgraph);
  if (h->bstage_done) (void)hipEventDestroy(h->bstage_done);
  if (h->bstage) (void)hipHostFree(h->bstage);
  if (h->bws) (void)hipFree(h->bws);
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  if (h->ws) (void)hipFree(h->ws);
  if (h->dev_flags) (void)hipFree(h->dev_flags);
  delete h;
}

ntf_status ntf_device_flags(ntf_handle* h, void* stream, uint32_t* flags_out) {
  clear_error();
  NTF_GUARD(h);
  NTF_RETURN_IF(!flags_out, NTF_EINVAL, "flags_out is NULL");
  NTF_HIP(hipStreamSynchronize(as_stream(stream)));
  uint32_t v = 0;
  NTF_HIP(hipMemcpy(&v, h->dev_flags, sizeof(v), hipMemcpyDeviceToHost));
  NTF_HIP(hipMemset(h->dev_flags, 0, sizeof(uint32_t)));
  *flags_out = v;
  return NTF_OK;
}

ntf_status ntf_handle_set_wait_limit(ntf_handle* h, double seconds) {
  clear_error();
  NTF_RETURN_IF(!h, NTF_EINVAL, "handle is NULL");
  NTF_RETURN_IF(!(seconds >= 0.0 && seconds <= 60.0), NTF_EINVAL,
                "wait limit %g s outside [0, 60]", seconds);
  if (h->wait_limit_s != seconds) {
    DeviceGuard guard(h->device);
    NTF_RETURN_IF(!guard.ok, NTF_EDEVICE, "cannot select device %d", h->device);
    NTF_HIP(hipDeviceSynchronize());
    release_solve_graph(h);  // its A-HALS launches carry the old limit
    h->wait_limit_s = seconds;
  }
  return NTF_OK;
}

ntf_status ntf_norm2(ntf_handle* h, const ntf_tensor* T, double* out, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_tensor(T);
  if (st) return st;
  NTF_RETURN_IF(!out, NTF_EINVAL, "out is NULL");
  int64_t n = 1;
  for (int l = 0; l < T->order; ++l) n *= T->dims[l];
  st = ensure_workspace(h, sizeof(double) * norm2_partials() + 256);
  if (st) return st;
  NTF_HIP(launch_norm2(T->data, T->dtype, n, reinterpret_cast<double*>(h->ws), out,
                       as_stream(stream)));
  return NTF_OK;
}

ntf_status ntf_cast_bf16(ntf_handle* h, const float* src, uint16_t* dst, int64_t n,
                         void* stream) {
  clear_error();
  NTF_GUARD(h);
  NTF_RETURN_IF(n < 0, NTF_EINVAL, "n < 0");
  if (n == 0) return NTF_OK;
  NTF_RETURN_IF(!src || !dst, NTF_EINVAL, "src/dst is NULL");
  NTF_RETURN_IF(reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 8,
                NTF_EINVAL, "src must be 16-byte and dst 8-byte aligned");
  NTF_HIP(launch_cast_bf16(src, dst, n, as_stream(stream)));
  return NTF_OK;
}

ntf_status ntf_mttkrp(ntf_handle* h, const ntf_tensor* T, const float* const* A, int32_t r,
                      int32_t mode, float* P, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_tensor(T);
  if (st) return st;
  if ((st = check_rank(r))) return st;
  NTF_RETURN_IF(mode < 0 || mode >= T->order, NTF_EINVAL, "mode %d outside [0, %d)", mode,
                T->order);
  NTF_RETURN_IF(!A || !P, NTF_EINVAL, "factor array or output is NULL");
  FactorPtrs fp{};
  for (int l = 0; l < T->order; ++l) {
    if (l == mode) continue;
    NTF_RETURN_IF(!A[l], NTF_EINVAL, "factor %d is NULL", l);
    fp.p[l] = A[l];
  }
  fp.p[mode] = A[(mode + 1) % T->order];  // never read; keeps the slot non-null
  const MttkrpPlan pl =
      plan_mttkrp(*T, mode, r, h->num_cus, false, tuned_choice(h, *T, mode, r));
  NTF_RETURN_IF(pl.chunks >= (int64_t(1) << 31), NTF_EUNSUPPORTED, "reduction too long");
  st = ensure_workspace(h, pl.partial_floats() * sizeof(float) + 256);
  if (st) return st;
  NTF_HIP(launch_mttkrp(pl, T->data, fp, P, reinterpret_cast<float*>(h->ws), true,
                        as_stream(stream)));
  return NTF_OK;
}

ntf_status ntf_tucker_mttkrp(ntf_handle* h, const ntf_tucker* X, const float* const* A,
                             int32_t r, int32_t mode, float* P, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_tucker(X);
  if (st) return st;
  if ((st = check_rank(r))) return st;
  const int N = X->core.order;
  NTF_RETURN_IF(mode < 0 || mode >= N, NTF_EINVAL, "mode %d outside [0, %d)", mode, N);
  NTF_RETURN_IF(!A || !P, NTF_EINVAL, "factor array or output is NULL");
  for (int l = 0; l < N; ++l)
    NTF_RETURN_IF(l != mode && !A[l], NTF_EINVAL, "factor %d is NULL", l);
  const MttkrpPlan pl =
      plan_mttkrp(X->core, mode, r, h->num_cus, false, tuned_choice(h, X->core, mode, r));
  size_t qp = 1;
  for (int l = 0; l < N; ++l)
    qp = std::max(qp, tucker_proj_part_doubles(X->dims[l], int(X->core.dims[l]), r));
  Arena dry;
  float* Q[kMaxOrder] = {};
  for (int l = 0; l < N; ++l) dry.take<float>(size_t(X->core.dims[l]) * r);
  dry.take<float>(size_t(X->core.dims[mode]) * r);
  dry.take<float>(std::max<size_t>(pl.partial_floats(), 1));
  dry.take<double>(qp);
  if ((st = ensure_workspace(h, dry.off + 256))) return st;
  Arena ar{h->ws, 0};
  for (int l = 0; l < N; ++l) Q[l] = ar.take<float>(size_t(X->core.dims[l]) * r);
  float* Pc = ar.take<float>(size_t(X->core.dims[mode]) * r);
  float* part = ar.take<float>(std::max<size_t>(pl.partial_floats(), 1));
  double* qpart = ar.take<double>(qp);
  hipStream_t s = as_stream(stream);
  FactorPtrs fq{};
  for (int l = 0; l < N; ++l) {
    fq.p[l] = Q[l];
    if (l != mode)
      NTF_HIP(launch_tucker_proj(X->U[l], A[l], X->dims[l], int(X->core.dims[l]), r, Q[l],
                                 nullptr, qpart, s));
  }
  NTF_HIP(launch_mttkrp(pl, X->core.data, fq, Pc, part, true, s));
  NTF_HIP(launch_tucker_expand(X->U[mode], Pc, X->dims[mode], int(X->core.dims[mode]), r, P, s));
  return NTF_OK;
}

ntf_status ntf_tucker_norm2(ntf_handle* h, const ntf_tucker* X, double* out, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_tucker(X);
  if (st) return st;
  NTF_RETURN_IF(!out, NTF_EINVAL, "out is NULL");
  if ((st = ensure_workspace(h, tucker_norm_workspace_doubles(*X) * sizeof(double) + 256)))
    return st;
  NTF_HIP(launch_tucker_norm2(*X, reinterpret_cast<double*>(h->ws), out, as_stream(stream)));
  return NTF_OK;
}

ntf_status ntf_mttkrp_multi(ntf_handle* h, const ntf_tensor* T, const float* const* A,
                            int32_t r, int32_t mask, float* const* P, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_tensor(T);
  if (st) return st;
  if ((st = check_rank(r))) return st;
  const int N = T->order;
  NTF_RETURN_IF(mask <= 0 || mask >= (1 << N), NTF_EINVAL, "mode mask %d outside [1, 2^%d)",
                mask, N);
  NTF_RETURN_IF(!A || !P, NTF_EINVAL, "factor or output array is NULL");
  // every factor is read by some requested mode unless only that factor's mode is requested
  FactorPtrs fp{};
  for (int l = 0; l < N; ++l) {
    NTF_RETURN_IF(!A[l] && (mask & ~(1 << l)) != 0, NTF_EINVAL, "factor %d is NULL", l);
    fp.p[l] = A[l] ? A[l] : A[(l + 1) % N];
    NTF_RETURN_IF(((mask >> l) & 1) && !P[l], NTF_EINVAL, "output %d is NULL", l);
  }
  // 4-way bf16, every mode asked: the fused one-pass kernel where its shape applies
  if (mask == 15 && fused4_applies(*T, r)) {
    if ((st = ensure_workspace(h, fused4_workspace_floats(*T, r, h->num_cus) * 4 + 256)))
      return st;
    NTF_HIP(launch_fused4(*T, A, r, h->num_cus, P, reinterpret_cast<float*>(h->ws),
                          as_stream(stream)));
    return NTF_OK;
  }
  MttkrpPlan plans[kMaxOrder];
  size_t need = 0;
  for (int n = 0; n < N; ++n) {
    if (!((mask >> n) & 1)) continue;
    plans[n] = plan_mttkrp(*T, n, r, h->num_cus, false, tuned_choice(h, *T, n, r));
    NTF_RETURN_IF(plans[n].chunks >= (int64_t(1) << 31), NTF_EUNSUPPORTED,
                  "reduction too long");
    need = std::max(need, plans[n].partial_floats());
  }
  // 3-way, modes 1 and 2 both asked: one pass forms Y = T x_3 A_3, two folds finish them
  MttkrpPlan plan_y{};
  bool shared = false;
  if (N == 3 && (mask & 3) == 3) {
    plan_y = plan_mttkrp(*T, 0, r, h->num_cus, true);
    shared = use_shared_y(*T, r, plan_y) && plan_y.chunks < (int64_t(1) << 31);
  }
  Arena dry;
  float* part = nullptr;
  float* Y = nullptr;
  if (shared)
    need = std::max<size_t>(need, size_t(fold_i_splits(T->dims[0], T->dims[1], r)) *
                                      T->dims[1] * r);
  dry.take<float>(std::max<size_t>(need, 1));
  if (shared) dry.take<float>(size_t(T->dims[0]) * T->dims[1] * r + 64);
  if ((st = ensure_workspace(h, dry.off + 256))) return st;
  Arena ar{h->ws, 0};
  part = ar.take<float>(std::max<size_t>(need, 1));
  if (shared) Y = ar.take<float>(size_t(T->dims[0]) * T->dims[1] * r + 64);
  hipStream_t s = as_stream(stream);
  for (int n = 0; n < N; ++n) {
    if (!((mask >> n) & 1)) continue;
    if (shared && n == 0) {
      NTF_HIP(launch_mttkrp(plan_y, T->data, fp, P[0], part, true, s, Y));
      NTF_HIP(launch_fold_u(Y, A[1], T->dims[0], T->dims[1], r, P[0], s));
    } else if (shared && n == 1) {
      NTF_HIP(launch_fold_i(Y, A[0], T->dims[0], T->dims[1], r, part, P[1], s));
    } else {
      NTF_HIP(launch_mttkrp(plans[n], T->data, fp, P[n], part, true, s));
    }
  }
  return NTF_OK;
}

ntf_status ntf_mttkrp_autotune(ntf_handle* h, const ntf_tensor* T, const float* const* A,
                               int32_t r, int32_t mode, float* P, int32_t reps,
                               int32_t* kernel_out, int32_t* wm_out, float* ms_out,
                               void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_tensor(T);
  if (st) return st;
  if ((st = check_rank(r))) return st;
  NTF_RETURN_IF(mode < 0 || mode >= T->order, NTF_EINVAL, "mode %d outside [0, %d)", mode,
                T->order);
  NTF_RETURN_IF(!A || !P, NTF_EINVAL, "factor array or output is NULL");
  NTF_RETURN_IF(reps < 1 || reps > 1000, NTF_EINVAL, "reps %d outside [1, 1000]", reps);
  FactorPtrs fp{};
  for (int l = 0; l < T->order; ++l) {
    if (l == mode) continue;
    NTF_RETURN_IF(!A[l], NTF_EINVAL, "factor %d is NULL", l);
    fp.p[l] = A[l];
  }
  fp.p[mode] = A[(mode + 1) % T->order];
  MttkrpChoice cand[8];
  const int nc = mttkrp_candidates(*T, mode, r, cand, 8);
  MttkrpPlan plans[8];
  size_t need = 0;
  for (int c = 0; c < nc; ++c) {
    plans[c] = plan_mttkrp(*T, mode, r, h->num_cus, false, &cand[c]);
    NTF_RETURN_IF(plans[c].chunks >= (int64_t(1) << 31), NTF_EUNSUPPORTED,
                  "reduction too long");
    need = std::max(need, plans[c].partial_floats());
  }
  if ((st = ensure_workspace(h, need * sizeof(float) + 256))) return st;
  hipStream_t s = as_stream(stream);
  float* part = reinterpret_cast<float*>(h->ws);
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  NTF_HIP(hipEventCreate(&ev.a));
  NTF_HIP(hipEventCreate(&ev.b));
  int best = 0;
  float best_ms = 0.f;
  for (int c = 0; c < nc; ++c) {
    NTF_HIP(launch_mttkrp(plans[c], T->data, fp, P, part, true, s));  // warm-up
    NTF_HIP(hipEventRecord(ev.a, s));
    for (int k = 0; k < reps; ++k) NTF_HIP(launch_mttkrp(plans[c], T->data, fp, P, part, true, s));
    NTF_HIP(hipEventRecord(ev.b, s));
    NTF_HIP(hipEventSynchronize(ev.b));
    float ms = 0.f;
    NTF_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    ms /= float(reps);
    // the planner's default (candidate 0) is kept unless another shape is faster by more
    // than 3 % (timing noise would otherwise pick shapes at random)
    if (c == 0 || ms < best_ms * (best == 0 ? 0.97f : 1.f)) {
      best = c;
      best_ms = ms;
    }
  }
  // the result in P comes from the chosen shape
  NTF_HIP(launch_mttkrp(plans[best], T->data, fp, P, part, true, s));
  h->tune[tune_key(*T, mode, r)] = cand[best];
  release_solve_graph(h);  // cached solver graphs were built with the previous plans
  if (kernel_out) *kernel_out = cand[best].kernel;
  if (wm_out) *wm_out = cand[best].wm;
  if (ms_out) *ms_out = best_ms;
  return NTF_OK;
}

int64_t ntf_tune_export(ntf_handle* h, char* buf, int64_t cap) {
  if (!h) return -1;
  std::string text;
  for (const auto& kv : h->tune)
    text += kv.first + " " + std::to_string(kv.second.kernel) + " " +
            std::to_string(kv.second.wm) + "\n";
  const int64_t need = int64_t(text.size()) + 1;
  if (buf && cap >= need) std::memcpy(buf, text.c_str(), size_t(need));
  return need;
}

ntf_status ntf_tune_import(ntf_handle* h, const char* text) {
  clear_error();
  NTF_RETURN_IF(!h, NTF_EINVAL, "handle is NULL");
  NTF_RETURN_IF(!text, NTF_EINVAL, "text is NULL");
  std::map<std::string, MttkrpChoice> add;
  const char* q = text;
  int line = 0;
  while (*q) {
    const char* e = std::strchr(q, '\n');
    const std::string ln(q, e ? size_t(e - q) : std::strlen(q));
    q = e ? e + 1 : q + ln.size();
    ++line;
    if (ln.find_first_not_of(" \t\r") == std::string::npos) continue;
    char key[256];
    int kernel = -1, wm = -1;
    char extra = 0;
    const int got = std::sscanf(ln.c_str(), "%255s %d %d %c", key, &kernel, &wm, &extra);
    NTF_RETURN_IF(got != 3 || kernel < 0 || kernel > 2 || !(wm == 0 || wm == 1 || wm == 2 || wm == 4),
                  NTF_EINVAL, "tuning line %d is not '<key> <kernel 0..2> <wm 0|1|2|4>'", line);
    add[key] = MttkrpChoice{kernel, wm};
  }
  for (const auto& kv : add) h->tune[kv.first] = kv.second;
  if (!add.empty()) {
    DeviceGuard guard_(h->device);
    release_solve_graph(h);
  }
  return NTF_OK;
}

ntf_status ntf_gram(ntf_handle* h, const float* const* A, const int64_t* rows, int32_t nfac,
                    int32_t r, int32_t exclude, float* G32, double* G64, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_rank(r);
  if (st) return st;
  NTF_RETURN_IF(nfac < 1 || nfac > NTF_MAX_ORDER, NTF_EINVAL, "nfac %d outside [1, %d]", nfac,
                NTF_MAX_ORDER);
  NTF_RETURN_IF(exclude < -1 || exclude >= nfac, NTF_EINVAL, "exclude %d outside [-1, %d)",
                exclude, nfac);
  NTF_RETURN_IF(!A || !rows, NTF_EINVAL, "factor or rows array is NULL");
  NTF_RETURN_IF(!G32 && !G64, NTF_EINVAL, "both outputs are NULL");
  GramJob job{};
  HadamardJob hj{};
  Arena dry;
  for (int l = 0; l < nfac; ++l) {
    if (l == exclude) continue;
    NTF_RETURN_IF(!A[l], NTF_EINVAL, "factor %d is NULL", l);
    NTF_RETURN_IF(rows[l] < 1, NTF_EINVAL, "rows[%d] < 1", l);
    dry.take<double>(size_t(gram_chunks(rows[l], r)) * r * r);
  }
  st = ensure_workspace(h, dry.off + 256);
  if (st) return st;
  Arena ar{h->ws, 0};
  for (int l = 0; l < nfac; ++l) {
    if (l == exclude) continue;
    double* part = ar.take<double>(size_t(gram_chunks(rows[l], r)) * r * r);
    job.A[job.nfac] = A[l];
    job.out[job.nfac] = part;
    job.rows[job.nfac] = rows[l];
    job.nfac++;
    hj.part[hj.nfac] = part;
    hj.nchunks[hj.nfac] = gram_chunks(rows[l], r);
    hj.nfac++;
  }
  hipStream_t s = as_stream(stream);
  if (job.nfac > 0) NTF_HIP(launch_gram_partials(job, r, s));
  NTF_HIP(launch_hadamard(hj, r, G32, G64, nullptr, 0, s));
  return NTF_OK;
}

ntf_status ntf_hals_update(ntf_handle* h, float* W, const float* P, const float* G,
                           int64_t rows, int32_t r, int32_t max_sweeps, double tol,
                           int32_t* sweeps_done, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_rank(r);
  if (st) return st;
  NTF_RETURN_IF(!W || !P || !G, NTF_EINVAL, "W, P or G is NULL");
  NTF_RETURN_IF(rows < 1, NTF_EINVAL, "rows < 1");
  NTF_RETURN_IF(max_sweeps < 1 || max_sweeps > kMaxSweeps, NTF_EINVAL,
                "max_sweeps outside [1, %d]", kMaxSweeps);
  NTF_RETURN_IF(!(tol >= 0.0), NTF_EINVAL, "tol must be >= 0");
  NTF_RETURN_IF(!hals_supported(rows, r, h->num_cus), NTF_EUNSUPPORTED,
                "A-HALS kernel supports r <= 128 and at most 256 workgroups of rows");
  const int64_t nslots = hals_slot_count(rows, r, max_sweeps);
  st = ensure_workspace(h, size_t(nslots) * sizeof(double) + 256);
  if (st) return st;
  hipStream_t s = as_stream(stream);
  double* slots = reinterpret_cast<double*>(h->ws);
  NTF_HIP(launch_fill_sentinel(slots, nslots, s));
  HalsArgs a{};
  a.wait_limit_s = h->wait_limit_s;
  a.W0 = W;
  a.W = W;
  a.P = P;
  a.G = G;
  a.rows = rows;
  a.r = r;
  a.max_sweeps = max_sweeps;
  a.tol = tol;
  a.sweeps_out = sweeps_done;
  a.slots = slots;
  a.flags = h->dev_flags;
  NTF_HIP(launch_hals(a, h->num_cus, s));
  return NTF_OK;
}

ntf_status ntf_pgd_update(ntf_handle* h, float* W, const float* P, const float* G,
                          int64_t rows, int32_t r, int32_t steps, int32_t accel,
                          double* L_out, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_rank(r);
  if (st) return st;
  NTF_RETURN_IF(!W || !P || !G || !L_out, NTF_EINVAL, "W, P, G or L_out is NULL");
  NTF_RETURN_IF(rows < 1, NTF_EINVAL, "rows < 1");
  NTF_RETURN_IF(steps < 1 || steps > kMaxSweeps, NTF_EINVAL, "steps outside [1, %d]",
                kMaxSweeps);
  NTF_RETURN_IF(accel != 0 && accel != 1, NTF_EINVAL, "accel must be 0 or 1");
  NTF_RETURN_IF(r > 128, NTF_EUNSUPPORTED, "projected-gradient kernel supports r <= 128");
  if ((st = ensure_workspace(h, size_t(steps) * sizeof(float) + 256))) return st;
  PgdArgs a{};
  a.coef = reinterpret_cast<float*>(h->ws);
  a.W0 = W;
  a.W = W;
  a.P = P;
  a.G = G;
  a.L = L_out;
  a.rows = rows;
  a.r = r;
  a.steps = steps;
  a.accel = accel;
  NTF_HIP(launch_pgd(a, as_stream(stream)));
  return NTF_OK;
}

ntf_status ntf_admm_update(ntf_handle* h, float* W, const float* P, const float* G,
                           int64_t rows, int32_t r, int32_t max_steps, double tol,
                           int32_t* steps_done, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_rank(r);
  if (st) return st;
  NTF_RETURN_IF(!W || !P || !G, NTF_EINVAL, "W, P or G is NULL");
  NTF_RETURN_IF(rows < 1, NTF_EINVAL, "rows < 1");
  NTF_RETURN_IF(max_steps < 1 || max_steps > kMaxSweeps, NTF_EINVAL,
                "max_steps outside [1, %d]", kMaxSweeps);
  NTF_RETURN_IF(!(tol >= 0.0), NTF_EINVAL, "tol must be >= 0");
  NTF_RETURN_IF(r > 128, NTF_EUNSUPPORTED, "ADMM kernel supports r <= 128");
  NTF_RETURN_IF(max_steps > kAdmmMaxSteps, NTF_EUNSUPPORTED,
                "ADMM kernel runs at most %d steps per block", kAdmmMaxSteps);
  const int64_t nwg = admm_workgroups(rows, r);
  const size_t kb = align_up(size_t(r) * r * sizeof(float), 256);
  const size_t pb = align_up(size_t(max_steps) * nwg * sizeof(double), 256);
  if ((st = ensure_workspace(h, kb + pb + 512))) return st;
  AdmmArgs a{};
  a.K = reinterpret_cast<float*>(h->ws);
  a.part = reinterpret_cast<double*>(h->ws + kb);
  a.rho = reinterpret_cast<float*>(h->ws + kb + pb);
  a.steps_dev = reinterpret_cast<int32_t*>(h->ws + kb + pb + 256);
  a.W0 = W;
  a.W = W;
  a.P = P;
  a.G = G;
  a.rows = rows;
  a.r = r;
  a.max_steps = max_steps;
  a.tol = tol;
  a.steps_out = steps_done;
  NTF_HIP(launch_admm(a, as_stream(stream)));
  return NTF_OK;
}

ntf_status ntf_her_step(ntf_handle* h, ntf_her_op op, ntf_her_state* state,
                        const ntf_her_params* params, int32_t nblocks, const int64_t* rows,
                        int32_t r, float* const* A, float* const* A_new, float* const* A_hat,
                        int32_t block, const double* fhat, void* stream) {
  clear_error();
  NTF_GUARD(h);
  NTF_RETURN_IF(!state, NTF_EINVAL, "state is NULL");
  hipStream_t s = as_stream(stream);
  if (op == NTF_HER_INIT) {
    ntf_status st = check_params(params);
    if (st) return st;
    NTF_RETURN_IF(!fhat, NTF_EINVAL, "INIT needs fhat = F(A_0)");
    NTF_HIP(launch_her_init(state, *params, fhat, s));
    return NTF_OK;
  }
  ntf_status st = check_rank(r);
  if (st) return st;
  NTF_RETURN_IF(nblocks < 1 || nblocks > NTF_MAX_ORDER, NTF_EINVAL, "nblocks outside [1, %d]",
                NTF_MAX_ORDER);
  NTF_RETURN_IF(!rows || !A || !A_new || !A_hat, NTF_EINVAL, "block arrays are NULL");
  if (op == NTF_HER_EXTRAPOLATE) {
    NTF_RETURN_IF(block < 0 || block >= nblocks, NTF_EINVAL, "block %d outside [0, %d)", block,
                  nblocks);
    NTF_RETURN_IF(!A[block] || !A_new[block] || !A_hat[block], NTF_EINVAL,
                  "block %d has a NULL buffer", block);
    NTF_RETURN_IF(rows[block] < 1, NTF_EINVAL, "rows[%d] < 1", block);
    // projected (eq. extproj_her) unless params name Bro's scheme (Sec. 3.3)
    NTF_HIP(launch_extrapolate(A_new[block], A[block], A_hat[block], rows[block] * r,
                               &state->beta, s, !(params && params->scheme == 1)));
    return NTF_OK;
  }
  NTF_RETURN_IF(op != NTF_HER_DECIDE, NTF_EINVAL, "unknown op %d", int(op));
  if ((st = check_params(params))) return st;
  NTF_RETURN_IF(!fhat, NTF_EINVAL, "DECIDE needs fhat");
  SelectJob j{};
  j.nblocks = nblocks;
  for (int b = 0; b < nblocks; ++b) {
    NTF_RETURN_IF(!A[b] || !A_new[b] || !A_hat[b], NTF_EINVAL, "block %d has a NULL buffer", b);
    NTF_RETURN_IF(rows[b] < 1, NTF_EINVAL, "rows[%d] < 1", b);
    j.dst[b] = A[b];
    j.a_new[b] = A_new[b];
    j.a_hat[b] = A_hat[b];
    j.n[b] = rows[b] * r;
  }
  DecideArgs d{};
  d.st = state;
  d.p = *params;
  d.fhat = fhat;
  d.flags = h->dev_flags;
  d.order = nblocks;
  NTF_HIP(launch_her_decide(d, s));
  NTF_HIP(launch_select(j, state, s));
  return NTF_OK;
}

ntf_status ntf_error(ntf_handle* h, const double* normT2, const float* P, const float* A,
                     const double* G, int64_t rows, int32_t r, double* fhat, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_rank(r);
  if (st) return st;
  NTF_RETURN_IF(!normT2 || !P || !A || !G || !fhat, NTF_EINVAL, "NULL argument");
  NTF_RETURN_IF(rows < 1, NTF_EINVAL, "rows < 1");
  const int64_t np = error_partial_count(rows, r);
  st = ensure_workspace(h, size_t(np) * sizeof(double) + 256);
  if (st) return st;
  hipStream_t s = as_stream(stream);
  double* part = reinterpret_cast<double*>(h->ws);
  NTF_HIP(launch_error_partials(P, A, G, rows, r, part, s));
  NTF_HIP(launch_error_finalize(normT2, part, np, fhat, h->dev_flags, s));
  return NTF_OK;
}

ntf_status ntf_cp_loss(ntf_handle* h, const double* normT2, const float* P, const float* A,
                       const double* G, int64_t rows, int32_t r, double* loss, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_rank(r);
  if (st) return st;
  NTF_RETURN_IF(!normT2 || !P || !A || !G || !loss, NTF_EINVAL, "NULL argument");
  NTF_RETURN_IF(rows < 1, NTF_EINVAL, "rows < 1");
  const int64_t np = error_partial_count(rows, r);
  st = ensure_workspace(h, size_t(np) * sizeof(double) + 256);
  if (st) return st;
  hipStream_t s = as_stream(stream);
  double* part = reinterpret_cast<double*>(h->ws);
  NTF_HIP(launch_error_partials(P, A, G, rows, r, part, s));
  NTF_HIP(launch_error_finalize(normT2, part, np, loss, h->dev_flags, s, 1.0));
  return NTF_OK;
}

ntf_status ntf_cp_grad(ntf_handle* h, const float* A, const float* P, const double* G,
                       int64_t rows, int32_t r, const double* scale, float alpha, float* grad,
                       void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_rank(r);
  if (st) return st;
  NTF_RETURN_IF(!A || !P || !G || !grad, NTF_EINVAL, "NULL argument");
  NTF_RETURN_IF(rows < 1, NTF_EINVAL, "rows < 1");
  NTF_RETURN_IF(!std::isfinite(alpha), NTF_EINVAL, "alpha is not finite");
  NTF_HIP(launch_cp_grad(A, P, G, rows, r, scale, alpha, grad, as_stream(stream)));
  return NTF_OK;
}

}  // extern "C"

namespace {
ntf_status solve_batched_impl(ntf_handle* h, int32_t nprob, const ntf_problem* probs,
                              const ntf_her_params* params, int32_t iters, int32_t resume,
                              void* stream) {
  NTF_GUARD(h);
  NTF_RETURN_IF(nprob < 1 || nprob > 65535, NTF_EINVAL, "nprob %d outside [1, 65535]", nprob);
  NTF_RETURN_IF(!probs, NTF_EINVAL, "probs is NULL");
  NTF_RETURN_IF(iters < 0, NTF_EINVAL, "iters < 0");
  ntf_status st = check_params(params);
  if (st) return st;
  NTF_RETURN_IF(params->inner_solver != 0, NTF_EUNSUPPORTED,
                "the batched solver uses A-HALS blocks only (inner_solver 0)");
  NTF_RETURN_IF(params->scheme != 0, NTF_EUNSUPPORTED,
                "the batched solver uses HER's extrapolation only (scheme 0)");
  std::vector<BatchedProblem> bp(static_cast<size_t>(nprob));
  std::vector<int64_t> cost(static_cast<size_t>(nprob));
  size_t ws_bytes = 0;
  for (int b = 0; b < nprob; ++b) {
    const ntf_problem& q = probs[b];
    NTF_RETURN_IF(q.T.order != 3, NTF_EUNSUPPORTED, "problem %d: order %d (batched: 3-way)", b,
                  q.T.order);
    NTF_RETURN_IF(q.T.dtype != NTF_F32, NTF_EUNSUPPORTED, "problem %d: tensor must be float32",
                  b);
    NTF_RETURN_IF(!q.T.data, NTF_EINVAL, "problem %d: tensor data is NULL", b);
    NTF_RETURN_IF(q.r < 1 || q.r > kBatchedMaxRank, NTF_EUNSUPPORTED,
                  "problem %d: rank %d outside [1, %d]", b, q.r, kBatchedMaxRank);
    NTF_RETURN_IF(q.reserved != 0, NTF_EINVAL, "problem %d: reserved must be 0", b);
    NTF_RETURN_IF(resume && !q.state, NTF_EINVAL, "problem %d: resume needs a state", b);
    BatchedProblem& d = bp[size_t(b)];
    d.T = static_cast<const float*>(q.T.data);
    for (int n = 0; n < 3; ++n) {
      NTF_RETURN_IF(q.T.dims[n] < 1 || q.T.dims[n] > kBatchedMaxDim, NTF_EUNSUPPORTED,
                    "problem %d: dim %d = %lld outside [1, %d]", b, n,
                    static_cast<long long>(q.T.dims[n]), kBatchedMaxDim);
      NTF_RETURN_IF(!q.A[n], NTF_EINVAL, "problem %d: factor %d is NULL", b, n);
      d.I[n] = int(q.T.dims[n]);
      d.A[n] = q.A[n];
    }
    d.r = q.r;
    d.rb = (q.r + 3) / 4 * 4;
    d.state = q.state;
    d.tr_fhat = q.trace_fhat;
    d.tr_restart = q.trace_restart;
    d.tr_sweeps = q.trace_sweeps;
    ws_bytes = align_up(ws_bytes, 256) + batched_problem_bytes(d.I, d.rb);
    cost[size_t(b)] = int64_t(d.I[0]) * d.I[1] * d.I[2] * d.rb;
  }
  // largest problems first, so the per-problem launches start the long ones early
  std::vector<int32_t> order(static_cast<size_t>(nprob));
  for (int b = 0; b < nprob; ++b) order[size_t(b)] = b;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return cost[size_t(x)] > cost[size_t(y)]; });
  BatchedJob job{};
  job.probs = bp.data();
  job.order = order.data();
  job.nprob = nprob;
  job.resume = resume ? 1 : 0;
  job.params = *params;
  job.flags = h->dev_flags;
  const BatchedPlan pl = batched_plan(job);
  NTF_RETURN_IF(pl.lds_y > 150 * 1024 || pl.lds_last > 150 * 1024 || pl.lds_hals > 128 * 1024,
                NTF_EUNSUPPORTED, "problem set needs %zu bytes of LDS",
                std::max({pl.lds_y, pl.lds_last, pl.lds_hals}));
  const size_t desc_bytes = pl.bytes;
  const size_t need = align_up(desc_bytes, 256) + ws_bytes;
  hipStream_t s = as_stream(stream);
  if (need > h->bws_size) {
    NTF_HIP(hipDeviceSynchronize());
    if (h->bgraph) {
      (void)hipGraphExecDestroy(h->bgraph);
      h->bgraph = nullptr;
    }
    if (h->bws) (void)hipFree(h->bws);
    h->bws = nullptr;
    h->bws_size = 0;
    const size_t want = align_up(need + need / 4, size_t(1) << 20);
    if (hipMalloc(&h->bws, want) != hipSuccess) {
      (void)hipGetLastError();
      set_error("batched workspace allocation of %zu bytes failed", want);
      return NTF_ENOMEM;
    }
    h->bws_size = want;
  }
  if (!h->bstage_done) NTF_HIP(hipEventCreateWithFlags(&h->bstage_done, hipEventDisableTiming));
  // the staging area is rewritten only after its previous upload has completed
  NTF_HIP(hipEventSynchronize(h->bstage_done));
  if (desc_bytes > h->bstage_size) {
    if (h->bstage) (void)hipHostFree(h->bstage);
    h->bstage = nullptr;
    h->bstage_size = 0;
    NTF_HIP(hipHostMalloc(&h->bstage, desc_bytes, hipHostMallocDefault));
    h->bstage_size = desc_bytes;
  }
  size_t off = align_up(desc_bytes, 256);
  for (int b = 0; b < nprob; ++b) {
    off = align_up(off, 256);
    bp[size_t(b)].ws = h->bws + off;
    off += batched_problem_bytes(bp[size_t(b)].I, bp[size_t(b)].rb);
  }
  job.host_desc = h->bstage;
  job.dev_desc = h->bws;
  NTF_HIP(batched_upload(job, pl, s));
  NTF_HIP(hipEventRecord(h->bstage_done, s));
  NTF_HIP(batched_setup(job, pl, s));
  if (iters > 0) {
    // one outer iteration of every problem (a few grouped launches) is captured once into
    // a graph and replayed while the problem set and parameters are unchanged
    unsigned char key[sizeof(h->bgraph_key)] = {};
    {
      struct K {
        void* ws;
        int nprob, resume;
        ntf_her_params p;
        int64_t n_y, n_fu, n_fi, n_last, n_sum;
        size_t lds_y, lds_last, lds_hals;
        uint32_t* flags;
      } k{};
      k.ws = h->bws;
      k.nprob = nprob;
      k.resume = job.resume;
      k.p = *params;
      k.n_y = pl.n_y;
      k.n_fu = pl.n_fu;
      k.n_fi = pl.n_fi;
      k.n_last = pl.n_last;
      k.n_sum = pl.n_sum;
      k.lds_y = pl.lds_y;
      k.lds_last = pl.lds_last;
      k.lds_hals = pl.lds_hals;
      k.flags = h->dev_flags;
      static_assert(sizeof(K) <= sizeof(key), "graph key too small");
      std::memcpy(key, &k, sizeof(K));
    }
    if (!h->bgraph || std::memcmp(key, h->bgraph_key, sizeof(key)) != 0) {
      if (h->bgraph) {
        NTF_HIP(hipStreamSynchronize(s));
        (void)hipGraphExecDestroy(h->bgraph);
        h->bgraph = nullptr;
      }
      if (!h->capture_stream)
        NTF_HIP(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      NTF_HIP(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeRelaxed));
      const hipError_t le = batched_iteration(job, pl, h->capture_stream);
      const hipError_t ce = hipStreamEndCapture(h->capture_stream, &g);
      NTF_HIP(le);
      NTF_HIP(ce);
      const hipError_t ie = hipGraphInstantiate(&h->bgraph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      NTF_HIP(ie);
      std::memcpy(h->bgraph_key, key, sizeof(key));
    }
    for (int k = 0; k < iters; ++k) NTF_HIP(hipGraphLaunch(h->bgraph, s));
  }
  NTF_HIP(batched_final(job, pl, s));
  return NTF_OK;
}
}  // namespace

extern "C" {

ntf_status ntf_solve_batched(ntf_handle* h, int32_t nprob, const ntf_problem* probs,
                             const ntf_her_params* params, int32_t iters, int32_t resume,
                             void* stream) {
  clear_error();
  try {
    return solve_batched_impl(h, nprob, probs, params, iters, resume, stream);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return NTF_ENOMEM;
  }
}

ntf_status ntf_residual_norm2(ntf_handle* h, const ntf_tensor* T, const float* const* A,
                              int32_t r, double* out, void* stream) {
  clear_error();
  NTF_GUARD(h);
  ntf_status st = check_tensor(T);
  if (st) return st;
  if ((st = check_rank(r))) return st;
  NTF_RETURN_IF(!A || !out, NTF_EINVAL, "NULL argument");
  FactorPtrs fp{};
  for (int l = 0; l < T->order; ++l) {
    NTF_RETURN_IF(!A[l], NTF_EINVAL, "factor %d is NULL", l);
    fp.p[l] = A[l];
  }
  st = ensure_workspace(h, sizeof(double) * residual_partials() + 256);
  if (st) return st;
  NTF_HIP(launch_residual(*T, fp, r, reinterpret_cast<double*>(h->ws), out, as_stream(stream)));
  return NTF_OK;
}

}  // extern "C"
