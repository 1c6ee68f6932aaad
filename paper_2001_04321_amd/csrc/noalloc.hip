// Scratch-free MTTKRP: the same kernels and launch shapes as ntf_mttkrp, with the split
// partials in a static device array instead of the handle's workspace, so that the call
// allocates nothing (for callers that cannot allocate device memory: code under HIP
// graph capture, tight serving loops).
//
// The array is a file-scope __device__ variable: every GPU the library runs on holds its
// own copy, at its own address, until the process ends. Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol); it resolves the
// device address once per device, with that device current, and passes that pointer.
#include <mutex>

#include "ntf_internal.h"

// split partials [splits][I][r] of one call; 16 MiB
constexpr size_t kNoAllocScratchFloats = size_t(4) << 20;
static __device__ __align__(256) float scratch[kNoAllocScratchFloats];

namespace ntf {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float* g_scratch[kMaxDevices] = {};

}  // namespace

ntf_status noalloc_scratch_attach(int device) {
  NTF_RETURN_IF(device < 0 || device >= kMaxDevices, NTF_EUNSUPPORTED,
                "device index %d beyond the %d devices the scratch table covers", device,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return NTF_OK;
  DeviceGuard guard(device);
  NTF_RETURN_IF(!guard.ok, NTF_EDEVICE, "cannot select device %d", device);
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  NTF_RETURN_IF(e != hipSuccess || !p, NTF_EDEVICE,
                "hipGetSymbolAddress of the scratch array failed on device %d: %s", device,
                hipGetErrorString(e));
  g_scratch[device] = static_cast<float*>(p);
  return NTF_OK;
}

}  // namespace ntf

using namespace ntf;

extern "C" ntf_status ntf_mttkrp_noalloc(ntf_handle* h, const ntf_tensor* T,
                                         const float* const* A, int32_t r, int32_t mode,
                                         float* P, void* stream) {
  clear_error();
  NTF_RETURN_IF(!h, NTF_EINVAL, "handle is NULL");
  DeviceGuard guard(h->device);
  NTF_RETURN_IF(!guard.ok, NTF_EDEVICE, "cannot select device %d", h->device);
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
  NTF_RETURN_IF(pl.partial_floats() > kNoAllocScratchFloats, NTF_EUNSUPPORTED,
                "mode %d of this tensor at rank %d needs %zu floats of split partials; the "
                "scratch-free call holds at most %zu (use ntf_mttkrp)",
                mode, r, pl.partial_floats(), kNoAllocScratchFloats);
  if ((st = noalloc_scratch_attach(h->device))) return st;
  float* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    ptr = g_scratch[h->device];
  }
  // every (split, row, column) of the partials is written by exactly one workgroup before
  // the reduction reads it, so nothing needs clearing between calls
  NTF_HIP(launch_mttkrp(pl, T->data, fp, P, ptr, true, static_cast<hipStream_t>(stream)));
  return NTF_OK;
}
