// The no-allocation entry point (for callers that cannot allocate device
// memory: code under graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  Its workspace is a static device array of this
// translation unit; every call on a GPU shares that GPU's copy.
#include <mutex>
#include <vector>

#include "sfd.h"
#include "sfd_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of each GPU's copy of the array (the array's name is a
// host-side stand-in, not a device address): taken once per device, with
// that device current.
std::mutex g_mu;
std::vector<void*> g_ptr;

}  // namespace

extern "C" {

size_t sfd_noalloc_capacity(void) { return kScratchBytes; }

sfd_status sfd_reconstruct_noalloc(sfd_plan_t plan, const void* holo, const double* z_or_null, void* const* out,
                                   hipStream_t stream) {
  if (!plan) return sfd::set_error(SFD_ERR_INVALID_ARG, "plan is NULL");
  size_t need = 0;
  sfd_status st = sfd_workspace_size(plan, &need);
  if (st != SFD_OK) return st;
  if (need > kScratchBytes) {
    const std::string msg = "the plan needs a " + std::to_string(need) + "-byte workspace; the no-allocation scratch holds " +
                            std::to_string(kScratchBytes) + " bytes (use sfd_reconstruct with a workspace)";
    return sfd::set_error(SFD_ERR_WORKSPACE, msg.c_str());
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return sfd::set_error(SFD_ERR_HIP, hipGetErrorString(e));
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_ptr.size() <= dev) g_ptr.resize(dev + 1, nullptr);
    if (!g_ptr[dev]) {
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return sfd::set_error(SFD_ERR_HIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
      g_ptr[dev] = ptr;
    }
    ptr = g_ptr[dev];
  }
  return sfd::reconstruct_impl(plan, holo, z_or_null, out, ptr, kScratchBytes, stream, true);
}

}  // extern "C"
