// Library contexts (include/sweep.h): a context binds plans and batches to one
// HIP device; every call on them makes that device current for its duration
// and restores the caller's device afterwards.
//
// The context is also where the library sets up the static device workspace of
// sweep_forward_noalloc: `scratch` below, one copy per GPU the library runs
// on, held until the process ends. In host code the array's name is a host
// stand-in, not a device address; its address on each device is looked up
// here once per device (with that device current) and only that pointer is
// ever handed to kernels or copies.
#include <mutex>
#include <string>

#include "internal.h"
#include "plan.h"

namespace sweep {
namespace {
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on `device` (which must be current); looked up
// on the first call for that device and kept.
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("scratch_address: device index out of range");
    return SWEEP_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    SWEEP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      set_error("hipGetSymbolAddress returned a null address for the scratch array");
      return SWEEP_EHIP;
    }
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return SWEEP_OK;
}
}  // namespace sweep

using namespace sweep;

extern "C" int sweep_ctx_create(sweep_ctx** out, int hip_device) try {
  if (!out) {
    set_error("sweep_ctx_create: null argument");
    return SWEEP_EINVAL;
  }
  *out = nullptr;
  int n = 0;
  SWEEP_HIP(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n) {
    set_error("sweep_ctx_create: device " + std::to_string(hip_device) + " outside [0, " +
              std::to_string(n) + ")");
    return SWEEP_EINVAL;
  }
  DeviceGuard g(hip_device);
  if (!g.ok) {
    set_error("sweep_ctx_create: hipSetDevice failed");
    return SWEEP_EHIP;
  }
  hipDeviceProp_t prop;
  SWEEP_HIP(hipGetDeviceProperties(&prop, hip_device));
  void* sp = nullptr;
  const int rc = scratch_address(hip_device, &sp);
  if (rc) return rc;
  sweep_ctx* c = new sweep_ctx();
  c->device = hip_device;
  const std::string name(prop.gcnArchName);
  c->arch = name.substr(0, name.find(':'));
  c->scratch = sp;
  *out = c;
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_ctx_create")

extern "C" void sweep_ctx_destroy(sweep_ctx* ctx) { delete ctx; }

extern "C" int sweep_ctx_device(const sweep_ctx* ctx) { return ctx ? ctx->device : -1; }
