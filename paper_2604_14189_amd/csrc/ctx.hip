// Library contexts (include/sweep.h): a context binds plans and batches to one
// HIP device; every call on them makes that device current for its duration
// and restores the caller's device afterwards.
#include <string>

#include "internal.h"
#include "plan.h"

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
  sweep_ctx* c = new sweep_ctx();
  c->device = hip_device;
  const std::string name(prop.gcnArchName);
  c->arch = name.substr(0, name.find(':'));
  *out = c;
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_ctx_create")

extern "C" void sweep_ctx_destroy(sweep_ctx* ctx) { delete ctx; }

extern "C" int sweep_ctx_device(const sweep_ctx* ctx) { return ctx ? ctx->device : -1; }
