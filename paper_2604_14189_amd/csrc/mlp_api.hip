// C-ABI of the MLP velocity model and of the Adam optimiser (include/sweep.h).
#include <string>

#include "mlp.h"

using namespace sweep;

extern "C" size_t sweep_mlp_param_count(void) { return kMlpParams; }
extern "C" size_t sweep_mlp_pack_count(void) { return kMlpPack; }
extern "C" size_t sweep_mlp_workspace_bytes(int npoints) try {
  return npoints > 0 ? mlp_workspace_bytes(npoints) : 0;
}
SWEEP_ABI_CATCH_SIZE("sweep_mlp_workspace_bytes")

extern "C" int sweep_mlp_encode(const float* d_B, int nx, int nz, uint16_t* d_feats,
                                void* stream) try {
  if (!d_B || !d_feats || nx < 1 || nz < 1) {
    set_error("sweep_mlp_encode: bad argument");
    return SWEEP_EINVAL;
  }
  return mlp_launch_encode(d_B, nx, nz, d_feats, (hipStream_t)stream);
}
SWEEP_ABI_CATCH("sweep_mlp_encode")

extern "C" int sweep_mlp_cast(const float* d_theta, uint16_t* d_wpack, void* stream) try {
  if (!d_theta || !d_wpack) {
    set_error("sweep_mlp_cast: null pointer");
    return SWEEP_EINVAL;
  }
  return mlp_launch_cast(d_theta, d_wpack, (hipStream_t)stream);
}
SWEEP_ABI_CATCH("sweep_mlp_cast")

extern "C" int sweep_mlp_forward(const uint16_t* d_wpack, const float* d_theta,
                                 const uint16_t* d_feats, int npoints, float vmin, float vscale,
                                 float* d_v, void* d_work, size_t work_bytes, void* stream) try {
  if (!d_wpack || !d_theta || !d_feats || !d_v || !d_work || npoints < 1) {
    set_error("sweep_mlp_forward: bad argument");
    return SWEEP_EINVAL;
  }
  if (work_bytes < mlp_workspace_bytes(npoints)) {
    set_error("sweep_mlp_forward: workspace too small");
    return SWEEP_ENOMEM;
  }
  return mlp_launch_forward(d_wpack, d_theta, d_feats, npoints, vmin, vscale, d_v,
                            mlp_carve(d_work, npoints), (hipStream_t)stream);
}
SWEEP_ABI_CATCH("sweep_mlp_forward")

extern "C" int sweep_mlp_backward(const uint16_t* d_wpack, const uint16_t* d_feats, int npoints,
                                  float vscale, const float* d_dv, float* d_grad, void* d_work,
                                  size_t work_bytes, void* stream) try {
  if (!d_wpack || !d_feats || !d_dv || !d_grad || !d_work || npoints < 1) {
    set_error("sweep_mlp_backward: bad argument");
    return SWEEP_EINVAL;
  }
  if (work_bytes < mlp_workspace_bytes(npoints)) {
    set_error("sweep_mlp_backward: workspace too small");
    return SWEEP_ENOMEM;
  }
  return mlp_launch_backward(d_wpack, d_feats, npoints, vscale, d_dv, d_grad,
                             mlp_carve(d_work, npoints), (hipStream_t)stream);
}
SWEEP_ABI_CATCH("sweep_mlp_backward")

extern "C" int sweep_adam_step(float* d_theta, float* d_m, float* d_v, const float* d_g,
                               size_t n, float lr, float b1, float b2, float eps, int t,
                               void* stream) try {
  if (!d_theta || !d_m || !d_v || !d_g || t < 1 || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1)) {
    set_error("sweep_adam_step: bad argument");
    return SWEEP_EINVAL;
  }
  return launch_adam(d_theta, d_m, d_v, d_g, n, lr, b1, b2, eps, t, (hipStream_t)stream);
}
SWEEP_ABI_CATCH("sweep_adam_step")
