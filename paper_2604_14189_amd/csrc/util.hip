// Small device utilities: fills, copies and the L2 misfit (deterministic
// two-stage reduction in float64). Fills are kernels rather than memset nodes
// so that a captured hipGraph replays them correctly.
#include "internal.h"

namespace sweep {
namespace {

__global__ void fill_kernel(float* p, size_t n, float v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill64_kernel(double* p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void copy_kernel(float4* __restrict__ d, const float4* __restrict__ s, size_t n4) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

__global__ void copy1_kernel(float* __restrict__ d, const float* __restrict__ s, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

unsigned grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

constexpr int kMisfitBlocks = 1024;

// Stage 1: each block reduces a fixed, contiguous chunk, so the summation order
// depends only on n.
__global__ void misfit_stage1(const float* __restrict__ pred, const float* __restrict__ obs,
                              float* resid, size_t n, double* partial) {
  __shared__ double red[256];
  const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const size_t b0 = (size_t)blockIdx.x * chunk;
  const size_t b1 = b0 + chunk < n ? b0 + chunk : n;
  double acc = 0.0;
  for (size_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
    const float r = pred[i] - obs[i];
    resid[i] = r;
    acc += (double)r * (double)r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void misfit_stage2(const double* partial, int nb, double* J) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *J = 0.5 * red[0];
}

}  // namespace

int launch_fill(float* p, size_t n, float v, hipStream_t s) {
  if (n == 0) return SWEEP_OK;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int launch_fill_f64(double* p, size_t n, double v, hipStream_t s) {
  if (n == 0) return SWEEP_OK;
  hipLaunchKernelGGL(fill64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int launch_copy(float* dst, const float* src, size_t n, hipStream_t s) {
  if (n == 0) return SWEEP_OK;
  if (((uintptr_t)dst % 16 == 0) && ((uintptr_t)src % 16 == 0) && n % 4 == 0)
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n / 4)), dim3(256), 0, s, (float4*)dst,
                       (const float4*)src, n / 4);
  else
    hipLaunchKernelGGL(copy1_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, src, n);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

}  // namespace sweep

extern "C" size_t sweep_l2_misfit_scratch_bytes(size_t) try {
  return sweep::kMisfitBlocks * sizeof(double);
}
SWEEP_ABI_CATCH_SIZE("sweep_l2_misfit_scratch_bytes")

extern "C" int sweep_l2_misfit(const float* d_pred, const float* d_obs, float* d_resid,
                               double* d_J, size_t n, void* d_scratch, void* stream) try {
  using namespace sweep;
  if (!d_pred || !d_obs || !d_resid || !d_J || !d_scratch) {
    set_error("sweep_l2_misfit: null pointer");
    return SWEEP_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  double* partial = (double*)d_scratch;
  hipLaunchKernelGGL(misfit_stage1, dim3(kMisfitBlocks), dim3(256), 0, s, d_pred, d_obs,
                     d_resid, n, partial);
  hipLaunchKernelGGL(misfit_stage2, dim3(1), dim3(256), 0, s, (const double*)partial,
                     kMisfitBlocks, d_J);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_l2_misfit")
