// Internal declarations of the MLP velocity model (not part of the C-ABI).
#pragma once

#include <cmath>
#include <cstdint>

#include "internal.h"

namespace sweep {

constexpr int kMlpFreq = 64;               // random Fourier frequencies
constexpr int kMlpFeat = 2 * kMlpFreq;     // cos and sin features
constexpr int kMlpWidth = 256;             // hidden width (4 hidden layers)
constexpr int kMlpChunk = 1024;            // rows per split-K chunk of the reductions

// float32 parameter vector: W1 [256][128], b1, W2, b2, W3, b3, W4, b4, w5 [256], b5
constexpr size_t kTh1 = 0;
constexpr size_t kThB1 = 32768;
constexpr size_t kThHidden[3] = {33024, 98816, 164608};
constexpr size_t kThBHidden[3] = {98560, 164352, 230144};
constexpr size_t kTh5 = 230400;
constexpr size_t kThB5 = 230656;
constexpr size_t kMlpParams = 230657;

// bfloat16 weight pack: W1, W2..W4 [out][in], W2^T..W4^T [in][out], w5
constexpr size_t kWp1 = 0;
constexpr size_t kWpHidden[3] = {32768, 98304, 163840};
constexpr size_t kWpHiddenT[3] = {229376, 294912, 360448};
constexpr size_t kWp5 = 425984;
constexpr size_t kMlpPack = 426240;

struct MlpWork {
  uint16_t* H[4];   // hidden activations (forward stash), [M][256] bf16
  float* y;         // pre-sigmoid output [M]
  uint16_t* dZ[4];  // pre-activation gradients of hidden layers 1..4 [M][256] bf16
  float* pW;        // split-K partials of dW [nchunk][256][256]
  float* pB;        // partials of the bias / output-layer gradients
  int nchunk;
};

size_t mlp_workspace_bytes(int M);
MlpWork mlp_carve(void* work, int M);
int mlp_launch_encode(const float* B, int nx, int nz, uint16_t* feats, hipStream_t s);
int mlp_launch_cast(const float* theta, uint16_t* wp, hipStream_t s);
int mlp_launch_forward(const uint16_t* wp, const float* theta, const uint16_t* feats, int M,
                       float vmin, float vscale, float* v, const MlpWork& w, hipStream_t s);
int mlp_launch_backward(const uint16_t* wp, const uint16_t* feats, int M, float vscale,
                        const float* dv, float* grad, const MlpWork& w, hipStream_t s);
int launch_adam(float* theta, float* m, float* v, const float* g, size_t n, float lr, float b1,
                float b2, float eps, int t, hipStream_t s);

}  // namespace sweep
