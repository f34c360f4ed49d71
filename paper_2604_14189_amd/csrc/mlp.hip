// Fourier-feature MLP velocity model on gfx950 (the neural-network velocity
// representation of the paper's workflows, Sec. 1): 2-D coordinates -> 64
// random Fourier frequencies (cos, sin: 128 features) -> 4 x 256 ReLU -> 1,
// v = vmin + vscale sigmoid(y). Matrix products run on the bf16 matrix cores
// (v_mfma_f32_32x32x16_bf16) with float32 accumulation; features, weights,
// hidden activations and back-propagated pre-activation gradients are stored as
// bfloat16 (round to nearest even), biases and everything else as float32.
//
// MFMA 32x32x16 operand layout (lane l of a wave64): A holds row l%32 and the 8
// reduction indices (l/32)*8 .. +7; B holds column l%32 and the same 8
// reduction indices; the 16 accumulators of lane l are rows 8i + (l/32)*4 + j,
// column l%32 (element 4i + j).
#include "mlp.h"

namespace sweep {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest, ties to even
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, v);
}

// --------------------------------------------------------------------------
// gamma[m] = [cos(2 pi B x_m), sin(2 pi B x_m)], x_m = (i/(nx-1), j/(nz-1))
// --------------------------------------------------------------------------
__global__ void mlp_encode_kernel(const float* B, int nx, int nz, uint16_t* feats) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t M = (size_t)nx * nz;
  if (t >= M * kMlpFreq) return;
  const size_t m = t / kMlpFreq;
  const int f = (int)(t % kMlpFreq);
  const int i = (int)(m % nx), j = (int)(m / nx);
  const double x = nx > 1 ? (double)i / (nx - 1) : 0.0;
  const double z = nz > 1 ? (double)j / (nz - 1) : 0.0;
  const double ph = 2.0 * M_PI * ((double)B[2 * f] * x + (double)B[2 * f + 1] * z);
  feats[m * kMlpFeat + f] = f2bf((float)cos(ph));
  feats[m * kMlpFeat + kMlpFreq + f] = f2bf((float)sin(ph));
}

// bf16 copies of the weights: W_l [out][in] and, for layers 2..4, W_l^T [in][out]
__global__ void mlp_cast_kernel(const float* theta, uint16_t* wp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kMlpWidth * kMlpFeat) wp[kWp1 + t] = f2bf(theta[kTh1 + t]);
  const int n2 = kMlpWidth * kMlpWidth;
  if (t < n2) {
    const int n = t / kMlpWidth, k = t % kMlpWidth;
    for (int l = 0; l < 3; ++l) {
      const uint16_t v = f2bf(theta[kThHidden[l] + t]);
      wp[kWpHidden[l] + t] = v;
      wp[kWpHiddenT[l] + k * kMlpWidth + n] = v;
    }
  }
  if (t < kMlpWidth) wp[kWp5 + t] = f2bf(theta[kTh5 + t]);
}

// --------------------------------------------------------------------------
// out[M][256] = epilogue(X[M][R] . Bm[256][R]^T)
//   mode 0 (forward): relu(acc + bias[c]) -> bf16
//   mode 1 (backward dX): acc * [mask[m][c] > 0] -> bf16
// Work-group: 128 rows x 128 columns; wave w: rows (w & 1) * 64, columns
// (w >> 1) * 64, as 2 x 2 accumulator tiles of 32 x 32. The reduction runs in
// chunks of 32: the A (128 x 32) and B (128 x 32) chunks are staged in LDS,
// double-buffered, each loaded with 16-byte global loads one chunk ahead of
// the matrix instructions that use it. LDS rows are padded to 40 bf16 (80 B),
// so the 32 rows read by a half-wave fall in different banks. Rows past M are
// clamped to M - 1, computed and not stored (no per-lane guard on the loads).
// --------------------------------------------------------------------------
constexpr int kGK = 32;       // reduction chunk
constexpr int kGS = kGK + 8;  // LDS row stride (bf16)
constexpr int kGL = 128 * kGK / 8 / 256;  // 16-byte loads per thread per operand and chunk

template <int MODE, int R>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(const uint16_t* __restrict__ X,
                                                       const uint16_t* __restrict__ Bm, int M,
                                                       const float* __restrict__ bias,
                                                       const uint16_t* __restrict__ mask,
                                                       uint16_t* __restrict__ out) {
  constexpr int NC = R / kGK;
  static_assert(R % kGK == 0 && kGL == 2, "gemm geometry");
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][128 * kGS];
  __shared__ __attribute__((aligned(16))) uint16_t sB[2][128 * kGS];
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int rb = blockIdx.x * 128, cb = blockIdx.y * 128;
  uint4 ga[kGL], gb[kGL];
  auto gload = [&](int c) {
#pragma unroll
    for (int j = 0; j < kGL; ++j) {
      const int sg = tid + 256 * j, row = sg >> 2, kk = c * kGK + 8 * (sg & 3);
      ga[j] = *reinterpret_cast<const uint4*>(X + (size_t)min(rb + row, M - 1) * R + kk);
      gb[j] = *reinterpret_cast<const uint4*>(Bm + (size_t)(cb + row) * R + kk);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < kGL; ++j) {
      const int sg = tid + 256 * j, row = sg >> 2, kk = 8 * (sg & 3);
      *reinterpret_cast<uint4*>(&sA[buf][row * kGS + kk]) = ga[j];
      *reinterpret_cast<uint4*>(&sB[buf][row * kGS + kk]) = gb[j];
    }
  };
  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx16{0};
  const int ar = (w & 1) * 64 + (l & 31), br = (w >> 1) * 64 + (l & 31);
  gload(0);
  lstore(0);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int u = c & 1;
    if (c + 1 < NC) gload(c + 1);
#pragma unroll
    for (int ks = 0; ks < kGK / 16; ++ks) {
      const int ko = ks * 16 + 8 * (l >> 5);
      const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&sA[u][ar * kGS + ko]);
      const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&sA[u][(ar + 32) * kGS + ko]);
      const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(&sB[u][br * kGS + ko]);
      const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(&sB[u][(br + 32) * kGS + ko]);
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (c + 1 < NC) lstore(u ^ 1);
    __syncthreads();
  }
  // mode 1: the 16 mask values of each accumulator tile are loaded together
  // (rows past M clamped) before that tile's stores, instead of each waiting
  // behind the previous stores
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      const floatx16& a = acc[ti][tj];
      const int r0 = rb + (w & 1) * 64 + 32 * ti;
      const int col = cb + (w >> 1) * 64 + 32 * tj + (l & 31);
      const float bc = MODE == 0 ? bias[col] : 0.0f;
      uint16_t mk[16];
      if (MODE == 1) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int row = min(r0 + 8 * (q >> 2) + (l >> 5) * 4 + (q & 3), M - 1);
          mk[q] = mask[(size_t)row * kMlpWidth + col];
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = r0 + 8 * i + (l >> 5) * 4 + j;
          float v = a[4 * i + j];
          if (MODE == 0) {
            v = fmaxf(v + bc, 0.0f);
          } else {
            v = bf2f(mk[4 * i + j]) > 0.0f ? v : 0.0f;
          }
          if (row < M) out[(size_t)row * kMlpWidth + col] = f2bf(v);
        }
    }
}

// y_m = h4_m . w5 + b5 (float32, fixed order), v_m = vmin + vscale sigmoid(y_m)
__global__ void mlp_head_fwd_kernel(const uint16_t* __restrict__ H, const uint16_t* w5,
                                    const float* b5, int M, float vmin, float vscale, float* y,
                                    float* v) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const uint16_t* h = H + (size_t)m * kMlpWidth;
  float acc = 0.0f;
  for (int k = 0; k < kMlpWidth; k += 8) {
    const uint4 q = *reinterpret_cast<const uint4*>(h + k);
    const uint16_t* e = reinterpret_cast<const uint16_t*>(&q);
#pragma unroll
    for (int t = 0; t < 8; ++t) acc = fmaf(bf2f(e[t]), bf2f(w5[k + t]), acc);
  }
  const float yy = acc + b5[0];
  y[m] = yy;
  v[m] = vmin + vscale / (1.0f + expf(-yy));
}

constexpr int kMlpThreads = 256;

// Per-chunk reductions over rows: one work-group per chunk of kMlpChunk rows.
// Thread t takes columns 4 (t % 64) .. +3 (8-byte loads) of rows g, g+4, g+8,
// ... of the chunk (g = t / 64), so the rows' loads are independent; the four
// row groups are added in LDS in a fixed order (results are deterministic).
constexpr int kRowGroups = kMlpThreads / (kMlpWidth / 4);
static_assert(kRowGroups == 4, "4 row groups of 64 column quads");
__device__ __forceinline__ void unpack4(uint2 v, float (&f)[4]) {
  f[0] = bf2f((uint16_t)(v.x & 0xffffu));
  f[1] = bf2f((uint16_t)(v.x >> 16));
  f[2] = bf2f((uint16_t)(v.y & 0xffffu));
  f[3] = bf2f((uint16_t)(v.y >> 16));
}
__device__ __forceinline__ uint2 pack4(const float (&f)[4]) {
  return make_uint2((uint32_t)f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16),
                    (uint32_t)f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16));
}
// Sums red[g][c] over the row groups in order and writes them to dst[c].
__device__ __forceinline__ void sum_groups(float (*red)[kMlpWidth + 1], float* dst, int n) {
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += kMlpThreads)
    dst[c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// dy_m = dv_m vscale s (1 - s); dZ4 = bf16(dy w5 [h4 > 0]); per-chunk partial
// sums of dy h4 (-> grad w5) and of dy (-> grad b5).
__global__ __launch_bounds__(kMlpThreads) void mlp_head_bwd_kernel(const float* dv, const float* y,
                                                                   const uint16_t* __restrict__ H,
                                                                   const uint16_t* w5, int M,
                                                                   float vscale, uint16_t* dZ,
                                                                   float* partial) {
  __shared__ float red[kRowGroups][kMlpWidth + 1];
  const int q = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int m0 = blockIdx.x * kMlpChunk, m1 = min(M, m0 + kMlpChunk);
  float wk[4], accw[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  unpack4(*reinterpret_cast<const uint2*>(w5 + 4 * q), wk);
  float accb = 0.0f;
#pragma unroll 4
  for (int m = m0 + g; m < m1; m += kRowGroups) {
    const float s = 1.0f / (1.0f + expf(-y[m]));
    const float dy = dv[m] * vscale * s * (1.0f - s);
    float h[4], z[4];
    unpack4(*reinterpret_cast<const uint2*>(H + (size_t)m * kMlpWidth + 4 * q), h);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      accw[j] = fmaf(dy, h[j], accw[j]);
      z[j] = h[j] > 0.0f ? dy * wk[j] : 0.0f;
    }
    accb += dy;
    *reinterpret_cast<uint2*>(dZ + (size_t)m * kMlpWidth + 4 * q) = pack4(z);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) red[g][4 * q + j] = accw[j];
  if (q == 0) red[g][kMlpWidth] = accb;
  sum_groups(red, partial + (size_t)blockIdx.x * (kMlpWidth + 1), kMlpWidth + 1);
}

// per-chunk column sums of dZ (-> bias gradient)
__global__ __launch_bounds__(kMlpThreads) void mlp_colsum_kernel(const uint16_t* __restrict__ dZ,
                                                                 int M, float* partial) {
  __shared__ float red[kRowGroups][kMlpWidth + 1];
  const int q = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int m0 = blockIdx.x * kMlpChunk, m1 = min(M, m0 + kMlpChunk);
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 8
  for (int m = m0 + g; m < m1; m += kRowGroups) {
    float v[4];
    unpack4(*reinterpret_cast<const uint2*>(dZ + (size_t)m * kMlpWidth + 4 * q), v);
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] += v[j];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) red[g][4 * q + j] = acc[j];
  sum_groups(red, partial + (size_t)blockIdx.x * kMlpWidth, kMlpWidth);
}

// partial[chunk][n][k] = sum over the chunk's rows m of dZ[m][n] H[m][k]
// (A = dZ^T, B = H, reduction over m). Work-group: 64 x 64 output tile, wave w
// one 32x32 tile at (n: (w&1)*32, k: (w>>1)*32).
__global__ __launch_bounds__(256) void mlp_dw_kernel(const uint16_t* __restrict__ dZ,
                                                     const uint16_t* __restrict__ H, int K, int M,
                                                     float* partial) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n0 = blockIdx.x * 64 + (w & 1) * 32;
  const int k0 = blockIdx.y * 64 + (w >> 1) * 32;
  const int m0 = blockIdx.z * kMlpChunk, m1 = min(M, m0 + kMlpChunk);
  const int nn = n0 + (l & 31), kk = k0 + (l & 31);
  const int mofs = (l >> 5) * 8;
  floatx16 acc = {0};
  for (int m = m0; m < m1; m += 16) {
    bf16x8 a, b;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int mm = m + mofs + t;
      const bool ok = mm < m1;
      const uint16_t av = ok ? dZ[(size_t)mm * kMlpWidth + nn] : (uint16_t)0;
      const uint16_t bv = ok ? H[(size_t)mm * K + kk] : (uint16_t)0;
      a[t] = __builtin_bit_cast(__bf16, av);
      b[t] = __builtin_bit_cast(__bf16, bv);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  float* out = partial + (size_t)blockIdx.z * kMlpWidth * K;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + 8 * i + (l >> 5) * 4 + j;
      out[(size_t)n * K + kk] = acc[4 * i + j];
    }
}

// dst[e] = sum over chunks c of partial[c * stride + off + e], in float64: four
// independent accumulators over c mod 4 (so the loads overlap), added in order.
__global__ void mlp_reduce_strided_kernel(const float* partial, int nchunk, int stride, int off,
                                          int len, float* dst) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const float* p = partial + off + e;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int c = 0;
  for (; c + 4 <= nchunk; c += 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] += (double)p[(size_t)(c + j) * stride];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if (c + j < nchunk) acc[j] += (double)p[(size_t)(c + j) * stride];
  dst[e] = (float)(((acc[0] + acc[1]) + acc[2]) + acc[3]);
}
__global__ void mlp_reduce_kernel(const float* partial, int nchunk, int len, float* dst) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const float* p = partial + e;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int c = 0;
  for (; c + 4 <= nchunk; c += 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] += (double)p[(size_t)(c + j) * len];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if (c + j < nchunk) acc[j] += (double)p[(size_t)(c + j) * len];
  dst[e] = (float)(((acc[0] + acc[1]) + acc[2]) + acc[3]);
}

// Adam with bias correction: c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
__global__ void adam_kernel(float* theta, float* m, float* v, const float* g, size_t n,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace

size_t mlp_workspace_bytes(int M) {
  const size_t Mz = (size_t)M;
  const int nch = (M + kMlpChunk - 1) / kMlpChunk;
  size_t off = 0;
  off = align_up(off + 4 * Mz * kMlpWidth * 2);  // H1..H4 (bf16)
  off = align_up(off + Mz * 4);                  // y
  off = align_up(off + 4 * Mz * kMlpWidth * 2);  // dZ1..dZ4 (bf16)
  off = align_up(off + (size_t)nch * kMlpWidth * kMlpWidth * 4);  // dW partials
  off = align_up(off + (size_t)nch * (kMlpWidth + 1) * 4);        // head / bias partials
  return off;
}

MlpWork mlp_carve(void* work, int M) {
  MlpWork w;
  const size_t Mz = (size_t)M;
  const int nch = (M + kMlpChunk - 1) / kMlpChunk;
  char* b = static_cast<char*>(work);
  size_t off = 0;
  for (int l = 0; l < 4; ++l) w.H[l] = reinterpret_cast<uint16_t*>(b + off) + (size_t)l * Mz * kMlpWidth;
  off = align_up(off + 4 * Mz * kMlpWidth * 2);
  w.y = reinterpret_cast<float*>(b + off);
  off = align_up(off + Mz * 4);
  for (int l = 0; l < 4; ++l) w.dZ[l] = reinterpret_cast<uint16_t*>(b + off) + (size_t)l * Mz * kMlpWidth;
  off = align_up(off + 4 * Mz * kMlpWidth * 2);
  w.pW = reinterpret_cast<float*>(b + off);
  off = align_up(off + (size_t)nch * kMlpWidth * kMlpWidth * 4);
  w.pB = reinterpret_cast<float*>(b + off);
  w.nchunk = nch;
  return w;
}

int mlp_launch_encode(const float* B, int nx, int nz, uint16_t* feats, hipStream_t s) {
  const size_t n = (size_t)nx * nz * kMlpFreq;
  hipLaunchKernelGGL(mlp_encode_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B, nx,
                     nz, feats);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int mlp_launch_cast(const float* theta, uint16_t* wp, hipStream_t s) {
  const int n = kMlpWidth * kMlpWidth;
  hipLaunchKernelGGL(mlp_cast_kernel, dim3((n + 255) / 256), dim3(256), 0, s, theta, wp);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int mlp_launch_forward(const uint16_t* wp, const float* theta, const uint16_t* feats, int M,
                       float vmin, float vscale, float* v, const MlpWork& w, hipStream_t s) {
  const dim3 g((M + 127) / 128, kMlpWidth / 128);
  hipLaunchKernelGGL((mlp_gemm_kernel<0, kMlpFeat>), g, dim3(256), 0, s, feats, wp + kWp1, M,
                     theta + kThB1, (const uint16_t*)nullptr, w.H[0]);
  for (int l = 0; l < 3; ++l)
    hipLaunchKernelGGL((mlp_gemm_kernel<0, kMlpWidth>), g, dim3(256), 0, s,
                       (const uint16_t*)w.H[l], wp + kWpHidden[l], M, theta + kThBHidden[l],
                       (const uint16_t*)nullptr, w.H[l + 1]);
  hipLaunchKernelGGL(mlp_head_fwd_kernel, dim3((M + 255) / 256), dim3(256), 0, s,
                     (const uint16_t*)w.H[3], wp + kWp5, theta + kThB5, M, vmin, vscale, w.y, v);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int mlp_launch_backward(const uint16_t* wp, const uint16_t* feats, int M, float vscale,
                        const float* dv, float* grad, const MlpWork& w, hipStream_t s) {
  const int nch = w.nchunk;
  // output layer
  hipLaunchKernelGGL(mlp_head_bwd_kernel, dim3(nch), dim3(256), 0, s, dv, (const float*)w.y,
                     (const uint16_t*)w.H[3], wp + kWp5, M, vscale, w.dZ[3], w.pB);
  hipLaunchKernelGGL(mlp_reduce_strided_kernel, dim3(2), dim3(256), 0, s, (const float*)w.pB,
                     nch, kMlpWidth + 1, 0, kMlpWidth + 1, grad + kTh5);
  // hidden layers 4..1: dW = dZ^T H_prev, db = colsum dZ, dZ_prev = (dZ W) [H_prev > 0]
  for (int l = 3; l >= 0; --l) {
    const uint16_t* dz = w.dZ[l];
    const uint16_t* hprev = l == 0 ? feats : w.H[l - 1];
    const int K = l == 0 ? kMlpFeat : kMlpWidth;
    const size_t wofs = l == 0 ? kTh1 : kThHidden[l - 1];
    const size_t bofs = l == 0 ? kThB1 : kThBHidden[l - 1];
    hipLaunchKernelGGL(mlp_dw_kernel, dim3(kMlpWidth / 64, K / 64, nch), dim3(256), 0, s, dz, hprev,
                       K, M, w.pW);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kMlpWidth * K + 255) / 256), dim3(256), 0, s,
                       (const float*)w.pW, nch, kMlpWidth * K, grad + wofs);
    hipLaunchKernelGGL(mlp_colsum_kernel, dim3(nch), dim3(256), 0, s, dz, M, w.pB);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3(1), dim3(256), 0, s, (const float*)w.pB, nch,
                       kMlpWidth, grad + bofs);
    if (l > 0) {
      const dim3 g((M + 127) / 128, kMlpWidth / 128);
      hipLaunchKernelGGL((mlp_gemm_kernel<1, kMlpWidth>), g, dim3(256), 0, s, dz,
                         wp + kWpHiddenT[l - 1], M, (const float*)nullptr,
                         (const uint16_t*)w.H[l - 1], w.dZ[l - 1]);
    }
  }
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int launch_adam(float* theta, float* m, float* v, const float* g, size_t n, float lr, float b1,
                float b2, float eps, int t, hipStream_t s) {
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, t)));
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, m, v,
                     g, n, lr, b1, b2, eps, c1, c2);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

}  // namespace sweep
