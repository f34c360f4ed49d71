// Device building blocks of the 8th-order stencil kernels (acoustic and VTI):
// the Fornberg (1988) central weights, the centred-difference second
// derivative and the first derivative, streaming loads and stores, and the
// C-PML strip indexing.
#pragma once

#include "internal.h"

namespace sweep {

// Fornberg (1988) 8th-order central weights.
// Second derivative, centred-difference form: sum_k a_k [(f_{+k}-f_0)+(f_{-k}-f_0)].
constexpr float kA1 = 8.0f / 5.0f;
constexpr float kA2 = -1.0f / 5.0f;
constexpr float kA3 = 8.0f / 315.0f;
constexpr float kA4 = -1.0f / 560.0f;
// First derivative: sum_k b_k (f_{+k} - f_{-k}).
constexpr float kB1 = 4.0f / 5.0f;
constexpr float kB2 = -1.0f / 5.0f;
constexpr float kB3 = 4.0f / 105.0f;
constexpr float kB4 = -1.0f / 280.0f;

// The library is built with -ffp-contract=off and every fused multiply-add is
// written out, so each kernel variant rounds identically (results are bitwise
// independent of the tiling).
__device__ __forceinline__ float d2c(float c, float p1, float m1, float p2, float m2, float p3,
                                     float m3, float p4, float m4) {
  float s = kA1 * ((p1 - c) + (m1 - c));
  s = fmaf(kA2, (p2 - c) + (m2 - c), s);
  s = fmaf(kA3, (p3 - c) + (m3 - c), s);
  return fmaf(kA4, (p4 - c) + (m4 - c), s);
}

__device__ __forceinline__ float d1c(float p1, float m1, float p2, float m2, float p3, float m3,
                                     float p4, float m4) {
  float s = kB1 * (p1 - m1);
  s = fmaf(kB2, p2 - m2, s);
  s = fmaf(kB3, p3 - m3, s);
  return fmaf(kB4, p4 - m4, s);
}

// Per-cell streams that a step touches exactly once (p^{n-1} in, p^{n+1} out,
// B^n, the gradient partial) carry the non-temporal hint, so they do not evict
// the halo lines that neighbouring tiles read again from L2.
__device__ __forceinline__ float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }

// Guarded load: f[i] where ok, else 0. Every lane issues the load (from
// `safe`, any valid address, where !ok) and the value is selected afterwards.
// Written as a branch, a guarded load has to complete before the other path
// writes its register, which serialises a sequence of them.
__device__ __forceinline__ float ldz(const float* f, size_t i, bool ok, const float* safe) {
  const float v = *(ok ? f + i : safe);
  return ok ? v : 0.0f;
}
__device__ __forceinline__ float ldz_nt(const float* f, size_t i, bool ok, const float* safe) {
  const float v = ld_nt(ok ? f + i : safe);
  return ok ? v : 0.0f;
}

// ldz32 with the non-temporal hint.
__device__ __forceinline__ float ldz32_nt(const float* f, unsigned i, bool ok) {
  const float v = ld_nt(&u32at(f, i));
  return ok ? v : 0.0f;
}

// Stencils on a strided LDS array centred at f.
__device__ __forceinline__ float d2s(const float* f, int st) {
  return d2c(f[0], f[st], f[-st], f[2 * st], f[-2 * st], f[3 * st], f[-3 * st], f[4 * st],
             f[-4 * st]);
}
__device__ __forceinline__ float d1s(const float* f, int st) {
  return d1c(f[st], f[-st], f[2 * st], f[-2 * st], f[3 * st], f[-3 * st], f[4 * st],
             f[-4 * st]);
}

// Column of an x-strip memory variable, or -1 outside the strip.
__device__ __forceinline__ int xstrip_col(int gx, int NX, int P) {
  if (gx < P) return gx;
  if (gx >= NX - P) return gx - (NX - 2 * P);
  return -1;
}
// Row of a z-strip memory variable, or -1 outside the strip.
__device__ __forceinline__ int zstrip_row(int gz, int NZ, int P) {
  if (gz < P) return gz;
  if (gz >= NZ - P) return gz - (NZ - 2 * P);
  return -1;
}

}  // namespace sweep
