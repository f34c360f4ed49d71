// Acoustic step kernels for gfx950: the constant-density wave equation
// (Sec. 3.1.2, Eq. 2) advanced with the leapfrog update of the paper's step
// function (Sec. 2.1), an 8th-order Laplacian and a C-PML absorbing pad, and the
// exact transpose of that recurrence for the adjoint (Sec. 1).
//
// Scaled form used on the GPU (h folded into the coefficients):
//   Cs = (v dt / h)^2, D2' = h^2 D2, D1' = h D1, psi' = h psi, zeta' = h^2 zeta,
//   B' = h^2 B, so p^{n+1} = 2 p^n - p^{n-1} + Cs B'^n + (dt/h)^2 s_n e_src.
//
// Decomposition of one step. B' = D2' p + Ex + Ez, where the C-PML part
//   Ex = D1x' psi_x + zeta_x   is non-zero only in the x band (columns within
//   P+4 of the left/right edges) and Ez likewise in the z band. Per step:
//   1. band kernels (x, then z): update the memory variables and fold the pad
//      terms into the previous field in place, p^{n-1} <- p^{n-1} - Cs E;
//   2. main kernel over the whole grid: p^{n+1} = 2 p^n - p^{n-1} + Cs D2' p^n,
//      source injection and receiver recording.
// The adjoint is the same split of the transposed recurrence. The main kernel
// stages a 4-cell halo tile of the field in LDS and keeps RZ rows per thread in
// registers; the band kernels are 1-D along their axis (a wave per row segment
// for x, a 64-column slab for z) and touch only the band cells.
#include "internal.h"

namespace sweep {
namespace {

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
__device__ __forceinline__ bool in_xband(int gx, int NX, int P) {
  return P > 0 && (gx < P + 4 || gx >= NX - P - 4);
}
__device__ __forceinline__ bool in_zband(int gz, int NZ, int P) {
  return P > 0 && (gz < P + 4 || gz >= NZ - P - 4);
}

// ---------------------------------------------------------------------------
// Model preparation: edge-replicated padding, Cs = (v dt/h)^2, C-PML tables.
// ---------------------------------------------------------------------------
__global__ void ac_prep_kernel(const float* __restrict__ v, float* __restrict__ vpad,
                               float* __restrict__ Cs, int nx, int nz, int P, double r) {
  const int NX = nx + 2 * P, NZ = nz + 2 * P;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= NX || j >= NZ) return;
  const int ii = min(max(i - P, 0), nx - 1);
  const int jj = min(max(j - P, 0), nz - 1);
  const double vv = v[(size_t)jj * nx + ii];
  vpad[(size_t)j * NX + i] = (float)vv;
  const double c = vv * r;
  Cs[(size_t)j * NX + i] = (float)(c * c);
}

// C-PML recursion coefficients at integer node i of an axis of length n with
// `pad` absorbing cells at both ends (Collino-Tsogka / Komatitsch-Martin form,
// quadratic damping, linearly decreasing alpha, kappa = 1).
__device__ void pml_coeffs(int i, int n, int pad, double h, double dt, double vmax, double f0,
                           double R, float* a, float* b) {
  double xi = 0.0;
  const double L = pad > 0 ? pad * h : 1.0;
  if (pad > 0 && i < pad) xi = (pad - i) * h;
  if (pad > 0 && i > n - 1 - pad) xi = (i - (n - 1 - pad)) * h;
  const double d0 = -3.0 * vmax * log(R) / (2.0 * L);
  const double d = xi > 0.0 ? d0 * (xi / L) * (xi / L) : 0.0;
  const double alpha = M_PI * f0 * (1.0 - xi / L);
  const double bb = exp(-(d + alpha) * dt);
  b[i] = (float)bb;
  a[i] = d > 0.0 ? (float)(d / (d + alpha) * (bb - 1.0)) : 0.0f;
}

__global__ void ac_tables_kernel(float* ax, float* bx, float* az, float* bz, int NX, int NZ,
                                 int P, double h, double dt, double vmax, double f0, double R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NX) pml_coeffs(i, NX, P, h, dt, vmax, f0, R, ax, bx);
  if (i < NZ) pml_coeffs(i, NZ, P, h, dt, vmax, f0, R, az, bz);
}

// ---------------------------------------------------------------------------
// Main kernels: a 64 x TZ tile per work-group, TZ = 4 RZ; thread (lx, w) owns
// column lx and rows [w RZ, w RZ + RZ). Tiles whose 4-cell halo lies inside
// the grid take unguarded loads; edge tiles zero-fill outside the grid.
// ---------------------------------------------------------------------------
template <int RZ>
struct MainTile {
  static constexpr int TZ = 4 * RZ;
  static constexpr int LW = kTX + 8;
  static constexpr int LH = TZ + 8;
};

// Stage f (or g * f, pointwise) on the tile plus a 4-cell halo. Every thread
// issues all of its loads before the first LDS store, so a work-group keeps
// ~12 (or ~24 for the product) loads per lane in flight instead of one.
template <int RZ, bool kProduct>
__device__ __forceinline__ void stage_box(float* s, const float* __restrict__ f,
                                          const float* __restrict__ g, int x0, int z0, int NX,
                                          int NZ, bool inside) {
  using T = MainTile<RZ>;
  constexpr int N = T::LH * T::LW;
  constexpr int K = (N + kThreads - 1) / kThreads;
  const int tid = threadIdx.x;
  float v[K], u[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = tid + k * kThreads;
    const int r = e / T::LW;
    const int c = e - r * T::LW;
    const int gx = x0 - 4 + c, gz = z0 - 4 + r;
    const bool ok = e < N && (inside || (gx >= 0 && gx < NX && gz >= 0 && gz < NZ));
    const size_t idx = ok ? (size_t)gz * NX + gx : 0;
    v[k] = ok ? f[idx] : 0.0f;
    if (kProduct) u[k] = ok ? g[idx] : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = tid + k * kThreads;
    if (e < N) s[e] = kProduct ? u[k] * v[k] : v[k];
  }
}

template <int RZ>
__device__ __forceinline__ void ac_fwd_main_body(const AcStep& a, const int bx, const int by, const int bz) {
  using T = MainTile<RZ>;
  __shared__ float sp[T::LH * T::LW];
  const int tid = threadIdx.x;
  const int lx = tid & 63;
  const int zb = (tid >> 6) * RZ;
  const int tile = bx;
  const int shot = by;
  const int NX = a.NX, NZ = a.NZ, P = a.P;
  const size_t plane = (size_t)NX * NZ;
  const int x0 = (tile % a.tiles_x) * kTX, z0 = (tile / a.tiles_x) * T::TZ;
  const bool inside = x0 >= 4 && x0 + kTX + 4 <= NX && z0 >= 4 && z0 + T::TZ + 4 <= NZ;
  const int gx = x0 + lx;

  // the per-cell operands are fetched first so their latency overlaps the
  // staging of the halo tile
  float pp[RZ], cs[RZ], bo[RZ];
  const bool xb = in_xband(gx, NX, P);
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const int gz = z0 + zb + r;
    pp[r] = 0.0f;
    cs[r] = 0.0f;
    bo[r] = 0.0f;
    if (inside || (gx < NX && gz < NZ)) {
      const int idx = gz * NX + gx;
      pp[r] = a.prev[shot * plane + idx];
      cs[r] = a.Cs[idx];
      if (a.B_out && (xb || in_zband(gz, NZ, P))) bo[r] = a.B_out[shot * plane + idx];
    }
  }
  stage_box<RZ, false>(sp, a.cur + shot * plane, nullptr, x0, z0, NX, NZ, inside);
  __syncthreads();

  float win[RZ + 8];
#pragma unroll
  for (int m = 0; m < RZ + 8; ++m) win[m] = sp[(zb + m) * T::LW + lx + 4];

  const int src = a.src_cell[shot];
  const float sw = a.w * a.wavelet[(size_t)shot * a.nt + a.n];
  float out[RZ];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const float* row = &sp[(zb + r + 4) * T::LW + lx + 4];
    const float c = win[r + 4];
    const float sx = d2c(c, row[1], row[-1], row[2], row[-2], row[3], row[-3], row[4], row[-4]);
    const float sz = d2c(c, win[r + 5], win[r + 3], win[r + 6], win[r + 2], win[r + 7],
                         win[r + 1], win[r + 8], win[r]);
    const float L = sx + sz;
    const int gz = z0 + zb + r;
    float pn = 0.0f;
    if (inside || (gx < NX && gz < NZ)) {
      const int idx = gz * NX + gx;
      const size_t gi = shot * plane + idx;
      pn = fmaf(cs[r], L, 2.0f * c - pp[r]);
      if (idx == src) pn += sw;
      a.next[gi] = pn;
      if (a.B_out) a.B_out[gi] = (xb || in_zband(gz, NZ, P)) ? L + bo[r] : L;
    }
    out[r] = pn;
  }

  // receivers in this tile record p^{n+1}
  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  const int e0 = ro[0], e1 = ro[1];
  if (a.gathers && e1 > e0) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RZ; ++r) sp[(zb + r) * kTX + lx] = out[r];
    __syncthreads();
    float* dst = a.gathers + ((size_t)shot * a.nt + a.n) * a.nrec;
    for (int e = e0 + tid; e < e1; e += kThreads) {
      const int2 en = a.rec_ent[e];
      dst[en.y] = sp[en.x];
    }
  }
}

// Adds r_{n-1} at the receivers of this (shot, tile) to the staged lambda values
// st[local] (run heads handle several receivers on one cell, in receiver order).
__device__ __forceinline__ void inject_residual(const AcStep& a, int shot, int tile, float* st) {
  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  const int e0 = ro[0], e1 = ro[1];
  const float* r = a.resid + ((size_t)shot * a.nt + (a.n - 1)) * a.nrec;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += kThreads) {
    const int2 en = a.rec_ent[e];
    if (e == e0 || a.rec_ent[e - 1].x != en.x) {
      float acc = st[en.x];
      for (int k = e; k < e1 && a.rec_ent[k].x == en.x; ++k) acc += r[a.rec_ent[k].y];
      st[en.x] = acc;
    }
  }
}

// lambda^n = 2 lambda^{n+1} - lambda^{n+2}' + D2'(Cs lambda^{n+1}), where the band
// kernels already subtracted their pad terms from lambda^{n+2}' in place;
// g += lambda^{n+1} B'^n; then r_{n-1} is injected at the receivers.
template <int RZ>
__device__ __forceinline__ void ac_adj_main_body(const AcStep& a, const int bx, const int by, const int bz) {
  using T = MainTile<RZ>;
  __shared__ float sq[T::LH * T::LW];
  const int tid = threadIdx.x;
  const int lx = tid & 63;
  const int zb = (tid >> 6) * RZ;
  const int tile = bx;
  const int shot = by;
  const int NX = a.NX, NZ = a.NZ;
  const size_t plane = (size_t)NX * NZ;
  const int x0 = (tile % a.tiles_x) * kTX, z0 = (tile / a.tiles_x) * T::TZ;
  const bool inside = x0 >= 4 && x0 + kTX + 4 <= NX && z0 >= 4 && z0 + T::TZ + 4 <= NZ;
  const int gx = x0 + lx;

  float p1[RZ], pp[RZ], bb[RZ], gg[RZ];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const int gz = z0 + zb + r;
    p1[r] = pp[r] = bb[r] = gg[r] = 0.0f;
    if (inside || (gx < NX && gz < NZ)) {
      const size_t gi = shot * plane + (size_t)gz * NX + gx;
      p1[r] = a.cur[gi];
      pp[r] = a.prev[gi];
      bb[r] = a.B_in[gi];
      if (!a.g_init) gg[r] = a.g[gi];
    }
  }
  stage_box<RZ, true>(sq, a.cur + shot * plane, a.Cs, x0, z0, NX, NZ, inside);
  __syncthreads();

  float win[RZ + 8];
#pragma unroll
  for (int m = 0; m < RZ + 8; ++m) win[m] = sq[(zb + m) * T::LW + lx + 4];

  float out[RZ];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const float* row = &sq[(zb + r + 4) * T::LW + lx + 4];
    const float c = win[r + 4];
    const float sxx = d2c(c, row[1], row[-1], row[2], row[-2], row[3], row[-3], row[4], row[-4]);
    const float szz = d2c(c, win[r + 5], win[r + 3], win[r + 6], win[r + 2], win[r + 7],
                          win[r + 1], win[r + 8], win[r]);
    const int gz = z0 + zb + r;
    float lam = 0.0f;
    if (inside || (gx < NX && gz < NZ)) {
      const size_t gi = shot * plane + (size_t)gz * NX + gx;
      const float gb = p1[r] * bb[r];
      a.g[gi] = a.g_init ? gb : gg[r] + gb;
      lam = ((2.0f * p1[r] - pp[r]) + sxx) + szz;
    }
    out[r] = lam;
  }

  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  if (a.n >= 1 && ro[1] > ro[0]) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RZ; ++r) sq[(zb + r) * kTX + lx] = out[r];
    __syncthreads();
    inject_residual(a, shot, tile, sq);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RZ; ++r) out[r] = sq[(zb + r) * kTX + lx];
  }
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const int gz = z0 + zb + r;
    if (inside || (gx < NX && gz < NZ)) a.next[shot * plane + (size_t)gz * NX + gx] = out[r];
  }
}

// ---------------------------------------------------------------------------
// x band (columns within P+4 of the left/right edges, all rows). One wave per
// (row, chunk): lane l holds column c0 - 8 + l; a chunk produces up to 48
// outputs (lanes 8 .. 8+W) and reads an 8-cell halo on each side.
// ---------------------------------------------------------------------------
constexpr int kChunk = 48;

// Rows handled by one wave of an x-band work-group (a work-group covers
// 4 * kXRows consecutive rows of one chunk). All global operands of a wave's
// rows are loaded before any of them is used.
constexpr int kXRows = 4;

// psi_x^n, zeta_x^n and Ex = D1x' psi_x^n + zeta_x^n; p^{n-1} -= Cs Ex.
__device__ __forceinline__ void ac_fwd_xband_body(const AcStep& a, const int bx, const int by, const int bz) {
  __shared__ float sp[4][kXRows][64];
  __shared__ float ss[4][kXRows][64];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int2 ch = a.xchunks[bx];
  const int shot = bz;
  const int NX = a.NX, NZ = a.NZ, P = a.P, P2 = 2 * P;
  const int gx = ch.x - 8 + l;
  const size_t plane = (size_t)NX * NZ;
  const bool own = l >= 8 && l < 8 + ch.y;
  const bool col_ok = gx >= 0 && gx < NX;
  const int col0 = col_ok ? xstrip_col(gx, NX, P) : -1;
  const float axv = col0 >= 0 ? a.ax[gx] : 0.0f, bxv = col0 >= 0 ? a.bx[gx] : 0.0f;
  const int gz0 = (by * 4 + w) * kXRows;
  float pv[kXRows], psio[kXRows], zo[kXRows], cs[kXRows], pp[kXRows];
#pragma unroll
  for (int rr = 0; rr < kXRows; ++rr) {
    const int gz = gz0 + rr;
    const bool in_grid = col_ok && gz < NZ;
    const bool strip = in_grid && col0 >= 0;
    const size_t si = shot * (size_t)NZ * P2 + (size_t)gz * P2 + (strip ? col0 : 0);
    const size_t gi = shot * plane + (size_t)gz * NX + (in_grid ? gx : 0);
    pv[rr] = in_grid ? a.cur[gi] : 0.0f;
    psio[rr] = (strip && l >= 4 && l < 60) ? a.psx_in[si] : 0.0f;
    zo[rr] = (strip && own) ? a.zex_in[si] : 0.0f;
    cs[rr] = (in_grid && own) ? a.Cs[(size_t)gz * NX + gx] : 0.0f;
    pp[rr] = (in_grid && own) ? a.prev_adj[gi] : 0.0f;
  }
#pragma unroll
  for (int rr = 0; rr < kXRows; ++rr) sp[w][rr][l] = pv[rr];
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < kXRows; ++rr) {
    const int gz = gz0 + rr;
    const bool strip = col0 >= 0 && gz < NZ;
    float psi = 0.0f;
    if (strip && l >= 4 && l < 60) {
      psi = fmaf(axv, d1s(&sp[w][rr][l], 1), bxv * psio[rr]);
      if (own) a.psx_out[shot * (size_t)NZ * P2 + (size_t)gz * P2 + col0] = psi;
    }
    ss[w][rr][l] = psi;
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < kXRows; ++rr) {
    const int gz = gz0 + rr;
    if (!(own && col_ok && gz < NZ)) continue;
    const float d1p = d1s(&ss[w][rr][l], 1);
    float E = d1p;
    if (col0 >= 0) {
      const float Q = d2s(&sp[w][rr][l], 1) + d1p;
      const float zeta = fmaf(axv, Q, bxv * zo[rr]);
      a.zex_out[shot * (size_t)NZ * P2 + (size_t)gz * P2 + col0] = zeta;
      E = d1p + zeta;
    }
    const size_t gi = shot * plane + (size_t)gz * NX + gx;
    a.prev_adj[gi] = fmaf(-cs[rr], E, pp[rr]);
    if (a.B_out) a.B_out[gi] = E;
  }
}

// Adjoint of the x band: zbar = Z + q, Qbar = q + a_x zbar (q = Cs lambda^{n+1}),
// psbar = Psi - D1x' Qbar, Eadj = D2x'(a_x zbar) - D1x'(a_x psbar);
// lambda^{n+2}' -= Eadj; Psi <- b_x psbar, Z <- b_x zbar.
__device__ __forceinline__ void ac_adj_xband_body(const AcStep& a, const int bx, const int by, const int bz) {
  __shared__ float sQ[4][kXRows][64];
  __shared__ float sS[4][kXRows][64];
  __shared__ float sT[4][kXRows][64];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int2 ch = a.xchunks[bx];
  const int shot = bz;
  const int NX = a.NX, NZ = a.NZ, P = a.P, P2 = 2 * P;
  const int gx = ch.x - 8 + l;
  const size_t plane = (size_t)NX * NZ;
  const bool own = l >= 8 && l < 8 + ch.y;
  const bool col_ok = gx >= 0 && gx < NX;
  const int col0 = col_ok ? xstrip_col(gx, NX, P) : -1;
  const float axv = col0 >= 0 ? a.ax[gx] : 0.0f, bxv = col0 >= 0 ? a.bx[gx] : 0.0f;
  const int gz0 = (by * 4 + w) * kXRows;
  float lv[kXRows], cv[kXRows], zi[kXRows], psi_in[kXRows], pp[kXRows];
#pragma unroll
  for (int rr = 0; rr < kXRows; ++rr) {
    const int gz = gz0 + rr;
    const bool in_grid = col_ok && gz < NZ;
    const bool strip = in_grid && col0 >= 0;
    const size_t si = shot * (size_t)NZ * P2 + (size_t)gz * P2 + (strip ? col0 : 0);
    const size_t gi = shot * plane + (size_t)gz * NX + (in_grid ? gx : 0);
    lv[rr] = in_grid ? a.cur[gi] : 0.0f;
    cv[rr] = in_grid ? a.Cs[(size_t)gz * NX + gx] : 0.0f;
    zi[rr] = strip ? a.zex_in[si] : 0.0f;
    psi_in[rr] = (strip && l >= 4 && l < 60) ? a.psx_in[si] : 0.0f;
    pp[rr] = (in_grid && own) ? a.prev_adj[gi] : 0.0f;
  }
#pragma unroll
  for (int rr = 0; rr < kXRows; ++rr) {
    const int gz = gz0 + rr;
    float q = cv[rr] * lv[rr];
    float sv = 0.0f;
    if (col0 >= 0 && gz < NZ) {
      const float zb = zi[rr] + q;
      sv = axv * zb;
      q = q + sv;
      if (own) a.zex_out[shot * (size_t)NZ * P2 + (size_t)gz * P2 + col0] = bxv * zb;
    }
    sQ[w][rr][l] = q;
    sS[w][rr][l] = sv;
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < kXRows; ++rr) {
    const int gz = gz0 + rr;
    float t = 0.0f;
    if (col0 >= 0 && gz < NZ && l >= 4 && l < 60) {
      const float psb = psi_in[rr] - d1s(&sQ[w][rr][l], 1);
      t = axv * psb;
      if (own) a.psx_out[shot * (size_t)NZ * P2 + (size_t)gz * P2 + col0] = bxv * psb;
    }
    sT[w][rr][l] = t;
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < kXRows; ++rr) {
    const int gz = gz0 + rr;
    if (!(own && col_ok && gz < NZ)) continue;
    const float E = d2s(&sS[w][rr][l], 1) - d1s(&sT[w][rr][l], 1);
    a.prev_adj[shot * plane + (size_t)gz * NX + gx] = pp[rr] - E;
  }
}

// ---------------------------------------------------------------------------
// z band (rows within P+4 of the top/bottom edges, all columns). A work-group
// covers 64 columns x up to 48 output rows with an 8-row halo above and below;
// wave w handles the LDS rows congruent to w mod 4, and issues all of its
// global loads of a phase before using any of them.
// ---------------------------------------------------------------------------
constexpr int kZRows = kChunk + 16;
constexpr int kZStage = kZRows / 4;       // staged rows per wave (64 / 4)
constexpr int kZPsi = (kZRows - 8) / 4;   // psi rows per wave
constexpr int kZOut = kChunk / 4;         // output rows per wave

__device__ __forceinline__ void ac_fwd_zband_body(const AcStep& a, const int bx, const int by, const int bz) {
  __shared__ float sp[kZRows * kTX];
  __shared__ float ss[kZRows * kTX];
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int2 ch = a.zchunks[by];
  const int x0 = bx * kTX, gx = x0 + c;
  const int shot = bz;
  const int NX = a.NX, NZ = a.NZ, P = a.P;
  const bool col_ok = gx < NX;
  const size_t plane = (size_t)NX * NZ;
  const size_t zs_plane = (size_t)2 * P * NX;
  const int rows = ch.y + 16;  // LDS row r <-> grid row ch.x - 8 + r
  {
    float v[kZStage];
#pragma unroll
    for (int k = 0; k < kZStage; ++k) {
      const int r = w + 4 * k, gz = ch.x - 8 + r;
      const bool ok = col_ok && r < rows && gz >= 0 && gz < NZ;
      v[k] = ok ? a.cur[shot * plane + (size_t)gz * NX + gx] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kZStage; ++k) sp[(w + 4 * k) * kTX + c] = v[k];
  }
  __syncthreads();
  {
    float old[kZPsi];
#pragma unroll
    for (int k = 0; k < kZPsi; ++k) {
      const int r = 4 + w + 4 * k, gz = ch.x - 8 + r;
      const int row = (col_ok && r < rows - 4 && gz >= 0 && gz < NZ) ? zstrip_row(gz, NZ, P) : -1;
      old[k] = row >= 0 ? a.psz_in[shot * zs_plane + (size_t)row * NX + gx] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kZPsi; ++k) {
      const int r = 4 + w + 4 * k, gz = ch.x - 8 + r;
      const int row = (col_ok && r < rows - 4 && gz >= 0 && gz < NZ) ? zstrip_row(gz, NZ, P) : -1;
      float psi = 0.0f;
      if (row >= 0) {
        psi = fmaf(a.az[gz], d1s(&sp[r * kTX + c], kTX), a.bz[gz] * old[k]);
        if (r >= 8 && r < 8 + ch.y) a.psz_out[shot * zs_plane + (size_t)row * NX + gx] = psi;
      }
      ss[r * kTX + c] = psi;
    }
  }
  __syncthreads();
  float zo[kZOut], cs[kZOut], pp[kZOut], bo[kZOut];
  const bool xb = in_xband(gx, NX, P);
#pragma unroll
  for (int k = 0; k < kZOut; ++k) {
    const int r = 8 + w + 4 * k, gz = ch.x - 8 + r;
    const bool ok = col_ok && r < 8 + ch.y && gz < NZ;
    const int row = ok ? zstrip_row(gz, NZ, P) : -1;
    const size_t kk = ok ? (size_t)gz * NX + gx : 0;
    zo[k] = row >= 0 ? a.zez_in[shot * zs_plane + (size_t)row * NX + gx] : 0.0f;
    cs[k] = ok ? a.Cs[kk] : 0.0f;
    pp[k] = ok ? a.prev_adj[shot * plane + kk] : 0.0f;
    bo[k] = (ok && a.B_out && xb) ? a.B_out[shot * plane + kk] : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < kZOut; ++k) {
    const int r = 8 + w + 4 * k, gz = ch.x - 8 + r;
    if (!(col_ok && r < 8 + ch.y && gz < NZ)) continue;
    const float d1p = d1s(&ss[r * kTX + c], kTX);
    float E = d1p;
    const int row = zstrip_row(gz, NZ, P);
    if (row >= 0) {
      const float Q = d2s(&sp[r * kTX + c], kTX) + d1p;
      const float zeta = fmaf(a.az[gz], Q, a.bz[gz] * zo[k]);
      a.zez_out[shot * zs_plane + (size_t)row * NX + gx] = zeta;
      E = d1p + zeta;
    }
    const size_t gi = shot * plane + (size_t)gz * NX + gx;
    a.prev_adj[gi] = fmaf(-cs[k], E, pp[k]);
    if (a.B_out) a.B_out[gi] = xb ? bo[k] + E : E;
  }
}

__device__ __forceinline__ void ac_adj_zband_body(const AcStep& a, const int bx, const int by, const int bz) {
  __shared__ float sQ[kZRows * kTX];
  __shared__ float sS[kZRows * kTX];
  __shared__ float sT[kZRows * kTX];
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int2 ch = a.zchunks[by];
  const int x0 = bx * kTX, gx = x0 + c;
  const int shot = bz;
  const int NX = a.NX, NZ = a.NZ, P = a.P;
  const bool col_ok = gx < NX;
  const size_t plane = (size_t)NX * NZ;
  const size_t zs_plane = (size_t)2 * P * NX;
  const int rows = ch.y + 16;
  {
    float lv[kZStage], cv[kZStage], zi[kZStage];
#pragma unroll
    for (int k = 0; k < kZStage; ++k) {
      const int r = w + 4 * k, gz = ch.x - 8 + r;
      const bool ok = col_ok && r < rows && gz >= 0 && gz < NZ;
      const size_t kk = ok ? (size_t)gz * NX + gx : 0;
      const int row = ok ? zstrip_row(gz, NZ, P) : -1;
      lv[k] = ok ? a.cur[shot * plane + kk] : 0.0f;
      cv[k] = ok ? a.Cs[kk] : 0.0f;
      zi[k] = row >= 0 ? a.zez_in[shot * zs_plane + (size_t)row * NX + gx] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kZStage; ++k) {
      const int r = w + 4 * k, gz = ch.x - 8 + r;
      const bool ok = col_ok && r < rows && gz >= 0 && gz < NZ;
      const int row = ok ? zstrip_row(gz, NZ, P) : -1;
      float q = cv[k] * lv[k], sv = 0.0f;
      if (row >= 0) {
        const float zb = zi[k] + q;
        sv = a.az[gz] * zb;
        q = q + sv;
        if (r >= 8 && r < 8 + ch.y) a.zez_out[shot * zs_plane + (size_t)row * NX + gx] = a.bz[gz] * zb;
      }
      sQ[r * kTX + c] = q;
      sS[r * kTX + c] = sv;
    }
  }
  __syncthreads();
  {
    float pin[kZPsi];
#pragma unroll
    for (int k = 0; k < kZPsi; ++k) {
      const int r = 4 + w + 4 * k, gz = ch.x - 8 + r;
      const int row = (col_ok && r < rows - 4 && gz >= 0 && gz < NZ) ? zstrip_row(gz, NZ, P) : -1;
      pin[k] = row >= 0 ? a.psz_in[shot * zs_plane + (size_t)row * NX + gx] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kZPsi; ++k) {
      const int r = 4 + w + 4 * k, gz = ch.x - 8 + r;
      const int row = (col_ok && r < rows - 4 && gz >= 0 && gz < NZ) ? zstrip_row(gz, NZ, P) : -1;
      float t = 0.0f;
      if (row >= 0) {
        const float psb = pin[k] - d1s(&sQ[r * kTX + c], kTX);
        t = a.az[gz] * psb;
        if (r >= 8 && r < 8 + ch.y) a.psz_out[shot * zs_plane + (size_t)row * NX + gx] = a.bz[gz] * psb;
      }
      sT[r * kTX + c] = t;
    }
  }
  __syncthreads();
  float pp[kZOut];
#pragma unroll
  for (int k = 0; k < kZOut; ++k) {
    const int r = 8 + w + 4 * k, gz = ch.x - 8 + r;
    const bool ok = col_ok && r < 8 + ch.y && gz < NZ;
    pp[k] = ok ? a.prev_adj[shot * plane + (size_t)gz * NX + gx] : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < kZOut; ++k) {
    const int r = 8 + w + 4 * k, gz = ch.x - 8 + r;
    if (!(col_ok && r < 8 + ch.y && gz < NZ)) continue;
    const float E = d2s(&sS[r * kTX + c], kTX) - d1s(&sT[r * kTX + c], kTX);
    a.prev_adj[shot * plane + (size_t)gz * NX + gx] = pp[k] - E;
  }
}

// ---------------------------------------------------------------------------
// Kernel entry points: one plan (block coordinates from the launch grid) or a
// batch of plans of different shapes in one launch (the flat block index is
// split by the per-plan block counts of this launch).
// ---------------------------------------------------------------------------
template <int RZ>
__global__ __launch_bounds__(kThreads) void ac_fwd_main(AcStep a) {
  ac_fwd_main_body<RZ>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}
template <int RZ>
__global__ __launch_bounds__(kThreads) void ac_adj_main(AcStep a) {
  ac_adj_main_body<RZ>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}
__global__ __launch_bounds__(kThreads) void ac_fwd_xband(AcStep a) {
  ac_fwd_xband_body(a, blockIdx.x, blockIdx.y, blockIdx.z);
}
__global__ __launch_bounds__(kThreads) void ac_adj_xband(AcStep a) {
  ac_adj_xband_body(a, blockIdx.x, blockIdx.y, blockIdx.z);
}
__global__ __launch_bounds__(kThreads) void ac_fwd_zband(AcStep a) {
  ac_fwd_zband_body(a, blockIdx.x, blockIdx.y, blockIdx.z);
}
__global__ __launch_bounds__(kThreads) void ac_adj_zband(AcStep a) {
  ac_adj_zband_body(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// plan index and the block coordinates inside that plan's grid
struct BatchCoord {
  int p, x, y, z;
};
__device__ __forceinline__ BatchCoord batch_coord(const AcBatch& b) {
  const int f = blockIdx.x;
  int p = 0;
  while (p + 1 < b.nplans && f >= b.base[p + 1]) ++p;
  const int l = f - b.base[p];
  BatchCoord c;
  c.p = p;
  c.x = l % b.gx[p];
  c.y = (l / b.gx[p]) % b.gy[p];
  c.z = l / (b.gx[p] * b.gy[p]);
  return c;
}

template <int RZ>
__global__ __launch_bounds__(kThreads) void ac_fwd_main_batch(AcBatch b) {
  const BatchCoord c = batch_coord(b);
  ac_fwd_main_body<RZ>(b.step[c.p], c.x, c.y, c.z);
}
template <int RZ>
__global__ __launch_bounds__(kThreads) void ac_adj_main_batch(AcBatch b) {
  const BatchCoord c = batch_coord(b);
  ac_adj_main_body<RZ>(b.step[c.p], c.x, c.y, c.z);
}
__global__ __launch_bounds__(kThreads) void ac_fwd_xband_batch(AcBatch b) {
  const BatchCoord c = batch_coord(b);
  ac_fwd_xband_body(b.step[c.p], c.x, c.y, c.z);
}
__global__ __launch_bounds__(kThreads) void ac_adj_xband_batch(AcBatch b) {
  const BatchCoord c = batch_coord(b);
  ac_adj_xband_body(b.step[c.p], c.x, c.y, c.z);
}
__global__ __launch_bounds__(kThreads) void ac_fwd_zband_batch(AcBatch b) {
  const BatchCoord c = batch_coord(b);
  ac_fwd_zband_body(b.step[c.p], c.x, c.y, c.z);
}
__global__ __launch_bounds__(kThreads) void ac_adj_zband_batch(AcBatch b) {
  const BatchCoord c = batch_coord(b);
  ac_adj_zband_body(b.step[c.p], c.x, c.y, c.z);
}

// ---------------------------------------------------------------------------
// Adjoint start: lambda^{nt}[rec] += r_{nt-1} (receiver order, so coincident
// receivers add up deterministically), after the state was zero-filled.
// ---------------------------------------------------------------------------
__global__ void ac_inject_last(float* lam, size_t plane, const int* rec_cell,
                               const float* resid, int nshots, int nt, int nrec) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshots) return;
  const float* r = resid + ((size_t)s * nt + (nt - 1)) * nrec;
  for (int k = 0; k < nrec; ++k) lam[s * plane + rec_cell[(size_t)s * nrec + k]] += r[k];
}

// tot[c] += sum_s gpart[s][c], shots in order (float64).
__global__ void ac_fold_kernel(double* tot, const float* __restrict__ gpart, int nshots,
                               size_t plane) {
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= plane) return;
  double acc = tot[c];
  for (int s = 0; s < nshots; ++s) acc += (double)gpart[s * plane + c];
  tot[c] = acc;
}

// grad[jj][ii] = sum over padded cells replicating model cell (ii, jj) of
// 2 v dt^2/h^2 * dJ/dCs (the chain rule of Cs = (v dt/h)^2 and of edge padding).
__global__ void ac_finish_kernel(const double* tot, const float* vpad, float* grad, int nx,
                                 int nz, int P, int NX, double scale) {
  const int ii = blockIdx.x * blockDim.x + threadIdx.x;
  const int jj = blockIdx.y;
  if (ii >= nx || jj >= nz) return;
  const int NZ = nz + 2 * P;
  const int i0 = ii == 0 ? 0 : ii + P, i1 = ii == nx - 1 ? NX - 1 : ii + P;
  const int j0 = jj == 0 ? 0 : jj + P, j1 = jj == nz - 1 ? NZ - 1 : jj + P;
  double acc = 0.0;
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) {
      const size_t c = (size_t)j * NX + i;
      acc += scale * (double)vpad[c] * tot[c];
    }
  grad[(size_t)jj * nx + ii] = (float)acc;
}

// ev (optional): start/stop event pairs recorded around the main launch
// (ev[0], ev[1]) and the two band launches (ev[2], ev[3]).
template <int RZ, bool kAdj>
int launch_step(const AcStep& a, hipStream_t s, hipEvent_t* ev) {
  if (a.n_xchunks > 0 || a.n_zchunks > 0) {
    if (ev) SWEEP_HIP(hipEventRecord(ev[2], s));
    if (a.n_xchunks > 0) {
      const dim3 g(a.n_xchunks, (a.NZ + 4 * kXRows - 1) / (4 * kXRows), a.nshots);
      if (kAdj)
        hipLaunchKernelGGL(ac_adj_xband, g, dim3(kThreads), 0, s, a);
      else
        hipLaunchKernelGGL(ac_fwd_xband, g, dim3(kThreads), 0, s, a);
    }
    if (a.n_zchunks > 0) {
      const dim3 g((a.NX + kTX - 1) / kTX, a.n_zchunks, a.nshots);
      if (kAdj)
        hipLaunchKernelGGL(ac_adj_zband, g, dim3(kThreads), 0, s, a);
      else
        hipLaunchKernelGGL(ac_fwd_zband, g, dim3(kThreads), 0, s, a);
    }
    if (ev) SWEEP_HIP(hipEventRecord(ev[3], s));
  }
  if (ev) SWEEP_HIP(hipEventRecord(ev[0], s));
  const dim3 g(a.ntiles, a.nshots);
  if (kAdj)
    hipLaunchKernelGGL(ac_adj_main<RZ>, g, dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(ac_fwd_main<RZ>, g, dim3(kThreads), 0, s, a);
  if (ev) SWEEP_HIP(hipEventRecord(ev[1], s));
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

// One batched step over the active plans `steps[0..n)` (all with the same rz).
template <int RZ, bool kAdj>
int launch_step_batch(const AcStep* steps, int n, hipStream_t s) {
  AcBatch b;
  // band kernels: x band, then z band, then the main kernel (as for one plan)
  for (int phase = 0; phase < 3; ++phase) {
    b.nplans = 0;
    b.base[0] = 0;
    for (int q = 0; q < n; ++q) {
      const AcStep& a = steps[q];
      int gx, gy, gz;
      if (phase == 0) {
        gx = a.n_xchunks;
        gy = (a.NZ + 4 * kXRows - 1) / (4 * kXRows);
        gz = a.nshots;
      } else if (phase == 1) {
        gx = (a.NX + kTX - 1) / kTX;
        gy = a.n_zchunks;
        gz = a.nshots;
      } else {
        gx = a.ntiles;
        gy = a.nshots;
        gz = 1;
      }
      if (gx <= 0 || gy <= 0 || gz <= 0) continue;
      const int k = b.nplans++;
      b.step[k] = a;
      b.gx[k] = gx;
      b.gy[k] = gy;
      b.base[k + 1] = b.base[k] + gx * gy * gz;
    }
    if (b.nplans == 0) continue;
    const dim3 g(b.base[b.nplans]);
    if (phase == 0) {
      if (kAdj)
        hipLaunchKernelGGL(ac_adj_xband_batch, g, dim3(kThreads), 0, s, b);
      else
        hipLaunchKernelGGL(ac_fwd_xband_batch, g, dim3(kThreads), 0, s, b);
    } else if (phase == 1) {
      if (kAdj)
        hipLaunchKernelGGL(ac_adj_zband_batch, g, dim3(kThreads), 0, s, b);
      else
        hipLaunchKernelGGL(ac_fwd_zband_batch, g, dim3(kThreads), 0, s, b);
    } else {
      if (kAdj)
        hipLaunchKernelGGL(ac_adj_main_batch<RZ>, g, dim3(kThreads), 0, s, b);
      else
        hipLaunchKernelGGL(ac_fwd_main_batch<RZ>, g, dim3(kThreads), 0, s, b);
    }
  }
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

}  // namespace

int ac_launch_prep(const float* v, float* vpad, float* Cs, float* ax, float* bx, float* az,
                   float* bz, int nx, int nz, int P, double h, double dt, double vmax,
                   double f0, double R, hipStream_t s) {
  const int NX = nx + 2 * P, NZ = nz + 2 * P;
  hipLaunchKernelGGL(ac_prep_kernel, dim3((NX + 255) / 256, NZ), dim3(256), 0, s, v, vpad, Cs,
                     nx, nz, P, dt / h);
  const int nmax = NX > NZ ? NX : NZ;
  hipLaunchKernelGGL(ac_tables_kernel, dim3((nmax + 255) / 256), dim3(256), 0, s, ax, bx, az,
                     bz, NX, NZ, P, h, dt, vmax, f0, R);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int ac_launch_fwd(const AcStep& a, int rz, hipStream_t s, hipEvent_t* ev) {
  switch (rz) {
    case 1: return launch_step<1, false>(a, s, ev);
    case 2: return launch_step<2, false>(a, s, ev);
    case 4: return launch_step<4, false>(a, s, ev);
    case 8: return launch_step<8, false>(a, s, ev);
  }
  set_error("unsupported rz");
  return SWEEP_EINVAL;
}

int ac_launch_adj(const AcStep& a, int rz, hipStream_t s, hipEvent_t* ev) {
  switch (rz) {
    case 1: return launch_step<1, true>(a, s, ev);
    case 2: return launch_step<2, true>(a, s, ev);
    case 4: return launch_step<4, true>(a, s, ev);
    case 8: return launch_step<8, true>(a, s, ev);
  }
  set_error("unsupported rz");
  return SWEEP_EINVAL;
}

int ac_launch_adj_init(float* lam_cur, float* lam_prev, size_t plane_elems, float* aux,
                       size_t aux_elems, const int* rec_cell, const float* resid, int nshots,
                       int nt, int nrec, hipStream_t s) {
  int rc;
  if ((rc = launch_fill(lam_cur, plane_elems, 0.0f, s))) return rc;
  if ((rc = launch_fill(lam_prev, plane_elems, 0.0f, s))) return rc;
  if (aux_elems && (rc = launch_fill(aux, aux_elems, 0.0f, s))) return rc;
  const size_t plane = plane_elems / (size_t)nshots;
  if (nrec > 0)
    hipLaunchKernelGGL(ac_inject_last, dim3((nshots + 63) / 64), dim3(64), 0, s, lam_cur, plane,
                       rec_cell, resid, nshots, nt, nrec);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int ac_launch_fold(double* tot, const float* gpart, int nshots, size_t plane, hipStream_t s) {
  hipLaunchKernelGGL(ac_fold_kernel, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, s, tot,
                     gpart, nshots, plane);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int ac_launch_finish(const double* tot, const float* vpad, float* grad, int nx, int nz, int P,
                     int NX, double scale, hipStream_t s) {
  hipLaunchKernelGGL(ac_finish_kernel, dim3((nx + 255) / 256, nz), dim3(256), 0, s, tot, vpad,
                     grad, nx, nz, P, NX, scale);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

}  // namespace sweep

namespace sweep {

int ac_launch_fwd_batch(const AcStep* steps, int n, int rz, hipStream_t s) {
  switch (rz) {
    case 1: return launch_step_batch<1, false>(steps, n, s);
    case 2: return launch_step_batch<2, false>(steps, n, s);
    case 4: return launch_step_batch<4, false>(steps, n, s);
    case 8: return launch_step_batch<8, false>(steps, n, s);
  }
  set_error("unsupported rz");
  return SWEEP_EINVAL;
}

int ac_launch_adj_batch(const AcStep* steps, int n, int rz, hipStream_t s) {
  switch (rz) {
    case 1: return launch_step_batch<1, true>(steps, n, s);
    case 2: return launch_step_batch<2, true>(steps, n, s);
    case 4: return launch_step_batch<4, true>(steps, n, s);
    case 8: return launch_step_batch<8, true>(steps, n, s);
  }
  set_error("unsupported rz");
  return SWEEP_EINVAL;
}

}  // namespace sweep
