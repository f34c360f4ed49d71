// Acoustic step kernels for gfx950: the constant-density wave equation
// (Sec. 3.1.2, Eq. 2) advanced with the leapfrog update of the paper's step
// function (Sec. 2.1), an 8th-order Laplacian and a C-PML absorbing pad, and the
// exact transpose of that recurrence for the adjoint (Sec. 1).
//
// Scaled form used on the GPU (h folded into the coefficients):
//   Cs = (v dt / h)^2, D2' = h^2 D2, D1' = h D1, psi' = h psi, zeta' = h^2 zeta,
//   B' = h^2 B, so p^{n+1} = 2 p^n - p^{n-1} + Cs B'^n + (dt/h)^2 s_n e_src.
//
// Every work-group covers a 64-column x TZ-row tile of one shot. Interior tiles
// (the tile and its 4-cell halo clear of the pad) run the plain update with a
// halo tile of p staged in LDS and TZ/4 rows per thread held in registers, so
// each HBM array is read once per cell. Tiles touching the pad run a general
// kernel that stages p with an 8-cell halo and computes the memory variables
// for the halo redundantly; memory variables are double-buffered so no
// work-group reads a value another one is overwriting in the same launch.
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
// independent of the tiling and of which kernel handles a cell).
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
// Forward step, interior tiles. TZ = 4 RZ rows; thread (lx, wz) owns column lx
// and rows [wz RZ, wz RZ + RZ) of the tile.
// ---------------------------------------------------------------------------
template <int RZ>
__global__ __launch_bounds__(kThreads) void ac_fwd_interior(AcStep a) {
  constexpr int TZ = 4 * RZ;
  constexpr int LW = kTX + 8;
  constexpr int LH = TZ + 8;
  __shared__ float sp[LH * LW];

  const int tid = threadIdx.x;
  const int lx = tid & 63;
  const int zb = (tid >> 6) * RZ;
  const int t = blockIdx.x;
  const int tx = a.int_tx0 + t % a.int_ntx;
  const int tz = a.int_tz0 + t / a.int_ntx;
  const int tile = tz * a.tiles_x + tx;
  const int shot = blockIdx.y;
  const int NX = a.NX;
  const size_t plane = (size_t)NX * a.NZ;
  const int x0 = tx * kTX, z0 = tz * TZ;
  const float* __restrict__ cur = a.cur + shot * plane;

  {  // stage p^n with a 4-cell halo (entirely inside the grid)
    const float* base = cur + (size_t)(z0 - 4) * NX + (x0 - 4);
    for (int e = tid; e < LH * LW; e += kThreads) {
      const int r = e / LW;
      const int c = e - r * LW;
      sp[e] = base[(size_t)r * NX + c];
    }
  }
  __syncthreads();

  float win[RZ + 8];
#pragma unroll
  for (int m = 0; m < RZ + 8; ++m) win[m] = sp[(zb + m) * LW + lx + 4];

  const int gx = x0 + lx;
  const int src = a.src_cell[shot];
  const float sw = a.w * a.wavelet[(size_t)shot * a.nt + a.n];
  float out[RZ];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const float* row = &sp[(zb + r + 4) * LW + lx + 4];
    const float c = win[r + 4];
    const float sx = d2c(c, row[1], row[-1], row[2], row[-2], row[3], row[-3], row[4], row[-4]);
    const float sz = d2c(c, win[r + 5], win[r + 3], win[r + 6], win[r + 2], win[r + 7],
                         win[r + 1], win[r + 8], win[r]);
    const float B = sx + sz;
    const int idx = (z0 + zb + r) * NX + gx;
    const size_t gi = shot * plane + idx;
    const float pp = a.prev[gi];
    float pn = fmaf(a.Cs[idx], B, 2.0f * c - pp);
    if (idx == src) pn += sw;
    a.next[gi] = pn;
    if (a.B_out) a.B_out[gi] = B;
    if (a.ck_cur) {
      a.ck_cur[gi] = c;
      a.ck_prev[gi] = pp;
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

// ---------------------------------------------------------------------------
// Forward step, tiles touching the pad (general form with memory variables).
// ---------------------------------------------------------------------------
template <int TZ>
__global__ __launch_bounds__(kThreads) void ac_fwd_frame(AcStep a) {
  constexpr int PW = kTX + 16;  // p with an 8-cell halo
  constexpr int PH = TZ + 16;
  constexpr int XW = kTX + 8;   // psi_x on the tile rows, 4-cell x halo
  constexpr int ZH = TZ + 8;    // psi_z on the tile columns, 4-cell z halo
  __shared__ float sp[PH * PW];
  __shared__ float sx[TZ * XW];
  __shared__ float sz[ZH * kTX];
  __shared__ float st[TZ * kTX];

  const int tid = threadIdx.x;
  const int tile = a.frame_tiles[blockIdx.x];
  const int shot = blockIdx.y;
  const int NX = a.NX, NZ = a.NZ, P = a.P, P2 = 2 * a.P;
  const size_t plane = (size_t)NX * NZ;
  const size_t xs_plane = (size_t)NZ * P2;
  const size_t zs_plane = (size_t)P2 * NX;
  const int x0 = (tile % a.tiles_x) * kTX;
  const int z0 = (tile / a.tiles_x) * TZ;
  const float* __restrict__ cur = a.cur + shot * plane;

  for (int e = tid; e < PH * PW; e += kThreads) {
    const int lz = e / PW, lc = e - lz * PW;
    const int gx = x0 - 8 + lc, gz = z0 - 8 + lz;
    sp[e] = (gx >= 0 && gx < NX && gz >= 0 && gz < NZ) ? cur[(size_t)gz * NX + gx] : 0.0f;
  }
  __syncthreads();

  // psi_x^n = b_x psi_x^{n-1} + a_x D1x' p^n on the tile rows, columns x0-4 .. x0+67
  for (int e = tid; e < TZ * XW; e += kThreads) {
    const int lz = e / XW, lc = e - lz * XW;
    const int gx = x0 - 4 + lc, gz = z0 + lz;
    float v = 0.0f;
    if (gz < NZ && gx >= 0 && gx < NX) {
      const int col = xstrip_col(gx, NX, P);
      if (col >= 0) {
        const float* q = &sp[(lz + 8) * PW + lc + 4];
        const float d1 = d1c(q[1], q[-1], q[2], q[-2], q[3], q[-3], q[4], q[-4]);
        const size_t si = shot * xs_plane + (size_t)gz * P2 + col;
        const float old = a.psx_in[si];
        v = fmaf(a.ax[gx], d1, a.bx[gx] * old);
        if (lc >= 4 && lc < 4 + kTX) {
          a.psx_out[si] = v;
          if (a.ck_psx) a.ck_psx[si] = old;
        }
      }
    }
    sx[e] = v;
  }
  // psi_z^n on the tile columns, rows z0-4 .. z0+TZ+3
  for (int e = tid; e < ZH * kTX; e += kThreads) {
    const int lz = e / kTX, lc = e - lz * kTX;
    const int gx = x0 + lc, gz = z0 - 4 + lz;
    float v = 0.0f;
    if (gx < NX && gz >= 0 && gz < NZ) {
      const int row = zstrip_row(gz, NZ, P);
      if (row >= 0) {
        const float* q = &sp[(lz + 4) * PW + lc + 8];
        const float d1 = d1c(q[PW], q[-PW], q[2 * PW], q[-2 * PW], q[3 * PW], q[-3 * PW],
                             q[4 * PW], q[-4 * PW]);
        const size_t si = shot * zs_plane + (size_t)row * NX + gx;
        const float old = a.psz_in[si];
        v = fmaf(a.az[gz], d1, a.bz[gz] * old);
        if (lz >= 4 && lz < 4 + TZ) {
          a.psz_out[si] = v;
          if (a.ck_psz) a.ck_psz[si] = old;
        }
      }
    }
    sz[e] = v;
  }
  __syncthreads();

  const int src = a.src_cell[shot];
  const float sw = a.w * a.wavelet[(size_t)shot * a.nt + a.n];
  for (int e = tid; e < TZ * kTX; e += kThreads) {
    const int lz = e / kTX, lc = e - lz * kTX;
    const int gx = x0 + lc, gz = z0 + lz;
    float pn = 0.0f;
    if (gx < NX && gz < NZ) {
      const float* pc = &sp[(lz + 8) * PW + lc + 8];
      const float c = pc[0];
      const float d2x = d2c(c, pc[1], pc[-1], pc[2], pc[-2], pc[3], pc[-3], pc[4], pc[-4]);
      const float d2z = d2c(c, pc[PW], pc[-PW], pc[2 * PW], pc[-2 * PW], pc[3 * PW],
                            pc[-3 * PW], pc[4 * PW], pc[-4 * PW]);
      const float* qx = &sx[lz * XW + lc + 4];
      const float* qz = &sz[(lz + 4) * kTX + lc];
      const float Qx = d2x + d1c(qx[1], qx[-1], qx[2], qx[-2], qx[3], qx[-3], qx[4], qx[-4]);
      const float Qz = d2z + d1c(qz[kTX], qz[-kTX], qz[2 * kTX], qz[-2 * kTX], qz[3 * kTX],
                                 qz[-3 * kTX], qz[4 * kTX], qz[-4 * kTX]);
      float zx = 0.0f, zz = 0.0f;
      const int col = xstrip_col(gx, NX, P);
      if (col >= 0) {
        const size_t si = shot * xs_plane + (size_t)gz * P2 + col;
        const float old = a.zex_in[si];
        zx = fmaf(a.ax[gx], Qx, a.bx[gx] * old);
        a.zex_out[si] = zx;
        if (a.ck_zex) a.ck_zex[si] = old;
      }
      const int row = zstrip_row(gz, NZ, P);
      if (row >= 0) {
        const size_t si = shot * zs_plane + (size_t)row * NX + gx;
        const float old = a.zez_in[si];
        zz = fmaf(a.az[gz], Qz, a.bz[gz] * old);
        a.zez_out[si] = zz;
        if (a.ck_zez) a.ck_zez[si] = old;
      }
      const float B = ((Qx + zx) + Qz) + zz;
      const int idx = gz * NX + gx;
      const size_t gi = shot * plane + idx;
      const float pp = a.prev[gi];
      pn = fmaf(a.Cs[idx], B, 2.0f * c - pp);
      if (idx == src) pn += sw;
      a.next[gi] = pn;
      if (a.B_out) a.B_out[gi] = B;
      if (a.ck_cur) {
        a.ck_cur[gi] = c;
        a.ck_prev[gi] = pp;
      }
    }
    st[e] = pn;
  }

  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  const int e0 = ro[0], e1 = ro[1];
  if (a.gathers && e1 > e0) {
    __syncthreads();
    float* dst = a.gathers + ((size_t)shot * a.nt + a.n) * a.nrec;
    for (int e = e0 + tid; e < e1; e += kThreads) {
      const int2 en = a.rec_ent[e];
      dst[en.y] = st[en.x];
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

// ---------------------------------------------------------------------------
// Adjoint step, interior tiles: lambda^n = 2 lambda^{n+1} - lambda^{n+2}
// + D2'(Cs lambda^{n+1}); g += lambda^{n+1} B'^n; then r_{n-1} is injected.
// ---------------------------------------------------------------------------
template <int RZ>
__global__ __launch_bounds__(kThreads) void ac_adj_interior(AcStep a) {
  constexpr int TZ = 4 * RZ;
  constexpr int LW = kTX + 8;
  constexpr int LH = TZ + 8;
  __shared__ float sq[LH * LW];

  const int tid = threadIdx.x;
  const int lx = tid & 63;
  const int zb = (tid >> 6) * RZ;
  const int t = blockIdx.x;
  const int tx = a.int_tx0 + t % a.int_ntx;
  const int tz = a.int_tz0 + t / a.int_ntx;
  const int tile = tz * a.tiles_x + tx;
  const int shot = blockIdx.y;
  const int NX = a.NX;
  const size_t plane = (size_t)NX * a.NZ;
  const int x0 = tx * kTX, z0 = tz * TZ;
  const float* __restrict__ cur = a.cur + shot * plane;

  {  // stage q = Cs lambda^{n+1} with a 4-cell halo
    const size_t off = (size_t)(z0 - 4) * NX + (x0 - 4);
    for (int e = tid; e < LH * LW; e += kThreads) {
      const int r = e / LW;
      const int c = e - r * LW;
      const size_t k = off + (size_t)r * NX + c;
      sq[e] = a.Cs[k] * cur[k];
    }
  }
  __syncthreads();

  float win[RZ + 8];
#pragma unroll
  for (int m = 0; m < RZ + 8; ++m) win[m] = sq[(zb + m) * LW + lx + 4];

  const int gx = x0 + lx;
  float out[RZ];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const float* row = &sq[(zb + r + 4) * LW + lx + 4];
    const float c = win[r + 4];
    const float sxx = d2c(c, row[1], row[-1], row[2], row[-2], row[3], row[-3], row[4], row[-4]);
    const float szz = d2c(c, win[r + 5], win[r + 3], win[r + 6], win[r + 2], win[r + 7],
                          win[r + 1], win[r + 8], win[r]);
    const int idx = (z0 + zb + r) * NX + gx;
    const size_t gi = shot * plane + idx;
    const float p1 = a.cur[gi];
    const float gb = p1 * a.B_in[gi];
    a.g[gi] = a.g_init ? gb : a.g[gi] + gb;
    // same association as the frame kernel, so a cell's value does not depend
    // on which kernel updates it
    out[r] = ((2.0f * p1 - a.prev[gi]) + sxx) + szz;
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
  for (int r = 0; r < RZ; ++r) a.next[shot * plane + (size_t)(z0 + zb + r) * NX + gx] = out[r];
}

// ---------------------------------------------------------------------------
// Adjoint step, tiles touching the pad (exact transpose of ac_fwd_frame):
//   zbar = Z + Cs P1, Qbar = Cs P1 + a zbar, psbar = Psi - D1' Qbar,
//   lambda = 2 P1 - P1prev + D2x' Qbar_x + D2z' Qbar_z - D1x'(a_x psbar_x) - D1z'(a_z psbar_z),
//   Psi <- b psbar, Z <- b zbar (kept only inside the strips, where a != 0).
// ---------------------------------------------------------------------------
template <int TZ>
__global__ __launch_bounds__(kThreads) void ac_adj_frame(AcStep a) {
  constexpr int QXW = kTX + 16;  // Qbar_x: tile rows, 8-cell x halo
  constexpr int QZH = TZ + 16;   // Qbar_z: tile columns, 8-cell z halo
  constexpr int TXW = kTX + 8;   // a_x psbar_x: 4-cell x halo
  constexpr int TZH = TZ + 8;    // a_z psbar_z: 4-cell z halo
  __shared__ float sqx[TZ * QXW];
  __shared__ float sqz[QZH * kTX];
  __shared__ float stx[TZ * TXW];
  __shared__ float stz[TZH * kTX];
  __shared__ float st[TZ * kTX];

  const int tid = threadIdx.x;
  const int tile = a.frame_tiles[blockIdx.x];
  const int shot = blockIdx.y;
  const int NX = a.NX, NZ = a.NZ, P = a.P, P2 = 2 * a.P;
  const size_t plane = (size_t)NX * NZ;
  const size_t xs_plane = (size_t)NZ * P2;
  const size_t zs_plane = (size_t)P2 * NX;
  const int x0 = (tile % a.tiles_x) * kTX;
  const int z0 = (tile / a.tiles_x) * TZ;
  const float* __restrict__ cur = a.cur + shot * plane;

  for (int e = tid; e < TZ * QXW; e += kThreads) {
    const int lz = e / QXW, lc = e - lz * QXW;
    const int gx = x0 - 8 + lc, gz = z0 + lz;
    float q = 0.0f;
    if (gx >= 0 && gx < NX && gz < NZ) {
      const size_t k = (size_t)gz * NX + gx;
      const float cp = a.Cs[k] * cur[k];
      q = cp;
      const int col = xstrip_col(gx, NX, P);
      if (col >= 0) {
        const size_t si = shot * xs_plane + (size_t)gz * P2 + col;
        const float zb = a.zex_in[si] + cp;
        q = fmaf(a.ax[gx], zb, cp);
        if (lc >= 8 && lc < 8 + kTX) a.zex_out[si] = a.bx[gx] * zb;
      }
    }
    sqx[e] = q;
  }
  for (int e = tid; e < QZH * kTX; e += kThreads) {
    const int lz = e / kTX, lc = e - lz * kTX;
    const int gx = x0 + lc, gz = z0 - 8 + lz;
    float q = 0.0f;
    if (gx < NX && gz >= 0 && gz < NZ) {
      const size_t k = (size_t)gz * NX + gx;
      const float cp = a.Cs[k] * cur[k];
      q = cp;
      const int row = zstrip_row(gz, NZ, P);
      if (row >= 0) {
        const size_t si = shot * zs_plane + (size_t)row * NX + gx;
        const float zb = a.zez_in[si] + cp;
        q = fmaf(a.az[gz], zb, cp);
        if (lz >= 8 && lz < 8 + TZ) a.zez_out[si] = a.bz[gz] * zb;
      }
    }
    sqz[e] = q;
  }
  __syncthreads();

  for (int e = tid; e < TZ * TXW; e += kThreads) {
    const int lz = e / TXW, lc = e - lz * TXW;
    const int gx = x0 - 4 + lc, gz = z0 + lz;
    float t = 0.0f;
    if (gx >= 0 && gx < NX && gz < NZ) {
      const int col = xstrip_col(gx, NX, P);
      if (col >= 0) {
        const float* q = &sqx[lz * QXW + lc + 4];
        const size_t si = shot * xs_plane + (size_t)gz * P2 + col;
        const float psb =
            a.psx_in[si] - d1c(q[1], q[-1], q[2], q[-2], q[3], q[-3], q[4], q[-4]);
        t = a.ax[gx] * psb;
        if (lc >= 4 && lc < 4 + kTX) a.psx_out[si] = a.bx[gx] * psb;
      }
    }
    stx[e] = t;
  }
  for (int e = tid; e < TZH * kTX; e += kThreads) {
    const int lz = e / kTX, lc = e - lz * kTX;
    const int gx = x0 + lc, gz = z0 - 4 + lz;
    float t = 0.0f;
    if (gx < NX && gz >= 0 && gz < NZ) {
      const int row = zstrip_row(gz, NZ, P);
      if (row >= 0) {
        const float* q = &sqz[(lz + 4) * kTX + lc];
        const size_t si = shot * zs_plane + (size_t)row * NX + gx;
        const float psb = a.psz_in[si] - d1c(q[kTX], q[-kTX], q[2 * kTX], q[-2 * kTX],
                                             q[3 * kTX], q[-3 * kTX], q[4 * kTX], q[-4 * kTX]);
        t = a.az[gz] * psb;
        if (lz >= 4 && lz < 4 + TZ) a.psz_out[si] = a.bz[gz] * psb;
      }
    }
    stz[e] = t;
  }
  __syncthreads();

  for (int e = tid; e < TZ * kTX; e += kThreads) {
    const int lz = e / kTX, lc = e - lz * kTX;
    const int gx = x0 + lc, gz = z0 + lz;
    float lam = 0.0f;
    if (gx < NX && gz < NZ) {
      const float* qx = &sqx[lz * QXW + lc + 8];
      const float* qz = &sqz[(lz + 8) * kTX + lc];
      const float* tx = &stx[lz * TXW + lc + 4];
      const float* tz = &stz[(lz + 4) * kTX + lc];
      const float d2x =
          d2c(qx[0], qx[1], qx[-1], qx[2], qx[-2], qx[3], qx[-3], qx[4], qx[-4]);
      const float d2z = d2c(qz[0], qz[kTX], qz[-kTX], qz[2 * kTX], qz[-2 * kTX], qz[3 * kTX],
                            qz[-3 * kTX], qz[4 * kTX], qz[-4 * kTX]);
      const float d1x = d1c(tx[1], tx[-1], tx[2], tx[-2], tx[3], tx[-3], tx[4], tx[-4]);
      const float d1z = d1c(tz[kTX], tz[-kTX], tz[2 * kTX], tz[-2 * kTX], tz[3 * kTX],
                            tz[-3 * kTX], tz[4 * kTX], tz[-4 * kTX]);
      const size_t gi = shot * plane + (size_t)gz * NX + gx;
      const float p1 = a.cur[gi];
      const float gb = p1 * a.B_in[gi];
      a.g[gi] = a.g_init ? gb : a.g[gi] + gb;
      lam = (((2.0f * p1 - a.prev[gi]) + d2x) + d2z) - d1x - d1z;
    }
    st[e] = lam;
  }
  __syncthreads();
  if (a.n >= 1) {
    inject_residual(a, shot, tile, st);
    __syncthreads();
  }
  for (int e = tid; e < TZ * kTX; e += kThreads) {
    const int lz = e / kTX, lc = e - lz * kTX;
    const int gx = x0 + lc, gz = z0 + lz;
    if (gx < NX && gz < NZ) a.next[shot * plane + (size_t)gz * NX + gx] = st[e];
  }
}

// ---------------------------------------------------------------------------
// Adjoint start: zero the adjoint state, then lambda^{nt}[rec] = r_{nt-1}
// (receiver order, so coincident receivers add up deterministically).
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

// ev (optional): start/stop event pairs recorded around the interior launch
// (ev[0], ev[1]) and the frame launch (ev[2], ev[3]).
template <int RZ>
int launch_fwd_rz(const AcStep& a, int n_int, hipStream_t s, hipEvent_t* ev) {
  constexpr int TZ = 4 * RZ;
  if (n_int > 0) {
    if (ev) SWEEP_HIP(hipEventRecord(ev[0], s));
    hipLaunchKernelGGL(ac_fwd_interior<RZ>, dim3(n_int, a.nshots), dim3(kThreads), 0, s, a);
    if (ev) SWEEP_HIP(hipEventRecord(ev[1], s));
  }
  if (a.n_frame > 0) {
    if (ev) SWEEP_HIP(hipEventRecord(ev[2], s));
    hipLaunchKernelGGL(ac_fwd_frame<TZ>, dim3(a.n_frame, a.nshots), dim3(kThreads), 0, s, a);
    if (ev) SWEEP_HIP(hipEventRecord(ev[3], s));
  }
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

template <int RZ>
int launch_adj_rz(const AcStep& a, int n_int, hipStream_t s, hipEvent_t* ev) {
  constexpr int TZ = 4 * RZ;
  if (n_int > 0) {
    if (ev) SWEEP_HIP(hipEventRecord(ev[0], s));
    hipLaunchKernelGGL(ac_adj_interior<RZ>, dim3(n_int, a.nshots), dim3(kThreads), 0, s, a);
    if (ev) SWEEP_HIP(hipEventRecord(ev[1], s));
  }
  if (a.n_frame > 0) {
    if (ev) SWEEP_HIP(hipEventRecord(ev[2], s));
    hipLaunchKernelGGL(ac_adj_frame<TZ>, dim3(a.n_frame, a.nshots), dim3(kThreads), 0, s, a);
    if (ev) SWEEP_HIP(hipEventRecord(ev[3], s));
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

int ac_launch_fwd(const AcStep& a, int rz, int n_int, hipStream_t s, hipEvent_t* ev) {
  switch (rz) {
    case 1: return launch_fwd_rz<1>(a, n_int, s, ev);
    case 2: return launch_fwd_rz<2>(a, n_int, s, ev);
    case 4: return launch_fwd_rz<4>(a, n_int, s, ev);
    case 8: return launch_fwd_rz<8>(a, n_int, s, ev);
  }
  set_error("unsupported rz");
  return SWEEP_EINVAL;
}

int ac_launch_adj(const AcStep& a, int rz, int n_int, hipStream_t s, hipEvent_t* ev) {
  switch (rz) {
    case 1: return launch_adj_rz<1>(a, n_int, s, ev);
    case 2: return launch_adj_rz<2>(a, n_int, s, ev);
    case 4: return launch_adj_rz<4>(a, n_int, s, ev);
    case 8: return launch_adj_rz<8>(a, n_int, s, ev);
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
