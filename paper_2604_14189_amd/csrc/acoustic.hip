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
//   P+4 of the left/right edges) and Ez likewise in the z band. The grid is cut
//   into 64 x TZ tiles (TZ = 4 RZ). Tiles with no band cell form a rectangle and
//   are advanced by the interior kernel, which computes only the leapfrog with
//   D2' p (16 bytes per cell); the frame of tiles around it is advanced by the
//   PML kernel, which does the whole update of its cells in one pass: psi on a
//   4-cell halo ring in LDS, then zeta, B' and p^{n+1}. Both kernels record
//   receivers and inject the source of their own tiles. At a cell outside the
//   band every C-PML term is an exact zero, so both kernels produce the same
//   bits there and results do not depend on the tiling.
// The adjoint is the same split of the transposed recurrence. Work-groups are
// spread over the XCDs in contiguous runs of tiles (see xcd_spread).
#include "fd.h"
#include "internal.h"

namespace sweep {
namespace {

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

// Born model perturbation on the padded grid: dCs = d(Cs)/dv . dv =
// 2 v dv (dt/h)^2, with dv edge-replicated into the pad like v.
__global__ void ac_born_prep_kernel(const float* __restrict__ v, const float* __restrict__ dv,
                                    float* __restrict__ dCs, int nx, int nz, int P, double r) {
  const int NX = nx + 2 * P, NZ = nz + 2 * P;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= NX || j >= NZ) return;
  const int ii = min(max(i - P, 0), nx - 1);
  const int jj = min(max(j - P, 0), nz - 1);
  const size_t k = (size_t)jj * nx + ii;
  dCs[(size_t)j * NX + i] = (float)(2.0 * (double)v[k] * (double)dv[k] * r * r);
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
// Tiles and work-group placement.
// ---------------------------------------------------------------------------
// The frame (tiles outside the interior rectangle) is split in two sets.
// x frame: the tile columns left and right of the rectangle, all rows; these
// are exactly the columns with an x-strip cell within 4 cells.
// z frame: the columns of the rectangle, in the rows above and below it.
// With an empty rectangle (itx0 = itx1 = itz0 = itz1 = 0) the x frame is the
// whole grid and the z frame is empty.
__device__ __forceinline__ int xframe_tile(const AcStep& a, int f) {
  const int nl = a.itx0, per = nl + (a.tiles_x - a.itx1);
  const int tz = f / per, k = f % per;
  return tz * a.tiles_x + (k < nl ? k : a.itx1 + (k - nl));
}
__device__ __forceinline__ int zframe_tile(const AcStep& a, int f) {
  const int w = a.itx1 - a.itx0;
  const int rr = f / w;
  const int tz = rr < a.itz0 ? rr : a.itz1 + (rr - a.itz0);
  return tz * a.tiles_x + a.itx0 + f % w;
}

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
    const unsigned idx = ok ? (unsigned)(gz * NX + gx) : 0u;
    v[k] = ok ? u32at(f, idx) : 0.0f;
    if (kProduct) u[k] = ok ? u32at(g, idx) : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = tid + k * kThreads;
    if (e < N) s[e] = kProduct ? u[k] * v[k] : v[k];
  }
}

// Receivers of (shot, tile) in the block's rows [row0, row0 + 4 RZ) of the tile
// record p^{n+1}: the outputs are staged in st (64 x 4 RZ) and each CSR entry
// (local index (row within the tile) * 64 + column) copies one of them.
template <int RZ>
__device__ __forceinline__ void record_receivers(const AcStep& a, int shot, int tile, int row0,
                                                 const float* out, float* st) {
  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  const int e0 = ro[0], e1 = ro[1];
  if (!a.gathers || e1 <= e0) return;
  const int lx = threadIdx.x & 63, zb = (threadIdx.x >> 6) * RZ;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RZ; ++r) st[(zb + r) * kTX + lx] = out[r];
  __syncthreads();
  float* dst = a.gathers + ((size_t)shot * a.nt + a.n) * a.nrec;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += kThreads) {
    const int2 en = a.rec_ent[e];
    const int r = en.x >> 6;
    if (r >= row0 && r < row0 + 4 * RZ) dst[en.y] = st[en.x - row0 * kTX];
  }
}

// Adds r_{n-1} at the receivers of this (shot, tile) in rows [row0, row0 + nrows)
// to the staged lambda values st[local - row0 * 64] (run heads handle several
// receivers on one cell, in receiver order; a cell's entries are contiguous).
__device__ __forceinline__ void inject_residual(const AcStep& a, int shot, int tile, int row0,
                                                int nrows, float* st) {
  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  const int e0 = ro[0], e1 = ro[1];
  const float* r = a.resid + ((size_t)shot * a.nt + (a.n - 1)) * a.nrec;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += kThreads) {
    const int2 en = a.rec_ent[e];
    const int row = en.x >> 6;
    if (row < row0 || row >= row0 + nrows) continue;
    if (e == e0 || a.rec_ent[e - 1].x != en.x) {
      float acc = st[en.x - row0 * kTX];
      for (int k = e; k < e1 && a.rec_ent[k].x == en.x; ++k) acc += r[a.rec_ent[k].y];
      st[en.x - row0 * kTX] = acc;
    }
  }
}

// Writes lambda^n of the tile, after injecting r_{n-1} at its receivers.
template <int RZ>
__device__ __forceinline__ void adj_store(const AcStep& a, int shot, int tile, int row0, int x0,
                                          int z0, float* out, float* st) {
  const int lx = threadIdx.x & 63, zb = (threadIdx.x >> 6) * RZ;
  const int NX = a.NX, NZ = a.NZ;
  const size_t plane = (size_t)NX * NZ;
  float* next = a.next + shot * plane;
  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  if (a.resid && a.n >= 1 && ro[1] > ro[0]) {  // no residual: nothing injected (timing runs)
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RZ; ++r) st[(zb + r) * kTX + lx] = out[r];
    __syncthreads();
    inject_residual(a, shot, tile, row0, 4 * RZ, st);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RZ; ++r) out[r] = st[(zb + r) * kTX + lx];
  }
  const int gx = x0 + lx;
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const int gz = z0 + zb + r;
    if (gx < NX && gz < NZ) st_nt(&u32at(next, (unsigned)(gz * NX + gx)), out[r]);
  }
}

// ---------------------------------------------------------------------------
// Interior kernels: a 64 x TZ tile per work-group; thread (lx, w) owns column
// lx and rows [w RZ, w RZ + RZ), kept as a register window for the z stencil.
// ---------------------------------------------------------------------------
// p^{n+1} = 2 p^n - p^{n-1} + Cs D2' p^n (+ source); B'^n = D2' p^n if kept.
// kBorn: the perturbation step of Born modelling, p^{n+1} += dCs B'^n_background.
template <int RZ, bool kBorn = false>
__device__ __forceinline__ void ac_fwd_int_body(const AcStep& a, const int tile, const int shot) {
  using T = MainTile<RZ>;
  __shared__ float sp[T::LH * T::LW];
  const int tid = threadIdx.x;
  const int lx = tid & 63;
  const int zb = (tid >> 6) * RZ;
  const int NX = a.NX, NZ = a.NZ;
  const size_t plane = (size_t)NX * NZ;
  const int x0 = (tile % a.tiles_x) * kTX, z0 = (tile / a.tiles_x) * T::TZ;
  const bool inside = x0 >= 4 && x0 + kTX + 4 <= NX && z0 >= 4 && z0 + T::TZ + 4 <= NZ;
  const int gx = x0 + lx;

  // the per-cell operands are fetched first so their latency overlaps the
  // staging of the halo tile
  float pp[RZ], cs[RZ], bd[kBorn ? RZ : 1], bb[kBorn ? RZ : 1];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const int gz = z0 + zb + r;
    pp[r] = 0.0f;
    cs[r] = 0.0f;
    if (kBorn) bd[r] = bb[r] = 0.0f;
    if (inside || (gx < NX && gz < NZ)) {
      const unsigned idx = (unsigned)(gz * NX + gx);
      pp[r] = ld_nt(&u32at(a.prev + shot * plane, idx));
      cs[r] = u32at(a.Cs, idx);
      if (kBorn) {
        bd[r] = u32at(a.bdC, idx);
        bb[r] = ld_nt(&u32at(a.bB + shot * plane, idx));
      }
    }
  }
  // source cell and sample with the first loads (a later wait on them would
  // also wait for this tile's stores)
  const int src = a.src_cell[shot];
  const float sw = a.w * a.wavelet[(size_t)shot * a.nt + a.n];
  stage_box<RZ, false>(sp, a.cur + shot * plane, nullptr, x0, z0, NX, NZ, inside);
  __syncthreads();

  float win[RZ + 8];
#pragma unroll
  for (int m = 0; m < RZ + 8; ++m) win[m] = sp[(zb + m) * T::LW + lx + 4];

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
      pn = fmaf(cs[r], L, 2.0f * c - pp[r]);
      if (kBorn) pn += bd[r] * bb[r];
      if (idx == src) pn += sw;
      st_nt(&u32at(a.next + shot * plane, (unsigned)idx), pn);
      if (a.B_out) st_nt(&u32at(a.B_out + shot * plane, (unsigned)idx), L);
    }
    out[r] = pn;
  }
  record_receivers<RZ>(a, shot, tile, 0, out, sp);
}

// lambda^n = 2 lambda^{n+1} - lambda^{n+2} + D2'(Cs lambda^{n+1});
// g += lambda^{n+1} B'^n; then r_{n-1} is injected at the receivers.
template <int RZ>
__device__ __forceinline__ void ac_adj_int_body(const AcStep& a, const int tile, const int shot) {
  using T = MainTile<RZ>;
  __shared__ float sq[T::LH * T::LW];
  const int tid = threadIdx.x;
  const int lx = tid & 63;
  const int zb = (tid >> 6) * RZ;
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
      const unsigned gi = (unsigned)(gz * NX + gx);
      p1[r] = u32at(a.cur + shot * plane, gi);
      pp[r] = ld_nt(&u32at(a.prev + shot * plane, gi));
      bb[r] = ld_nt(&u32at(a.B_in + shot * plane, gi));
      if (!a.g_init) gg[r] = ld_nt(&u32at(a.g + shot * plane, gi));
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
      const unsigned gi = (unsigned)(gz * NX + gx);
      const float gb = p1[r] * bb[r];
      st_nt(&u32at(a.g + shot * plane, gi), a.g_init ? gb : gg[r] + gb);
      lam = ((2.0f * p1[r] - pp[r]) + sxx) + szz;
    }
    out[r] = lam;
  }
  adj_store<RZ>(a, shot, tile, 0, x0, z0, out, sq);
}

// ---------------------------------------------------------------------------
// PML kernels: the frame tiles, whole update in one pass. A work-group takes
// rows [row0, row0 + 4 RZ) of one frame tile (a frame tile is split into
// a.nsub such pieces), so its register and LDS footprint is set by its own RZ.
// Most frame tiles meet the strips of one axis only; the body is specialised
// on which axes have a strip cell within 4 cells of the piece (HX, HZ), and
// the other axis reduces exactly to the plain second difference.
// ---------------------------------------------------------------------------
template <int RZ, bool HX, bool HZ>
struct PmlGeom {
  static constexpr int TZ = 4 * RZ;
  static constexpr int hx = HX ? 8 : 4;  // halo of the staged field along x
  static constexpr int hz = HZ ? 8 : 4;  // and along z
  static constexpr int BW = kTX + 2 * hx;
  static constexpr int BH = TZ + 2 * hz;
  static constexpr int XW = kTX + 8;     // x ring (4-column halo)
  static constexpr int ZH = TZ + 8;      // z ring (4-row halo)
  // forward LDS: field box, psi_x ring, psi_z ring, C-PML (a, b) along the
  // box columns and rows
  static constexpr int NB = BH * BW;
  static constexpr int NPX = HX ? TZ * XW : 0;
  static constexpr int NPZ = HZ ? ZH * kTX : 0;
  static constexpr int kFwdFloats = NB + NPX + NPZ + 2 * BW + 2 * BH;
  // adjoint LDS: Qbar_x (tile rows, x halo hx), Qbar_z (tile columns, z halo hz),
  // T rings, C-PML (a, b) along the box columns and rows
  static constexpr int NQX = TZ * BW;
  static constexpr int NQZ = BH * kTX;
  static constexpr int kAdjFloats = NQX + NQZ + NPX + NPZ + 2 * BW + 2 * BH;
};

// LDS floats of the PML kernels: x frame (largest general variant, both axes)
// and z frame (field box with an 8-row and 4-column halo)
template <int RZ>
struct PmlLds {
  static constexpr int kFwd = PmlGeom<RZ, true, true>::kFwdFloats;
  static constexpr int kAdj = PmlGeom<RZ, true, true>::kAdjFloats;
  static constexpr int kZFwd = PmlGeom<RZ, false, true>::kFwdFloats;
  static constexpr int kZAdj = PmlGeom<RZ, false, true>::kAdjFloats;
  static constexpr int get(bool adj, bool z) {
    return z ? (adj ? kZAdj : kZFwd) : (adj ? kAdj : kFwd);
  }
};

// Whether the piece [x0, x0+64) x [z0, z0+TZ) has an x-strip (z-strip) cell
// within 4 cells along x (z).
__device__ __forceinline__ bool near_xstrip(int x0, int NX, int P) {
  return P > 0 && (x0 - 4 < P || x0 + kTX + 4 > NX - P);
}
__device__ __forceinline__ bool near_zstrip(int z0, int TZ, int NZ, int P) {
  return P > 0 && (z0 - 4 < P || z0 + TZ + 4 > NZ - P);
}

// Forward. psi_x^n = b_x psi_x^{n-1} + a_x D1x' p^n on the tile rows and a
// 4-column halo, psi_z^n likewise on the tile columns and a 4-row halo (zero
// outside the strips); then per cell
//   Bx = D2x' p + D1x' psi_x (+ zeta_x^n, zeta_x^n = b_x zeta_x^{n-1} + a_x (D2x' p + D1x' psi_x)
//   in the x strip), Bz likewise, B' = Bx + Bz, p^{n+1} = 2 p^n - p^{n-1} + Cs B'.
template <int RZ, bool HX, bool HZ, bool kBorn = false>
__device__ __forceinline__ void ac_fwd_pml_body(const AcStep& a, const int tile, const int shot,
                                                const int row0, float* lds) {
  using G = PmlGeom<RZ, HX, HZ>;
  constexpr int TZ = G::TZ, BW = G::BW, XW = G::XW, hx = G::hx, hz = G::hz;
  constexpr int NB = G::NB, KB = (NB + kThreads - 1) / kThreads;
  constexpr int NPX = G::NPX, KPX = (NPX + kThreads - 1) / kThreads;
  constexpr int NPZ = G::NPZ, KPZ = (NPZ + kThreads - 1) / kThreads;
  float* sb = lds;              // p^n: rows z0-hz .., columns x0-hx ..
  float* spx = lds + NB;        // psi_x^n: tile rows, columns x0-4 ..
  float* spz = lds + NB + NPX;  // psi_z^n: rows z0-4 .., tile columns
  float* tax = spz + NPZ;       // a_x, b_x at the box columns; a_z, b_z at the box rows
  float* tbx = tax + BW;
  float* taz = tbx + BW;
  float* tbz = taz + G::BH;
  const int tid = threadIdx.x;
  const int lx = tid & 63;
  const int zb = (tid >> 6) * RZ;
  const int NX = a.NX, NZ = a.NZ, P = a.P, P2 = 2 * P;
  const size_t plane = (size_t)NX * NZ;
  const size_t xsp = (size_t)NZ * P2, zsp = (size_t)P2 * NX;
  const int x0 = (tile % a.tiles_x) * kTX, z0 = (tile / a.tiles_x) * a.tz + row0;
  const int gx = x0 + lx;
  const float* cur = a.cur + shot * plane;

  // all global loads of the step are issued before the first use
  float vb[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int e = tid + k * kThreads;
    const int r = e / BW, c = e - (e / BW) * BW;
    const int gz = z0 - hz + r, gxx = x0 - hx + c;
    const bool ok = e < NB && gxx >= 0 && gxx < NX && gz >= 0 && gz < NZ;
    vb[k] = ok ? u32at(cur, (unsigned)(gz * NX + gxx)) : 0.0f;
  }
  float opx[HX ? KPX : 1], opz[HZ ? KPZ : 1];
  if constexpr (HX) {
#pragma unroll
    for (int k = 0; k < KPX; ++k) {
      const int e = tid + k * kThreads;
      const int r = e / XW, c = e - (e / XW) * XW;
      const int gz = z0 + r, gxx = x0 - 4 + c;
      const int col = (e < NPX && gz < NZ && gxx >= 0 && gxx < NX) ? xstrip_col(gxx, NX, P) : -1;
      opx[k] = col >= 0 ? u32at(a.psx_in + shot * xsp, (unsigned)(gz * P2 + col)) : 0.0f;
    }
  }
  if constexpr (HZ) {
#pragma unroll
    for (int k = 0; k < KPZ; ++k) {
      const int e = tid + k * kThreads;
      const int r = e >> 6, c = e & 63;
      const int gz = z0 - 4 + r, gxx = x0 + c;
      const int row = (e < NPZ && gxx < NX && gz >= 0 && gz < NZ) ? zstrip_row(gz, NZ, P) : -1;
      opz[k] = row >= 0 ? u32at(a.psz_in + shot * zsp, (unsigned)(row * NX + gxx)) : 0.0f;
    }
  }
  // C-PML coefficients of the box columns (threads 0..BW-1) and rows (128..)
  float ta = 0.0f, tb = 0.0f;
  if (tid < BW) {
    const int gxx = x0 - hx + tid;
    if (HX && gxx >= 0 && gxx < NX) {
      ta = a.ax[gxx];
      tb = a.bx[gxx];
    }
  } else if (tid >= 128 && tid < 128 + G::BH) {
    const int gz = z0 - hz + (tid - 128);
    if (HZ && gz >= 0 && gz < NZ) {
      ta = a.az[gz];
      tb = a.bz[gz];
    }
  }
  const int src = a.src_cell[shot];
  const float sw = a.w * a.wavelet[(size_t)shot * a.nt + a.n];
  const int xcol = (HX && gx < NX) ? xstrip_col(gx, NX, P) : -1;
  float pp[RZ], cs[RZ], zx[RZ], zz[RZ], bd[kBorn ? RZ : 1], bb[kBorn ? RZ : 1];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const int gz = z0 + zb + r;
    const bool ok = gx < NX && gz < NZ;
    const unsigned idx = ok ? (unsigned)(gz * NX + gx) : 0u;
    pp[r] = ok ? ld_nt(&u32at(a.prev + shot * plane, idx)) : 0.0f;
    cs[r] = ok ? u32at(a.Cs, idx) : 0.0f;
    if (kBorn) {
      bd[r] = ok ? u32at(a.bdC, idx) : 0.0f;
      bb[r] = ok ? ld_nt(&u32at(a.bB + shot * plane, idx)) : 0.0f;
    }
    zx[r] = (HX && ok && xcol >= 0) ? u32at(a.zex_in + shot * xsp, (unsigned)(gz * P2 + xcol)) : 0.0f;
    const int zrow = (HZ && ok) ? zstrip_row(gz, NZ, P) : -1;
    zz[r] = zrow >= 0 ? u32at(a.zez_in + shot * zsp, (unsigned)(zrow * NX + gx)) : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int e = tid + k * kThreads;
    if (e < NB) sb[e] = vb[k];
  }
  if (tid < BW) {
    tax[tid] = ta;
    tbx[tid] = tb;
  } else if (tid >= 128 && tid < 128 + G::BH) {
    taz[tid - 128] = ta;
    tbz[tid - 128] = tb;
  }
  __syncthreads();

  // memory variables on the halo rings (written back for the piece's own cells)
  if constexpr (HX) {
#pragma unroll
    for (int k = 0; k < KPX; ++k) {
      const int e = tid + k * kThreads;
      if (e >= NPX) break;
      const int r = e / XW, c = e - (e / XW) * XW;
      const int gz = z0 + r, gxx = x0 - 4 + c;
      const int col = (gz < NZ && gxx >= 0 && gxx < NX) ? xstrip_col(gxx, NX, P) : -1;
      float ps = 0.0f;
      if (col >= 0) {
        ps = fmaf(tax[c + hx - 4], d1s(&sb[(r + hz) * BW + c + hx - 4], 1), tbx[c + hx - 4] * opx[k]);
        if (c >= 4 && c < 4 + kTX) u32at(a.psx_out + shot * xsp, (unsigned)(gz * P2 + col)) = ps;
      }
      spx[e] = ps;
    }
  }
  if constexpr (HZ) {
#pragma unroll
    for (int k = 0; k < KPZ; ++k) {
      const int e = tid + k * kThreads;
      if (e >= NPZ) break;
      const int r = e >> 6, c = e & 63;
      const int gz = z0 - 4 + r, gxx = x0 + c;
      const int row = (gxx < NX && gz >= 0 && gz < NZ) ? zstrip_row(gz, NZ, P) : -1;
      float ps = 0.0f;
      if (row >= 0) {
        ps = fmaf(taz[r + hz - 4], d1s(&sb[(r + hz - 4) * BW + c + hx], BW), tbz[r + hz - 4] * opz[k]);
        if (r >= 4 && r < 4 + TZ) u32at(a.psz_out + shot * zsp, (unsigned)(row * NX + gxx)) = ps;
      }
      spz[e] = ps;
    }
  }
  __syncthreads();

  float win[RZ + 8];
#pragma unroll
  for (int m = 0; m < RZ + 8; ++m) win[m] = sb[(zb + hz - 4 + m) * BW + lx + hx];
  float out[RZ];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const float* row = &sb[(zb + r + hz) * BW + lx + hx];
    const float c = win[r + 4];
    const float sx = d2c(c, row[1], row[-1], row[2], row[-2], row[3], row[-3], row[4], row[-4]);
    const float sz = d2c(c, win[r + 5], win[r + 3], win[r + 6], win[r + 2], win[r + 7],
                         win[r + 1], win[r + 8], win[r]);
    float Bx = sx, Bz = sz;
    if constexpr (HX) Bx = sx + d1s(&spx[(zb + r) * XW + lx + 4], 1);
    if constexpr (HZ) Bz = sz + d1s(&spz[(zb + r + 4) * kTX + lx], kTX);
    const int gz = z0 + zb + r;
    float pn = 0.0f;
    if (gx < NX && gz < NZ) {
      const int idx = gz * NX + gx;
      if (HX && xcol >= 0) {
        const float zeta = fmaf(tax[lx + hx], Bx, tbx[lx + hx] * zx[r]);
        u32at(a.zex_out + shot * xsp, (unsigned)(gz * P2 + xcol)) = zeta;
        Bx = Bx + zeta;
      }
      const int zrow = HZ ? zstrip_row(gz, NZ, P) : -1;
      if (zrow >= 0) {
        const float zeta = fmaf(taz[zb + r + hz], Bz, tbz[zb + r + hz] * zz[r]);
        u32at(a.zez_out + shot * zsp, (unsigned)(zrow * NX + gx)) = zeta;
        Bz = Bz + zeta;
      }
      const float B = Bx + Bz;
      pn = fmaf(cs[r], B, 2.0f * c - pp[r]);
      if (kBorn) pn += bd[r] * bb[r];
      if (idx == src) pn += sw;
      st_nt(&u32at(a.next + shot * plane, (unsigned)idx), pn);
      if (a.B_out) st_nt(&u32at(a.B_out + shot * plane, (unsigned)idx), B);
    }
    out[r] = pn;
  }
  record_receivers<RZ>(a, shot, tile, row0, out, sb);
}

// Adjoint. With q = Cs lambda^{n+1}: in the x strip zbar_x = Z_x + q and
// Qbar_x = q + a_x zbar_x (elsewhere Qbar_x = q), on the tile rows and an
// 8-column halo; psbar_x = Psi_x - D1x' Qbar_x and T_x = a_x psbar_x on a
// 4-column halo (zero outside the strip); z likewise. Then per cell
//   lambda^n = 2 lambda^{n+1} - lambda^{n+2} + D2x' Qbar_x + D2z' Qbar_z - D1x' T_x - D1z' T_z,
// the memory variables become Z = b zbar, Psi = b psbar, and g += lambda^{n+1} B'^n.
template <int RZ, bool HX, bool HZ>
__device__ __forceinline__ void ac_adj_pml_body(const AcStep& a, const int tile, const int shot,
                                                const int row0, float* lds) {
  using G = PmlGeom<RZ, HX, HZ>;
  constexpr int TZ = G::TZ, BW = G::BW, XW = G::XW, hx = G::hx, hz = G::hz;
  constexpr int NQX = G::NQX, KQX = (NQX + kThreads - 1) / kThreads;
  constexpr int NQZ = G::NQZ, KQZ = (NQZ + kThreads - 1) / kThreads;
  constexpr int NTX = G::NPX, KTX = (NTX + kThreads - 1) / kThreads;
  constexpr int NTZ = G::NPZ, KTZ = (NTZ + kThreads - 1) / kThreads;
  float* sqx = lds;                     // Qbar_x: tile rows, columns x0-hx ..
  float* sqz = lds + NQX;               // Qbar_z: rows z0-hz .., tile columns
  float* stx = lds + NQX + NQZ;         // T_x: tile rows, columns x0-4 ..
  float* stz = lds + NQX + NQZ + NTX;   // T_z: rows z0-4 .., tile columns
  float* tax = stz + NTZ;               // a_x, b_x at the box columns (x0-hx ..),
  float* tbx = tax + BW;                // a_z, b_z at the box rows (z0-hz ..)
  float* taz = tbx + BW;
  float* tbz = taz + G::BH;
  const int tid = threadIdx.x;
  const int lx = tid & 63;
  const int zb = (tid >> 6) * RZ;
  const int NX = a.NX, NZ = a.NZ, P = a.P, P2 = 2 * P;
  const size_t plane = (size_t)NX * NZ;
  const size_t xsp = (size_t)NZ * P2, zsp = (size_t)P2 * NX;
  const int x0 = (tile % a.tiles_x) * kTX, z0 = (tile / a.tiles_x) * a.tz + row0;
  const int gx = x0 + lx;
  const float* cur = a.cur + shot * plane;

  // C-PML coefficients of the box columns (threads 0..BW-1) and rows (128..),
  // written to LDS tables before Qbar is formed (registers are not held for
  // a and b of every ring item)
  float ta = 0.0f, tb = 0.0f;
  if (tid < BW) {
    const int gxx = x0 - hx + tid;
    if (HX && gxx >= 0 && gxx < NX) {
      ta = a.ax[gxx];
      tb = a.bx[gxx];
    }
  } else if (tid >= 128 && tid < 128 + G::BH) {
    const int gz = z0 - hz + (tid - 128);
    if (HZ && gz >= 0 && gz < NZ) {
      ta = a.az[gz];
      tb = a.bz[gz];
    }
  }
  {
    float lx_[KQX], cx_[KQX], zx_[HX ? KQX : 1];
#pragma unroll
    for (int k = 0; k < KQX; ++k) {
      const int e = tid + k * kThreads;
      const int r = e / BW, c = e - (e / BW) * BW;
      const int gz = z0 + r, gxx = x0 - hx + c;
      const bool ok = e < NQX && gz < NZ && gxx >= 0 && gxx < NX;
      const unsigned idx = ok ? (unsigned)(gz * NX + gxx) : 0u;
      lx_[k] = ok ? u32at(cur, idx) : 0.0f;
      cx_[k] = ok ? u32at(a.Cs, idx) : 0.0f;
      if constexpr (HX) {
        const int col = ok ? xstrip_col(gxx, NX, P) : -1;
        zx_[k] = col >= 0 ? u32at(a.zex_in + shot * xsp, (unsigned)(gz * P2 + col)) : 0.0f;
      }
    }
    float lz_[KQZ], cz_[KQZ], zz_[HZ ? KQZ : 1];
#pragma unroll
    for (int k = 0; k < KQZ; ++k) {
      const int e = tid + k * kThreads;
      const int r = e >> 6, c = e & 63;
      const int gz = z0 - hz + r, gxx = x0 + c;
      const bool ok = e < NQZ && gxx < NX && gz >= 0 && gz < NZ;
      const unsigned idx = ok ? (unsigned)(gz * NX + gxx) : 0u;
      lz_[k] = ok ? u32at(cur, idx) : 0.0f;
      cz_[k] = ok ? u32at(a.Cs, idx) : 0.0f;
      if constexpr (HZ) {
        const int row = ok ? zstrip_row(gz, NZ, P) : -1;
        zz_[k] = row >= 0 ? u32at(a.zez_in + shot * zsp, (unsigned)(row * NX + gxx)) : 0.0f;
      }
    }
    if (tid < BW) {
      tax[tid] = ta;
      tbx[tid] = tb;
    } else if (tid >= 128 && tid < 128 + G::BH) {
      taz[tid - 128] = ta;
      tbz[tid - 128] = tb;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KQX; ++k) {
      const int e = tid + k * kThreads;
      if (e >= NQX) break;
      float q = cx_[k] * lx_[k];
      if constexpr (HX) {
        const int r = e / BW, c = e - (e / BW) * BW;
        const int gz = z0 + r, gxx = x0 - hx + c;
        const int col = (gz < NZ && gxx >= 0 && gxx < NX) ? xstrip_col(gxx, NX, P) : -1;
        if (col >= 0) {
          const float zbar = zx_[k] + q;
          q = q + tax[c] * zbar;
          if (c >= hx && c < hx + kTX)
            u32at(a.zex_out + shot * xsp, (unsigned)(gz * P2 + col)) = tbx[c] * zbar;
        }
      }
      sqx[e] = q;
    }
#pragma unroll
    for (int k = 0; k < KQZ; ++k) {
      const int e = tid + k * kThreads;
      if (e >= NQZ) break;
      float q = cz_[k] * lz_[k];
      if constexpr (HZ) {
        const int r = e >> 6, c = e & 63;
        const int gz = z0 - hz + r, gxx = x0 + c;
        const int row = (gxx < NX && gz >= 0 && gz < NZ) ? zstrip_row(gz, NZ, P) : -1;
        if (row >= 0) {
          const float zbar = zz_[k] + q;
          q = q + taz[r] * zbar;
          if (r >= hz && r < hz + TZ)
            u32at(a.zez_out + shot * zsp, (unsigned)(row * NX + gxx)) = tbz[r] * zbar;
        }
      }
      sqz[e] = q;
    }
  }
  // Psi^{in} of the halo rings and the per-cell operands
  float ox[HX ? KTX : 1], oz[HZ ? KTZ : 1];
  if constexpr (HX) {
#pragma unroll
    for (int k = 0; k < KTX; ++k) {
      const int e = tid + k * kThreads;
      const int r = e / XW, c = e - (e / XW) * XW;
      const int gz = z0 + r, gxx = x0 - 4 + c;
      const int col = (e < NTX && gz < NZ && gxx >= 0 && gxx < NX) ? xstrip_col(gxx, NX, P) : -1;
      ox[k] = col >= 0 ? u32at(a.psx_in + shot * xsp, (unsigned)(gz * P2 + col)) : 0.0f;
    }
  }
  if constexpr (HZ) {
#pragma unroll
    for (int k = 0; k < KTZ; ++k) {
      const int e = tid + k * kThreads;
      const int r = e >> 6, c = e & 63;
      const int gz = z0 - 4 + r, gxx = x0 + c;
      const int row = (e < NTZ && gxx < NX && gz >= 0 && gz < NZ) ? zstrip_row(gz, NZ, P) : -1;
      oz[k] = row >= 0 ? u32at(a.psz_in + shot * zsp, (unsigned)(row * NX + gxx)) : 0.0f;
    }
  }
  // per-cell operands: branch-free where the body has no x-strip cells (measured
  // faster there); as a guarded block in the x-strip bodies (fewer registers)
  float p1[RZ], pp[RZ], bb[RZ], gg[RZ];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const int gz = z0 + zb + r;
    const bool ok = gx < NX && gz < NZ;
    if constexpr (!HX) {
      const unsigned gi = ok ? (unsigned)(gz * NX + gx) : 0u;
      p1[r] = ldz32(cur, gi, ok);
      pp[r] = ldz32_nt(a.prev + shot * plane, gi, ok);
      bb[r] = ldz32_nt(a.B_in + shot * plane, gi, ok);
      gg[r] = ldz32_nt(a.g + shot * plane, gi, ok && !a.g_init);
    } else {
      p1[r] = pp[r] = bb[r] = gg[r] = 0.0f;
      if (ok) {
        const unsigned gi = (unsigned)(gz * NX + gx);
        p1[r] = u32at(cur, gi);
        pp[r] = ld_nt(&u32at(a.prev + shot * plane, gi));
        bb[r] = ld_nt(&u32at(a.B_in + shot * plane, gi));
        if (!a.g_init) gg[r] = ld_nt(&u32at(a.g + shot * plane, gi));
      }
    }
  }
  __syncthreads();

  if constexpr (HX) {
#pragma unroll
    for (int k = 0; k < KTX; ++k) {
      const int e = tid + k * kThreads;
      if (e >= NTX) break;
      const int r = e / XW, c = e - (e / XW) * XW;
      const int gz = z0 + r, gxx = x0 - 4 + c;
      const int col = (gz < NZ && gxx >= 0 && gxx < NX) ? xstrip_col(gxx, NX, P) : -1;
      float t = 0.0f;
      if (col >= 0) {
        const float psb = ox[k] - d1s(&sqx[r * BW + c + hx - 4], 1);
        t = tax[c + hx - 4] * psb;
        if (c >= 4 && c < 4 + kTX)
          u32at(a.psx_out + shot * xsp, (unsigned)(gz * P2 + col)) = tbx[c + hx - 4] * psb;
      }
      stx[e] = t;
    }
  }
  if constexpr (HZ) {
#pragma unroll
    for (int k = 0; k < KTZ; ++k) {
      const int e = tid + k * kThreads;
      if (e >= NTZ) break;
      const int r = e >> 6, c = e & 63;
      const int gz = z0 - 4 + r, gxx = x0 + c;
      const int row = (gxx < NX && gz >= 0 && gz < NZ) ? zstrip_row(gz, NZ, P) : -1;
      float t = 0.0f;
      if (row >= 0) {
        const float psb = oz[k] - d1s(&sqz[(r + hz - 4) * kTX + c], kTX);
        t = taz[r + hz - 4] * psb;
        if (r >= 4 && r < 4 + TZ)
          u32at(a.psz_out + shot * zsp, (unsigned)(row * NX + gxx)) = tbz[r + hz - 4] * psb;
      }
      stz[e] = t;
    }
  }
  if constexpr (HX || HZ) __syncthreads();

  float out[RZ];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const float dxx = d2s(&sqx[(zb + r) * BW + lx + hx], 1);
    const float dzz = d2s(&sqz[(zb + r + hz) * kTX + lx], kTX);
    float tx = 0.0f, tz = 0.0f;
    if constexpr (HX) tx = d1s(&stx[(zb + r) * XW + lx + 4], 1);
    if constexpr (HZ) tz = d1s(&stz[(zb + r + 4) * kTX + lx], kTX);
    const int gz = z0 + zb + r;
    float lam = 0.0f;
    if (gx < NX && gz < NZ) {
      const unsigned gi = (unsigned)(gz * NX + gx);
      const float gb = p1[r] * bb[r];
      st_nt(&u32at(a.g + shot * plane, gi), a.g_init ? gb : gg[r] + gb);
      lam = ((2.0f * p1[r] - pp[r]) + dxx) + dzz;
      if constexpr (HX) lam = lam - tx;
      if constexpr (HZ) lam = lam - tz;
    }
    out[r] = lam;
  }
  adj_store<RZ>(a, shot, tile, row0, x0, z0, out, sqz);
}

// ---------------------------------------------------------------------------
// Deep runs: two time steps per pass. A deep tile has no C-PML cell within 4
// cells and no source or receiver within 4 cells (for any shot), so the first
// step can be recomputed on a 4-cell ring around it from the field with an
// 8-cell halo. A run is a chunk of consecutive deep tiles of one tile column;
// one work-group marches down it H rows at a time (H = kMH). Per iteration it
//   1. computes step 1 (p^{n+1} / lambda^n) on H new rows, 72 columns wide
//      (the strip and its 4-column ring), from p^n rows held in LDS;
//   2. computes step 2 (p^{n+2} / lambda^{n-1}) on the H rows starting 4 above;
//   3. stores the next H rows of p^n (80 columns), loaded into registers one
//      iteration earlier.
// LDS holds both levels in circular buffers of 3H slots. Rows move by H per
// iteration, so the slots repeat every 3 iterations; the first slots are also
// written 3H rows further on, which keeps every stencil window contiguous.
// Only the ring rows at the start of a run and the 4-column side rings are
// computed twice, and only the 8-cell halo rows and columns are read twice
// (from L2). The per-cell arithmetic is that of the interior kernel, so both
// steps give the same bits as two single steps. HBM traffic per cell and two
// steps: 20 bytes forward (28 saving B), 36 adjoint.
// ---------------------------------------------------------------------------
constexpr int kMH = 16;                               // rows per iteration
constexpr int kMS = 3 * kMH;                          // slots of a circular buffer
constexpr int kMA = kTX + 16;                         // level-n columns: x0-8 .. x0+71
constexpr int kMB = kTX + 8;                          // step-1 columns: x0-4 .. x0+67
constexpr int kNA = kMH * kMA;                        // cells of H level-n rows
constexpr int kKA = (kNA + kThreads - 1) / kThreads;  // per thread
constexpr int kR2 = kMH / 4;                          // step-2 rows per thread
constexpr int kPB = (kMH + 16) / kMH;                 // level-n blocks of the prologue
static_assert(kThreads == 4 * kTX && (kMH == 8 || kMH == 16), "march geometry");

// Slot arithmetic, with rows relative to the run's first row za:
//   level-n row za-8+j is in slot j mod 3H, step-1 row za-4+j in slot j mod 3H.
// Iteration i (rows r = za + H i):
//   step 1 writes rows [r+4, r+H+4) from slot (8 + H i) mod 3H (wrapping), and
//     reads level n rows [r, r+H+8), a window from the same slot;
//   step 2 reads step-1 rows [r-4, r+H+4), a window from slot H i mod 3H, and
//     level n rows [r, r+H);
//   level n rows [r+H+8, r+2H+8) are stored as one block from slot
//     (16 + H (i+1)) mod 3H, a multiple of H.
// Level-n slots [0, H) are duplicated at 3H, step-1 slots [0, 8) at 3H; every
// window then stays below 3H + H (level n) or 3H + 8 (step 1).
__device__ __forceinline__ int m_win1(int i) { return (8 + kMH * i) % kMS; }
__device__ __forceinline__ int m_win2(int i) { return (kMH * i) % kMS; }
__device__ __forceinline__ int m_put(int i) { return (16 + kMH * (i + 1)) % kMS; }

// Loads H rows [z, z+H) x [x0-8, x0+72) of a level-n field. A run's 8-cell
// halo lies inside the grid, so the loads need no guard; rows past zlim (which
// only feed results that are not kept) are clamped to zlim - 1. The loads are
// unconditional on purpose: a load under a per-lane condition must complete
// before the other branch writes its register, which serialises them.
__device__ __forceinline__ void march_load_a(const float* f, int z, int zlim, int x0, int NX,
                                             float (&v)[kKA]) {
#pragma unroll
  for (int k = 0; k < kKA; ++k) {
    const int e = threadIdx.x + k * kThreads;
    const int r = e / kMA, c = e - (e / kMA) * kMA;
    const int gz = min(z + r, zlim - 1), gx = x0 - 8 + c;
    v[k] = f[(unsigned)(gz * NX + gx)];
  }
}

// Writes them to slot s (a multiple of H; slot 0 also at 3H); with w, the
// products w v (w loaded by march_load_a from the same rows).
__device__ __forceinline__ void march_put_a(float* sa, int s, const float (&v)[kKA]) {
#pragma unroll
  for (int k = 0; k < kKA; ++k) {
    const int e = threadIdx.x + k * kThreads;
    if (e < kNA) {
      sa[s * kMA + e] = v[k];
      if (s == 0) sa[kMS * kMA + e] = v[k];
    }
  }
}
__device__ __forceinline__ void march_put_a(float* sa, int s, const float (&w)[kKA],
                                            const float (&v)[kKA]) {
#pragma unroll
  for (int k = 0; k < kKA; ++k) {
    const int e = threadIdx.x + k * kThreads;
    if (e < kNA) {
      const float q = w[k] * v[k];
      sa[s * kMA + e] = q;
      if (s == 0) sa[kMS * kMA + e] = q;
    }
  }
}

// Step-1 cells of an H x 72 block. The 64 strip columns go to the threads as
// in step 2 (column lx, rows wz .. wz+H/4-1), so a wave reads consecutive LDS
// words and takes the vertical stencil from a register window. The 8 ring
// columns (4 each side) are spread over the first 2H lanes of every wave.
constexpr int kRL = 2 * kMH;  // ring lanes per wave
struct MarchCells {
  int rr, rc;   // this lane's ring cell: row, step-1 column (0..3, 68..71)
  bool ring;    // lane takes a ring cell
  __device__ __forceinline__ MarchCells() {
    const int lane = threadIdx.x & 63;
    const int q = (lane & (kRL - 1)) + kRL * (threadIdx.x >> 6);
    ring = lane < kRL;
    rr = q >> 3;
    const int c = q & 7;
    rc = c < 4 ? c : c + kTX;
  }
};

// Geometry of one march (a run of one shot).
// Plane offsets fit in 32 bits; the per-shot planes are addressed from
// work-group-uniform base pointers. The march indexes them with a 32-bit
// element index widened per lane: the scalar-base byte-offset form (u32at)
// cut the adjoint pass's vector instructions by 16 % but made it 0.9 % slower. wz is uniform within a wave (a wave is 64
// consecutive threads), which readfirstlane tells the compiler, so branches on
// it are scalar.
struct March {
  int NX, NZ, x0, za, zb, nit, alim, blim, lx, wz;
  size_t base;
  __device__ __forceinline__ March(const AcStep& a, const int2 run, const int shot) {
    NX = a.NX;
    NZ = a.NZ;
    base = (size_t)shot * NX * NZ;
    x0 = run.x * kTX;
    za = (run.y & 0xffff) * a.tz;
    zb = za + (run.y >> 16) * a.tz;
    nit = (zb - za + kMH - 1) / kMH;
    alim = zb + 8;
    blim = zb + 4;
    lx = threadIdx.x & 63;
    wz = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6) * kR2);
  }
};

// Per-thread step-1 inputs of one field for rows [z, z+H): the strip cells
// (column lx, rows wz..) and the ring cell (rows past zlim clamped, as above).
struct StepIn {
  float v[kR2], ring;
};
__device__ __forceinline__ void march_load_b(const March& m, const MarchCells& mc, const float* f,
                                             int z, bool nt, StepIn& in) {
#pragma unroll
  for (int j = 0; j < kR2; ++j) {
    const int gz = min(z + m.wz + j, m.blim - 1);
    const float* p = &f[(unsigned)(gz * m.NX + m.x0 + m.lx)];
    in.v[j] = nt ? ld_nt(p) : *p;
  }
  const int gz = min(z + mc.rr, m.blim - 1);
  const float* p = &f[(unsigned)(gz * m.NX + m.x0 - 4 + mc.rc)];
  in.ring = nt ? ld_nt(p) : *p;
}

// Slot of step-1 row offset r from window slot w (wrapping at 3H).
__device__ __forceinline__ int m_wrap(int w, int r) {
  const int s = w + r;
  return s >= kMS ? s - kMS : s;
}

// Laplacian parts of the interior update at the cell of LDS row `row` (a
// pointer to the cell), with the vertical neighbours from the register window
// w (centre w[j + 4]); the same operations in the same order as d2s.
template <int NW>
__device__ __forceinline__ float lap_x(const float* row, const float (&w)[NW], int j) {
  return d2c(w[j + 4], row[1], row[-1], row[2], row[-2], row[3], row[-3], row[4], row[-4]);
}
template <int NW>
__device__ __forceinline__ float lap_z(const float (&w)[NW], int j) {
  return d2c(w[j + 4], w[j + 5], w[j + 3], w[j + 6], w[j + 2], w[j + 7], w[j + 1], w[j + 8], w[j]);
}

// p^{n+1} on step-1 rows [z, z+nrows) (level-n window from slot wa, whose first
// row is z - 4; results from slot wb), stored at the run's own cells.
__device__ __forceinline__ void march_fwd_step1(const AcStep& a, const March& m,
                                                const MarchCells& mc, const float* sa, float* sb,
                                                int wa, int wb, int z, int nrows,
                                                const StepIn& pm, const StepIn& cs) {
  // strip cells
  float w[kR2 + 8];
#pragma unroll
  for (int t = 0; t < kR2 + 8; ++t) w[t] = sa[(wa + m.wz + t) * kMA + m.lx + 8];
#pragma unroll
  for (int j = 0; j < kR2; ++j) {
    const int rj = m.wz + j;
    if (rj >= nrows) continue;
    const float* row = &sa[(wa + 4 + rj) * kMA + m.lx + 8];
    const float L = lap_x(row, w, j) + lap_z(w, j);
    const float pn = fmaf(cs.v[j], L, 2.0f * w[j + 4] - pm.v[j]);
    const int s = m_wrap(wb, rj);
    sb[s * kMB + m.lx + 4] = pn;
    if (s < 8) sb[(s + kMS) * kMB + m.lx + 4] = pn;
    const int gz = z + rj;
    if (gz >= m.za && gz < m.zb) {
      const unsigned gi = gz * m.NX + m.x0 + m.lx;
      st_nt(&(a.next + m.base)[gi], pn);
      if (a.B_out) st_nt(&(a.B_out + m.base)[gi], L);
    }
  }
  // ring cells (not stored: they belong to neighbouring strips)
  if (mc.ring && mc.rr < nrows) {
    const float* f = &sa[(wa + 4 + mc.rr) * kMA + mc.rc + 4];
    const float L = d2s(f, 1) + d2s(f, kMA);
    const float pn = fmaf(cs.ring, L, 2.0f * f[0] - pm.ring);
    const int s = m_wrap(wb, mc.rr);
    sb[s * kMB + mc.rc] = pn;
    if (s < 8) sb[(s + kMS) * kMB + mc.rc] = pn;
  }
}

// Iteration i of the forward march. pm/cs: step-1 inputs of this iteration,
// refilled with those of iteration i+2; put: level-n rows stored at the end of
// this iteration; load: filled with those of iteration i+1.
__device__ __forceinline__ void march_fwd_iter(const AcStep& a, const March& m,
                                               const MarchCells& mc, float* sa, float* sb, int i,
                                               StepIn& pm, StepIn& cs, const float (&put)[kKA],
                                               float (&load)[kKA]) {
  const float* cur = a.cur + m.base;
  const float* prev = a.prev + m.base;
  const int r = m.za + kMH * i;
  const int w1 = m_win1(i), w2 = m_win2(i);
  float c2[kR2];
#pragma unroll
  for (int j = 0; j < kR2; ++j) {
    const int gz = min(r + m.wz + j, m.zb - 1);
    c2[j] = a.Cs[(unsigned)(gz * m.NX + m.x0 + m.lx)];
  }
  march_fwd_step1(a, m, mc, sa, sb, w1, w1, r + 4, kMH, pm, cs);
  march_load_b(m, mc, prev, r + 2 * kMH + 4, true, pm);
  march_load_b(m, mc, a.Cs, r + 2 * kMH + 4, false, cs);
  march_load_a(cur, r + 2 * kMH + 8, m.alim, m.x0, m.NX, load);
  __syncthreads();
  // step 2 on rows [r, r+H)
  float w[kR2 + 8];
#pragma unroll
  for (int t = 0; t < kR2 + 8; ++t) w[t] = sb[(w2 + m.wz + t) * kMB + m.lx + 4];
#pragma unroll
  for (int j = 0; j < kR2; ++j) {
    const int gz = r + m.wz + j;
    if (gz >= m.zb) continue;
    const float* row = &sb[(w2 + 4 + m.wz + j) * kMB + m.lx + 4];
    const float L = lap_x(row, w, j) + lap_z(w, j);
    const float pn = fmaf(c2[j], L, 2.0f * w[j + 4] - sa[(w1 + m.wz + j) * kMA + m.lx + 8]);
    const unsigned gi = gz * m.NX + m.x0 + m.lx;
    st_nt(&(a.next2 + m.base)[gi], pn);
    if (a.B_out2) st_nt(&(a.B_out2 + m.base)[gi], L);
  }
  march_put_a(sa, m_put(i), put);
  __syncthreads();
}

// The march keeps two sets of in-flight registers and alternates them between
// iterations (a copy from one set to the other would wait for its loads).
__device__ __forceinline__ void ac_march_fwd(const AcStep& a, const int2 run, const int shot) {
  __shared__ float sa[(kMS + kMH) * kMA];  // p^n
  __shared__ float sb[(kMS + 8) * kMB];    // p^{n+1}
  const March m(a, run, shot);
  const MarchCells mc;
  const float* cur = a.cur + m.base;
  const float* prev = a.prev + m.base;

  // prologue: level n rows [za-8, za+H+8), step 1 on rows [za-4, za+4)
  float va[kPB][kKA], n0[kKA], n1[kKA];
  StepIn pm0, cs0, pm1, cs1;
#pragma unroll
  for (int b = 0; b < kPB; ++b) march_load_a(cur, m.za - 8 + kMH * b, m.alim, m.x0, m.NX, va[b]);
  march_load_b(m, mc, prev, m.za - 4, true, pm1);
  march_load_b(m, mc, a.Cs, m.za - 4, false, cs1);
  march_load_b(m, mc, prev, m.za + 4, true, pm0);
  march_load_b(m, mc, a.Cs, m.za + 4, false, cs0);
  march_load_a(cur, m.za + kMH + 8, m.alim, m.x0, m.NX, n0);
#pragma unroll
  for (int b = 0; b < kPB; ++b) march_put_a(sa, kMH * b, va[b]);
  __syncthreads();
  march_fwd_step1(a, m, mc, sa, sb, 0, 0, m.za - 4, 8, pm1, cs1);
  march_load_b(m, mc, prev, m.za + kMH + 4, true, pm1);
  march_load_b(m, mc, a.Cs, m.za + kMH + 4, false, cs1);

  for (int i = 0; i < m.nit; i += 2) {
    march_fwd_iter(a, m, mc, sa, sb, i, pm0, cs0, n0, n1);
    if (i + 1 < m.nit) march_fwd_iter(a, m, mc, sa, sb, i + 1, pm1, cs1, n1, n0);
  }
}

// Step-1 inputs of the adjoint: lambda^{n+1}, lambda^{n+2} and Cs.
struct AdjIn {
  StepIn l1, l2, cr;
};
__device__ __forceinline__ void march_adj_load_b(const AcStep& a, const March& m,
                                                 const MarchCells& mc, int z, AdjIn& v) {
  march_load_b(m, mc, a.cur + m.base, z, false, v.l1);
  march_load_b(m, mc, a.prev + m.base, z, true, v.l2);
  march_load_b(m, mc, a.Cs, z, false, v.cr);
}
// Level-n rows of the adjoint: lambda^{n+1} and Cs (multiplied when stored).
struct AdjRows {
  float l[kKA], c[kKA];
};
__device__ __forceinline__ void march_adj_load_a(const AcStep& a, const March& m, int z,
                                                 AdjRows& v) {
  march_load_a(a.cur + m.base, z, m.alim, m.x0, m.NX, v.l);
  march_load_a(a.Cs, z, m.alim, m.x0, m.NX, v.c);
}

// lambda^n on step-1 rows [z, z+nrows) from q = Cs lambda^{n+1} (window from
// slot wa, first row z - 4): Cs lambda^n and lambda^n from slot wb, stored at
// the run's own cells.
__device__ __forceinline__ void march_adj_step1(const AcStep& a, const March& m,
                                                const MarchCells& mc, const float* sq, float* sb,
                                                float* sl, int wa, int wb, int z, int nrows,
                                                const AdjIn& in) {
  float w[kR2 + 8];
#pragma unroll
  for (int t = 0; t < kR2 + 8; ++t) w[t] = sq[(wa + m.wz + t) * kMA + m.lx + 8];
#pragma unroll
  for (int j = 0; j < kR2; ++j) {
    const int rj = m.wz + j;
    if (rj >= nrows) continue;
    const float* row = &sq[(wa + 4 + rj) * kMA + m.lx + 8];
    const float lam = ((2.0f * in.l1.v[j] - in.l2.v[j]) + lap_x(row, w, j)) + lap_z(w, j);
    const int s = m_wrap(wb, rj);
    const float cl = in.cr.v[j] * lam;
    sb[s * kMB + m.lx + 4] = cl;
    sl[s * kTX + m.lx] = lam;
    if (s < 8) {
      sb[(s + kMS) * kMB + m.lx + 4] = cl;
      sl[(s + kMS) * kTX + m.lx] = lam;
    }
    const int gz = z + rj;
    if (gz >= m.za && gz < m.zb) st_nt(&(a.next + m.base)[(unsigned)(gz * m.NX + m.x0 + m.lx)], lam);
  }
  if (mc.ring && mc.rr < nrows) {
    const float* f = &sq[(wa + 4 + mc.rr) * kMA + mc.rc + 4];
    const float lam = ((2.0f * in.l1.ring - in.l2.ring) + d2s(f, 1)) + d2s(f, kMA);
    const int s = m_wrap(wb, mc.rr);
    const float cl = in.cr.ring * lam;
    sb[s * kMB + mc.rc] = cl;
    if (s < 8) sb[(s + kMS) * kMB + mc.rc] = cl;
  }
}

__device__ __forceinline__ void march_adj_iter(const AcStep& a, const March& m,
                                               const MarchCells& mc, float* sq, float* sb,
                                               float* sl, int i, AdjIn& in, const AdjRows& put,
                                               AdjRows& load) {
  const int r = m.za + kMH * i;
  const int w1 = m_win1(i), w2 = m_win2(i);
  float p1[kR2], b1[kR2], b2[kR2], gg[kR2];
  const bool gacc = !a.g_init;
#pragma unroll
  for (int j = 0; j < kR2; ++j) {
    const int gz = min(r + m.wz + j, m.zb - 1);
    const unsigned gi = gz * m.NX + m.x0 + m.lx;
    p1[j] = (a.cur + m.base)[gi];
    b1[j] = ld_nt(&(a.B_in + m.base)[gi]);
    b2[j] = ld_nt(&(a.B_in2 + m.base)[gi]);
    gg[j] = gacc ? ld_nt(&(a.g + m.base)[gi]) : 0.0f;
  }
  march_adj_step1(a, m, mc, sq, sb, sl, w1, w1, r + 4, kMH, in);
  march_adj_load_b(a, m, mc, r + 2 * kMH + 4, in);
  march_adj_load_a(a, m, r + 2 * kMH + 8, load);
  __syncthreads();
  // step 2 on rows [r, r+H) and the gradient of both steps
  float w[kR2 + 8];
#pragma unroll
  for (int t = 0; t < kR2 + 8; ++t) w[t] = sb[(w2 + m.wz + t) * kMB + m.lx + 4];
#pragma unroll
  for (int j = 0; j < kR2; ++j) {
    const int gz = r + m.wz + j;
    if (gz >= m.zb) continue;
    const int s = w2 + 4 + m.wz + j;
    const float* row = &sb[s * kMB + m.lx + 4];
    const float lam_n = sl[s * kTX + m.lx];
    const float lam = ((2.0f * lam_n - p1[j]) + lap_x(row, w, j)) + lap_z(w, j);
    const unsigned gi = gz * m.NX + m.x0 + m.lx;
    const float gb = p1[j] * b1[j];
    const float g1 = a.g_init ? gb : gg[j] + gb;
    st_nt(&(a.g + m.base)[gi], g1 + lam_n * b2[j]);
    st_nt(&(a.next2 + m.base)[gi], lam);
  }
  march_put_a(sq, m_put(i), put.c, put.l);
  __syncthreads();
}

// Reverse steps n and n-1; g += lambda^{n+1} B'^n + lambda^n B'^{n-1}.
__device__ __forceinline__ void ac_march_adj(const AcStep& a, const int2 run, const int shot) {
  __shared__ float sq[(kMS + kMH) * kMA];  // q = Cs lambda^{n+1}
  __shared__ float sb[(kMS + 8) * kMB];    // Cs lambda^n
  __shared__ float sl[(kMS + 8) * kTX];    // lambda^n on the strip's own columns
  const March m(a, run, shot);
  const MarchCells mc;

  AdjRows va[kPB], n0, n1;
  AdjIn in0, in1;
#pragma unroll
  for (int b = 0; b < kPB; ++b) march_adj_load_a(a, m, m.za - 8 + kMH * b, va[b]);
  march_adj_load_b(a, m, mc, m.za - 4, in1);
  march_adj_load_b(a, m, mc, m.za + 4, in0);
  march_adj_load_a(a, m, m.za + kMH + 8, n0);
#pragma unroll
  for (int b = 0; b < kPB; ++b) march_put_a(sq, kMH * b, va[b].c, va[b].l);
  __syncthreads();
  march_adj_step1(a, m, mc, sq, sb, sl, 0, 0, m.za - 4, 8, in1);
  march_adj_load_b(a, m, mc, m.za + kMH + 4, in1);

  for (int i = 0; i < m.nit; i += 2) {
    march_adj_iter(a, m, mc, sq, sb, sl, i, in0, n0, n1);
    if (i + 1 < m.nit) march_adj_iter(a, m, mc, sq, sb, sl, i + 1, in1, n1, n0);
  }
}

template <bool kAdj>
__global__ __launch_bounds__(kThreads) void ac_march_kernel(AcStep a) {
  const int l = xcd_spread(blockIdx.x, gridDim.x);
  const int2 run = a.drun[l % a.n_run];
  const int shot = l / a.n_run;
  if (kAdj)
    ac_march_adj(a, run, shot);
  else
    ac_march_fwd(a, run, shot);
}

// ---------------------------------------------------------------------------
// Kernel entry points: one plan (1-D grid over kind tiles x shots) or a batch
// of plans of different shapes in one launch (the flat block index is split by
// the per-plan block counts of this launch).
// ---------------------------------------------------------------------------
template <int RZ, bool kAdj, bool kBorn = false>
__device__ __forceinline__ void run_interior(const AcStep& a, int l) {
  const int tile = a.ilist[l % a.n_int];
  const int shot = l / a.n_int;
  if (kAdj)
    ac_adj_int_body<RZ>(a, tile, shot);
  else
    ac_fwd_int_body<RZ, kBorn>(a, tile, shot);
}

// Frame pieces: kZ selects the z frame (its pieces meet z strips only) or the
// x frame (general body, specialised on the strips near the piece).
template <int RZ, bool kAdj, bool kZ, bool kBorn = false>
__device__ __forceinline__ void run_frame(const AcStep& a, int l, float* lds) {
  const int nk = (kZ ? a.n_zf : a.n_xf) * a.nsub;
  const int t = l % nk, shot = l / nk;
  const int tile = kZ ? zframe_tile(a, t / a.nsub) : xframe_tile(a, t / a.nsub);
  const int row0 = (t % a.nsub) * 4 * RZ;
  if (kZ) {
    if (kAdj)
      ac_adj_pml_body<RZ, false, true>(a, tile, shot, row0, lds);
    else
      ac_fwd_pml_body<RZ, false, true, kBorn>(a, tile, shot, row0, lds);
    return;
  }
  const int x0 = (tile % a.tiles_x) * kTX, z0 = (tile / a.tiles_x) * a.tz + row0;
  const bool hx = near_xstrip(x0, a.NX, a.P), hz = near_zstrip(z0, 4 * RZ, a.NZ, a.P);
  if (kAdj) {
    if (hx && hz)
      ac_adj_pml_body<RZ, true, true>(a, tile, shot, row0, lds);
    else if (hx)
      ac_adj_pml_body<RZ, true, false>(a, tile, shot, row0, lds);
    else if (hz)
      ac_adj_pml_body<RZ, false, true>(a, tile, shot, row0, lds);
    else
      ac_adj_pml_body<RZ, false, false>(a, tile, shot, row0, lds);
  } else {
    if (hx && hz)
      ac_fwd_pml_body<RZ, true, true, kBorn>(a, tile, shot, row0, lds);
    else if (hx)
      ac_fwd_pml_body<RZ, true, false, kBorn>(a, tile, shot, row0, lds);
    else if (hz)
      ac_fwd_pml_body<RZ, false, true, kBorn>(a, tile, shot, row0, lds);
    else
      ac_fwd_pml_body<RZ, false, false, kBorn>(a, tile, shot, row0, lds);
  }
}

template <int RZ, bool kAdj>
__global__ __launch_bounds__(kThreads) void ac_int_kernel(AcStep a) {
  run_interior<RZ, kAdj>(a, xcd_spread(blockIdx.x, gridDim.x));
}

// The x-frame kernels at prz = 4 need 97 (forward) and 101 (adjoint) VGPRs,
// 4 waves per SIMD; capped at 96 they hold 5 (the adjoint spills one VGPR,
// which costs less than the extra wave gains).
template <int RZ, bool kAdj, bool kZ>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(!kZ && RZ == 4 ? 5 : 1))) void ac_pml_kernel(AcStep a) {
  __shared__ float lds[PmlLds<RZ>::get(kAdj, kZ)];
  run_frame<RZ, kAdj, kZ>(a, xcd_spread(blockIdx.x, gridDim.x), lds);
}

// Born perturbation steps (single steps; the frame and interior tile sets as
// in the forward).
template <int RZ>
__global__ __launch_bounds__(kThreads) void ac_born_int_kernel(AcStep a) {
  run_interior<RZ, false, true>(a, xcd_spread(blockIdx.x, gridDim.x));
}

template <int RZ, bool kZ>
__global__ __launch_bounds__(kThreads) void ac_born_pml_kernel(AcStep a) {
  __shared__ float lds[PmlLds<RZ>::get(false, kZ)];
  run_frame<RZ, false, kZ, true>(a, xcd_spread(blockIdx.x, gridDim.x), lds);
}

// plan of flat block f in a batched launch, and f's index inside that plan
__device__ __forceinline__ int batch_plan(const AcBatch& b, int& f) {
  int p = 0;
  while (p + 1 < b.nplans && f >= b.base[p + 1]) ++p;
  f -= b.base[p];
  return p;
}

template <int RZ, bool kAdj>
__global__ __launch_bounds__(kThreads) void ac_int_batch_kernel(AcBatch b) {
  int f = xcd_spread(blockIdx.x, gridDim.x);
  const int p = batch_plan(b, f);
  run_interior<RZ, kAdj>(b.step[p], f);
}

template <int RZ, bool kAdj, bool kZ>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(!kZ && RZ == 4 ? 5 : 1))) void ac_pml_batch_kernel(AcBatch b) {
  __shared__ float lds[PmlLds<RZ>::get(kAdj, kZ)];
  int f = xcd_spread(blockIdx.x, gridDim.x);
  const int p = batch_plan(b, f);
  run_frame<RZ, kAdj, kZ>(b.step[p], f, lds);
}

template <bool kAdj>
__global__ __launch_bounds__(kThreads) void ac_march_batch_kernel(AcBatch b) {
  int f = xcd_spread(blockIdx.x, gridDim.x);
  const int p = batch_plan(b, f);
  const AcStep& a = b.step[p];
  const int2 run = a.drun[f % a.n_run];
  const int shot = f / a.n_run;
  if (kAdj)
    ac_march_adj(a, run, shot);
  else
    ac_march_fwd(a, run, shot);
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

// Encoded shots (several sources per simulation): after step n the step
// kernels, which inject no source for such plans, have written p^{n+1}; one
// thread per shot adds its sources' terms w s_{k,n} in the order k = 0 ..
// nsrc-1 (coincident sources add up deterministically) and records again the
// receivers that sit on a source cell (co_off / co_rec: CSR per shot).
__global__ void ac_inject_encoded(float* next, size_t plane, const int* src_cell,
                                  const float* wav, int nsrc, int nt, int n, float w, int nshots,
                                  const int* co_off, const int* co_rec, const int* rec_cell,
                                  float* gathers, int nrec) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshots) return;
  float* f = next + (size_t)s * plane;
  const int* sc = src_cell + (size_t)s * nsrc;
  const float* ws = wav + (size_t)s * nsrc * nt;
  for (int k = 0; k < nsrc; ++k) {
    const float sw = w * ws[(size_t)k * nt + n];
    f[sc[k]] += sw;
  }
  if (!gathers) return;
  float* g = gathers + ((size_t)s * nt + n) * nrec;
  for (int e = co_off[s]; e < co_off[s + 1]; ++e) {
    const int r = co_rec[e];
    g[r] = f[rec_cell[(size_t)s * nrec + r]];
  }
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

template <bool kAdj>
void launch_interior(const AcStep& a, int rz, dim3 g, hipStream_t s) {
  switch (rz) {
    case 1: hipLaunchKernelGGL((ac_int_kernel<1, kAdj>), g, dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((ac_int_kernel<2, kAdj>), g, dim3(kThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL((ac_int_kernel<4, kAdj>), g, dim3(kThreads), 0, s, a); break;
    default: hipLaunchKernelGGL((ac_int_kernel<8, kAdj>), g, dim3(kThreads), 0, s, a); break;
  }
}

template <bool kAdj, bool kZ>
void launch_frame(const AcStep& a, int prz, dim3 g, hipStream_t s) {
  switch (prz) {
    case 1: hipLaunchKernelGGL((ac_pml_kernel<1, kAdj, kZ>), g, dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((ac_pml_kernel<2, kAdj, kZ>), g, dim3(kThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL((ac_pml_kernel<4, kAdj, kZ>), g, dim3(kThreads), 0, s, a); break;
    default: hipLaunchKernelGGL((ac_pml_kernel<8, kAdj, kZ>), g, dim3(kThreads), 0, s, a); break;
  }
}

template <bool kAdj>
void launch_interior_batch(const AcBatch& b, int rz, dim3 g, hipStream_t s) {
  switch (rz) {
    case 1: hipLaunchKernelGGL((ac_int_batch_kernel<1, kAdj>), g, dim3(kThreads), 0, s, b); break;
    case 2: hipLaunchKernelGGL((ac_int_batch_kernel<2, kAdj>), g, dim3(kThreads), 0, s, b); break;
    case 4: hipLaunchKernelGGL((ac_int_batch_kernel<4, kAdj>), g, dim3(kThreads), 0, s, b); break;
    default: hipLaunchKernelGGL((ac_int_batch_kernel<8, kAdj>), g, dim3(kThreads), 0, s, b); break;
  }
}

template <bool kAdj, bool kZ>
void launch_frame_batch(const AcBatch& b, int prz, dim3 g, hipStream_t s) {
  switch (prz) {
    case 1: hipLaunchKernelGGL((ac_pml_batch_kernel<1, kAdj, kZ>), g, dim3(kThreads), 0, s, b); break;
    case 2: hipLaunchKernelGGL((ac_pml_batch_kernel<2, kAdj, kZ>), g, dim3(kThreads), 0, s, b); break;
    case 4: hipLaunchKernelGGL((ac_pml_batch_kernel<4, kAdj, kZ>), g, dim3(kThreads), 0, s, b); break;
    default: hipLaunchKernelGGL((ac_pml_batch_kernel<8, kAdj, kZ>), g, dim3(kThreads), 0, s, b); break;
  }
}

// ev (optional): start/stop event pairs around the interior launch (ev[0],
// ev[1]), the z-frame launch (ev[2], ev[3]) and the x-frame launch (ev[4],
// ev[5]); a null pair is not recorded. a.nsub = a.tz / (4 prz).
template <bool kAdj>
int launch_step(const AcStep& a, int rz, int prz, hipStream_t s, hipEvent_t* ev) {
  if (a.n_zf > 0) {
    if (ev && ev[2]) SWEEP_HIP(hipEventRecord(ev[2], s));
    launch_frame<kAdj, true>(a, prz, dim3(a.n_zf * a.nsub * a.nshots), s);
    if (ev && ev[3]) SWEEP_HIP(hipEventRecord(ev[3], s));
  }
  if (a.n_xf > 0) {
    if (ev && ev[4]) SWEEP_HIP(hipEventRecord(ev[4], s));
    launch_frame<kAdj, false>(a, prz, dim3(a.n_xf * a.nsub * a.nshots), s);
    if (ev && ev[5]) SWEEP_HIP(hipEventRecord(ev[5], s));
  }
  if (a.n_int > 0) {
    if (ev && ev[0]) SWEEP_HIP(hipEventRecord(ev[0], s));
    launch_interior<kAdj>(a, rz, dim3(a.n_int * a.nshots), s);
    if (ev && ev[1]) SWEEP_HIP(hipEventRecord(ev[1], s));
  }
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

// One batched step over the active plans `steps[0..n)` (all with the same rz and
// prz): one launch per tile set (z frame, x frame, interior) for all plans.
// Plans with more than kPlansPerLaunch members with work take one launch per
// group of kPlansPerLaunch of them, in plan order.
template <bool kAdj>
int launch_step_batch(const AcStep* steps, int n, int rz, int prz, hipStream_t s) {
  AcBatch b;
  for (int phase = 0; phase < 3; ++phase) {
    for (int q = 0; q < n;) {
      b.nplans = 0;
      b.base[0] = 0;
      for (; q < n && b.nplans < kPlansPerLaunch; ++q) {
        const AcStep& a = steps[q];
        const int blocks =
            (phase == 0 ? a.n_zf * a.nsub : phase == 1 ? a.n_xf * a.nsub : a.n_int) * a.nshots;
        if (blocks <= 0) continue;
        const int k = b.nplans++;
        b.step[k] = a;
        b.base[k + 1] = b.base[k] + blocks;
      }
      if (b.nplans == 0) continue;
      const dim3 g(b.base[b.nplans]);
      if (phase == 0)
        launch_frame_batch<kAdj, true>(b, prz, g, s);
      else if (phase == 1)
        launch_frame_batch<kAdj, false>(b, prz, g, s);
      else
        launch_interior_batch<kAdj>(b, rz, g, s);
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

int ac_launch_tables(float* ax, float* bx, float* az, float* bz, int NX, int NZ, int P,
                     double h, double dt, double vmax, double f0, double R, hipStream_t s) {
  const int nmax = NX > NZ ? NX : NZ;
  hipLaunchKernelGGL(ac_tables_kernel, dim3((nmax + 255) / 256), dim3(256), 0, s, ax, bx, az,
                     bz, NX, NZ, P, h, dt, vmax, f0, R);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int ac_launch_deep(const AcStep& a, bool adj, hipStream_t s, hipEvent_t* ev) {
  if (a.n_run <= 0) return SWEEP_OK;
  const dim3 g(a.n_run * a.nshots);
  if (ev && ev[0]) SWEEP_HIP(hipEventRecord(ev[0], s));
  if (adj)
    hipLaunchKernelGGL((ac_march_kernel<true>), g, dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((ac_march_kernel<false>), g, dim3(kThreads), 0, s, a);
  if (ev && ev[1]) SWEEP_HIP(hipEventRecord(ev[1], s));
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

// Two-step passes of several plans in one launch (plans with no deep run are
// left out).
int ac_launch_deep_batch(const AcStep* steps, int n, bool adj, hipStream_t s) {
  AcBatch b;
  for (int q = 0; q < n;) {
    b.nplans = 0;
    b.base[0] = 0;
    for (; q < n && b.nplans < kPlansPerLaunch; ++q) {
      const AcStep& a = steps[q];
      if (a.n_run <= 0) continue;
      const int k = b.nplans++;
      b.step[k] = a;
      b.base[k + 1] = b.base[k] + a.n_run * a.nshots;
    }
    if (b.nplans == 0) continue;
    const dim3 g(b.base[b.nplans]);
    if (adj)
      hipLaunchKernelGGL((ac_march_batch_kernel<true>), g, dim3(kThreads), 0, s, b);
    else
      hipLaunchKernelGGL((ac_march_batch_kernel<false>), g, dim3(kThreads), 0, s, b);
  }
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

static bool valid_rz(int rz, int prz) {
  return (rz == 1 || rz == 2 || rz == 4 || rz == 8) &&
         (prz == 1 || prz == 2 || prz == 4 || prz == 8) && prz <= rz;
}

int ac_launch_fwd(const AcStep& a, int rz, int prz, hipStream_t s, hipEvent_t* ev) {
  if (!valid_rz(rz, prz)) {
    set_error("unsupported rz / pml_rz");
    return SWEEP_EINVAL;
  }
  return launch_step<false>(a, rz, prz, s, ev);
}

template <bool kZ>
void launch_born_frame(const AcStep& a, int prz, dim3 g, hipStream_t s) {
  switch (prz) {
    case 1: hipLaunchKernelGGL((ac_born_pml_kernel<1, kZ>), g, dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((ac_born_pml_kernel<2, kZ>), g, dim3(kThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL((ac_born_pml_kernel<4, kZ>), g, dim3(kThreads), 0, s, a); break;
    default: hipLaunchKernelGGL((ac_born_pml_kernel<8, kZ>), g, dim3(kThreads), 0, s, a); break;
  }
}

int ac_launch_born(const AcStep& a, int rz, int prz, hipStream_t s) {
  if (!valid_rz(rz, prz)) {
    set_error("unsupported rz / pml_rz");
    return SWEEP_EINVAL;
  }
  if (!a.bdC || !a.bB) {
    set_error("Born step without its perturbation operands");
    return SWEEP_EINVAL;
  }
  if (a.n_zf > 0) launch_born_frame<true>(a, prz, dim3(a.n_zf * a.nsub * a.nshots), s);
  if (a.n_xf > 0) launch_born_frame<false>(a, prz, dim3(a.n_xf * a.nsub * a.nshots), s);
  if (a.n_int > 0) {
    const dim3 g(a.n_int * a.nshots);
    switch (rz) {
      case 1: hipLaunchKernelGGL((ac_born_int_kernel<1>), g, dim3(kThreads), 0, s, a); break;
      case 2: hipLaunchKernelGGL((ac_born_int_kernel<2>), g, dim3(kThreads), 0, s, a); break;
      case 4: hipLaunchKernelGGL((ac_born_int_kernel<4>), g, dim3(kThreads), 0, s, a); break;
      default: hipLaunchKernelGGL((ac_born_int_kernel<8>), g, dim3(kThreads), 0, s, a); break;
    }
  }
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int ac_launch_born_prep(const float* v, const float* dv, float* dCs, int nx, int nz, int P,
                        double h, double dt, hipStream_t s) {
  const int NX = nx + 2 * P, NZ = nz + 2 * P;
  hipLaunchKernelGGL(ac_born_prep_kernel, dim3((NX + 255) / 256, NZ), dim3(256), 0, s, v, dv, dCs,
                     nx, nz, P, dt / h);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int ac_launch_adj(const AcStep& a, int rz, int prz, hipStream_t s, hipEvent_t* ev) {
  if (!valid_rz(rz, prz)) {
    set_error("unsupported rz / pml_rz");
    return SWEEP_EINVAL;
  }
  return launch_step<true>(a, rz, prz, s, ev);
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

int ac_launch_inject_encoded(float* next, size_t plane, const int* src_cell, const float* wav,
                             int nsrc, int nt, int n, float w, int nshots, const int* co_off,
                             const int* co_rec, const int* rec_cell, float* gathers, int nrec,
                             hipStream_t s) {
  hipLaunchKernelGGL(ac_inject_encoded, dim3((nshots + 63) / 64), dim3(64), 0, s, next, plane,
                     src_cell, wav, nsrc, nt, n, w, nshots, co_off, co_rec, rec_cell, gathers,
                     nrec);
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

int ac_launch_fwd_batch(const AcStep* steps, int n, int rz, int prz, hipStream_t s) {
  if (!valid_rz(rz, prz)) {
    set_error("unsupported rz / pml_rz");
    return SWEEP_EINVAL;
  }
  return launch_step_batch<false>(steps, n, rz, prz, s);
}

int ac_launch_adj_batch(const AcStep* steps, int n, int rz, int prz, hipStream_t s) {
  if (!valid_rz(rz, prz)) {
    set_error("unsupported rz / pml_rz");
    return SWEEP_EINVAL;
  }
  return launch_step_batch<true>(steps, n, rz, prz, s);
}

}  // namespace sweep
