// Elastic step kernels for gfx950: the isotropic velocity-stress system
// (Sec. 3.5, Eq. 12) on a staggered grid, 4th order in space, with C-PML and an
// optional free surface, and the exact transpose of that recurrence.
//
// Nodes of the values stored at [j][i]: txx, tzz at (i, j); vx at (i+1/2, j);
// vz at (i, j+1/2); txz at (i+1/2, j+1/2). Derivatives (c1 = 9/8, c2 = -1/24):
//   Dx+ f = c1 (f[i+1]-f[i]) + c2 (f[i+2]-f[i-1])    integer -> half
//   Dx- g = c1 (g[i]-g[i-1]) + c2 (g[i+1]-g[i-2])    half -> integer
// zero outside the grid; along z at a free surface the stress images
// tzz[-k] = -tzz[k], txz[-k-1] = -txz[k] are folded into the first rows and the
// velocity z-derivatives that would reach above the surface fall back to the
// 2nd-order difference. Each of the eight derivatives carries a C-PML memory
// variable psi <- b psi + a D f, stored over the whole grid but touched only
// where a != 0.
//
// Forward step: velocity kernel (vx, vz), receiver gather, stress kernel
// (txx, tzz, txz, explosive source). Every step kernel has a fluid variant
// (kFluid, the first-order acoustic system at vs = 0): there mu = 0, so txz
// stays 0, and the shear stress, its four memory variables and the mu
// partials of the adjoint enter only through products with 0. The variant
// drops them; every other value is formed by the same operations, so it gives
// the elastic kernels' results at vs = 0 while moving about a fifth fewer
// bytes forward and a quarter fewer in reverse. Reverse step (gather form of the
// transpose): adjoint-stress kernel (updates the velocity adjoints from the
// stress adjoints), residual injection, adjoint-velocity kernel. Away from the
// surface the transposes are (Dx+)^T = -Dx-, (Dx-)^T = -Dx+ (and along z); on the
// first four rows below a free surface they use tap tables derived on the host
// from the forward taps.
#include "elastic.h"

namespace sweep {
namespace {

constexpr float C1 = 9.0f / 8.0f;
constexpr float C2 = -1.0f / 24.0f;

// ---------------------------------------------------------------------------
// Tiles: 64 columns x kElTZ rows per work-group, thread (lx, w) owns column lx
// and rows [w kElRZ, w kElRZ + kElRZ). The fields (or derived quantities) a
// kernel differentiates are staged in LDS on the tile plus a 2-cell halo, zero
// outside the grid, so the stencils read LDS and every global load is
// coalesced and issued once per tile.
// ---------------------------------------------------------------------------
constexpr int kElRZ = 4;
constexpr int kElTZ = 4 * kElRZ;
constexpr int kElBW = kTX + 4;
constexpr int kElBH = kElTZ + 4;
constexpr int kElBox = kElBW * kElBH;
constexpr int kElK = (kElBox + kThreads - 1) / kThreads;

// value at grid cell (i, j) of a staged box whose first cell is (x0-2, z0-2)
struct Box {
  const float* s;
  int x0, z0;
  __device__ __forceinline__ float operator()(int i, int j) const {
    return s[(j - z0 + 2) * kElBW + (i - x0 + 2)];
  }
};

template <class F>
__device__ __forceinline__ float bdxp(const F& f, int i, int j) {
  return fmaf(C2, f(i + 2, j) - f(i - 1, j), C1 * (f(i + 1, j) - f(i, j)));
}
template <class F>
__device__ __forceinline__ float bdxm(const F& f, int i, int j) {
  return fmaf(C2, f(i + 1, j) - f(i - 2, j), C1 * (f(i, j) - f(i - 1, j)));
}
template <class F>
__device__ __forceinline__ float bdzp(const F& f, int i, int j) {
  return fmaf(C2, f(i, j + 2) - f(i, j - 1), C1 * (f(i, j + 1) - f(i, j)));
}
template <class F>
__device__ __forceinline__ float bdzm(const F& f, int i, int j) {
  return fmaf(C2, f(i, j + 1) - f(i, j - 2), C1 * (f(i, j) - f(i, j - 1)));
}
// z derivatives with the free-surface rules on rows 0 and 1
template <class F>
__device__ __forceinline__ float bdz_tzz(const F& f, int i, int j, int fs) {
  if (fs && j == 0)  // tzz[-1] = -tzz[1]
    return fmaf(C2, f(i, 2), fmaf(C1 + C2, f(i, 1), -C1 * f(i, 0)));
  return bdzp(f, i, j);
}
template <class F>
__device__ __forceinline__ float bdz_txz(const F& f, int i, int j, int fs) {
  if (fs && j == 0)  // txz[-1] = -txz[0], txz[-2] = -txz[1]
    return fmaf(2.0f * C2, f(i, 1), 2.0f * C1 * f(i, 0));
  if (fs && j == 1)  // txz[-1] = -txz[0]
    return fmaf(C2, f(i, 2), fmaf(-C1 + C2, f(i, 0), C1 * f(i, 1)));
  return bdzm(f, i, j);
}
template <class F>
__device__ __forceinline__ float bdz_vx(const F& f, int i, int j, int fs) {
  if (fs && j == 0) return f(i, 1) - f(i, 0);
  return bdzp(f, i, j);
}
template <class F>
__device__ __forceinline__ float bdz_vz(const F& f, int i, int j, int fs) {
  if (fs && j == 0) return 0.0f;
  if (fs && j == 1) return f(i, 1) - f(i, 0);
  return bdzm(f, i, j);
}

// tile and shot of this work-group (1-D launch over tiles x shots)
struct ElTile {
  int x0, z0, shot;
};
__device__ __forceinline__ ElTile el_tile(const ElStep& a) {
  const int f = xcd_spread(blockIdx.x, gridDim.x);
  const int tx = (a.NX + kTX - 1) / kTX, tz = (a.NZ + kElTZ - 1) / kElTZ;
  const int t = f % (tx * tz);
  ElTile r;
  r.shot = f / (tx * tz);
  r.x0 = (t % tx) * kTX;
  r.z0 = (t / tx) * kElTZ;
  return r;
}

// Guarded load without a per-lane branch: every lane loads (from `safe`, any
// valid address, where !ok) and the value is selected afterwards. Written as a
// branch, a guarded load must complete before the other path writes its
// register, which serialises a sequence of them. The reverse kernels address
// with 64-bit per-lane offsets like this: the scalar-base form (u32at, as in
// the forward kernels) made their step 3 % slower.
__device__ __forceinline__ float ldz(const float* f, size_t i, bool ok, const float* safe) {
  const float v = *(ok ? f + i : safe);
  return ok ? v : 0.0f;
}

// Stages NF shot fields on the tile plus the halo: dst[q][box] = src[q][cell].
template <int NF>
__device__ __forceinline__ void el_stage(float (*dst)[kElBox], const float* const* src, int x0,
                                         int z0, int NX, int NZ) {
  float v[NF][kElK];
#pragma unroll
  for (int k = 0; k < kElK; ++k) {
    const int e = threadIdx.x + k * kThreads;
    const int r = e / kElBW, c = e - (e / kElBW) * kElBW;
    const int gx = x0 - 2 + c, gz = z0 - 2 + r;
    const bool ok = e < kElBox && gx >= 0 && gx < NX && gz >= 0 && gz < NZ;
    const unsigned q = ok ? (unsigned)(gz * NX + gx) : 0u;
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f][k] = ldz32(src[f], q, ok);
  }
#pragma unroll
  for (int k = 0; k < kElK; ++k) {
    const int e = threadIdx.x + k * kThreads;
    if (e < kElBox) {
#pragma unroll
      for (int f = 0; f < NF; ++f) dst[f][e] = v[f][k];
    }
  }
}

// Per-thread cell geometry of a tile: column i (clamped ic for loads), rows
// jb .. jb + kElRZ - 1 (jb is the same for the whole wave, which readfirstlane
// tells the compiler, so the row coefficients are scalar loads and branches on
// them are uniform).
struct ElCells {
  int i, ic, jb;
  __device__ __forceinline__ ElCells(const ElTile& T, int NX) {
    i = T.x0 + (threadIdx.x & 63);
    ic = min(i, NX - 1);
    jb = T.z0 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * kElRZ;
  }
};

// The stress update is txx += dt (cxx_x exx + cxx_z ezz), tzz += dt (czz_x exx +
// czz_z ezz). Away from a free surface cxx_x = czz_z = lambda + 2 mu and
// cxx_z = czz_x = lambda; on the free-surface row cxx_x = M and the other three
// are 0. So czz_x = cxx_z everywhere, and czz_z (of row j) follows from cxx_x:
// the kernels read two coefficient planes instead of four.
__device__ __forceinline__ float czz_z(const ElStep& a, int j, float cxx_x) {
  return a.fs && j == 0 ? 0.0f : cxx_x;
}

// C-PML update with a preloaded memory variable: psi <- b psi + a G where
// a != 0 (stored), returns G + psi; G elsewhere.
__device__ __forceinline__ float cpml_p(float* psi, unsigned k, float G, float a, float b, float p0,
                                        bool store) {
  if (a == 0.0f) return G;
  const float p = fmaf(a, G, b * p0);
  if (store) u32at(psi, k) = p;
  return G + p;
}

// ---------------------------------------------------------------------------
// forward: velocity update  vx += dt bx (Dx+ txx + Dz- txz), vz += dt bz (Dx- txz + Dz+ tzz)
// All global loads of a thread (staging, then its cells' operands and memory
// variables) are issued before its first store.
// ---------------------------------------------------------------------------
template <bool kFluid>
__global__ __launch_bounds__(256) void el_vel_kernel(ElStep a) {
  constexpr int NF = kFluid ? 2 : 3;
  __shared__ float sb[NF][kElBox];
  const ElTile T = el_tile(a);
  const int NX = a.NX, NZ = a.NZ;
  const size_t plane = (size_t)NX * NZ;
  const size_t so = (size_t)T.shot * plane;
  {
    const float* src[3] = {a.txx + so, a.tzz + so, a.txz + so};
    el_stage<NF>(sb, src, T.x0, T.z0, NX, NZ);
  }
  const ElCells C(T, NX);
  const float axh = a.axh[C.ic], bxh = a.bxh[C.ic], axi = a.axi[C.ic], bxi = a.bxi[C.ic];
  const bool wxh = __any(axh != 0.0f), wxi = __any(axi != 0.0f);
  float ovx[kElRZ], ovz[kElRZ], cbx[kElRZ], cbz[kElRZ], p0[kElRZ], p1[kElRZ], p2[kElRZ],
      p3[kElRZ];
  float azi[kElRZ], bzi[kElRZ], azh[kElRZ], bzh[kElRZ];
#pragma unroll
  for (int r = 0; r < kElRZ; ++r) {
    const int jc = min(C.jb + r, NZ - 1);
    const unsigned k = (unsigned)(jc * NX + C.ic);
    ovx[r] = u32at(a.vx + so, k);
    ovz[r] = u32at(a.vz + so, k);
    cbx[r] = u32at(a.bx, k);
    cbz[r] = u32at(a.bz, k);
    azi[r] = a.azi[jc];
    bzi[r] = a.bzi[jc];
    azh[r] = a.azh[jc];
    bzh[r] = a.bzh[jc];
    p0[r] = wxh ? u32at(a.ps[0] + so, k) : 0.0f;
    p1[r] = !kFluid && azi[r] != 0.0f ? u32at(a.ps[1] + so, k) : 0.0f;
    p2[r] = !kFluid && wxi ? u32at(a.ps[2] + so, k) : 0.0f;
    p3[r] = azh[r] != 0.0f ? u32at(a.ps[3] + so, k) : 0.0f;
  }
  __syncthreads();
  const Box txx{sb[0], T.x0, T.z0}, tzz{sb[1], T.x0, T.z0}, txz{sb[NF - 1], T.x0, T.z0};
  const int i = C.i;
  const float ih = a.ih;
#pragma unroll
  for (int r = 0; r < kElRZ; ++r) {
    const int j = C.jb + r;
    if (i >= NX || j >= NZ) continue;
    const unsigned k = (unsigned)(j * NX + i);
    const float Ga = bdxp(txx, i, j) * ih;
    const float Gd = bdz_tzz(tzz, i, j, a.fs) * ih;
    float fvx = cpml_p(a.ps[0] + so, k, Ga, axh, bxh, p0[r], true);
    float fvz = cpml_p(a.ps[3] + so, k, Gd, azh[r], bzh[r], p3[r], true);
    if (!kFluid) {
      const float Gb = bdz_txz(txz, i, j, a.fs) * ih;
      const float Gc = bdxm(txz, i, j) * ih;
      fvx = fvx + cpml_p(a.ps[1] + so, k, Gb, azi[r], bzi[r], p1[r], true);
      fvz = cpml_p(a.ps[2] + so, k, Gc, axi, bxi, p2[r], true) + fvz;
    }
    u32at(a.vx + so, k) = fmaf(a.dt * cbx[r], fvx, ovx[r]);
    u32at(a.vz + so, k) = fmaf(a.dt * cbz[r], fvz, ovz[r]);
    if (a.tr[0]) {
      u32at(a.tr[0] + so, k) = fvx;
      u32at(a.tr[1] + so, k) = fvz;
    }
  }
}

// gathers[shot][n][r] = (vx, vz) at the receiver cell (v^{n+1/2})
__global__ void el_record_kernel(ElStep a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.nshots * a.nrec) return;
  const int s = t / a.nrec, r = t - s * a.nrec;
  const size_t plane = (size_t)a.NX * a.NZ;
  const size_t k = (size_t)s * plane + a.rec_cell[t];
  float* d = a.gathers + (((size_t)s * a.nt + a.n) * a.nrec + r) * 2;
  d[0] = a.vx[k];
  d[1] = a.vz[k];
}

// ---------------------------------------------------------------------------
// forward: stress update and explosive source
// ---------------------------------------------------------------------------
template <bool kFluid>
__global__ __launch_bounds__(256) void el_str_kernel(ElStep a) {
  __shared__ float sb[2][kElBox];
  const ElTile T = el_tile(a);
  const int NX = a.NX, NZ = a.NZ;
  const size_t plane = (size_t)NX * NZ;
  const int shot = T.shot;
  const size_t so = (size_t)shot * plane;
  {
    const float* src[2] = {a.vx + so, a.vz + so};
    el_stage<2>(sb, src, T.x0, T.z0, NX, NZ);
  }
  const ElCells C(T, NX);
  const float axi = a.axi[C.ic], bxi = a.bxi[C.ic], axh = a.axh[C.ic], bxh = a.bxh[C.ic];
  const bool wxi = __any(axi != 0.0f), wxh = __any(axh != 0.0f);
  float otxx[kElRZ], otzz[kElRZ], otxz[kElRZ], cxx_x[kElRZ], cxx_z[kElRZ], mxz[kElRZ],
      p4[kElRZ], p5[kElRZ], p6[kElRZ], p7[kElRZ];
  float azi[kElRZ], bzi[kElRZ], azh[kElRZ], bzh[kElRZ];
#pragma unroll
  for (int r = 0; r < kElRZ; ++r) {
    const int jc = min(C.jb + r, NZ - 1);
    const unsigned k = (unsigned)(jc * NX + C.ic);
    otxx[r] = u32at(a.txx + so, k);
    otzz[r] = u32at(a.tzz + so, k);
    otxz[r] = kFluid ? 0.0f : u32at(a.txz + so, k);
    cxx_x[r] = u32at(a.cxx_x, k);
    cxx_z[r] = u32at(a.cxx_z, k);
    mxz[r] = kFluid ? 0.0f : u32at(a.mxz, k);
    azi[r] = a.azi[jc];
    bzi[r] = a.bzi[jc];
    azh[r] = a.azh[jc];
    bzh[r] = a.bzh[jc];
    p4[r] = wxi ? u32at(a.ps[4] + so, k) : 0.0f;
    p5[r] = azi[r] != 0.0f ? u32at(a.ps[5] + so, k) : 0.0f;
    p6[r] = !kFluid && azh[r] != 0.0f ? u32at(a.ps[6] + so, k) : 0.0f;
    p7[r] = !kFluid && wxh ? u32at(a.ps[7] + so, k) : 0.0f;
  }
  const int src = a.src_cell[shot];
  const float sw = a.w * a.wavelet[(size_t)shot * a.nt + a.n];
  __syncthreads();
  const Box vx{sb[0], T.x0, T.z0}, vz{sb[1], T.x0, T.z0};
  const int i = C.i;
  const float ih = a.ih, dt = a.dt;
#pragma unroll
  for (int r = 0; r < kElRZ; ++r) {
    const int j = C.jb + r;
    if (i >= NX || j >= NZ) continue;
    const unsigned k = (unsigned)(j * NX + i);
    const float Ge = bdxm(vx, i, j) * ih;
    const float Gf = bdz_vz(vz, i, j, a.fs) * ih;
    const float exx = cpml_p(a.ps[4] + so, k, Ge, axi, bxi, p4[r], true);
    const float ezz = cpml_p(a.ps[5] + so, k, Gf, azi[r], bzi[r], p5[r], true);
    float txx = otxx[r] + dt * fmaf(cxx_x[r], exx, cxx_z[r] * ezz);
    float tzz = otzz[r] + dt * fmaf(cxx_z[r], exx, czz_z(a, j, cxx_x[r]) * ezz);
    if ((int)k == src) {
      txx += sw;
      tzz += sw * u32at(a.smask, k);
    }
    u32at(a.txx + so, k) = txx;
    u32at(a.tzz + so, k) = tzz;
    if (a.tr[2]) {
      u32at(a.tr[2] + so, k) = exx;
      u32at(a.tr[3] + so, k) = ezz;
    }
    if (!kFluid) {
      const float Gg = bdz_vx(vx, i, j, a.fs) * ih;
      const float Gh = bdxp(vz, i, j) * ih;
      const float exz = cpml_p(a.ps[6] + so, k, Gg, azh[r], bzh[r], p6[r], true) +
                        cpml_p(a.ps[7] + so, k, Gh, axh, bxh, p7[r], true);
      u32at(a.txz + so, k) = fmaf(dt * mxz[r], exz, otxz[r]);
      if (a.tr[2]) u32at(a.tr[4] + so, k) = exz;
    }
  }
}

// ---------------------------------------------------------------------------
// Reverse step. With ebar = dt (stress coefficient) x (stress adjoint) and the
// C-PML adjoint t = Psi + ebar, the derivative input adjoint is ebar + a t and
// Psi <- b t. The velocity adjoints collect the transposed derivatives of those.
// ---------------------------------------------------------------------------

// Transposed z-derivative of g at row j: standard (-Dz- or -Dz+) away from a
// free surface, otherwise the host-derived taps of the first four rows (their
// offsets lie within two rows).
template <class F>
__device__ __forceinline__ float dzT(const ElStep& a, int kind, int j, F g, bool minus_dzm) {
  if (a.fs && j < 4) {
    float acc = 0.0f;
    const int n = a.tt_cnt[kind][j];
    for (int e = 0; e < n; ++e) acc = fmaf(a.tt_w[kind][j][e], g(j + a.tt_off[kind][j][e]), acc);
    return acc;
  }
  // -(Dz-) g = -[c1 (g_j - g_{j-1}) + c2 (g_{j+1} - g_{j-2})]
  // -(Dz+) g = -[c1 (g_{j+1} - g_j) + c2 (g_{j+2} - g_{j-1})]
  if (minus_dzm) return -fmaf(C2, g(j + 1) - g(j - 2), C1 * (g(j) - g(j - 1)));
  return -fmaf(C2, g(j + 2) - g(j - 1), C1 * (g(j + 1) - g(j)));
}

// The reverse kernels split the box cells of a tile between the threads: a
// thread stages its own cells (box column lx + 2, rows kElRZ w + 2 ..
// kElRZ w + kElRZ + 1) and keeps their raw values in registers for its own
// update, and up to kElKH of the kElHalo halo cells (the two rows above and
// below the tile, the two columns left and right of it). Reading its own
// cells again after the LDS phase would miss L2: by then the other resident
// work-groups' reads have evicted them.
constexpr int kElHalo = kElBox - kTX * kElTZ;
constexpr int kElKH = (kElHalo + kThreads - 1) / kThreads;
static_assert(kElBW == kTX + 4 && kElBH == kElTZ + 4 && kThreads == 4 * kTX, "tile geometry");

// box index of halo cell h < kElHalo
__device__ __forceinline__ int el_halo_cell(int h) {
  if (h < 2 * kElBW) return h;                                // rows 0, 1
  if (h < 4 * kElBW) return h + (kElBH - 4) * kElBW;          // the last two rows
  const int q = h - 4 * kElBW, c = q & 3;                     // columns 0, 1, 66, 67
  return (2 + (q >> 2)) * kElBW + (c < 2 ? c : kTX + c);
}
// box index of this thread's own cell in row r of its rows
__device__ __forceinline__ int el_own_cell(int r) {
  return ((int)(threadIdx.x >> 6) * kElRZ + r + 2) * kElBW + (int)(threadIdx.x & 63) + 2;
}

// Raw inputs of one box cell of the stress-adjoint staging (zero outside the
// grid or where !valid; every lane takes part, as the C-PML tests are votes
// of the wave).
struct AdjS {
  float txx, tzz, txz, cxx_x, czz_x, cxx_z, czz_z, mxz, ax, az, azh, axh, q4, q5, q6, q7;
};
template <bool kFluid>
__device__ __forceinline__ void adj_s_load(const ElStep& a, size_t so, int e, bool valid, int x0,
                                           int z0, AdjS& v) {
  const int r = e / kElBW, c = e - (e / kElBW) * kElBW;
  const int gx = x0 - 2 + c, gz = z0 - 2 + r;
  const bool ok = valid && gx >= 0 && gx < a.NX && gz >= 0 && gz < a.NZ;
  const size_t q = ok ? (size_t)gz * a.NX + gx : 0;
  const int cx = ok ? gx : 0, cz = ok ? gz : 0;
  v.txx = ldz(a.txx + so, q, ok, a.txx);
  v.tzz = ldz(a.tzz + so, q, ok, a.tzz);
  v.txz = kFluid ? 0.0f : ldz(a.txz + so, q, ok, a.txz);
  v.cxx_x = ldz(a.cxx_x, q, ok, a.cxx_x);
  v.cxx_z = ldz(a.cxx_z, q, ok, a.cxx_z);
  v.czz_x = v.cxx_z;
  v.czz_z = czz_z(a, gz, v.cxx_x);
  v.mxz = kFluid ? 0.0f : ldz(a.mxz, q, ok, a.mxz);
  v.ax = ldz(a.axi, cx, ok, a.axi);
  v.az = ldz(a.azi, cz, ok, a.azi);
  v.azh = kFluid ? 0.0f : ldz(a.azh, cz, ok, a.azh);
  v.axh = kFluid ? 0.0f : ldz(a.axh, cx, ok, a.axh);
  // memory variables only where a wave has a C-PML cell (wave-uniform branch)
  v.q4 = __any(v.ax != 0.0f) ? ldz(a.ps_in[4] + so, q, ok, a.ps_in[4]) : 0.0f;
  v.q5 = __any(v.az != 0.0f) ? ldz(a.ps_in[5] + so, q, ok, a.ps_in[5]) : 0.0f;
  v.q6 = !kFluid && __any(v.azh != 0.0f) ? ldz(a.ps_in[6] + so, q, ok, a.ps_in[6]) : 0.0f;
  v.q7 = !kFluid && __any(v.axh != 0.0f) ? ldz(a.ps_in[7] + so, q, ok, a.ps_in[7]) : 0.0f;
}
// ebar of the three stress-step inputs: dt (stress coefficients) x (stress adjoints)
__device__ __forceinline__ float adj_ex(const AdjS& v, float dt) {
  return dt * fmaf(v.cxx_x, v.txx, v.czz_x * v.tzz);
}
__device__ __forceinline__ float adj_ez(const AdjS& v, float dt) {
  return dt * fmaf(v.cxx_z, v.txx, v.czz_z * v.tzz);
}
__device__ __forceinline__ float adj_exz(const AdjS& v, float dt) { return dt * v.mxz * v.txz; }

// derivative-input adjoints gbe (exx input), gbf (ezz), gbg (Dz vx of exz),
// gbh (Dx vz of exz) of box cell e (outside the grid every operand is 0, so
// every value is 0 too)
template <bool kFluid>
__device__ __forceinline__ void adj_s_put(float (*sb)[kElBox], int e, float dt, const AdjS& v) {
  const float e1 = adj_ex(v, dt), e2 = adj_ez(v, dt);
  sb[0][e] = v.ax == 0.0f ? e1 : fmaf(v.ax, v.q4 + e1, e1);
  sb[1][e] = v.az == 0.0f ? e2 : fmaf(v.az, v.q5 + e2, e2);
  if (!kFluid) {
    const float e3 = adj_exz(v, dt);
    sb[2][e] = v.azh == 0.0f ? e3 : fmaf(v.azh, v.q6 + e3, e3);
    sb[3][e] = v.axh == 0.0f ? e3 : fmaf(v.axh, v.q7 + e3, e3);
  }
}

template <bool kFluid>
__global__ __launch_bounds__(256) void el_adj_s_kernel(ElStep a) {
  __shared__ float sb[kFluid ? 2 : 4][kElBox];
  const ElTile T = el_tile(a);
  const int NX = a.NX, NZ = a.NZ;
  const size_t plane = (size_t)NX * NZ;
  const size_t so = (size_t)T.shot * plane;
  const float dt = a.dt, ih = a.ih;
  AdjS hv[kElKH], ov[kElRZ];
#pragma unroll
  for (int k = 0; k < kElKH; ++k) {
    const int h = (int)threadIdx.x + k * kThreads;
    adj_s_load<kFluid>(a, so, h < kElHalo ? el_halo_cell(h) : 0, h < kElHalo, T.x0, T.z0,
                       hv[k]);
  }
#pragma unroll
  for (int r = 0; r < kElRZ; ++r)
    adj_s_load<kFluid>(a, so, el_own_cell(r), true, T.x0, T.z0, ov[r]);
#pragma unroll
  for (int k = 0; k < kElKH; ++k) {
    const int h = (int)threadIdx.x + k * kThreads;
    if (h < kElHalo) adj_s_put<kFluid>(sb, el_halo_cell(h), dt, hv[k]);
  }
#pragma unroll
  for (int r = 0; r < kElRZ; ++r) adj_s_put<kFluid>(sb, el_own_cell(r), dt, ov[r]);
  const ElCells C(T, NX);
  const float bxi = a.bxi[C.ic], bxh = a.bxh[C.ic];
  const bool gacc = !a.g_init;
  float ovx[kElRZ], ovz[kElRZ], fexx[kElRZ], fezz[kElRZ], fexz[kElRZ], g0[kElRZ], g1[kElRZ],
      g2[kElRZ], bzi[kElRZ], bzh[kElRZ];
#pragma unroll
  for (int r = 0; r < kElRZ; ++r) {
    const int jc = min(C.jb + r, NZ - 1);
    const size_t k = (size_t)jc * NX + C.ic;
    ovx[r] = a.vx[so + k];
    ovz[r] = a.vz[so + k];
    bzi[r] = a.bzi[jc];
    bzh[r] = a.bzh[jc];
    fexx[r] = a.trc[2][so + k];
    fezz[r] = a.trc[3][so + k];
    fexz[r] = kFluid ? 0.0f : a.trc[4][so + k];
    g0[r] = gacc ? a.g[0][so + k] : 0.0f;
    g1[r] = !kFluid && gacc ? a.g[1][so + k] : 0.0f;
    g2[r] = !kFluid && gacc ? a.g[2][so + k] : 0.0f;
  }
  const float dml = a.fs ? a.dM_dl[C.ic] : 0.0f, dmm = a.fs ? a.dM_dm[C.ic] : 0.0f;
  __syncthreads();
  const Box gbe{sb[0], T.x0, T.z0}, gbf{sb[1], T.x0, T.z0}, gbg{sb[kFluid ? 0 : 2], T.x0, T.z0},
      gbh{sb[kFluid ? 1 : 3], T.x0, T.z0};
  const int i = C.i;
#pragma unroll
  for (int r = 0; r < kElRZ; ++r) {
    const int j = C.jb + r;
    if (i >= NX || j >= NZ) continue;
    const size_t k = (size_t)j * NX + i;
    // Vx += (Dx-)^T gbe + (Dz+ of vx)^T gbg ;  (Dx-)^T = -Dx+
    // (the exz terms are absent in a fluid)
    const float dxe = -fmaf(C2, gbe(i + 2, j) - gbe(i - 1, j), C1 * (gbe(i + 1, j) - gbe(i, j)));
    // Vz += (Dz- of vz)^T gbf + (Dx+)^T gbh ;  (Dx+)^T = -Dx-
    const float dzf = dzT(a, 3, j, [&](int jj) { return gbf(i, jj); }, false);
    if (kFluid) {
      a.vx[so + k] = ovx[r] + dxe * ih;
      a.vz[so + k] = ovz[r] + dzf * ih;
    } else {
      const float dzg = dzT(a, 2, j, [&](int jj) { return gbg(i, jj); }, true);
      const float dxh =
          -fmaf(C2, gbh(i + 1, j) - gbh(i - 2, j), C1 * (gbh(i, j) - gbh(i - 1, j)));
      a.vx[so + k] = ovx[r] + (dxe + dzg) * ih;
      a.vz[so + k] = ovz[r] + (dzf + dxh) * ih;
    }

    // own cell: memory-variable adjoints and the coefficient gradients
    const AdjS& v = ov[r];
    const float ex = adj_ex(v, dt), ez = adj_ez(v, dt), exz = adj_exz(v, dt);
    if (v.ax != 0.0f) a.ps_out[4][so + k] = bxi * (v.q4 + ex);
    if (v.az != 0.0f) a.ps_out[5][so + k] = bzi[r] * (v.q5 + ez);
    if (!kFluid && v.azh != 0.0f) a.ps_out[6][so + k] = bzh[r] * (v.q6 + exz);
    if (!kFluid && v.axh != 0.0f) a.ps_out[7][so + k] = bxh * (v.q7 + exz);
    float glam, gmu;
    if (a.fs && j == 0) {
      // txx += dt M exx with M = 4 mu (lambda + mu) / (lambda + 2 mu)
      const float gM = dt * v.txx * fexx[r];
      glam = gM * dml;
      gmu = gM * dmm;
    } else {
      glam = dt * (v.txx + v.tzz) * (fexx[r] + fezz[r]);
      gmu = 2.0f * dt * fmaf(v.txx, fexx[r], v.tzz * fezz[r]);
    }
    // a fluid has no mu partials (the gradient finish weighs them by vs = 0;
    // their planes stay zero)
    const float gmxz = dt * v.txz * fexz[r];
    if (a.g_init) {
      a.g[0][so + k] = glam;
      if (!kFluid) {
        a.g[1][so + k] = gmu;
        a.g[2][so + k] = gmxz;
      }
    } else {
      a.g[0][so + k] = g0[r] + glam;
      if (!kFluid) {
        a.g[1][so + k] = g1[r] + gmu;
        a.g[2][so + k] = g2[r] + gmxz;
      }
    }
  }
}

// residual injection into the velocity adjoints: entries sorted by (shot, cell, r);
// the first entry of each run of equal cells adds the whole run in order.
__global__ void el_inject_kernel(ElStep a, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int tot = a.nshots * a.nrec;
  if (e >= tot) return;
  const int4 en = a.rec_sorted[e];  // (shot, cell, r, -)
  if (e > 0) {
    const int4 pv = a.rec_sorted[e - 1];
    if (pv.x == en.x && pv.y == en.y) return;
  }
  const size_t plane = (size_t)a.NX * a.NZ;
  const size_t k = (size_t)en.x * plane + en.y;
  float ax = a.vx[k], az = a.vz[k];
  for (int q = e; q < tot; ++q) {
    const int4 c = a.rec_sorted[q];
    if (c.x != en.x || c.y != en.y) break;
    const float* r = a.resid + (((size_t)c.x * a.nt + n) * a.nrec + c.z) * 2;
    ax += r[0];
    az += r[1];
  }
  a.vx[k] = ax;
  a.vz[k] = az;
}

// Raw inputs of one box cell of the velocity-adjoint staging (as AdjS).
struct AdjV {
  float vx, vz, bx, bz, axh, az, ax, azh, q0, q1, q2, q3;
};
template <bool kFluid>
__device__ __forceinline__ void adj_v_load(const ElStep& a, size_t so, int e, bool valid, int x0,
                                           int z0, AdjV& v) {
  const int r = e / kElBW, c = e - (e / kElBW) * kElBW;
  const int gx = x0 - 2 + c, gz = z0 - 2 + r;
  const bool ok = valid && gx >= 0 && gx < a.NX && gz >= 0 && gz < a.NZ;
  const size_t q = ok ? (size_t)gz * a.NX + gx : 0;
  const int cx = ok ? gx : 0, cz = ok ? gz : 0;
  v.vx = ldz(a.vx + so, q, ok, a.vx);
  v.vz = ldz(a.vz + so, q, ok, a.vz);
  v.bx = ldz(a.bx, q, ok, a.bx);
  v.bz = ldz(a.bz, q, ok, a.bz);
  v.axh = ldz(a.axh, cx, ok, a.axh);
  v.az = kFluid ? 0.0f : ldz(a.azi, cz, ok, a.azi);
  v.ax = kFluid ? 0.0f : ldz(a.axi, cx, ok, a.axi);
  v.azh = ldz(a.azh, cz, ok, a.azh);
  v.q0 = __any(v.axh != 0.0f) ? ldz(a.ps_in[0] + so, q, ok, a.ps_in[0]) : 0.0f;
  v.q1 = !kFluid && __any(v.az != 0.0f) ? ldz(a.ps_in[1] + so, q, ok, a.ps_in[1]) : 0.0f;
  v.q2 = !kFluid && __any(v.ax != 0.0f) ? ldz(a.ps_in[2] + so, q, ok, a.ps_in[2]) : 0.0f;
  v.q3 = __any(v.azh != 0.0f) ? ldz(a.ps_in[3] + so, q, ok, a.ps_in[3]) : 0.0f;
}
// derivative-input adjoints of the velocity step: gba (Dx txx of vx), gbb (Dz
// txz of vx), gbc (Dx txz of vz), gbd (Dz tzz of vz)
// (a fluid keeps gba and gbd only, in planes 0 and 1)
template <bool kFluid>
__device__ __forceinline__ void adj_v_put(float (*sb)[kElBox], int e, float dt, const AdjV& v) {
  const float kx = dt * v.bx * v.vx;
  const float kz = dt * v.bz * v.vz;
  sb[0][e] = v.axh == 0.0f ? kx : fmaf(v.axh, v.q0 + kx, kx);
  sb[kFluid ? 1 : 3][e] = v.azh == 0.0f ? kz : fmaf(v.azh, v.q3 + kz, kz);
  if (!kFluid) {
    sb[1][e] = v.az == 0.0f ? kx : fmaf(v.az, v.q1 + kx, kx);
    sb[2][e] = v.ax == 0.0f ? kz : fmaf(v.ax, v.q2 + kz, kz);
  }
}

template <bool kFluid>
__global__ __launch_bounds__(256) void el_adj_v_kernel(ElStep a) {
  __shared__ float sb[kFluid ? 2 : 4][kElBox];
  const ElTile T = el_tile(a);
  const int NX = a.NX, NZ = a.NZ;
  const size_t plane = (size_t)NX * NZ;
  const size_t so = (size_t)T.shot * plane;
  const float dt = a.dt, ih = a.ih;
  AdjV hv[kElKH], ov[kElRZ];
#pragma unroll
  for (int k = 0; k < kElKH; ++k) {
    const int h = (int)threadIdx.x + k * kThreads;
    adj_v_load<kFluid>(a, so, h < kElHalo ? el_halo_cell(h) : 0, h < kElHalo, T.x0, T.z0,
                       hv[k]);
  }
#pragma unroll
  for (int r = 0; r < kElRZ; ++r)
    adj_v_load<kFluid>(a, so, el_own_cell(r), true, T.x0, T.z0, ov[r]);
#pragma unroll
  for (int k = 0; k < kElKH; ++k) {
    const int h = (int)threadIdx.x + k * kThreads;
    if (h < kElHalo) adj_v_put<kFluid>(sb, el_halo_cell(h), dt, hv[k]);
  }
#pragma unroll
  for (int r = 0; r < kElRZ; ++r) adj_v_put<kFluid>(sb, el_own_cell(r), dt, ov[r]);
  const ElCells C(T, NX);
  const float bxh = a.bxh[C.ic], bxi = a.bxi[C.ic];
  const bool gacc = !a.g_init;
  float otxx[kElRZ], otzz[kElRZ], otxz[kElRZ], f0[kElRZ], f1[kElRZ], g3[kElRZ], g4[kElRZ],
      bzi[kElRZ], bzh[kElRZ];
#pragma unroll
  for (int r = 0; r < kElRZ; ++r) {
    const int jc = min(C.jb + r, NZ - 1);
    const size_t k = (size_t)jc * NX + C.ic;
    otxx[r] = a.txx[so + k];
    otzz[r] = a.tzz[so + k];
    otxz[r] = kFluid ? 0.0f : a.txz[so + k];
    bzi[r] = a.bzi[jc];
    bzh[r] = a.bzh[jc];
    f0[r] = a.trc[0][so + k];
    f1[r] = a.trc[1][so + k];
    g3[r] = gacc ? a.g[3][so + k] : 0.0f;
    g4[r] = gacc ? a.g[4][so + k] : 0.0f;
  }
  __syncthreads();
  const Box gba{sb[0], T.x0, T.z0}, gbb{sb[1], T.x0, T.z0}, gbc{sb[kFluid ? 0 : 2], T.x0, T.z0},
      gbd{sb[kFluid ? 1 : 3], T.x0, T.z0};
  const int i = C.i;
#pragma unroll
  for (int r = 0; r < kElRZ; ++r) {
    const int j = C.jb + r;
    if (i >= NX || j >= NZ) continue;
    const size_t k = (size_t)j * NX + i;
    // Txx += (Dx+)^T gba = -Dx- gba
    const float dxa = -fmaf(C2, gba(i + 1, j) - gba(i - 2, j), C1 * (gba(i, j) - gba(i - 1, j)));
    // Tzz += (Dz+ of tzz)^T gbd
    const float dzd = dzT(a, 0, j, [&](int jj) { return gbd(i, jj); }, true);
    a.txx[so + k] = otxx[r] + dxa * ih;
    a.tzz[so + k] = otzz[r] + dzd * ih;
    if (!kFluid) {
      // Txz += (Dz- of txz)^T gbb + (Dx-)^T gbc = ... - Dx+ gbc (a fluid's txz
      // adjoint reaches nothing: its only use is weighed by mu = 0)
      const float dzb = dzT(a, 1, j, [&](int jj) { return gbb(i, jj); }, false);
      const float dxc =
          -fmaf(C2, gbc(i + 2, j) - gbc(i - 1, j), C1 * (gbc(i + 1, j) - gbc(i, j)));
      a.txz[so + k] = otxz[r] + (dzb + dxc) * ih;
    }

    const AdjV& v = ov[r];
    const float kx = dt * v.bx * v.vx, kz = dt * v.bz * v.vz;
    if (v.axh != 0.0f) a.ps_out[0][so + k] = bxh * (v.q0 + kx);
    if (!kFluid && v.az != 0.0f) a.ps_out[1][so + k] = bzi[r] * (v.q1 + kx);
    if (!kFluid && v.ax != 0.0f) a.ps_out[2][so + k] = bxi * (v.q2 + kz);
    if (v.azh != 0.0f) a.ps_out[3][so + k] = bzh[r] * (v.q3 + kz);
    const float gbx = dt * v.vx * f0[r];
    const float gbz = dt * v.vz * f1[r];
    if (a.g_init) {
      a.g[3][so + k] = gbx;
      a.g[4][so + k] = gbz;
    } else {
      a.g[3][so + k] = g3[r] + gbx;
      a.g[4][so + k] = g4[r] + gbz;
    }
  }
}

// ---------------------------------------------------------------------------
// Material preparation: padded vp, vs, rho, lambda, mu; buoyancies; harmonic
// mu at txz nodes; stress coefficients (free-surface row uses M); C-PML tables.
// A fluid model holds (vp, rho) and has vs = 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double el_vs(const float* model, size_t mn, size_t m, int fluid) {
  return fluid ? 0.0 : (double)model[mn + m];
}
__device__ __forceinline__ double el_rho(const float* model, size_t mn, size_t m, int fluid) {
  return (double)model[(fluid ? 1 : 2) * mn + m];
}

__global__ void el_prep_kernel(const float* model, ElCoef c, int nx, int nz, int P, int top,
                               int NX, int NZ, int fs, int fluid) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= NX || j >= NZ) return;
  const size_t mn = (size_t)nx * nz;
  const int ii = min(max(i - P, 0), nx - 1), jj = min(max(j - top, 0), nz - 1);
  const size_t m = (size_t)jj * nx + ii, k = (size_t)j * NX + i;
  const double vp = model[m], vs = el_vs(model, mn, m, fluid), rho = el_rho(model, mn, m, fluid);
  const double mu = rho * vs * vs, lam = rho * (vp * vp - 2.0 * vs * vs);
  c.vp[k] = (float)vp;
  c.vs[k] = (float)vs;
  c.rho[k] = (float)rho;
  c.lam[k] = (float)lam;
  c.mu[k] = (float)mu;
  if (fs && j == 0) {
    const double d = lam + 2.0 * mu;
    c.cxx_x[k] = d > 0 ? (float)(4.0 * mu * (lam + mu) / d) : 0.0f;
    c.cxx_z[k] = c.czz_x[k] = c.czz_z[k] = 0.0f;
    c.smask[k] = 0.0f;
    c.dM_dl[i] = d > 0 ? (float)(4.0 * mu * mu / (d * d)) : 0.0f;
    c.dM_dm[i] = d > 0 ? (float)(4.0 * (lam * lam + 2.0 * lam * mu + 2.0 * mu * mu) / (d * d)) : 0.0f;
  } else {
    c.cxx_x[k] = c.czz_z[k] = (float)(lam + 2.0 * mu);
    c.cxx_z[k] = c.czz_x[k] = (float)lam;
    c.smask[k] = 1.0f;
  }
}

// buoyancies and the harmonic-mean shear modulus need neighbouring cells: a
// second pass over the padded grid (values re-read from the edge-replicated model)
__device__ __forceinline__ size_t el_model_index(int i, int j, int nx, int nz, int P, int top) {
  const int mi = min(max(i - P, 0), nx - 1), mj = min(max(j - top, 0), nz - 1);
  return (size_t)mj * nx + mi;
}

__global__ void el_prep2_kernel(const float* model, ElCoef c, int nx, int nz, int P, int top,
                                int NX, int NZ, int fluid) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= NX || j >= NZ) return;
  const size_t mn = (size_t)nx * nz;
  auto rho_at = [&](int ii, int jj) -> double {
    return el_rho(model, mn, el_model_index(ii, jj, nx, nz, P, top), fluid);
  };
  auto mu_at = [&](int ii, int jj) -> double {
    const size_t m = el_model_index(ii, jj, nx, nz, P, top);
    const double vs = el_vs(model, mn, m, fluid), rho = el_rho(model, mn, m, fluid);
    return rho * vs * vs;
  };
  const int i1 = min(i + 1, NX - 1), j1 = min(j + 1, NZ - 1);
  const size_t k = (size_t)j * NX + i;
  const double r0 = rho_at(i, j);
  c.bx[k] = (float)(2.0 / (r0 + rho_at(i1, j)));
  c.bz[k] = (float)(2.0 / (r0 + rho_at(i, j1)));
  const double m00 = mu_at(i, j), m10 = mu_at(i1, j), m01 = mu_at(i, j1), m11 = mu_at(i1, j1);
  c.mxz[k] = (m00 > 0 && m10 > 0 && m01 > 0 && m11 > 0)
                 ? (float)(4.0 / (1.0 / m00 + 1.0 / m10 + 1.0 / m01 + 1.0 / m11))
                 : 0.0f;
}

// C-PML coefficients at node x = i + shift of an axis of n cells with lo / hi pads
__device__ void el_pml(int i, double shift, int n, int lo, int hi, double h, double dt,
                       double vmax, double f0, double R, float* a, float* b) {
  const double x = i + shift;
  double xi = 0.0, L = 1.0;
  if (lo > 0 && x < lo) {
    xi = (lo - x) * h;
    L = lo * h;
  } else if (hi > 0 && x > n - 1 - hi) {
    xi = (x - (n - 1 - hi)) * h;
    L = hi * h;
  }
  if (xi > L) xi = L;
  const double d0 = -3.0 * vmax * log(R) / (2.0 * L);
  const double d = xi > 0.0 ? d0 * (xi / L) * (xi / L) : 0.0;
  const double alpha = M_PI * f0 * (1.0 - xi / L);
  const double bb = exp(-(d + alpha) * dt);
  b[i] = (float)bb;
  a[i] = d > 0.0 ? (float)(d / (d + alpha) * (bb - 1.0)) : 0.0f;
}

__global__ void el_tables_kernel(ElCoef c, int NX, int NZ, int P, int top, double h, double dt,
                                 double vmax, double f0, double R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NX) {
    el_pml(i, 0.0, NX, P, P, h, dt, vmax, f0, R, c.axi, c.bxi);
    el_pml(i, 0.5, NX, P, P, h, dt, vmax, f0, R, c.axh, c.bxh);
  }
  if (i < NZ) {
    el_pml(i, 0.0, NZ, top, P, h, dt, vmax, f0, R, c.azi, c.bzi);
    el_pml(i, 0.5, NZ, top, P, h, dt, vmax, f0, R, c.azh, c.bzh);
  }
}

// tot_q += sum over shots of the FP32 partial q (q = 0..4), float64
__global__ void el_fold_kernel(double* tot, const float* gpart, int nshots, size_t plane) {
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (c >= plane) return;
  double acc = tot[q * plane + c];
  for (int s = 0; s < nshots; ++s) acc += (double)gpart[((size_t)q * nshots + s) * plane + c];
  tot[q * plane + c] = acc;
}

// Chain rule on the padded grid for one padded cell:
//   lambda = rho (vp^2 - 2 vs^2), mu = rho vs^2; mu_xz = harmonic mean of 4 mu;
//   b = 2/(rho_a + rho_b). Returns (gvp, gvs, grho).
__device__ void el_chain_cell(const double* tot, size_t plane, const ElCoef& c, int i, int j,
                              int NX, int NZ, double* out) {
  const size_t q = (size_t)j * NX + i;
  double gl = tot[q], gm = tot[plane + q], gr = 0.0;
  const double muq = c.mu[q];
  // contributions of the txz nodes and buoyancy nodes whose stencil uses cell q
  for (int dj = -1; dj <= 0; ++dj)
    for (int di = -1; di <= 0; ++di) {
      const int ki = i + di, kj = j + dj;
      if (ki < 0 || kj < 0) continue;
      const int k1i = min(ki + 1, NX - 1), k1j = min(kj + 1, NZ - 1);
      const size_t k = (size_t)kj * NX + ki;
      // multiplicity of q among the four mu cells of txz node k
      const int mult = (ki == i && kj == j) + (k1i == i && kj == j) + (ki == i && k1j == j) +
                       (k1i == i && k1j == j);
      const double mxz = c.mxz[k];
      if (mult && mxz > 0.0 && muq > 0.0)
        gm += mult * tot[2 * plane + k] * mxz * mxz / (4.0 * muq * muq);
      // buoyancy bx at k uses rho at (ki, kj) and (k1i, kj); bz at (ki, kj), (ki, k1j)
      if (kj == j) {
        const int mb = (ki == i) + (k1i == i);
        const double b = c.bx[k];
        gr += mb * tot[3 * plane + k] * (-0.5 * b * b);
      }
      if (ki == i) {
        const int mb = (kj == j) + (k1j == j);
        const double b = c.bz[k];
        gr += mb * tot[4 * plane + k] * (-0.5 * b * b);
      }
    }
  const double vp = c.vp[q], vs = c.vs[q], rho = c.rho[q];
  out[0] = gl * 2.0 * rho * vp;
  out[1] = gl * (-4.0 * rho * vs) + gm * 2.0 * rho * vs;
  out[2] = gl * (vp * vp - 2.0 * vs * vs) + gm * vs * vs + gr;
}

__global__ void el_finish_kernel(const double* tot, ElCoef c, float* grad, int nx, int nz, int P,
                                 int top, int NX, int NZ, int fluid) {
  const int ii = blockIdx.x * blockDim.x + threadIdx.x;
  const int jj = blockIdx.y;
  if (ii >= nx || jj >= nz) return;
  const size_t plane = (size_t)NX * NZ;
  const int i0 = ii == 0 ? 0 : ii + P, i1 = ii == nx - 1 ? NX - 1 : ii + P;
  const int j0 = jj == 0 ? 0 : jj + top, j1 = jj == nz - 1 ? NZ - 1 : jj + top;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) {
      double o[3];
      el_chain_cell(tot, plane, c, i, j, NX, NZ, o);
      acc[0] += o[0];
      acc[1] += o[1];
      acc[2] += o[2];
    }
  const size_t mn = (size_t)nx * nz, m = (size_t)jj * nx + ii;
  grad[m] = (float)acc[0];
  if (fluid) {  // (vp, rho); the vs term vanishes at vs = 0
    grad[mn + m] = (float)acc[2];
  } else {
    grad[mn + m] = (float)acc[1];
    grad[2 * mn + m] = (float)acc[2];
  }
}

dim3 grid_of(const ElStep& a) {
  return dim3(((a.NX + kTX - 1) / kTX) * ((a.NZ + kElTZ - 1) / kElTZ) * a.nshots);
}

}  // namespace

int el_launch_prep(const float* model, const ElCoef& c, int nx, int nz, int P, int fs, int fluid,
                   double h, double dt, double vmax, double f0, double R, hipStream_t s) {
  const int top = fs ? 0 : P;
  const int NX = nx + 2 * P, NZ = nz + top + P;
  hipLaunchKernelGGL(el_prep_kernel, dim3((NX + 255) / 256, NZ), dim3(256), 0, s, model, c, nx,
                     nz, P, top, NX, NZ, fs, fluid);
  hipLaunchKernelGGL(el_prep2_kernel, dim3((NX + 255) / 256, NZ), dim3(256), 0, s, model, c, nx,
                     nz, P, top, NX, NZ, fluid);
  const int nmax = NX > NZ ? NX : NZ;
  hipLaunchKernelGGL(el_tables_kernel, dim3((nmax + 255) / 256), dim3(256), 0, s, c, NX, NZ, P,
                     top, h, dt, vmax, f0, R);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int el_launch_fwd(const ElStep& a, hipStream_t s, hipEvent_t* ev) {
  if (ev) SWEEP_HIP(hipEventRecord(ev[0], s));
  if (a.fluid)
    hipLaunchKernelGGL(el_vel_kernel<true>, grid_of(a), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(el_vel_kernel<false>, grid_of(a), dim3(256), 0, s, a);
  if (a.gathers && a.nrec > 0)
    hipLaunchKernelGGL(el_record_kernel, dim3((a.nshots * a.nrec + 255) / 256), dim3(256), 0, s,
                       a);
  if (a.fluid)
    hipLaunchKernelGGL(el_str_kernel<true>, grid_of(a), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(el_str_kernel<false>, grid_of(a), dim3(256), 0, s, a);
  if (ev) SWEEP_HIP(hipEventRecord(ev[1], s));
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int el_launch_adj(const ElStep& a, hipStream_t s, hipEvent_t* ev) {
  if (ev) SWEEP_HIP(hipEventRecord(ev[0], s));
  if (a.fluid)
    hipLaunchKernelGGL(el_adj_s_kernel<true>, grid_of(a), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(el_adj_s_kernel<false>, grid_of(a), dim3(256), 0, s, a);
  if (a.nrec > 0)
    hipLaunchKernelGGL(el_inject_kernel, dim3((a.nshots * a.nrec + 255) / 256), dim3(256), 0, s,
                       a, a.n);
  if (a.fluid)
    hipLaunchKernelGGL(el_adj_v_kernel<true>, grid_of(a), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(el_adj_v_kernel<false>, grid_of(a), dim3(256), 0, s, a);
  if (ev) SWEEP_HIP(hipEventRecord(ev[1], s));
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int el_launch_fold(double* tot, const float* gpart, int nshots, size_t plane, hipStream_t s) {
  hipLaunchKernelGGL(el_fold_kernel, dim3((unsigned)((plane + 255) / 256), 5), dim3(256), 0, s,
                     tot, gpart, nshots, plane);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int el_launch_finish(const double* tot, const ElCoef& c, float* grad, int nx, int nz, int P,
                     int fs, int fluid, hipStream_t s) {
  const int top = fs ? 0 : P;
  const int NX = nx + 2 * P, NZ = nz + top + P;
  hipLaunchKernelGGL(el_finish_kernel, dim3((nx + 255) / 256, nz), dim3(256), 0, s, tot, c, grad,
                     nx, nz, P, top, NX, NZ, fluid);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

}  // namespace sweep
