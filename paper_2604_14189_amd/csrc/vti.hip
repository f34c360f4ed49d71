// Pseudo-acoustic VTI step kernels for gfx950 (Sec. 3.3.1, Eq. 5): the
// acoustic scheme's 8th-order operators and per-axis C-PML with separate x and
// z coefficients, the auxiliary field G = F / dt^2 advanced by the same
// leapfrog, and the mixed term D2x' D2z' G; then the exact transpose for the
// adjoint. Scaled form and data layout: vti.h.
//
// One work-group of 256 lanes takes one 64 x 16 tile of one shot. It stages
// P^n (float64 in memory) as its float32 part hi and the bfloat16 rounding of
// the rest, lo, with an 8-cell halo, and G^n with a 4-cell halo in LDS (all
// global loads of a lane are issued before its first LDS store), computes the
// C-PML memory
// variables psi on a 4-cell ring only when a strip lies within 4 cells (a
// block-uniform test), D2z' G on the tile rows and a 4-column ring, and then
// each lane finishes its four cells from LDS. P^{n+1} and G^{n+1} overwrite
// P^{n-1} and G^{n-1} at the lane's own cells (each is read there only).
#include "fd.h"
#include "internal.h"
#include "vti.h"

namespace sweep {
namespace {

constexpr int kTZ = kVtiTZ;            // tile rows
constexpr int kRZ = kTZ / 4;           // rows per lane
constexpr int PW = kTX + 16;           // 8-cell-halo box: 80 x 32
constexpr int PH = kTZ + 16;
constexpr int GW = kTX + 8;            // 4-cell-halo box: 72 x 24
constexpr int GH = kTZ + 8;

__device__ __forceinline__ bool in_grid(int gx, int gz, int NX, int NZ) {
  return gx >= 0 && gx < NX && gz >= 0 && gz < NZ;
}

// Stage field f on the box [x0 - hx, x0 + 64 + hx) x [z0 - hz, z0 + 16 + hz)
// of W x H cells, zero outside the grid; all loads of a lane first, then its
// LDS stores.
template <int W, int H, class T>
__device__ __forceinline__ void stage(T* s, const T* __restrict__ f, int x0, int z0, int hx,
                                      int hz, int NX, int NZ) {
  constexpr int N = W * H;
  constexpr int K = (N + kThreads - 1) / kThreads;
  T v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * kThreads;
    const int r = e / W, c = e - r * W;
    const int gx = x0 - hx + c, gz = z0 - hz + r;
    const bool ok = e < N && in_grid(gx, gz, NX, NZ);
    v[k] = ok ? u32at(f, (unsigned)(gz * NX + gx)) : T(0);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * kThreads;
    if (e < N) s[e] = v[k];
  }
}

// P = hi + lo: hi = float(P), lo = P - hi rounded to bfloat16 (round to
// nearest even; lo is finite and far from the float range's ends).
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short b) {
  return __uint_as_float((unsigned)b << 16);
}

// Stage float64 field f as hi (float) and lo (bfloat16) boxes, as stage does.
template <int W, int H>
__device__ __forceinline__ void stage_split(float* hi, unsigned short* lo,
                                            const double* __restrict__ f, int x0, int z0, int hx,
                                            int hz, int NX, int NZ) {
  constexpr int N = W * H;
  constexpr int K = (N + kThreads - 1) / kThreads;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * kThreads;
    const int r = e / W, c = e - r * W;
    const int gx = x0 - hx + c, gz = z0 - hz + r;
    const bool ok = e < N && in_grid(gx, gz, NX, NZ);
    v[k] = ok ? u32at(f, (unsigned)(gz * NX + gx)) : 0.0;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * kThreads;
    if (e < N) {
      const float h = (float)v[k];
      hi[e] = h;
      lo[e] = bf16_bits((float)(v[k] - (double)h));
    }
  }
}

// D2' of P from the hi and lo boxes (both centred on the same cell): the two
// parts' second differences in float32, summed.
__device__ __forceinline__ float d2p(const float* hi, const unsigned short* lo, int st) {
  const float l = d2c(bf16_val(lo[0]), bf16_val(lo[st]), bf16_val(lo[-st]), bf16_val(lo[2 * st]),
                      bf16_val(lo[-2 * st]), bf16_val(lo[3 * st]), bf16_val(lo[-3 * st]),
                      bf16_val(lo[4 * st]), bf16_val(lo[-4 * st]));
  return d2s(hi, st) + l;
}

// 8th-order centred-difference second derivative in float64 (for G).
__device__ __forceinline__ double d2d(const double* f, int st) {
  const double c = f[0];
  double s = (8.0 / 5.0) * ((f[st] - c) + (f[-st] - c));
  s = fma(-1.0 / 5.0, (f[2 * st] - c) + (f[-2 * st] - c), s);
  s = fma(8.0 / 315.0, (f[3 * st] - c) + (f[-3 * st] - c), s);
  return fma(-1.0 / 560.0, (f[4 * st] - c) + (f[-4 * st] - c), s);
}

// Receivers of (shot, tile) record the staged values st[local] (64 x 16).
__device__ __forceinline__ void vti_record(const VtiStep& a, int shot, int tile,
                                           const float* st) {
  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  float* dst = a.gathers + ((size_t)shot * a.nt + a.n) * a.nrec;
  for (int e = ro[0] + (int)threadIdx.x; e < ro[1]; e += kThreads) {
    const int2 en = a.rec_ent[e];
    dst[en.y] = st[en.x];
  }
}

__global__ __launch_bounds__(kThreads) void vti_fwd_kernel(VtiStep a) {
  __shared__ float sP[PH * PW];            // P^n: hi, 8-cell halo
  __shared__ unsigned short sPl[PH * PW];  // and lo
  // G^n (float64, 4-cell halo); once each lane holds its cells' G^n and its
  // share of D2z' G^n (tile rows, 4-column ring) in registers, the same
  // memory holds that D2z' G^n
  __shared__ double sG[GH * GW];
  double* sT = sG;
  static_assert(kTZ * GW <= GH * GW, "D2z' G box fits in the G box");
  __shared__ float sX[kTZ * GW];  // psi_x^n on the tile rows, 4-column ring
  __shared__ float sZ[GH * kTX];  // psi_z^n on the tile columns, 4-row ring
  const int f = xcd_spread(blockIdx.x, gridDim.x);
  const int shot = f / a.n_pml, tile = a.tl[a.n_int + f - shot * a.n_pml];
  const int NX = a.NX, NZ = a.NZ, P = a.P, P2 = 2 * a.P;
  const size_t plane = (size_t)NX * NZ, base = (size_t)shot * plane;
  const int x0 = (tile % a.tiles_x) * kTX, z0 = (tile / a.tiles_x) * kTZ;
  const int tid = threadIdx.x, lx = tid & 63, zb = (tid >> 6) * kRZ;
  const bool hx = P > 0 && (x0 - 4 < P || x0 + kTX + 4 > NX - P);
  const bool hz = P > 0 && (z0 - 4 < P || z0 + kTZ + 4 > NZ - P);
  const int gx = x0 + lx;
  const int xcol = gx < NX ? xstrip_col(gx, NX, P) : -1;

  // own cells: P^n, old values, coefficients, zeta^{n-1}
  float ccx[kRZ], ccz[kRZ], ccm[kRZ], zx[kRZ], zz[kRZ];
  double pown[kRZ], pold[kRZ], gold[kRZ];
#pragma unroll
  for (int r = 0; r < kRZ; ++r) {
    const int gz = z0 + zb + r;
    const bool ok = gx < NX && gz < NZ;
    const unsigned idx = ok ? (unsigned)(gz * NX + gx) : 0u;
    pown[r] = ok ? u32at(a.pcur + base, idx) : 0.0;
    pold[r] = ok ? __builtin_nontemporal_load(&u32at(a.pprev + base, idx)) : 0.0;
    gold[r] = ok ? __builtin_nontemporal_load(&u32at(a.gprev + base, idx)) : 0.0;
    ccx[r] = ok ? u32at(a.cx, idx) : 0.0f;
    ccz[r] = ok ? u32at(a.cz, idx) : 0.0f;
    ccm[r] = ok ? u32at(a.cm, idx) : 0.0f;
    const int zrow = ok ? zstrip_row(gz, NZ, P) : -1;
    zx[r] = ok && xcol >= 0 ? u32at(a.zex_in + (size_t)shot * NZ * P2, (unsigned)(gz * P2 + xcol)) : 0.0f;
    zz[r] = zrow >= 0 ? u32at(a.zez_in + (size_t)shot * P2 * NX, (unsigned)(zrow * NX + gx)) : 0.0f;
  }
  stage_split<PW, PH>(sP, sPl, a.pcur + base, x0, z0, 8, 8, NX, NZ);
  stage<GW, GH>(sG, a.gcur + base, x0, z0, 4, 4, NX, NZ);
  __syncthreads();

  // psi^n = b psi^{n-1} + a D1' P^n on the rings (zero outside the strips)
  if (hx) {
    for (int e = tid; e < kTZ * GW; e += kThreads) {
      const int r = e / GW, c = e - r * GW;
      const int x = x0 - 4 + c, z = z0 + r;
      const int col = in_grid(x, z, NX, NZ) ? xstrip_col(x, NX, P) : -1;
      float psi = 0.0f;
      if (col >= 0) {
        const unsigned si = (unsigned)(z * P2 + col);
        psi = fmaf(a.bx[x], u32at(a.psx_in + (size_t)shot * NZ * P2, si), a.ax[x] * d1s(&sP[(r + 8) * PW + c + 4], 1));
        if (c >= 4 && c < 4 + kTX) u32at(a.psx_out + (size_t)shot * NZ * P2, si) = psi;
      }
      sX[e] = psi;
    }
  }
  if (hz) {
    for (int e = tid; e < GH * kTX; e += kThreads) {
      const int r = e / kTX, c = e - r * kTX;
      const int x = x0 + c, z = z0 - 4 + r;
      const int row = in_grid(x, z, NX, NZ) ? zstrip_row(z, NZ, P) : -1;
      float psi = 0.0f;
      if (row >= 0) {
        const unsigned si = (unsigned)(row * NX + x);
        psi = fmaf(a.bz[z], u32at(a.psz_in + (size_t)shot * P2 * NX, si), a.az[z] * d1s(&sP[(r + 4) * PW + c + 8], PW));
        if (r >= 4 && r < 4 + kTZ) u32at(a.psz_out + (size_t)shot * P2 * NX, si) = psi;
      }
      sZ[e] = psi;
    }
  }
  constexpr int KT = (kTZ * GW + kThreads - 1) / kThreads;
  double tz[KT], g0[kRZ];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int e = tid + k * kThreads, r = e / GW, c = e - r * GW;
    tz[k] = e < kTZ * GW ? d2d(&sG[(r + 4) * GW + c], GW) : 0.0;
  }
#pragma unroll
  for (int rr = 0; rr < kRZ; ++rr) g0[rr] = sG[(zb + rr + 4) * GW + lx + 4];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int e = tid + k * kThreads;
    if (e < kTZ * GW) sT[e] = tz[k];
  }
  __syncthreads();

  const int src = a.src_cell[shot];
  const float sw = a.w * a.wavelet[(size_t)shot * a.nt + a.n];
  float out[kRZ];
#pragma unroll
  for (int rr = 0; rr < kRZ; ++rr) {
    const int r = zb + rr, gz = z0 + r;
    const bool ok = gx < NX && gz < NZ;
    const unsigned idx = ok ? (unsigned)(gz * NX + gx) : 0u;
    const int pe = (r + 8) * PW + lx + 8;
    float qx = d2p(&sP[pe], &sPl[pe], 1), qz = d2p(&sP[pe], &sPl[pe], PW);
    if (hx) qx += d1s(&sX[r * GW + lx + 4], 1);
    if (hz) qz += d1s(&sZ[(r + 4) * kTX + lx], kTX);
    float bxv = qx, bzv = qz;
    if (ok && xcol >= 0) {
      const float zn = fmaf(a.bx[gx], zx[rr], a.ax[gx] * qx);
      u32at(a.zex_out + (size_t)shot * NZ * P2, (unsigned)(gz * P2 + xcol)) = zn;
      bxv = qx + zn;
    }
    const int zrow = ok ? zstrip_row(gz, NZ, P) : -1;
    if (zrow >= 0) {
      const float zn = fmaf(a.bz[gz], zz[rr], a.az[gz] * qz);
      u32at(a.zez_out + (size_t)shot * P2 * NX, (unsigned)(zrow * NX + gx)) = zn;
      bzv = qz + zn;
    }
    const float m = (float)d2d(&sT[r * GW + lx + 4], 1);
    const double p0 = pown[rr];
    double pn = 2.0 * p0 - pold[rr];
    pn = fma((double)ccx[rr], (double)bxv, pn);
    pn = fma((double)ccz[rr], (double)bzv, pn);
    pn = fma(-(double)ccm[rr], (double)m, pn);
    if (ok && (int)idx == src) pn += (double)sw;
    const double gn = (2.0 * g0[rr] - gold[rr]) + p0;
    out[rr] = (float)pn;
    if (ok) {
      __builtin_nontemporal_store(pn, &u32at(a.pprev + base, idx));
      __builtin_nontemporal_store(gn, &u32at(a.gprev + base, idx));
      if (a.tr[0]) {
        st_nt(&u32at(a.tr[0] + base, idx), bxv);
        st_nt(&u32at(a.tr[1] + base, idx), bzv);
        st_nt(&u32at(a.tr[2] + base, idx), m);
      }
    }
  }
  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  if (a.gathers && ro[1] > ro[0]) {
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < kRZ; ++rr) sP[(zb + rr) * kTX + lx] = out[rr];
    __syncthreads();
    vti_record(a, shot, tile, sP);
  }
}

// Reverse of step n (exact transpose of the forward kernel). With
// lambda^{n+1} = P1: qx = cx P1, Qbar_x = qx + a_x (Z_x + qx) in the x strip
// (qx elsewhere) on the tile rows and an 8-column ring; psbar_x = Psi_x -
// D1x' Qbar_x and T_x = a_x psbar_x on a 4-column ring; z likewise with cz;
//   lambda^n = 2 P1 - lambda^{n+2} + D2x' Qbar_x + D2z' Qbar_z - D1x' T_x - D1z' T_z + mu^{n+1},
//   mu^n     = 2 mu^{n+1} - mu^{n+2} - D2x' D2z' (cm P1),
// Psi = b psbar, Z = b (Z + q); g += P1 (Bx', Bz', -D2x'D2z'G^n); then r_{n-1}
// is added at the receivers.
__global__ __launch_bounds__(kThreads) void vti_adj_kernel(VtiStep a) {
  // lambda^{n+1} with an 8-cell halo; once the products are formed, the same
  // memory holds D2z'(cm lambda^{n+1}) (float64, tile rows, 4-column ring),
  // and at the end the staging of lambda^n for the residual injection
  __shared__ __align__(16) float sL[PH * PW];
  __shared__ float sQx[kTZ * PW];  // Qbar_x on the tile rows, 8-column ring
  __shared__ float sQz[PH * kTX];  // Qbar_z on the tile columns, 8-row ring
  __shared__ double sM[GH * GW];   // cm lambda^{n+1} (float64), 4-cell halo
  double* sU = reinterpret_cast<double*>(sL);
  static_assert(kTZ * GW * sizeof(double) <= PH * PW * sizeof(float), "sU fits in sL");
  __shared__ float sTx[kTZ * GW];  // T_x on the tile rows, 4-column ring
  __shared__ float sTz[GH * kTX];  // T_z on the tile columns, 4-row ring
  const int f = xcd_spread(blockIdx.x, gridDim.x);
  const int shot = f / a.n_pml, tile = a.tl[a.n_int + f - shot * a.n_pml];
  const int NX = a.NX, NZ = a.NZ, P = a.P, P2 = 2 * a.P;
  const size_t plane = (size_t)NX * NZ, base = (size_t)shot * plane;
  const int x0 = (tile % a.tiles_x) * kTX, z0 = (tile / a.tiles_x) * kTZ;
  const int tid = threadIdx.x, lx = tid & 63, zb = (tid >> 6) * kRZ;
  const bool hx = P > 0 && (x0 - 4 < P || x0 + kTX + 4 > NX - P);
  const bool hz = P > 0 && (z0 - 4 < P || z0 + kTZ + 4 > NZ - P);
  const int gx = x0 + lx;
  const int xcol = gx < NX ? xstrip_col(gx, NX, P) : -1;

  float l2[kRZ], ccx[kRZ], ccz[kRZ], zx[kRZ], zz[kRZ], t0[kRZ], t1[kRZ], t2[kRZ];
  double m1[kRZ], m2[kRZ];
#pragma unroll
  for (int r = 0; r < kRZ; ++r) {
    const int gz = z0 + zb + r;
    const bool ok = gx < NX && gz < NZ;
    const unsigned idx = ok ? (unsigned)(gz * NX + gx) : 0u;
    l2[r] = ok ? ld_nt(&u32at(a.prev + base, idx)) : 0.0f;
    m1[r] = ok ? u32at(a.mcur + base, idx) : 0.0;
    m2[r] = ok ? __builtin_nontemporal_load(&u32at(a.mprev + base, idx)) : 0.0;
    ccx[r] = ok ? u32at(a.cx, idx) : 0.0f;
    ccz[r] = ok ? u32at(a.cz, idx) : 0.0f;
    t0[r] = ok ? ld_nt(&u32at(a.trc[0] + base, idx)) : 0.0f;
    t1[r] = ok ? ld_nt(&u32at(a.trc[1] + base, idx)) : 0.0f;
    t2[r] = ok ? ld_nt(&u32at(a.trc[2] + base, idx)) : 0.0f;
    const int zrow = ok ? zstrip_row(gz, NZ, P) : -1;
    zx[r] = ok && xcol >= 0 ? u32at(a.zex_in + (size_t)shot * NZ * P2, (unsigned)(gz * P2 + xcol)) : 0.0f;
    zz[r] = zrow >= 0 ? u32at(a.zez_in + (size_t)shot * P2 * NX, (unsigned)(zrow * NX + gx)) : 0.0f;
  }
  // the coefficients of the three product boxes (and, in tiles near a strip,
  // the zeta adjoints there) are loaded with the lambda box, before any LDS
  // store, so a lane keeps all its loads in flight together
  constexpr int NQX = kTZ * PW, KQX = (NQX + kThreads - 1) / kThreads;
  constexpr int NQZ = PH * kTX, KQZ = (NQZ + kThreads - 1) / kThreads;
  constexpr int NM = GH * GW, KM = (NM + kThreads - 1) / kThreads;
  float vcx[KQX], vzx[KQX], vcz[KQZ], vzz[KQZ], vcm[KM];
#pragma unroll
  for (int k = 0; k < KQX; ++k) {
    const int e = tid + k * kThreads, r = e / PW, c = e - r * PW;
    const int x = x0 - 8 + c, z = z0 + r;
    const bool ok = e < NQX && in_grid(x, z, NX, NZ);
    vcx[k] = ok ? u32at(a.cx, (unsigned)(z * NX + x)) : 0.0f;
    const int col = ok && hx ? xstrip_col(x, NX, P) : -1;
    vzx[k] = col >= 0 ? u32at(a.zex_in + (size_t)shot * NZ * P2, (unsigned)(z * P2 + col)) : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < KQZ; ++k) {
    const int e = tid + k * kThreads, r = e / kTX, c = e - r * kTX;
    const int x = x0 + c, z = z0 - 8 + r;
    const bool ok = e < NQZ && in_grid(x, z, NX, NZ);
    vcz[k] = ok ? u32at(a.cz, (unsigned)(z * NX + x)) : 0.0f;
    const int row = ok && hz ? zstrip_row(z, NZ, P) : -1;
    vzz[k] = row >= 0 ? u32at(a.zez_in + (size_t)shot * P2 * NX, (unsigned)(row * NX + x)) : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    const int e = tid + k * kThreads, r = e / GW, c = e - r * GW;
    const int x = x0 - 4 + c, z = z0 - 4 + r;
    vcm[k] = e < NM && in_grid(x, z, NX, NZ) ? u32at(a.cm, (unsigned)(z * NX + x)) : 0.0f;
  }
  stage<PW, PH>(sL, a.cur + base, x0, z0, 8, 8, NX, NZ);
  __syncthreads();
  float l1v[kRZ];
#pragma unroll
  for (int rr = 0; rr < kRZ; ++rr) l1v[rr] = sL[(zb + rr + 8) * PW + lx + 8];

  // products with the coefficients, and the x / z memory terms of Qbar
  // (outside the grid every operand is 0)
#pragma unroll
  for (int k = 0; k < KQX; ++k) {
    const int e = tid + k * kThreads, r = e / PW, c = e - r * PW;
    if (e >= NQX) break;
    const float q = vcx[k] * sL[(r + 8) * PW + c];
    const int x = x0 - 8 + c;
    const int col = hx && x >= 0 && x < NX ? xstrip_col(x, NX, P) : -1;
    sQx[e] = col >= 0 ? q + a.ax[x] * (vzx[k] + q) : q;
  }
#pragma unroll
  for (int k = 0; k < KQZ; ++k) {
    const int e = tid + k * kThreads, r = e / kTX, c = e - r * kTX;
    if (e >= NQZ) break;
    const float q = vcz[k] * sL[r * PW + c + 8];
    const int z = z0 - 8 + r;
    const int row = hz && z >= 0 && z < NZ ? zstrip_row(z, NZ, P) : -1;
    sQz[e] = row >= 0 ? q + a.az[z] * (vzz[k] + q) : q;
  }
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    const int e = tid + k * kThreads, r = e / GW, c = e - r * GW;
    if (e >= NM) break;
    sM[e] = (double)vcm[k] * (double)sL[(r + 4) * PW + c + 4];
  }
  __syncthreads();

  if (hx) {
    for (int e = tid; e < kTZ * GW; e += kThreads) {
      const int r = e / GW, c = e - r * GW;
      const int x = x0 - 4 + c, z = z0 + r;
      const int col = in_grid(x, z, NX, NZ) ? xstrip_col(x, NX, P) : -1;
      float t = 0.0f;
      if (col >= 0) {
        const unsigned si = (unsigned)(z * P2 + col);
        const float psb = u32at(a.psx_in + (size_t)shot * NZ * P2, si) - d1s(&sQx[r * PW + c + 4], 1);
        t = a.ax[x] * psb;
        if (c >= 4 && c < 4 + kTX) u32at(a.psx_out + (size_t)shot * NZ * P2, si) = a.bx[x] * psb;
      }
      sTx[e] = t;
    }
  }
  if (hz) {
    for (int e = tid; e < GH * kTX; e += kThreads) {
      const int r = e / kTX, c = e - r * kTX;
      const int x = x0 + c, z = z0 - 4 + r;
      const int row = in_grid(x, z, NX, NZ) ? zstrip_row(z, NZ, P) : -1;
      float t = 0.0f;
      if (row >= 0) {
        const unsigned si = (unsigned)(row * NX + x);
        const float psb = u32at(a.psz_in + (size_t)shot * P2 * NX, si) - d1s(&sQz[(r + 4) * kTX + c], kTX);
        t = a.az[z] * psb;
        if (r >= 4 && r < 4 + kTZ) u32at(a.psz_out + (size_t)shot * P2 * NX, si) = a.bz[z] * psb;
      }
      sTz[e] = t;
    }
  }
  for (int e = tid; e < kTZ * GW; e += kThreads) {
    const int r = e / GW, c = e - r * GW;
    sU[e] = d2d(&sM[(r + 4) * GW + c], GW);
  }
  __syncthreads();

  float out[kRZ];
#pragma unroll
  for (int rr = 0; rr < kRZ; ++rr) {
    const int r = zb + rr, gz = z0 + r;
    const bool ok = gx < NX && gz < NZ;
    const unsigned idx = ok ? (unsigned)(gz * NX + gx) : 0u;
    const float l1 = l1v[rr];
    float lam = 2.0f * l1 - l2[rr];
    lam += d2s(&sQx[r * PW + lx + 8], 1);
    lam += d2s(&sQz[(r + 8) * kTX + lx], kTX);
    if (hx) lam -= d1s(&sTx[r * GW + lx + 4], 1);
    if (hz) lam -= d1s(&sTz[(r + 4) * kTX + lx], kTX);
    lam += (float)m1[rr];
    const double mu = (2.0 * m1[rr] - m2[rr]) - d2d(&sU[r * GW + lx + 4], 1);
    out[rr] = lam;
    if (!ok) continue;
    if (xcol >= 0)
      u32at(a.zex_out + (size_t)shot * NZ * P2, (unsigned)(gz * P2 + xcol)) = a.bx[gx] * (zx[rr] + ccx[rr] * l1);
    const int zrow = zstrip_row(gz, NZ, P);
    if (zrow >= 0)
      u32at(a.zez_out + (size_t)shot * P2 * NX, (unsigned)(zrow * NX + gx)) = a.bz[gz] * (zz[rr] + ccz[rr] * l1);
    __builtin_nontemporal_store(mu, &u32at(a.mprev + base, idx));
    float* g0 = &u32at(a.g + base, idx);
    float* g1 = &u32at(a.g + base + (size_t)a.nshots * plane, idx);
    float* g2 = &u32at(a.g + base + 2 * (size_t)a.nshots * plane, idx);
    if (a.g_init) {
      st_nt(g0, l1 * t0[rr]);
      st_nt(g1, l1 * t1[rr]);
      st_nt(g2, -(l1 * t2[rr]));
    } else {
      st_nt(g0, fmaf(l1, t0[rr], ld_nt(g0)));
      st_nt(g1, fmaf(l1, t1[rr], ld_nt(g1)));
      st_nt(g2, ld_nt(g2) - l1 * t2[rr]);
    }
  }
  // r_{n-1} at the receivers of this (shot, tile), coincident receivers in
  // receiver order, then lambda^n
  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  if (a.resid && a.n >= 1 && ro[1] > ro[0]) {
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < kRZ; ++rr) sL[(zb + rr) * kTX + lx] = out[rr];
    __syncthreads();
    const int e0 = ro[0], e1 = ro[1];
    const float* rv = a.resid + ((size_t)shot * a.nt + (a.n - 1)) * a.nrec;
    for (int e = e0 + tid; e < e1; e += kThreads) {
      const int2 en = a.rec_ent[e];
      if (e == e0 || a.rec_ent[e - 1].x != en.x) {
        float acc = sL[en.x];
        for (int k = e; k < e1 && a.rec_ent[k].x == en.x; ++k) acc += rv[a.rec_ent[k].y];
        sL[en.x] = acc;
      }
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < kRZ; ++rr) out[rr] = sL[(zb + rr) * kTX + lx];
  }
#pragma unroll
  for (int rr = 0; rr < kRZ; ++rr) {
    const int gz = z0 + zb + rr;
    if (gx < NX && gz < NZ) st_nt(&u32at(a.prev + base, (unsigned)(gz * NX + gx)), out[rr]);
  }
}

// Interior tiles: no C-PML strip within 4 cells, so every memory-variable
// term of the general kernels is an exact zero there and the rings that carry
// them are not needed. The same operations on the same values (so the same
// bits), with P^n staged with a 4-cell halo: about half the LDS of the
// general kernels and fewer registers, for more work-groups per CU.
__global__ __launch_bounds__(kThreads) void vti_fwd_int_kernel(VtiStep a) {
  __shared__ float sP[GH * GW];            // P^n: hi, 4-cell halo
  __shared__ unsigned short sPl[GH * GW];  // and lo
  // G^n (float64, 4-cell halo), then D2z' G^n (tile rows, 4-column ring)
  __shared__ double sG[GH * GW];
  double* sT = sG;
  const int f = xcd_spread(blockIdx.x, gridDim.x);
  const int shot = f / a.n_int, tile = a.tl[f - shot * a.n_int];
  const int NX = a.NX, NZ = a.NZ;
  const size_t plane = (size_t)NX * NZ, base = (size_t)shot * plane;
  const int x0 = (tile % a.tiles_x) * kTX, z0 = (tile / a.tiles_x) * kTZ;
  const int tid = threadIdx.x, lx = tid & 63, zb = (tid >> 6) * kRZ;
  const int gx = x0 + lx;

  float ccx[kRZ], ccz[kRZ], ccm[kRZ];
  double pown[kRZ], pold[kRZ], gold[kRZ];
#pragma unroll
  for (int r = 0; r < kRZ; ++r) {
    const int gz = z0 + zb + r;
    const bool ok = gx < NX && gz < NZ;
    const unsigned idx = ok ? (unsigned)(gz * NX + gx) : 0u;
    pown[r] = ok ? u32at(a.pcur + base, idx) : 0.0;
    pold[r] = ok ? __builtin_nontemporal_load(&u32at(a.pprev + base, idx)) : 0.0;
    gold[r] = ok ? __builtin_nontemporal_load(&u32at(a.gprev + base, idx)) : 0.0;
    ccx[r] = ok ? u32at(a.cx, idx) : 0.0f;
    ccz[r] = ok ? u32at(a.cz, idx) : 0.0f;
    ccm[r] = ok ? u32at(a.cm, idx) : 0.0f;
  }
  stage_split<GW, GH>(sP, sPl, a.pcur + base, x0, z0, 4, 4, NX, NZ);
  stage<GW, GH>(sG, a.gcur + base, x0, z0, 4, 4, NX, NZ);
  __syncthreads();
  constexpr int KT = (kTZ * GW + kThreads - 1) / kThreads;
  double tz[KT], g0[kRZ];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int e = tid + k * kThreads, r = e / GW, c = e - r * GW;
    tz[k] = e < kTZ * GW ? d2d(&sG[(r + 4) * GW + c], GW) : 0.0;
  }
#pragma unroll
  for (int rr = 0; rr < kRZ; ++rr) g0[rr] = sG[(zb + rr + 4) * GW + lx + 4];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int e = tid + k * kThreads;
    if (e < kTZ * GW) sT[e] = tz[k];
  }
  __syncthreads();

  const int src = a.src_cell[shot];
  const float sw = a.w * a.wavelet[(size_t)shot * a.nt + a.n];
  float out[kRZ];
#pragma unroll
  for (int rr = 0; rr < kRZ; ++rr) {
    const int r = zb + rr, gz = z0 + r;
    const bool ok = gx < NX && gz < NZ;
    const unsigned idx = ok ? (unsigned)(gz * NX + gx) : 0u;
    const int pe = (r + 4) * GW + lx + 4;
    const float bxv = d2p(&sP[pe], &sPl[pe], 1), bzv = d2p(&sP[pe], &sPl[pe], GW);
    const float m = (float)d2d(&sT[r * GW + lx + 4], 1);
    const double p0 = pown[rr];
    double pn = 2.0 * p0 - pold[rr];
    pn = fma((double)ccx[rr], (double)bxv, pn);
    pn = fma((double)ccz[rr], (double)bzv, pn);
    pn = fma(-(double)ccm[rr], (double)m, pn);
    if (ok && (int)idx == src) pn += (double)sw;
    const double gn = (2.0 * g0[rr] - gold[rr]) + p0;
    out[rr] = (float)pn;
    if (ok) {
      __builtin_nontemporal_store(pn, &u32at(a.pprev + base, idx));
      __builtin_nontemporal_store(gn, &u32at(a.gprev + base, idx));
      if (a.tr[0]) {
        st_nt(&u32at(a.tr[0] + base, idx), bxv);
        st_nt(&u32at(a.tr[1] + base, idx), bzv);
        st_nt(&u32at(a.tr[2] + base, idx), m);
      }
    }
  }
  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  if (a.gathers && ro[1] > ro[0]) {
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < kRZ; ++rr) sP[(zb + rr) * kTX + lx] = out[rr];
    __syncthreads();
    vti_record(a, shot, tile, sP);
  }
}

__global__ __launch_bounds__(kThreads) void vti_adj_int_kernel(VtiStep a) {
  __shared__ float sQx[kTZ * GW];  // cx lambda^{n+1} on the tile rows, 4-column ring
  __shared__ float sQz[GH * kTX];  // cz lambda^{n+1} on the tile columns, 4-row ring
  // cm lambda^{n+1} (float64, 4-cell halo), then D2z'(cm lambda^{n+1}) (tile
  // rows, 4-column ring)
  __shared__ double sM[GH * GW];
  double* sU = sM;
  const int f = xcd_spread(blockIdx.x, gridDim.x);
  const int shot = f / a.n_int, tile = a.tl[f - shot * a.n_int];
  const int NX = a.NX, NZ = a.NZ;
  const size_t plane = (size_t)NX * NZ, base = (size_t)shot * plane;
  const int x0 = (tile % a.tiles_x) * kTX, z0 = (tile / a.tiles_x) * kTZ;
  const int tid = threadIdx.x, lx = tid & 63, zb = (tid >> 6) * kRZ;
  const int gx = x0 + lx;

  // the lambda^{n+1} box and its coefficients, then the own cells' operands,
  // all before the first LDS store
  constexpr int NB = GH * GW, KB = (NB + kThreads - 1) / kThreads;
  float bl[KB], bcx[KB], bcz[KB], bcm[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int e = tid + k * kThreads, r = e / GW, c = e - r * GW;
    const int x = x0 - 4 + c, z = z0 - 4 + r;
    const bool ok = e < NB && in_grid(x, z, NX, NZ);
    const unsigned idx = ok ? (unsigned)(z * NX + x) : 0u;
    bl[k] = ok ? u32at(a.cur + base, idx) : 0.0f;
    bcx[k] = ok ? u32at(a.cx, idx) : 0.0f;
    bcz[k] = ok ? u32at(a.cz, idx) : 0.0f;
    bcm[k] = ok ? u32at(a.cm, idx) : 0.0f;
  }
  float l1v[kRZ], l2[kRZ], t0[kRZ], t1[kRZ], t2[kRZ];
  double m1[kRZ], m2[kRZ];
#pragma unroll
  for (int r = 0; r < kRZ; ++r) {
    const int gz = z0 + zb + r;
    const bool ok = gx < NX && gz < NZ;
    const unsigned idx = ok ? (unsigned)(gz * NX + gx) : 0u;
    l1v[r] = ok ? u32at(a.cur + base, idx) : 0.0f;
    l2[r] = ok ? ld_nt(&u32at(a.prev + base, idx)) : 0.0f;
    m1[r] = ok ? u32at(a.mcur + base, idx) : 0.0;
    m2[r] = ok ? __builtin_nontemporal_load(&u32at(a.mprev + base, idx)) : 0.0;
    t0[r] = ok ? ld_nt(&u32at(a.trc[0] + base, idx)) : 0.0f;
    t1[r] = ok ? ld_nt(&u32at(a.trc[1] + base, idx)) : 0.0f;
    t2[r] = ok ? ld_nt(&u32at(a.trc[2] + base, idx)) : 0.0f;
  }
  // products (outside the grid every operand is 0)
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int e = tid + k * kThreads, r = e / GW, c = e - r * GW;
    if (e >= NB) break;
    if (r >= 4 && r < 4 + kTZ) sQx[(r - 4) * GW + c] = bcx[k] * bl[k];
    if (c >= 4 && c < 4 + kTX) sQz[r * kTX + c - 4] = bcz[k] * bl[k];
    sM[e] = (double)bcm[k] * (double)bl[k];
  }
  __syncthreads();
  constexpr int KT = (kTZ * GW + kThreads - 1) / kThreads;
  double tu[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int e = tid + k * kThreads, r = e / GW, c = e - r * GW;
    tu[k] = e < kTZ * GW ? d2d(&sM[(r + 4) * GW + c], GW) : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int e = tid + k * kThreads;
    if (e < kTZ * GW) sU[e] = tu[k];
  }
  __syncthreads();

  float out[kRZ];
#pragma unroll
  for (int rr = 0; rr < kRZ; ++rr) {
    const int r = zb + rr, gz = z0 + r;
    const bool ok = gx < NX && gz < NZ;
    const unsigned idx = ok ? (unsigned)(gz * NX + gx) : 0u;
    const float l1 = l1v[rr];
    float lam = 2.0f * l1 - l2[rr];
    lam += d2s(&sQx[r * GW + lx + 4], 1);
    lam += d2s(&sQz[(r + 4) * kTX + lx], kTX);
    lam += (float)m1[rr];
    const double mu = (2.0 * m1[rr] - m2[rr]) - d2d(&sU[r * GW + lx + 4], 1);
    out[rr] = lam;
    if (!ok) continue;
    __builtin_nontemporal_store(mu, &u32at(a.mprev + base, idx));
    float* g0 = &u32at(a.g + base, idx);
    float* g1 = &u32at(a.g + base + (size_t)a.nshots * plane, idx);
    float* g2 = &u32at(a.g + base + 2 * (size_t)a.nshots * plane, idx);
    if (a.g_init) {
      st_nt(g0, l1 * t0[rr]);
      st_nt(g1, l1 * t1[rr]);
      st_nt(g2, -(l1 * t2[rr]));
    } else {
      st_nt(g0, fmaf(l1, t0[rr], ld_nt(g0)));
      st_nt(g1, fmaf(l1, t1[rr], ld_nt(g1)));
      st_nt(g2, ld_nt(g2) - l1 * t2[rr]);
    }
  }
  // r_{n-1} at the receivers of this (shot, tile), as in vti_adj_kernel
  const int* ro = a.rec_off + (size_t)shot * a.ntiles + tile;
  if (a.resid && a.n >= 1 && ro[1] > ro[0]) {
    __syncthreads();
    float* st = sQz;
#pragma unroll
    for (int rr = 0; rr < kRZ; ++rr) st[(zb + rr) * kTX + lx] = out[rr];
    __syncthreads();
    const int e0 = ro[0], e1 = ro[1];
    const float* rv = a.resid + ((size_t)shot * a.nt + (a.n - 1)) * a.nrec;
    for (int e = e0 + tid; e < e1; e += kThreads) {
      const int2 en = a.rec_ent[e];
      if (e == e0 || a.rec_ent[e - 1].x != en.x) {
        float acc = st[en.x];
        for (int k = e; k < e1 && a.rec_ent[k].x == en.x; ++k) acc += rv[a.rec_ent[k].y];
        st[en.x] = acc;
      }
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < kRZ; ++rr) out[rr] = st[(zb + rr) * kTX + lx];
  }
#pragma unroll
  for (int rr = 0; rr < kRZ; ++rr) {
    const int gz = z0 + zb + rr;
    if (gx < NX && gz < NZ) st_nt(&u32at(a.prev + base, (unsigned)(gz * NX + gx)), out[rr]);
  }
}

// Padded model (vv, v, eta; eta = 0 in the pad) and the coefficients, from
// model [3][nz][nx] = (vv, v, eta); r = dt / h.
__global__ void vti_prep_kernel(const float* __restrict__ model, float* __restrict__ pad,
                                float* __restrict__ cx, float* __restrict__ cz,
                                float* __restrict__ cm, int nx, int nz, int P, double r) {
  const int NX = nx + 2 * P, NZ = nz + 2 * P;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= NX || j >= NZ) return;
  const int ii = min(max(i - P, 0), nx - 1), jj = min(max(j - P, 0), nz - 1);
  const bool in_model = ii == i - P && jj == j - P;
  const size_t m = (size_t)jj * nx + ii, mn = (size_t)nx * nz, k = (size_t)j * NX + i;
  const size_t plane = (size_t)NX * NZ;
  const double vv = model[m], vn = model[mn + m], eta = in_model ? (double)model[2 * mn + m] : 0.0;
  pad[k] = (float)vv;
  pad[plane + k] = (float)vn;
  pad[2 * plane + k] = (float)eta;
  const double ax = vn * r, az = vv * r;
  cx[k] = (float)((1.0 + 2.0 * eta) * ax * ax);
  cz[k] = (float)(az * az);
  cm[k] = (float)(2.0 * eta * ax * ax * az * az);
}

__global__ void vti_fold_kernel(double* tot, const float* __restrict__ gpart, int nshots,
                                size_t plane) {
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (c >= plane) return;
  double acc = tot[q * plane + c];
  const float* gq = gpart + (size_t)q * nshots * plane;
  for (int s = 0; s < nshots; ++s) acc += (double)gq[s * plane + c];
  tot[q * plane + c] = acc;
}

// dJ/d(vv, v, eta) of model cell (ii, jj): the chain rule through (cx, cz, cm),
// summed over the padded cells that replicate the cell (vv and v); eta only at
// the cell itself (the pad holds eta = 0, which depends on no model value).
__global__ void vti_finish_kernel(const double* tot, const float* pad, float* grad, int nx,
                                  int nz, int P, double r) {
  const int ii = blockIdx.x * blockDim.x + threadIdx.x;
  const int jj = blockIdx.y;
  if (ii >= nx || jj >= nz) return;
  const int NX = nx + 2 * P, NZ = nz + 2 * P;
  const size_t plane = (size_t)NX * NZ, mn = (size_t)nx * nz;
  const int i0 = ii == 0 ? 0 : ii + P, i1 = ii == nx - 1 ? NX - 1 : ii + P;
  const int j0 = jj == 0 ? 0 : jj + P, j1 = jj == nz - 1 ? NZ - 1 : jj + P;
  const double r2 = r * r, r4 = r2 * r2;
  double gvv = 0.0, gvn = 0.0, geta = 0.0;
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) {
      const size_t c = (size_t)j * NX + i;
      const double vv = pad[c], vn = pad[plane + c], eta = pad[2 * plane + c];
      const double gx = tot[c], gz = tot[plane + c], gm = tot[2 * plane + c];
      gvv += gz * 2.0 * vv * r2 + gm * 4.0 * eta * vn * vn * vv * r4;
      gvn += gx * 2.0 * (1.0 + 2.0 * eta) * vn * r2 + gm * 4.0 * eta * vn * vv * vv * r4;
      if (i == ii + P && j == jj + P) geta += gx * 2.0 * vn * vn * r2 + gm * 2.0 * vn * vn * vv * vv * r4;
    }
  const size_t m = (size_t)jj * nx + ii;
  grad[m] = (float)gvv;
  grad[mn + m] = (float)gvn;
  grad[2 * mn + m] = (float)geta;
}

}  // namespace

int vti_launch_prep(const float* model, float* pad, float* cx, float* cz, float* cm, int nx,
                    int nz, int P, double h, double dt, hipStream_t s) {
  const int NX = nx + 2 * P, NZ = nz + 2 * P;
  hipLaunchKernelGGL(vti_prep_kernel, dim3((NX + 255) / 256, NZ), dim3(256), 0, s, model, pad, cx,
                     cz, cm, nx, nz, P, dt / h);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

bool vti_near_strip(int x0, int z0, int NX, int NZ, int P) {
  return P > 0 && (x0 - 4 < P || x0 + kTX + 4 > NX - P || z0 - 4 < P || z0 + kTZ + 4 > NZ - P);
}

// Within a step every tile reads only the current level around it and writes
// its own cells of the other buffers, so the two tile sets may run in either
// order.
int vti_launch_fwd(const VtiStep& a, hipStream_t s) {
  if (a.n_int > 0)
    hipLaunchKernelGGL(vti_fwd_int_kernel, dim3(a.n_int * a.nshots), dim3(kThreads), 0, s, a);
  if (a.n_pml > 0)
    hipLaunchKernelGGL(vti_fwd_kernel, dim3(a.n_pml * a.nshots), dim3(kThreads), 0, s, a);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int vti_launch_adj(const VtiStep& a, hipStream_t s) {
  if (a.n_int > 0)
    hipLaunchKernelGGL(vti_adj_int_kernel, dim3(a.n_int * a.nshots), dim3(kThreads), 0, s, a);
  if (a.n_pml > 0)
    hipLaunchKernelGGL(vti_adj_kernel, dim3(a.n_pml * a.nshots), dim3(kThreads), 0, s, a);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int vti_launch_fold(double* tot, const float* gpart, int nshots, size_t plane, hipStream_t s) {
  hipLaunchKernelGGL(vti_fold_kernel, dim3((unsigned)((plane + 255) / 256), 3), dim3(256), 0, s,
                     tot, gpart, nshots, plane);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

int vti_launch_finish(const double* tot, const float* pad, float* grad, int nx, int nz, int P,
                      double r, hipStream_t s) {
  hipLaunchKernelGGL(vti_finish_kernel, dim3((nx + 255) / 256, nz), dim3(256), 0, s, tot, pad, grad,
                     nx, nz, P, r);
  SWEEP_HIP(hipGetLastError());
  return SWEEP_OK;
}

}  // namespace sweep
