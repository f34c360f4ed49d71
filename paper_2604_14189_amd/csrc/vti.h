// Pseudo-acoustic VTI step (Sec. 3.3.1, Eq. 5): device-side view of one step of
// all shots of a plan, and the launchers (vti.hip). Not part of the C ABI.
#pragma once

#include "internal.h"

namespace sweep {

// Scaled form on the GPU (h and dt folded in): G = F / dt^2, and with
// r = dt / h,
//   cx = (1 + 2 eta) (v r)^2, cz = (vv r)^2, cm = 2 eta (v r)^2 (vv r)^2,
//   P^{n+1} = 2 P^n - P^{n-1} + cx Bx' + cz Bz' - cm D2x' D2z' G^n + r^2 s_n e_src,
//   G^{n+1} = 2 G^n - G^{n-1} + P^n,
// where Bx' = h^2 Bx (the x part of the acoustic C-PML Laplacian) and D' = h^k D.
// G, the double time integral of P, is several hundred times larger than P;
// the fourth-order mixed difference would amplify its float32 rounding noise
// (white, about 1e-5 of P per step in a test of the recurrence on the host),
// so G, its update and D2x'D2z'G are held in float64 and only cm D2x'D2z'G is
// rounded to float32. The adjoint of G, mu, accumulates D2x'D2z'(cm lambda)
// twice over time in the same way, so it and that mixed term are float64 too.
// P itself is float64 as well: rounding P^{n+1} to float32 every step injects
// white noise that D2x'D2z'G turns into an error of about 1e-3 .. 1e-2 in the
// eta gradient where eta = 0 (there no mixed term feeds back, and nothing
// bounds the low-frequency part that G sums up). The stencils stay float32:
// they take hi = float(P) and lo = P - hi (kept to bfloat16 in LDS, where
// it needs only a few bits) separately, so their result holds P's low bits
// too. The adjoint fields may stay float32 (their rounding moves the
// gradients by about 1e-6).
// Tiles are 64 x 16 cells; thread (lx, w) of a 256-thread work-group owns
// column lx and rows 4w .. 4w+3 of its tile.
constexpr int kVtiTZ = 16;

struct VtiStep {
  int NX, NZ, P, nt, nrec, nshots, n, tiles_x, ntiles;
  // tiles [0, n_int) of tl have no C-PML strip within 4 cells and take the
  // interior kernels; tiles [n_int, n_int + n_pml) take the general ones
  const int* tl;
  int n_int, n_pml;
  float w;  // (dt/h)^2, source scale
  const float* cx;
  const float* cz;
  const float* cm;
  const float* ax;
  const float* bx;
  const float* az;
  const float* bz;
  // forward: P^n (pcur), P^{n-1} in / P^{n+1} out (pprev), both float64; G
  // likewise. adjoint: lambda^{n+1} (cur), lambda^{n+2} in / lambda^n out
  // (prev); the adjoint of G (mu) likewise. The second field of each pair is
  // read and written at a thread's own cells only, so it is updated in place.
  const double* pcur;  // forward: P (float64)
  double* pprev;
  const float* cur;    // adjoint: lambda
  float* prev;
  const double* gcur;  // forward: G (float64)
  double* gprev;
  const double* mcur;  // adjoint: the adjoint of G (float64)
  double* mprev;
  // C-PML memory variables (x strips [shot][NZ][2P], z strips [shot][2P][NX]):
  // read *_in (n-1), write *_out (n)
  const float* psx_in;
  float* psx_out;
  const float* zex_in;
  float* zex_out;
  const float* psz_in;
  float* psz_out;
  const float* zez_in;
  float* zez_out;
  const int* src_cell;   // [nshots] padded linear index
  const float* wavelet;  // [nshots][nt]
  const int* rec_off;    // [nshots * ntiles + 1] CSR over (shot, 64 x 16 tile)
  const int2* rec_ent;   // (local cell index in the tile, receiver index)
  float* gathers;        // forward: [nshots][nt][nrec] or null
  const float* resid;    // adjoint: r_{n-1} injected into lambda^n (null: none)
  float* tr[3];          // forward: Bx', Bz', D2x'D2z'G^n of step n, [nshots][NZ][NX], or null
  const float* trc[3];   // adjoint: the same planes of the step being reversed
  float* g;              // adjoint: [3][nshots][NZ][NX] partials for cx, cz, cm
  int g_init;            // 1: g = ..., 0: g += ...
};

// interior (no C-PML strip within 4 cells of the 64 x 16 tile) or not, as the
// kernels test it
bool vti_near_strip(int x0, int z0, int NX, int NZ, int P);

int vti_launch_prep(const float* model, float* pad, float* cx, float* cz, float* cm, int nx,
                    int nz, int P, double h, double dt, hipStream_t s);
int vti_launch_fwd(const VtiStep& a, hipStream_t s);
int vti_launch_adj(const VtiStep& a, hipStream_t s);
int vti_launch_fold(double* tot, const float* gpart, int nshots, size_t plane, hipStream_t s);
int vti_launch_finish(const double* tot, const float* pad, float* grad, int nx, int nz, int P,
                      double r, hipStream_t s);

}  // namespace sweep
