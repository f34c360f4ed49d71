// Internal declarations of the elastic path (not part of the C-ABI).
#pragma once

#include "internal.h"

namespace sweep {

// Shared (per plan) coefficient arrays on the padded grid.
struct ElCoef {
  float *vp, *vs, *rho, *lam, *mu;              // [NZ][NX]
  float *bx, *bz, *mxz;                          // buoyancy at vx / vz nodes, mu at txz nodes
  float *cxx_x, *cxx_z, *czz_x, *czz_z, *smask;  // stress-update coefficients, tzz source mask
                                                 // (the step kernels derive czz_x, czz_z from
                                                 // cxx_z, cxx_x; see elastic.hip)
  float *dM_dl, *dM_dm;                          // [NX] free-surface modulus derivatives (row 0)
  float *axi, *bxi, *axh, *bxh;                  // [NX] C-PML, integer / half nodes
  float *azi, *bzi, *azh, *bzh;                  // [NZ]
};

// One time step (forward) or its reverse (adjoint) for all shots of a plan.
struct ElStep {
  int NX, NZ, nt, nrec, nshots, n, fs;
  int fluid;        // vs = 0 (first-order acoustic): the kernels' fluid variants
  float dt, w, ih;  // time step, source scale dt/h^2, 1/h
  const float *bx, *bz, *mxz, *cxx_x, *cxx_z, *smask, *dM_dl, *dM_dm;
  const float *axi, *bxi, *axh, *bxh, *azi, *bzi, *azh, *bzh;
  // fields [shot][NZ][NX]: forward state, or the adjoint state in the reverse pass
  float *vx, *vz, *txx, *tzz, *txz;
  float* ps[8];          // forward memory variables (updated in place)
  const float* ps_in[8]; // adjoint memory variables, read
  float* ps_out[8];      // adjoint memory variables, written
  float* tr[5];          // forward trace out (fvx, fvz, exx, ezz, exz) or null
  const float* trc[5];   // adjoint: trace of this step
  float* g[5];           // gradient partials (lambda, mu, mu_xz, bx, bz), [shot][plane] each
  int g_init;
  const int* src_cell;
  const float* wavelet;
  const int* rec_cell;    // [nshots][nrec]
  const int4* rec_sorted; // (shot, cell, r, 0) sorted
  float* gathers;         // [nshots][nt][nrec][2]
  const float* resid;
  // transposed z-taps of the first four rows under a free surface, per kind:
  // 0 Dz+ of tzz, 1 Dz- of txz, 2 Dz+ of vx, 3 Dz- of vz
  int tt_cnt[4][4];
  int tt_off[4][4][8];
  float tt_w[4][4][8];
};

// fluid: the model is (vp, rho) and vs = 0 (first-order acoustic); the
// gradient then has the planes (vp, rho).
int el_launch_prep(const float* model, const ElCoef& c, int nx, int nz, int P, int fs, int fluid,
                   double h, double dt, double vmax, double f0, double R, hipStream_t s);
int el_launch_fwd(const ElStep& a, hipStream_t s, hipEvent_t* ev);
int el_launch_adj(const ElStep& a, hipStream_t s, hipEvent_t* ev);
int el_launch_fold(double* tot, const float* gpart, int nshots, size_t plane, hipStream_t s);
int el_launch_finish(const double* tot, const ElCoef& c, float* grad, int nx, int nz, int P,
                     int fs, int fluid, hipStream_t s);

}  // namespace sweep
