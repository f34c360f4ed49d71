// FP64 CPU oracle: isotropic elastic velocity-stress system (Sec. 3.5, Eq. 12).
//
// TEST INFRASTRUCTURE ONLY (see oracle.h). The discretisation (the paper gives
// the PDE only):
//
//  * Staggered grid (Virieux 1986), 4th order in space (Levander 1988,
//    c1 = 9/8, c2 = -1/24). Padded grid NX = nx + 2P, NZ = nz + 2P (nz + P with
//    a free surface: no pad on top, model row 0 is the surface). Node of each
//    stored value [j][i]: txx, tzz at (i, j); vx at (i+1/2, j); vz at (i, j+1/2);
//    txz at (i+1/2, j+1/2).
//  * Derivatives (divided by h), zero outside the grid:
//      Dx+ f = c1 (f[i+1]-f[i]) + c2 (f[i+2]-f[i-1])   (integer -> half node)
//      Dx- g = c1 (g[i]-g[i-1]) + c2 (g[i+1]-g[i-2])   (half -> integer node)
//    and the same along j.
//  * Material: lambda = rho (vp^2 - 2 vs^2), mu = rho vs^2 at integer nodes;
//    buoyancy bx = 2/(rho[i]+rho[i+1]), bz = 2/(rho[j]+rho[j+1]) (the index past
//    the last cell is clamped); mu at txz nodes = harmonic mean of the 4
//    surrounding mu (0 if any is 0).
//  * C-PML (kappa = 1): each of the eight derivatives D f becomes D f + psi with
//    psi <- b psi + a D f, the profile taken at the derivative's output node.
//  * Step n (state v^{n-1/2}, tau^n):
//      vx += dt bx (Dx+ txx + Dz- txz),  vz += dt bz (Dx- txz + Dz+ tzz)
//      record (vx, vz) at the receivers (v^{n+1/2})
//      txx += dt [(l+2m) Dx- vx + l Dz- vz],  tzz += dt [l Dx- vx + (l+2m) Dz- vz]
//      txz += dt mu_xz (Dz+ vx + Dx+ vz)
//      txx[src] += (dt/h^2) s_n, tzz[src] += (dt/h^2) s_n   (explosive source)
//  * Free surface (Levander 1988 stress imaging): tzz = 0 on row 0 (never
//    updated); images tzz[-k] = -tzz[k], txz[-k-1] = -txz[k] in the velocity
//    update; txx on row 0 uses 4 mu (l + mu)/(l + 2 mu) Dx- vx; velocity
//    z-derivatives that would reach above the surface use the 2nd-order
//    difference (row 1 of Dz- vz, row 0 of Dz+ vx; Graves 1996).
//
// Every derivative is a list of taps (offset, weight) per output row; the
// adjoint applies the same taps in scatter form, so it is the exact transpose.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <vector>

#include "oracle.h"

namespace {

const double C1 = 9.0 / 8.0;
const double C2 = -1.0 / 24.0;

typedef std::vector<double> Arr;

struct G2 {
  int NX = 0, NZ = 0;
  size_t size() const { return (size_t)NX * NZ; }
  size_t idx(int i, int j) const { return (size_t)j * NX + i; }
};

// Derivative kinds: axis, direction, and which free-surface rule applies.
enum Kind {
  DXP,    // Dx+ (integer -> half x)
  DXM,    // Dx- (half -> integer x)
  DZP_T,  // Dz+ of tzz (velocity update), surface images
  DZM_T,  // Dz- of txz (velocity update), surface images
  DZP_V,  // Dz+ of vx (txz update), 2nd order on row 0 at a surface
  DZM_V,  // Dz- of vz (txx/tzz update), 2nd order on row 1, none on row 0
};

struct Tap {
  int off;
  double w;
};

// Taps of derivative `k` for output row j (offsets along the derivative axis).
int taps(Kind k, int j, bool fs, Tap* t) {
  switch (k) {
    case DXP:
      t[0] = {1, C1}; t[1] = {0, -C1}; t[2] = {2, C2}; t[3] = {-1, -C2};
      return 4;
    case DXM:
      t[0] = {0, C1}; t[1] = {-1, -C1}; t[2] = {1, C2}; t[3] = {-2, -C2};
      return 4;
    case DZP_T:
      if (fs && j == 0) {  // tzz[-1] = -tzz[1]
        t[0] = {1, C1 + C2}; t[1] = {0, -C1}; t[2] = {2, C2};
        return 3;
      }
      t[0] = {1, C1}; t[1] = {0, -C1}; t[2] = {2, C2}; t[3] = {-1, -C2};
      return 4;
    case DZM_T:
      if (fs && j == 0) {  // txz[-1] = -txz[0], txz[-2] = -txz[1]
        t[0] = {0, 2.0 * C1}; t[1] = {1, 2.0 * C2};
        return 2;
      }
      if (fs && j == 1) {  // txz[-1] = -txz[0]
        t[0] = {0, C1}; t[1] = {-1, -C1 + C2}; t[2] = {1, C2};
        return 3;
      }
      t[0] = {0, C1}; t[1] = {-1, -C1}; t[2] = {1, C2}; t[3] = {-2, -C2};
      return 4;
    case DZP_V:
      if (fs && j == 0) {
        t[0] = {1, 1.0}; t[1] = {0, -1.0};
        return 2;
      }
      t[0] = {1, C1}; t[1] = {0, -C1}; t[2] = {2, C2}; t[3] = {-1, -C2};
      return 4;
    case DZM_V:
      if (fs && j == 0) return 0;
      if (fs && j == 1) {
        t[0] = {0, 1.0}; t[1] = {-1, -1.0};
        return 2;
      }
      t[0] = {0, C1}; t[1] = {-1, -C1}; t[2] = {1, C2}; t[3] = {-2, -C2};
      return 4;
  }
  return 0;
}

bool is_x(Kind k) { return k == DXP || k == DXM; }

// out = D f  (gather form)
void dop(Kind k, const Arr& f, Arr& out, const G2& g, double h, bool fs) {
  Tap t[4];
  for (int j = 0; j < g.NZ; ++j) {
    const int nt = taps(k, j, fs, t);
    for (int i = 0; i < g.NX; ++i) {
      double s = 0.0;
      for (int q = 0; q < nt; ++q) {
        const int ii = is_x(k) ? i + t[q].off : i;
        const int jj = is_x(k) ? j : j + t[q].off;
        if (ii < 0 || ii >= g.NX || jj < 0 || jj >= g.NZ) continue;
        s += t[q].w * f[g.idx(ii, jj)];
      }
      out[g.idx(i, j)] = s / h;
    }
  }
}

// out += D^T gbar  (scatter form of the same taps)
void dopT(Kind k, const Arr& gbar, Arr& out, const G2& g, double h, bool fs) {
  Tap t[4];
  for (int j = 0; j < g.NZ; ++j) {
    const int nt = taps(k, j, fs, t);
    for (int i = 0; i < g.NX; ++i) {
      const double v = gbar[g.idx(i, j)] / h;
      if (v == 0.0) continue;
      for (int q = 0; q < nt; ++q) {
        const int ii = is_x(k) ? i + t[q].off : i;
        const int jj = is_x(k) ? j : j + t[q].off;
        if (ii < 0 || ii >= g.NX || jj < 0 || jj >= g.NZ) continue;
        out[g.idx(ii, jj)] += t[q].w * v;
      }
    }
  }
}

struct ElSetup {
  G2 g;
  int P = 0, nx = 0, nz = 0, nt = 0, nshots = 0, nrec = 0;
  bool fs = false;
  double h = 0, dt = 0, w = 0;  // w = dt / h^2: source scale
  Arr vp, vs, rho, lam, mu;     // padded, integer nodes
  Arr bx, bz, mxz;              // buoyancy at vx / vz nodes, mu at txz nodes
  Arr cxx_x, cxx_z, czz_x, czz_z;  // txx += dt (cxx_x exx + cxx_z ezz), tzz likewise
  Arr smask;                    // tzz source mask (0 on a surface row)
  Arr axi, bxi, axh, bxh, azi, bzi, azh, bzh;
  std::vector<size_t> src, rec;
};

int el_setup(const orc_problem* pb, const double* model, const int* src_xz, const int* rec_xz,
             ElSetup& S) {
  if (!pb || !model || pb->nx <= 0 || pb->nz <= 0 || pb->pml < 0 || pb->nt < 1 || pb->h <= 0 ||
      pb->dt <= 0 || pb->nshots < 1 || pb->nrec < 0)
    return -1;
  S.P = pb->pml;
  S.nx = pb->nx;
  S.nz = pb->nz;
  S.nt = pb->nt;
  S.nshots = pb->nshots;
  S.nrec = pb->nrec;
  S.fs = pb->free_surface != 0;
  S.h = pb->h;
  S.dt = pb->dt;
  S.w = pb->dt / (pb->h * pb->h);
  const int top = S.fs ? 0 : S.P;
  S.g.NX = pb->nx + 2 * S.P;
  S.g.NZ = pb->nz + top + S.P;
  const G2& g = S.g;
  const size_t N = g.size();
  S.vp.assign(N, 0);
  S.vs.assign(N, 0);
  S.rho.assign(N, 0);
  S.lam.assign(N, 0);
  S.mu.assign(N, 0);
  const size_t mn = (size_t)pb->nx * pb->nz;
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const int ii = std::min(std::max(i - S.P, 0), pb->nx - 1);
      const int jj = std::min(std::max(j - top, 0), pb->nz - 1);
      const size_t m = (size_t)jj * pb->nx + ii, k = g.idx(i, j);
      S.vp[k] = model[m];
      S.vs[k] = model[mn + m];
      S.rho[k] = model[2 * mn + m];
      S.mu[k] = S.rho[k] * S.vs[k] * S.vs[k];
      S.lam[k] = S.rho[k] * (S.vp[k] * S.vp[k] - 2.0 * S.vs[k] * S.vs[k]);
    }
  S.bx.assign(N, 0);
  S.bz.assign(N, 0);
  S.mxz.assign(N, 0);
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const int i1 = std::min(i + 1, g.NX - 1), j1 = std::min(j + 1, g.NZ - 1);
      const size_t k = g.idx(i, j);
      S.bx[k] = 2.0 / (S.rho[k] + S.rho[g.idx(i1, j)]);
      S.bz[k] = 2.0 / (S.rho[k] + S.rho[g.idx(i, j1)]);
      const double m00 = S.mu[k], m10 = S.mu[g.idx(i1, j)], m01 = S.mu[g.idx(i, j1)],
                   m11 = S.mu[g.idx(i1, j1)];
      S.mxz[k] = (m00 > 0 && m10 > 0 && m01 > 0 && m11 > 0)
                     ? 4.0 / (1.0 / m00 + 1.0 / m10 + 1.0 / m01 + 1.0 / m11)
                     : 0.0;
    }
  S.cxx_x.assign(N, 0);
  S.cxx_z.assign(N, 0);
  S.czz_x.assign(N, 0);
  S.czz_z.assign(N, 0);
  S.smask.assign(N, 1.0);
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const double l = S.lam[k], m = S.mu[k];
      if (S.fs && j == 0) {
        S.cxx_x[k] = (l + 2 * m) > 0 ? 4.0 * m * (l + m) / (l + 2.0 * m) : 0.0;
        S.smask[k] = 0.0;
      } else {
        S.cxx_x[k] = l + 2.0 * m;
        S.cxx_z[k] = l;
        S.czz_x[k] = l;
        S.czz_z[k] = l + 2.0 * m;
      }
    }
  const int NX = g.NX, NZ = g.NZ;
  for (Arr* a : {&S.axi, &S.bxi, &S.axh, &S.bxh}) a->assign(NX, 0);
  for (Arr* a : {&S.azi, &S.bzi, &S.azh, &S.bzh}) a->assign(NZ, 0);
  orc_pml_profile(NX, S.P, S.P, 0.0, pb->h, pb->dt, pb->pml_vmax, pb->pml_f0, pb->pml_R,
                  S.axi.data(), S.bxi.data());
  orc_pml_profile(NX, S.P, S.P, 0.5, pb->h, pb->dt, pb->pml_vmax, pb->pml_f0, pb->pml_R,
                  S.axh.data(), S.bxh.data());
  orc_pml_profile(NZ, top, S.P, 0.0, pb->h, pb->dt, pb->pml_vmax, pb->pml_f0, pb->pml_R,
                  S.azi.data(), S.bzi.data());
  orc_pml_profile(NZ, top, S.P, 0.5, pb->h, pb->dt, pb->pml_vmax, pb->pml_f0, pb->pml_R,
                  S.azh.data(), S.bzh.data());
  if (src_xz) {
    S.src.resize(S.nshots);
    for (int s = 0; s < S.nshots; ++s) {
      const int x = src_xz[2 * s], z = src_xz[2 * s + 1];
      if (x < 0 || x >= pb->nx || z < 0 || z >= pb->nz) return -1;
      S.src[s] = g.idx(x + S.P, z + top);
    }
  }
  if (rec_xz) {
    S.rec.resize((size_t)S.nshots * S.nrec);
    for (size_t r = 0; r < S.rec.size(); ++r) {
      const int x = rec_xz[2 * r], z = rec_xz[2 * r + 1];
      if (x < 0 || x >= pb->nx || z < 0 || z >= pb->nz) return -1;
      S.rec[r] = g.idx(x + S.P, z + top);
    }
  }
  return 0;
}

// State entering step n: v^{n-1/2}, tau^n and the eight memory variables.
struct ElState {
  Arr f[13];  // vx vz txx tzz txz psi_a .. psi_h
  void zeros(size_t n) {
    for (Arr& a : f) a.assign(n, 0.0);
  }
};
enum { VX, VZ, TXX, TZZ, TXZ, PA, PB, PC, PD, PE, PF, PG, PH };

// Forward quantities the gradient needs from step n.
struct ElTrace {
  Arr fvx, fvz, exx, ezz, exz;
  void alloc(size_t n) {
    fvx.assign(n, 0);
    fvz.assign(n, 0);
    exx.assign(n, 0);
    ezz.assign(n, 0);
    exz.assign(n, 0);
  }
};

// psi <- b psi + a G, returns G + psi (a, b indexed along x (ax) or z)
inline double cpml(double& psi, double G, double a, double b) {
  psi = b * psi + a * G;
  return G + psi;
}

// One forward step. `src_amp` is the source sample (0 for none); `extra_txx`,
// `extra_tzz`, `extra_txz`, `extra_vx`, `extra_vz` (may be null) are additional
// increments (Born sources). `tr` (may be null) receives the gradient terms.
struct Extra {
  const Arr *vx = nullptr, *vz = nullptr, *txx = nullptr, *tzz = nullptr, *txz = nullptr;
};

void el_step(const ElSetup& S, ElState& st, size_t src, double src_amp, const Extra& ex,
             ElTrace* tr, bool par, double* rec_out, const size_t* rec) {
  const G2& g = S.g;
  const size_t N = g.size();
  const double h = S.h, dt = S.dt;
  Arr Ga(N), Gb(N), Gc(N), Gd(N);
  dop(DXP, st.f[TXX], Ga, g, h, S.fs);
  dop(DZM_T, st.f[TXZ], Gb, g, h, S.fs);
  dop(DXM, st.f[TXZ], Gc, g, h, S.fs);
  dop(DZP_T, st.f[TZZ], Gd, g, h, S.fs);
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const double fvx = cpml(st.f[PA][k], Ga[k], S.axh[i], S.bxh[i]) +
                         cpml(st.f[PB][k], Gb[k], S.azi[j], S.bzi[j]);
      const double fvz = cpml(st.f[PC][k], Gc[k], S.axi[i], S.bxi[i]) +
                         cpml(st.f[PD][k], Gd[k], S.azh[j], S.bzh[j]);
      st.f[VX][k] += dt * S.bx[k] * fvx;
      st.f[VZ][k] += dt * S.bz[k] * fvz;
      if (ex.vx) st.f[VX][k] += (*ex.vx)[k];
      if (ex.vz) st.f[VZ][k] += (*ex.vz)[k];
      if (tr) {
        tr->fvx[k] = fvx;
        tr->fvz[k] = fvz;
      }
    }
  if (rec_out)
    for (int r = 0; r < S.nrec; ++r) {
      rec_out[2 * r] = st.f[VX][rec[r]];
      rec_out[2 * r + 1] = st.f[VZ][rec[r]];
    }
  Arr Ge(N), Gf(N), Gg(N), Gh(N);
  dop(DXM, st.f[VX], Ge, g, h, S.fs);
  dop(DZM_V, st.f[VZ], Gf, g, h, S.fs);
  dop(DZP_V, st.f[VX], Gg, g, h, S.fs);
  dop(DXP, st.f[VZ], Gh, g, h, S.fs);
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const double exx = cpml(st.f[PE][k], Ge[k], S.axi[i], S.bxi[i]);
      const double ezz = cpml(st.f[PF][k], Gf[k], S.azi[j], S.bzi[j]);
      const double exz = cpml(st.f[PG][k], Gg[k], S.azh[j], S.bzh[j]) +
                         cpml(st.f[PH][k], Gh[k], S.axh[i], S.bxh[i]);
      st.f[TXX][k] += dt * (S.cxx_x[k] * exx + S.cxx_z[k] * ezz);
      st.f[TZZ][k] += dt * (S.czz_x[k] * exx + S.czz_z[k] * ezz);
      st.f[TXZ][k] += dt * S.mxz[k] * exz;
      if (ex.txx) st.f[TXX][k] += (*ex.txx)[k];
      if (ex.tzz) st.f[TZZ][k] += (*ex.tzz)[k] * S.smask[k];
      if (ex.txz) st.f[TXZ][k] += (*ex.txz)[k];
      if (tr) {
        tr->exx[k] = exx;
        tr->ezz[k] = ezz;
        tr->exz[k] = exz;
      }
    }
  st.f[TXX][src] += S.w * src_amp;
  st.f[TZZ][src] += S.w * src_amp * S.smask[src];
}

// Gradients with respect to the coefficient fields of the step.
struct ElCoefGrad {
  Arr bx, bz, mxz, cxx_x, cxx_z, czz_x, czz_z;
  void alloc(size_t n) {
    for (Arr* a : {&bx, &bz, &mxz, &cxx_x, &cxx_z, &czz_x, &czz_z}) a->assign(n, 0.0);
  }
};

// Reverse of step n (exact transpose of el_step). A holds the adjoints of the
// step's outputs on entry and of its inputs on exit.
void el_adj_step(const ElSetup& S, ElState& A, const ElTrace& tr, const double* r_n,
                 const size_t* rec, size_t src, ElCoefGrad& cg, double* sbar) {
  const G2& g = S.g;
  const size_t N = g.size();
  const double h = S.h, dt = S.dt;
  if (sbar) *sbar = S.w * (A.f[TXX][src] + A.f[TZZ][src] * S.smask[src]);
  // stress phase
  Arr Gbe(N), Gbf(N), Gbg(N), Gbh(N);
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const double Txx = A.f[TXX][k], Tzz = A.f[TZZ][k], Txz = A.f[TXZ][k];
      cg.cxx_x[k] += dt * Txx * tr.exx[k];
      cg.cxx_z[k] += dt * Txx * tr.ezz[k];
      cg.czz_x[k] += dt * Tzz * tr.exx[k];
      cg.czz_z[k] += dt * Tzz * tr.ezz[k];
      cg.mxz[k] += dt * Txz * tr.exz[k];
      const double ebx = dt * (S.cxx_x[k] * Txx + S.czz_x[k] * Tzz);
      const double ebz = dt * (S.cxx_z[k] * Txx + S.czz_z[k] * Tzz);
      const double ebxz = dt * S.mxz[k] * Txz;
      // G + psi_new with psi_new = b psi_old + a G:  G gets e (1 + a), psi_old gets b e
      const double te = A.f[PE][k] + ebx, tf = A.f[PF][k] + ebz;
      const double tg = A.f[PG][k] + ebxz, th = A.f[PH][k] + ebxz;
      Gbe[k] = ebx + S.axi[i] * te;
      Gbf[k] = ebz + S.azi[j] * tf;
      Gbg[k] = ebxz + S.azh[j] * tg;
      Gbh[k] = ebxz + S.axh[i] * th;
      A.f[PE][k] = S.bxi[i] * te;
      A.f[PF][k] = S.bzi[j] * tf;
      A.f[PG][k] = S.bzh[j] * tg;
      A.f[PH][k] = S.bxh[i] * th;
    }
  dopT(DXM, Gbe, A.f[VX], g, h, S.fs);
  dopT(DZM_V, Gbf, A.f[VZ], g, h, S.fs);
  dopT(DZP_V, Gbg, A.f[VX], g, h, S.fs);
  dopT(DXP, Gbh, A.f[VZ], g, h, S.fs);
  // recording of v^{n+1/2}
  if (r_n)
    for (int r = 0; r < S.nrec; ++r) {
      A.f[VX][rec[r]] += r_n[2 * r];
      A.f[VZ][rec[r]] += r_n[2 * r + 1];
    }
  // velocity phase
  Arr Gba(N), Gbb(N), Gbc(N), Gbd(N);
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const double Vx = A.f[VX][k], Vz = A.f[VZ][k];
      cg.bx[k] += dt * Vx * tr.fvx[k];
      cg.bz[k] += dt * Vz * tr.fvz[k];
      const double kx = dt * S.bx[k] * Vx, kz = dt * S.bz[k] * Vz;
      const double ta = A.f[PA][k] + kx, tb = A.f[PB][k] + kx;
      const double tc = A.f[PC][k] + kz, td = A.f[PD][k] + kz;
      Gba[k] = kx + S.axh[i] * ta;
      Gbb[k] = kx + S.azi[j] * tb;
      Gbc[k] = kz + S.axi[i] * tc;
      Gbd[k] = kz + S.azh[j] * td;
      A.f[PA][k] = S.bxh[i] * ta;
      A.f[PB][k] = S.bzi[j] * tb;
      A.f[PC][k] = S.bxi[i] * tc;
      A.f[PD][k] = S.bzh[j] * td;
    }
  dopT(DXP, Gba, A.f[TXX], g, h, S.fs);
  dopT(DZM_T, Gbb, A.f[TXZ], g, h, S.fs);
  dopT(DXM, Gbc, A.f[TXZ], g, h, S.fs);
  dopT(DZP_T, Gbd, A.f[TZZ], g, h, S.fs);
}

// Chain the coefficient gradients to (vp, vs, rho) on the padded grid, then fold
// the pad onto the model edge cells; adds into grad[3][nz][nx].
void el_chain(const ElSetup& S, const ElCoefGrad& cg, double* grad) {
  const G2& g = S.g;
  const size_t N = g.size();
  Arr gl(N, 0.0), gm(N, 0.0), gr(N, 0.0);
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const double l = S.lam[k], m = S.mu[k];
      if (S.fs && j == 0) {
        // cxx_x = M(l, m) = 4 m (l + m) / (l + 2 m)
        const double d = l + 2.0 * m;
        if (d > 0) {
          gl[k] += cg.cxx_x[k] * 4.0 * m * m / (d * d);
          gm[k] += cg.cxx_x[k] * 4.0 * (l * l + 2.0 * l * m + 2.0 * m * m) / (d * d);
        }
      } else {
        gl[k] += cg.cxx_x[k] + cg.cxx_z[k] + cg.czz_x[k] + cg.czz_z[k];
        gm[k] += 2.0 * (cg.cxx_x[k] + cg.czz_z[k]);
      }
      // buoyancy: b = 2 / (rho_a + rho_b): db/drho = -b^2 / 2 on both cells
      const int i1 = std::min(i + 1, g.NX - 1), j1 = std::min(j + 1, g.NZ - 1);
      const double dbx = -0.5 * S.bx[k] * S.bx[k] * cg.bx[k];
      gr[k] += dbx;
      gr[g.idx(i1, j)] += dbx;
      const double dbz = -0.5 * S.bz[k] * S.bz[k] * cg.bz[k];
      gr[k] += dbz;
      gr[g.idx(i, j1)] += dbz;
      // harmonic mean: d mxz / d mu_q = mxz^2 / (4 mu_q^2)
      if (S.mxz[k] > 0) {
        const size_t q[4] = {k, g.idx(i1, j), g.idx(i, j1), g.idx(i1, j1)};
        for (size_t qq : q) gm[qq] += cg.mxz[k] * S.mxz[k] * S.mxz[k] / (4.0 * S.mu[qq] * S.mu[qq]);
      }
    }
  const size_t mn = (size_t)S.nx * S.nz;
  const int top = S.fs ? 0 : S.P;
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const double vp = S.vp[k], vs = S.vs[k], rho = S.rho[k];
      // lambda = rho (vp^2 - 2 vs^2), mu = rho vs^2
      const double gvp = gl[k] * 2.0 * rho * vp;
      const double gvs = gl[k] * (-4.0 * rho * vs) + gm[k] * 2.0 * rho * vs;
      const double grho = gl[k] * (vp * vp - 2.0 * vs * vs) + gm[k] * vs * vs + gr[k];
      const int ii = std::min(std::max(i - S.P, 0), S.nx - 1);
      const int jj = std::min(std::max(j - top, 0), S.nz - 1);
      const size_t m = (size_t)jj * S.nx + ii;
      grad[m] += gvp;
      grad[mn + m] += gvs;
      grad[2 * mn + m] += grho;
    }
}

void el_forward_shot(const ElSetup& S, int s, const double* wav, double* gath, double* snaps,
                     bool par) {
  ElState st;
  st.zeros(S.g.size());
  const size_t* rec = S.rec.empty() ? nullptr : &S.rec[(size_t)s * S.nrec];
  for (int n = 0; n < S.nt; ++n) {
    el_step(S, st, S.src[s], wav[n], Extra(), nullptr, par,
            gath ? gath + (size_t)n * S.nrec * 2 : nullptr, rec);
    if (snaps)
      for (int c = 0; c < 5; ++c)
        std::copy(st.f[c].begin(), st.f[c].end(), snaps + ((size_t)n * 5 + c) * S.g.size());
  }
}

void el_gradient_shot(const ElSetup& S, int s, const double* wav, const double* resid, int k,
                      ElCoefGrad& cg, double* sbar, double* gath, bool par) {
  const G2& g = S.g;
  const int nt = S.nt;
  if (k <= 0 || k > nt) k = nt;
  const int nseg = (nt + k - 1) / k;
  const size_t* rec = &S.rec[(size_t)s * S.nrec];
  std::vector<ElState> ck(nseg);
  ElState st;
  st.zeros(g.size());
  for (int n = 0; n < nt; ++n) {
    if (n % k == 0) ck[n / k] = st;
    el_step(S, st, S.src[s], wav[n], Extra(), nullptr, par,
            gath ? gath + (size_t)n * S.nrec * 2 : nullptr, rec);
  }
  cg.alloc(g.size());
  ElState A;
  A.zeros(g.size());
  std::vector<ElTrace> tr(k);
  for (ElTrace& t : tr) t.alloc(g.size());
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int n0 = sg * k, n1 = std::min(nt, n0 + k);
    ElState w = ck[sg];
    for (int n = n0; n < n1; ++n) el_step(S, w, S.src[s], wav[n], Extra(), &tr[n - n0], par, nullptr, rec);
    for (int n = n1 - 1; n >= n0; --n)
      el_adj_step(S, A, tr[n - n0], resid + (size_t)n * S.nrec * 2, rec, S.src[s], cg,
                  sbar ? sbar + n : nullptr);
  }
}

int threads_of(const orc_problem* pb) {
  return pb->nthreads > 0 ? pb->nthreads : omp_get_max_threads();
}

}  // namespace

extern "C" int orc_el_forward(const orc_problem* pb, const double* model, const int* src_xz,
                              const double* wavelet, const int* rec_xz, double* gathers) {
  ElSetup S;
  if (!src_xz || !rec_xz || !wavelet || !gathers) return -1;
  if (el_setup(pb, model, src_xz, rec_xz, S)) return -1;
  const bool inner = S.nshots == 1;
#pragma omp parallel for schedule(dynamic) num_threads(threads_of(pb)) if (!inner)
  for (int s = 0; s < S.nshots; ++s)
    el_forward_shot(S, s, wavelet + (size_t)s * S.nt, gathers + (size_t)s * S.nt * S.nrec * 2,
                    nullptr, inner);
  return 0;
}

extern "C" int orc_el_wavefield(const orc_problem* pb, const double* model, const int* src_xz,
                                const double* wavelet, double* snaps) {
  ElSetup S;
  if (!src_xz || !wavelet || !snaps) return -1;
  orc_problem one = *pb;
  one.nshots = 1;
  one.nrec = 0;
  if (el_setup(&one, model, src_xz, nullptr, S)) return -1;
  omp_set_num_threads(threads_of(pb));
  el_forward_shot(S, 0, wavelet, nullptr, snaps, true);
  return 0;
}

extern "C" int orc_el_gradient(const orc_problem* pb, const double* model, const int* src_xz,
                               const double* wavelet, const int* rec_xz, const double* resid,
                               double* grad, double* grad_wavelet, double* gathers) {
  ElSetup S;
  if (!src_xz || !rec_xz || !wavelet || !resid || !grad) return -1;
  if (el_setup(pb, model, src_xz, rec_xz, S)) return -1;
  const bool inner = S.nshots == 1;
  std::vector<ElCoefGrad> cg(S.nshots);
#pragma omp parallel for schedule(dynamic) num_threads(threads_of(pb)) if (!inner)
  for (int s = 0; s < S.nshots; ++s)
    el_gradient_shot(S, s, wavelet + (size_t)s * S.nt, resid + (size_t)s * S.nt * S.nrec * 2,
                     pb->ckpt_every, cg[s],
                     grad_wavelet ? grad_wavelet + (size_t)s * S.nt : nullptr,
                     gathers ? gathers + (size_t)s * S.nt * S.nrec * 2 : nullptr, inner);
  std::fill(grad, grad + 3 * (size_t)S.nx * S.nz, 0.0);
  for (int s = 0; s < S.nshots; ++s) el_chain(S, cg[s], grad);
  return 0;
}

extern "C" int orc_el_born(const orc_problem* pb, const double* model, const double* dmodel,
                           const int* src_xz, const double* wavelet, const int* rec_xz,
                           double* dgathers) {
  // Tangent-linear model (Eq. 17-18 in spirit): perturb (vp, vs, rho), linearise
  // every coefficient of the step, drive the perturbed fields with dcoef * field.
  ElSetup S, Sd;
  if (!dmodel || !src_xz || !rec_xz || !wavelet || !dgathers) return -1;
  if (el_setup(pb, model, src_xz, rec_xz, S)) return -1;
  const G2& g = S.g;
  const size_t N = g.size();
  const size_t mn = (size_t)S.nx * S.nz;
  const int top = S.fs ? 0 : S.P;
  // perturbation of the padded parameters
  Arr dvp(N), dvs(N), drho(N);
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const int ii = std::min(std::max(i - S.P, 0), S.nx - 1);
      const int jj = std::min(std::max(j - top, 0), S.nz - 1);
      const size_t m = (size_t)jj * S.nx + ii, k = g.idx(i, j);
      dvp[k] = dmodel[m];
      dvs[k] = dmodel[mn + m];
      drho[k] = dmodel[2 * mn + m];
    }
  Arr dl(N), dm(N);
  for (size_t k = 0; k < N; ++k) {
    dl[k] = drho[k] * (S.vp[k] * S.vp[k] - 2 * S.vs[k] * S.vs[k]) +
            S.rho[k] * (2 * S.vp[k] * dvp[k] - 4 * S.vs[k] * dvs[k]);
    dm[k] = drho[k] * S.vs[k] * S.vs[k] + S.rho[k] * 2 * S.vs[k] * dvs[k];
  }
  // perturbed coefficients
  Arr dbx(N), dbz(N), dmxz(N), dcxx_x(N), dcxx_z(N), dczz_x(N), dczz_z(N);
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const int i1 = std::min(i + 1, g.NX - 1), j1 = std::min(j + 1, g.NZ - 1);
      dbx[k] = -0.5 * S.bx[k] * S.bx[k] * (drho[k] + drho[g.idx(i1, j)]);
      dbz[k] = -0.5 * S.bz[k] * S.bz[k] * (drho[k] + drho[g.idx(i, j1)]);
      if (S.mxz[k] > 0) {
        const size_t q[4] = {k, g.idx(i1, j), g.idx(i, j1), g.idx(i1, j1)};
        double acc = 0;
        for (size_t qq : q) acc += dm[qq] / (S.mu[qq] * S.mu[qq]);
        dmxz[k] = S.mxz[k] * S.mxz[k] / 4.0 * acc;
      }
      const double l = S.lam[k], m = S.mu[k];
      if (S.fs && j == 0) {
        const double d = l + 2 * m;
        if (d > 0)
          dcxx_x[k] = 4.0 * m * m / (d * d) * dl[k] +
                      4.0 * (l * l + 2 * l * m + 2 * m * m) / (d * d) * dm[k];
      } else {
        dcxx_x[k] = dl[k] + 2 * dm[k];
        dcxx_z[k] = dl[k];
        dczz_x[k] = dl[k];
        dczz_z[k] = dl[k] + 2 * dm[k];
      }
    }
  const bool inner = S.nshots == 1;
#pragma omp parallel for schedule(dynamic) num_threads(threads_of(pb)) if (!inner)
  for (int s = 0; s < S.nshots; ++s) {
    ElState bg, pt;
    bg.zeros(N);
    pt.zeros(N);
    ElTrace tr;
    tr.alloc(N);
    Arr evx(N), evz(N), etxx(N), etzz(N), etxz(N);
    const size_t* rec = &S.rec[(size_t)s * S.nrec];
    double* out = dgathers + (size_t)s * S.nt * S.nrec * 2;
    for (int n = 0; n < S.nt; ++n) {
      // the perturbed velocity update uses the background force of this step and
      // the perturbed stress update uses the background strain of this step, so
      // the background step runs first and provides both through `tr`
      el_step(S, bg, S.src[s], wavelet[(size_t)s * S.nt + n], Extra(), &tr, inner, nullptr, rec);
      for (size_t k = 0; k < N; ++k) {
        evx[k] = S.dt * dbx[k] * tr.fvx[k];
        evz[k] = S.dt * dbz[k] * tr.fvz[k];
        etxx[k] = S.dt * (dcxx_x[k] * tr.exx[k] + dcxx_z[k] * tr.ezz[k]);
        etzz[k] = S.dt * (dczz_x[k] * tr.exx[k] + dczz_z[k] * tr.ezz[k]);
        etxz[k] = S.dt * dmxz[k] * tr.exz[k];
      }
      Extra ex;
      ex.vx = &evx;
      ex.vz = &evz;
      ex.txx = &etxx;
      ex.tzz = &etzz;
      ex.txz = &etxz;
      el_step(S, pt, S.src[s], 0.0, ex, nullptr, inner, out + (size_t)n * S.nrec * 2, rec);
    }
  }
  return 0;
}
