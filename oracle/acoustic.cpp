// FP64 CPU oracle: constant-density acoustic wave equation (Sec. 3.1.2, Eq. 2).
//
// TEST INFRASTRUCTURE ONLY (see oracle.h). Plain loops over whole arrays, in the
// order the recurrence is written in oracle/README.md; nothing is blocked, fused
// or reordered. The interior update is the leapfrog of the step function in
// Sec. 2.1, u_next = 2 u_now - u_pre + vp^2 dt^2 lap(u_now); the pad adds the
// C-PML memory terms, which reduce to that update wherever the damping is zero.
#include "oracle.h"
#include "stencil.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <vector>

using namespace orc;

// ---------------------------------------------------------------------------
// C-PML profile (Collino & Tsogka 2001; Komatitsch & Martin 2007 form, kappa=1):
//   xi = distance into the pad, L = pad thickness,
//   d = d0 (xi/L)^2, d0 = -3 vmax ln(R) / (2 L), alpha = pi f0 (1 - xi/L),
//   b = exp(-(d + alpha) dt), a = d (b - 1) / (d + alpha) where d > 0, else 0.
// ---------------------------------------------------------------------------
extern "C" int orc_pml_profile(int n, int lo_pad, int hi_pad, double shift, double h,
                               double dt, double vmax, double f0, double R, double* a,
                               double* b) {
  if (n <= 0 || lo_pad < 0 || hi_pad < 0 || !a || !b || h <= 0 || dt <= 0) return -1;
  for (int i = 0; i < n; ++i) {
    const double x = i + shift;
    double xi = 0.0, L = 1.0;
    if (lo_pad > 0 && x < lo_pad) {
      xi = (lo_pad - x) * h;
      L = lo_pad * h;
    } else if (hi_pad > 0 && x > (n - 1 - hi_pad)) {
      xi = (x - (n - 1 - hi_pad)) * h;
      L = hi_pad * h;
    }
    if (xi > L) xi = L;
    const double d0 = -3.0 * vmax * std::log(R) / (2.0 * L);
    const double d = (xi > 0.0) ? d0 * (xi / L) * (xi / L) : 0.0;
    const double alpha = M_PI * f0 * (1.0 - xi / L);
    b[i] = std::exp(-(d + alpha) * dt);
    a[i] = (d > 0.0) ? d / (d + alpha) * (b[i] - 1.0) : 0.0;
  }
  return 0;
}

extern "C" int orc_d2_1d(const double* f, int n, double h, double* out) {
  if (!f || !out || n <= 0) return -1;
  Grid2 g;
  g.NX = n;
  g.NZ = 1;
  Arr a(f, f + n);
  for (int i = 0; i < n; ++i) out[i] = d2x(a, g, i, 0, h);
  return 0;
}

extern "C" int orc_d1_1d(const double* f, int n, double h, double* out) {
  if (!f || !out || n <= 0) return -1;
  Grid2 g;
  g.NX = n;
  g.NZ = 1;
  Arr a(f, f + n);
  for (int i = 0; i < n; ++i) out[i] = d1x(a, g, i, 0, h);
  return 0;
}

namespace {

// Everything fixed for a problem: padded grid, C = (v dt)^2, profiles, geometry.
struct AcSetup {
  Grid2 g;
  int P = 0, nx = 0, nz = 0, nt = 0, nshots = 0, nrec = 0;
  double h = 0, dt = 0, w = 0;  // w = dt^2 / h^2 : source scaling
  Arr vpad, C, ax, bx, az, bz;
  int nsrc = 1;             // sources per shot
  std::vector<size_t> src;  // [nshots][nsrc] padded cell index
  std::vector<size_t> rec;  // [nshots][nrec] padded cell index
};

int make_setup(const orc_problem* pb, const double* v, const int* src_xz, const int* rec_xz,
               AcSetup& S, int nsrc = 1) {
  if (nsrc < 1) return -1;
  S.nsrc = nsrc;
  if (!pb || !v || pb->nx <= 0 || pb->nz <= 0 || pb->pml < 0 || pb->nt < 1 || pb->h <= 0 ||
      pb->dt <= 0 || pb->nshots < 1 || pb->nrec < 0)
    return -1;
  S.P = pb->pml;
  S.nx = pb->nx;
  S.nz = pb->nz;
  S.nt = pb->nt;
  S.nshots = pb->nshots;
  S.nrec = pb->nrec;
  S.h = pb->h;
  S.dt = pb->dt;
  S.w = pb->dt * pb->dt / (pb->h * pb->h);
  S.g.NX = pb->nx + 2 * S.P;
  S.g.NZ = pb->nz + 2 * S.P;
  const Grid2& g = S.g;
  S.vpad.assign(g.size(), 0.0);
  S.C.assign(g.size(), 0.0);
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const int ii = std::min(std::max(i - S.P, 0), pb->nx - 1);
      const int jj = std::min(std::max(j - S.P, 0), pb->nz - 1);
      const double vv = v[(size_t)jj * pb->nx + ii];
      S.vpad[g.idx(i, j)] = vv;
      S.C[g.idx(i, j)] = vv * vv * pb->dt * pb->dt;
    }
  S.ax.resize(g.NX);
  S.bx.resize(g.NX);
  S.az.resize(g.NZ);
  S.bz.resize(g.NZ);
  orc_pml_profile(g.NX, S.P, S.P, 0.0, pb->h, pb->dt, pb->pml_vmax, pb->pml_f0, pb->pml_R,
                  S.ax.data(), S.bx.data());
  orc_pml_profile(g.NZ, S.P, S.P, 0.0, pb->h, pb->dt, pb->pml_vmax, pb->pml_f0, pb->pml_R,
                  S.az.data(), S.bz.data());
  if (src_xz) {
    S.src.resize((size_t)S.nshots * nsrc);
    for (size_t q = 0; q < S.src.size(); ++q) {
      const int x = src_xz[2 * q], z = src_xz[2 * q + 1];
      if (x < 0 || x >= pb->nx || z < 0 || z >= pb->nz) return -1;
      S.src[q] = g.idx(x + S.P, z + S.P);
    }
  }
  if (rec_xz) {
    S.rec.resize((size_t)S.nshots * S.nrec);
    for (size_t r = 0; r < S.rec.size(); ++r) {
      const int x = rec_xz[2 * r], z = rec_xz[2 * r + 1];
      if (x < 0 || x >= pb->nx || z < 0 || z >= pb->nz) return -1;
      S.rec[r] = g.idx(x + S.P, z + S.P);
    }
  }
  return 0;
}

// Wavefield state entering step n: p0 = p^{n-1}, p1 = p^n, memory variables at n-1.
struct AcState {
  Arr p0, p1, psx, psz, zex, zez;
  void zeros(size_t n) {
    p0.assign(n, 0.0);
    p1.assign(n, 0.0);
    psx.assign(n, 0.0);
    psz.assign(n, 0.0);
    zex.assign(n, 0.0);
    zez.assign(n, 0.0);
  }
};

// One forward step n:
//   psi_x^n  = b_x psi_x^{n-1} + a_x D1x p^n           (and z)
//   Q_x      = D2x p^n + D1x psi_x^n                   (and z)
//   zeta_x^n = b_x zeta_x^{n-1} + a_x Q_x              (and z)
//   B^n      = Q_x + zeta_x^n + Q_z + zeta_z^n
//   p^{n+1}  = 2 p^n - p^{n-1} + C B^n  [+ extra]  + (dt^2/h^2) s_{k,n} e_{src k}
// with the source terms added in the order k = 0 .. ns-1 (several sources per
// simulation: an encoded shot). `extra` (may be null) is an additional field
// added to p^{n+1} (Born source); `Bout` (may be null) receives B^n.
void ac_step_multi(const AcSetup& S, AcState& st, const size_t* src, const double* s_n, int ns,
                   const Arr* extra, Arr* Bout, bool par) {
  const Grid2& g = S.g;
  const double h = S.h;
  Arr psx(g.size()), psz(g.size()), pn(g.size());
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      psx[k] = S.bx[i] * st.psx[k] + S.ax[i] * d1x(st.p1, g, i, j, h);
      psz[k] = S.bz[j] * st.psz[k] + S.az[j] * d1z(st.p1, g, i, j, h);
    }
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const double Qx = d2x(st.p1, g, i, j, h) + d1x(psx, g, i, j, h);
      const double Qz = d2z(st.p1, g, i, j, h) + d1z(psz, g, i, j, h);
      st.zex[k] = S.bx[i] * st.zex[k] + S.ax[i] * Qx;
      st.zez[k] = S.bz[j] * st.zez[k] + S.az[j] * Qz;
      const double B = Qx + st.zex[k] + Qz + st.zez[k];
      pn[k] = 2.0 * st.p1[k] - st.p0[k] + S.C[k] * B;
      if (extra) pn[k] += (*extra)[k];
      if (Bout) (*Bout)[k] = B;
    }
  for (int k = 0; k < ns; ++k) pn[src[k]] += S.w * s_n[k];
  st.psx.swap(psx);
  st.psz.swap(psz);
  st.p0.swap(st.p1);
  st.p1.swap(pn);
}

void ac_step(const AcSetup& S, AcState& st, size_t src, double s_n, const Arr* extra, Arr* Bout,
             bool par) {
  ac_step_multi(S, st, &src, &s_n, 1, extra, Bout, par);
}

// Step n of shot s with its nsrc sources (wavelets wav[k][nt]).
void ac_step_shot(const AcSetup& S, AcState& st, int s, const double* wav, int n, Arr* Bout,
                  bool par) {
  double sv[64];
  std::vector<double> big;
  double* v = sv;
  if (S.nsrc > 64) {
    big.resize(S.nsrc);
    v = big.data();
  }
  for (int k = 0; k < S.nsrc; ++k) v[k] = wav[(size_t)k * S.nt + n];
  ac_step_multi(S, st, &S.src[(size_t)s * S.nsrc], v, S.nsrc, nullptr, Bout, par);
}

// Adjoint state entering the reverse of step n: P1 = adjoint of p^{n+1},
// P0 = adjoint of p^n, PS / ZE = adjoints of psi^n / zeta^n.
struct AcAdj {
  Arr P1, P0, PSx, PSz, ZEx, ZEz;
  void zeros(size_t n) {
    P1.assign(n, 0.0);
    P0.assign(n, 0.0);
    PSx.assign(n, 0.0);
    PSz.assign(n, 0.0);
    ZEx.assign(n, 0.0);
    ZEz.assign(n, 0.0);
  }
};

// Reverse of step n, the exact transpose of ac_step (D2 is symmetric and D1 is
// antisymmetric on the zero-padded grid):
//   P1[rec] += r_n ;  sbar_n = (dt^2/h^2) P1[src] ;  g_C += P1 * B^n
//   zbar_x = ZE_x + C P1 ;  Qbar_x = C P1 + a_x zbar_x
//   psbar_x = PS_x - D1x Qbar_x
//   lambda = P0 + 2 P1 + D2x Qbar_x + D2z Qbar_z - D1x(a_x psbar_x) - D1z(a_z psbar_z)
//   (P1, P0, PS, ZE) <- (lambda, -P1, b psbar, b zbar)
void ac_adj_step(const AcSetup& S, AcAdj& A, const double* r_n, const size_t* rec, size_t src,
                 const Arr& B, Arr& gC, double* sbar, bool par) {
  const Grid2& g = S.g;
  const double h = S.h;
  for (int r = 0; r < S.nrec; ++r) A.P1[rec[r]] += r_n[r];
  if (sbar) *sbar = S.w * A.P1[src];
  for (size_t k = 0; k < g.size(); ++k) gC[k] += A.P1[k] * B[k];
  Arr zbx(g.size()), zbz(g.size()), qbx(g.size()), qbz(g.size());
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const double cp = S.C[k] * A.P1[k];
      zbx[k] = A.ZEx[k] + cp;
      zbz[k] = A.ZEz[k] + cp;
      qbx[k] = cp + S.ax[i] * zbx[k];
      qbz[k] = cp + S.az[j] * zbz[k];
    }
  Arr psbx(g.size()), psbz(g.size()), tx(g.size()), tz(g.size());
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      psbx[k] = A.PSx[k] - d1x(qbx, g, i, j, h);
      psbz[k] = A.PSz[k] - d1z(qbz, g, i, j, h);
      tx[k] = S.ax[i] * psbx[k];
      tz[k] = S.az[j] * psbz[k];
    }
  Arr lam(g.size());
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      lam[k] = A.P0[k] + 2.0 * A.P1[k] + d2x(qbx, g, i, j, h) + d2z(qbz, g, i, j, h) -
               d1x(tx, g, i, j, h) - d1z(tz, g, i, j, h);
    }
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      A.P0[k] = -A.P1[k];
      A.PSx[k] = S.bx[i] * psbx[k];
      A.PSz[k] = S.bz[j] * psbz[k];
      A.ZEx[k] = S.bx[i] * zbx[k];
      A.ZEz[k] = S.bz[j] * zbz[k];
    }
  A.P1.swap(lam);
}

// Forward for one shot; gathers (may be null) receive [nt][nrec].
void ac_forward_shot(const AcSetup& S, int s, const double* wav, double* gath, double* snaps,
                     bool par) {
  AcState st;
  st.zeros(S.g.size());
  const size_t* rec = S.rec.empty() ? nullptr : &S.rec[(size_t)s * S.nrec];
  for (int n = 0; n < S.nt; ++n) {
    ac_step_shot(S, st, s, wav, n, nullptr, par);
    if (gath)
      for (int r = 0; r < S.nrec; ++r) gath[(size_t)n * S.nrec + r] = st.p1[rec[r]];
    if (snaps) std::copy(st.p1.begin(), st.p1.end(), snaps + (size_t)n * S.g.size());
  }
}

// Gradient for one shot with checkpointing every k steps: returns gC (padded,
// dJ/dC for this shot) and optionally sbar[nt] and the forward gathers.
void ac_gradient_shot(const AcSetup& S, int s, const double* wav, const double* resid, int k,
                      Arr& gC, double* sbar, double* gath, bool par) {
  const Grid2& g = S.g;
  const int nt = S.nt;
  if (k <= 0 || k > nt) k = nt;
  const int nseg = (nt + k - 1) / k;
  const size_t* rec = &S.rec[(size_t)s * S.nrec];
  // forward, keeping the state entering every segment
  std::vector<AcState> ck(nseg);
  AcState st;
  st.zeros(g.size());
  for (int n = 0; n < nt; ++n) {
    if (n % k == 0) ck[n / k] = st;
    ac_step_shot(S, st, s, wav, n, nullptr, par);
    if (gath)
      for (int r = 0; r < S.nrec; ++r) gath[(size_t)n * S.nrec + r] = st.p1[rec[r]];
  }
  // reverse sweep, segment by segment
  gC.assign(g.size(), 0.0);
  AcAdj A;
  A.zeros(g.size());
  std::vector<Arr> Bseg(k, Arr(g.size()));
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int n0 = sg * k, n1 = std::min(nt, n0 + k);
    AcState w = ck[sg];
    for (int n = n0; n < n1; ++n) ac_step_shot(S, w, s, wav, n, &Bseg[n - n0], par);
    for (int n = n1 - 1; n >= n0; --n)
      ac_adj_step(S, A, resid + (size_t)n * S.nrec, rec, S.src[(size_t)s * S.nsrc], Bseg[n - n0],
                  gC, sbar ? sbar + n : nullptr, par);
  }
}

// dJ/dv on the model grid from dJ/dC on the padded grid:
// C = (v dt)^2 so dJ/dv = 2 v dt^2 dJ/dC; each pad cell copies an edge cell of
// the model, so its derivative is added back onto that edge cell.
void fold_gradient(const AcSetup& S, const Arr& gC, double* grad_v) {
  const Grid2& g = S.g;
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const int ii = std::min(std::max(i - S.P, 0), S.nx - 1);
      const int jj = std::min(std::max(j - S.P, 0), S.nz - 1);
      const size_t k = g.idx(i, j);
      grad_v[(size_t)jj * S.nx + ii] += 2.0 * S.vpad[k] * S.dt * S.dt * gC[k];
    }
}

}  // namespace

extern "C" int orc_ac_forward(const orc_problem* pb, const double* v, const int* src_xz,
                              const double* wavelet, const int* rec_xz, double* gathers) {
  AcSetup S;
  if (!src_xz || !rec_xz || !wavelet || !gathers) return -1;
  if (make_setup(pb, v, src_xz, rec_xz, S)) return -1;
  const int nth = default_threads(pb);
  const bool inner = S.nshots == 1;
#pragma omp parallel for schedule(dynamic) num_threads(nth) if (!inner)
  for (int s = 0; s < S.nshots; ++s)
    ac_forward_shot(S, s, wavelet + (size_t)s * S.nt, gathers + (size_t)s * S.nt * S.nrec,
                    nullptr, inner);
  return 0;
}

extern "C" int orc_ac_wavefield(const orc_problem* pb, const double* v, const int* src_xz,
                                const double* wavelet, double* snaps) {
  AcSetup S;
  if (!src_xz || !wavelet || !snaps) return -1;
  orc_problem one = *pb;
  one.nshots = 1;
  one.nrec = 0;
  if (make_setup(&one, v, src_xz, nullptr, S)) return -1;
  omp_set_num_threads(default_threads(pb));
  ac_forward_shot(S, 0, wavelet, nullptr, snaps, true);
  return 0;
}

extern "C" int orc_ac_gradient(const orc_problem* pb, const double* v, const int* src_xz,
                               const double* wavelet, const int* rec_xz, const double* resid,
                               double* grad_v, double* grad_wavelet, double* gathers) {
  AcSetup S;
  if (!src_xz || !rec_xz || !wavelet || !resid || !grad_v) return -1;
  if (make_setup(pb, v, src_xz, rec_xz, S)) return -1;
  const int nth = default_threads(pb);
  const bool inner = S.nshots == 1;
  std::vector<Arr> gC(S.nshots);
#pragma omp parallel for schedule(dynamic) num_threads(nth) if (!inner)
  for (int s = 0; s < S.nshots; ++s)
    ac_gradient_shot(S, s, wavelet + (size_t)s * S.nt,
                     resid + (size_t)s * S.nt * S.nrec, pb->ckpt_every, gC[s],
                     grad_wavelet ? grad_wavelet + (size_t)s * S.nt : nullptr,
                     gathers ? gathers + (size_t)s * S.nt * S.nrec : nullptr, inner);
  // sum over shots in shot order, then chain to v and fold the pad
  Arr tot(S.g.size(), 0.0);
  for (int s = 0; s < S.nshots; ++s)
    for (size_t k = 0; k < tot.size(); ++k) tot[k] += gC[s][k];
  std::fill(grad_v, grad_v + (size_t)S.nx * S.nz, 0.0);
  fold_gradient(S, tot, grad_v);
  return 0;
}

// Encoded shots: nsrc sources per simulation (src_xz [nshots][nsrc][2],
// wavelet [nshots][nsrc][nt]).
extern "C" int orc_ac_forward_encoded(const orc_problem* pb, int nsrc, const double* v,
                                      const int* src_xz, const double* wavelet,
                                      const int* rec_xz, double* gathers) {
  AcSetup S;
  if (!src_xz || !rec_xz || !wavelet || !gathers) return -1;
  if (make_setup(pb, v, src_xz, rec_xz, S, nsrc)) return -1;
  const int nth = default_threads(pb);
  const bool inner = S.nshots == 1;
#pragma omp parallel for schedule(dynamic) num_threads(nth) if (!inner)
  for (int s = 0; s < S.nshots; ++s)
    ac_forward_shot(S, s, wavelet + (size_t)s * nsrc * S.nt,
                    gathers + (size_t)s * S.nt * S.nrec, nullptr, inner);
  return 0;
}

extern "C" int orc_ac_gradient_encoded(const orc_problem* pb, int nsrc, const double* v,
                                       const int* src_xz, const double* wavelet,
                                       const int* rec_xz, const double* resid, double* grad_v) {
  AcSetup S;
  if (!src_xz || !rec_xz || !wavelet || !resid || !grad_v) return -1;
  if (make_setup(pb, v, src_xz, rec_xz, S, nsrc)) return -1;
  const int nth = default_threads(pb);
  const bool inner = S.nshots == 1;
  std::vector<Arr> gC(S.nshots);
#pragma omp parallel for schedule(dynamic) num_threads(nth) if (!inner)
  for (int s = 0; s < S.nshots; ++s)
    ac_gradient_shot(S, s, wavelet + (size_t)s * nsrc * S.nt, resid + (size_t)s * S.nt * S.nrec,
                     pb->ckpt_every, gC[s], nullptr, nullptr, inner);
  Arr tot(S.g.size(), 0.0);
  for (int s = 0; s < S.nshots; ++s)
    for (size_t k = 0; k < tot.size(); ++k) tot[k] += gC[s][k];
  std::fill(grad_v, grad_v + (size_t)S.nx * S.nz, 0.0);
  fold_gradient(S, tot, grad_v);
  return 0;
}

extern "C" int orc_ac_born(const orc_problem* pb, const double* v, const double* dv,
                           const int* src_xz, const double* wavelet, const int* rec_xz,
                           double* dgathers) {
  AcSetup S;
  if (!dv || !src_xz || !rec_xz || !wavelet || !dgathers) return -1;
  if (make_setup(pb, v, src_xz, rec_xz, S)) return -1;
  const Grid2& g = S.g;
  // dC = 2 v dt^2 dv on the padded grid (the pad replicates dv like v)
  Arr dC(g.size());
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const int ii = std::min(std::max(i - S.P, 0), S.nx - 1);
      const int jj = std::min(std::max(j - S.P, 0), S.nz - 1);
      const size_t k = g.idx(i, j);
      dC[k] = 2.0 * S.vpad[k] * S.dt * S.dt * dv[(size_t)jj * S.nx + ii];
    }
  const int nth = default_threads(pb);
  const bool inner = S.nshots == 1;
#pragma omp parallel for schedule(dynamic) num_threads(nth) if (!inner)
  for (int s = 0; s < S.nshots; ++s) {
    // background p and perturbation dp advance together; dp is driven by dC * B^n
    AcState bg, pert;
    bg.zeros(g.size());
    pert.zeros(g.size());
    Arr B(g.size()), src_term(g.size());
    const size_t* rec = &S.rec[(size_t)s * S.nrec];
    double* out = dgathers + (size_t)s * S.nt * S.nrec;
    for (int n = 0; n < S.nt; ++n) {
      ac_step(S, bg, S.src[s], wavelet[(size_t)s * S.nt + n], nullptr, &B, inner);
      for (size_t k = 0; k < g.size(); ++k) src_term[k] = dC[k] * B[k];
      ac_step(S, pert, S.src[s], 0.0, &src_term, nullptr, inner);
      for (int r = 0; r < S.nrec; ++r) out[(size_t)n * S.nrec + r] = pert.p1[rec[r]];
    }
  }
  return 0;
}
