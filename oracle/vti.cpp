// FP64 CPU oracle: pseudo-acoustic wave equation for 2-D VTI media (Sec. 3.3.1,
// Eq. 5).
//
// TEST INFRASTRUCTURE ONLY (see oracle.h). The paper gives the PDE pair
//   P_tt = (1 + 2 eta) v^2 P_xx + vv^2 P_zz - 2 eta v^2 vv^2 F_xxzz,  P = F_tt
// (v the NMO velocity, vv the vertical P velocity, eta the anisotropy
// parameter) and leaves the discretisation to its reference. The reading
// taken here (written out in oracle/README.md):
//  * both P and the auxiliary field F advance by the leapfrog of the acoustic
//    step; F^{n+1} = 2 F^n - F^{n-1} + dt^2 P^n is the centred form of P = F_tt;
//  * P_xx, P_zz are the 8th-order second derivatives of the acoustic scheme,
//    each with its axis's C-PML memory terms (one profile per axis, as there);
//    F_xxzz is the composition D2x(D2z F) of the same operators, zero outside
//    the grid;
//  * the model (vv, v, eta) is replicated from its edge cells into the pad,
//    except eta, which is 0 in the pad: the absorbing layer is elliptic
//    (v^2 P_xx + vv^2 P_zz), where the per-axis C-PML applies as it stands.
// With Cx = (1 + 2 eta) v^2 dt^2, Cz = vv^2 dt^2 and Cm = 2 eta v^2 vv^2 dt^2,
// step n is
//   psi, Q, zeta per axis exactly as in the acoustic step, Bx = Qx + zeta_x^n,
//   Bz = Qz + zeta_z^n, M^n = D2x D2z F^n,
//   P^{n+1} = 2 P^n - P^{n-1} + Cx Bx + Cz Bz - Cm M^n + (dt^2/h^2) s_n e_src,
//   F^{n+1} = 2 F^n - F^{n-1} + dt^2 P^n,  d_n = P^{n+1}[rec].
// Plain loops over whole arrays, nothing blocked or fused.
#include <omp.h>

#include <algorithm>
#include <cstddef>
#include <vector>

#include "oracle.h"
#include "stencil.h"

using namespace orc;

namespace {

struct VtiSetup {
  Grid2 g;
  int P = 0, nx = 0, nz = 0, nt = 0, nshots = 0, nrec = 0;
  double h = 0, dt = 0, w = 0;   // w = dt^2 / h^2: source scaling
  Arr vv, vn, eta;               // padded model (eta = 0 in the pad)
  Arr Cx, Cz, Cm;
  Arr ax, bx, az, bz;
  std::vector<size_t> src, rec;
};

// Model cell that padded cell (i, j) replicates, and whether (i, j) is a pad cell.
inline size_t model_cell(const VtiSetup& S, int i, int j, bool* pad) {
  const int ii = std::min(std::max(i - S.P, 0), S.nx - 1);
  const int jj = std::min(std::max(j - S.P, 0), S.nz - 1);
  *pad = (i - S.P) != ii || (j - S.P) != jj;
  return (size_t)jj * S.nx + ii;
}

int vti_setup(const orc_problem* pb, const double* model, const int* src_xz, const int* rec_xz,
              VtiSetup& S) {
  if (!pb || !model || pb->nx <= 0 || pb->nz <= 0 || pb->pml < 0 || pb->nt < 1 || pb->h <= 0 ||
      pb->dt <= 0 || pb->nshots < 1 || pb->nrec < 0 || pb->free_surface)
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
  const size_t mn = (size_t)pb->nx * pb->nz;
  for (Arr* a : {&S.vv, &S.vn, &S.eta, &S.Cx, &S.Cz, &S.Cm}) a->assign(g.size(), 0.0);
  const double dt2 = pb->dt * pb->dt;
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      bool pad = false;
      const size_t m = model_cell(S, i, j, &pad), k = g.idx(i, j);
      const double vv = model[m], vn = model[mn + m], et = pad ? 0.0 : model[2 * mn + m];
      if (et < 0.0) return -1;  // eta >= 0: the scheme's two modes stay real
      S.vv[k] = vv;
      S.vn[k] = vn;
      S.eta[k] = et;
      S.Cx[k] = (1.0 + 2.0 * et) * vn * vn * dt2;
      S.Cz[k] = vv * vv * dt2;
      S.Cm[k] = 2.0 * et * vn * vn * vv * vv * dt2;
    }
  for (Arr* a : {&S.ax, &S.bx}) a->assign(g.NX, 0.0);
  for (Arr* a : {&S.az, &S.bz}) a->assign(g.NZ, 0.0);
  orc_pml_profile(g.NX, S.P, S.P, 0.0, pb->h, pb->dt, pb->pml_vmax, pb->pml_f0, pb->pml_R,
                  S.ax.data(), S.bx.data());
  orc_pml_profile(g.NZ, S.P, S.P, 0.0, pb->h, pb->dt, pb->pml_vmax, pb->pml_f0, pb->pml_R,
                  S.az.data(), S.bz.data());
  if (src_xz) {
    S.src.resize(S.nshots);
    for (int s = 0; s < S.nshots; ++s) {
      const int x = src_xz[2 * s], z = src_xz[2 * s + 1];
      if (x < 0 || x >= pb->nx || z < 0 || z >= pb->nz) return -1;
      S.src[s] = g.idx(x + S.P, z + S.P);
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

// out = D2x D2z f (zero outside the grid in both passes)
void d2xz(const Arr& f, Arr& out, const Grid2& g, double h, bool par) {
  Arr t(g.size());
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) t[g.idx(i, j)] = d2z(f, g, i, j, h);
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) out[g.idx(i, j)] = d2x(t, g, i, j, h);
}

// State entering step n: P^{n-1}, P^n, F^{n-1}, F^n, memory variables at n-1.
struct VtiState {
  Arr p0, p1, f0, f1, psx, psz, zex, zez;
  void zeros(size_t n) {
    for (Arr* a : {&p0, &p1, &f0, &f1, &psx, &psz, &zex, &zez}) a->assign(n, 0.0);
  }
};

// The terms of step n that the gradient needs: Bx, Bz, M^n.
struct VtiTrace {
  Arr Bx, Bz, M;
};

void vti_step(const VtiSetup& S, VtiState& st, size_t src, double s_n, VtiTrace* tr, bool par) {
  const Grid2& g = S.g;
  const double h = S.h, dt2 = S.dt * S.dt;
  Arr psx(g.size()), psz(g.size()), pn(g.size()), fn(g.size()), M(g.size());
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      psx[k] = S.bx[i] * st.psx[k] + S.ax[i] * d1x(st.p1, g, i, j, h);
      psz[k] = S.bz[j] * st.psz[k] + S.az[j] * d1z(st.p1, g, i, j, h);
    }
  d2xz(st.f1, M, g, h, par);
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      const double Qx = d2x(st.p1, g, i, j, h) + d1x(psx, g, i, j, h);
      const double Qz = d2z(st.p1, g, i, j, h) + d1z(psz, g, i, j, h);
      st.zex[k] = S.bx[i] * st.zex[k] + S.ax[i] * Qx;
      st.zez[k] = S.bz[j] * st.zez[k] + S.az[j] * Qz;
      const double Bx = Qx + st.zex[k], Bz = Qz + st.zez[k];
      pn[k] = 2.0 * st.p1[k] - st.p0[k] + S.Cx[k] * Bx + S.Cz[k] * Bz - S.Cm[k] * M[k];
      fn[k] = 2.0 * st.f1[k] - st.f0[k] + dt2 * st.p1[k];
      if (tr) {
        tr->Bx[k] = Bx;
        tr->Bz[k] = Bz;
      }
    }
  pn[src] += S.w * s_n;
  if (tr) tr->M.swap(M);
  st.psx.swap(psx);
  st.psz.swap(psz);
  st.p0.swap(st.p1);
  st.p1.swap(pn);
  st.f0.swap(st.f1);
  st.f1.swap(fn);
}

// Adjoint state entering the reverse of step n: P1, H1 = adjoints of P^{n+1},
// F^{n+1}; P0, H0 = the parts of the adjoints of P^n, F^n that step n+1
// contributed (-P1, -H1 of that step); PS / ZE = adjoints of psi^n / zeta^n.
struct VtiAdj {
  Arr P1, P0, H1, H0, PSx, PSz, ZEx, ZEz;
  void zeros(size_t n) {
    for (Arr* a : {&P1, &P0, &H1, &H0, &PSx, &PSz, &ZEx, &ZEz}) a->assign(n, 0.0);
  }
};

// Reverse of step n, the exact transpose of vti_step (D2 symmetric, D1
// antisymmetric and D2x D2z symmetric on the zero-padded grid):
//   P1[rec] += r_n ; sbar_n = (dt^2/h^2) P1[src]
//   gCx += P1 Bx ; gCz += P1 Bz ; gCm -= P1 M^n
//   zbar_x = ZE_x + Cx P1 ; Qbar_x = Cx P1 + a_x zbar_x ; psbar_x = PS_x - D1x Qbar_x
//   (z likewise with Cz)
//   lambda = P0 + 2 P1 + D2x Qbar_x + D2z Qbar_z - D1x(a_x psbar_x) - D1z(a_z psbar_z) + dt^2 H1
//   mu     = H0 + 2 H1 - D2x D2z (Cm P1)
//   (P1, P0, H1, H0, PS, ZE) <- (lambda, -P1, mu, -H1, b psbar, b zbar)
void vti_adj_step(const VtiSetup& S, VtiAdj& A, const double* r_n, const size_t* rec, size_t src,
                  const VtiTrace& tr, Arr& gx, Arr& gz, Arr& gm, double* sbar, bool par) {
  const Grid2& g = S.g;
  const double h = S.h, dt2 = S.dt * S.dt;
  for (int r = 0; r < S.nrec; ++r) A.P1[rec[r]] += r_n[r];
  if (sbar) *sbar = S.w * A.P1[src];
  for (size_t k = 0; k < g.size(); ++k) {
    gx[k] += A.P1[k] * tr.Bx[k];
    gz[k] += A.P1[k] * tr.Bz[k];
    gm[k] -= A.P1[k] * tr.M[k];
  }
  Arr zbx(g.size()), zbz(g.size()), qbx(g.size()), qbz(g.size()), cm(g.size());
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      zbx[k] = A.ZEx[k] + S.Cx[k] * A.P1[k];
      zbz[k] = A.ZEz[k] + S.Cz[k] * A.P1[k];
      qbx[k] = S.Cx[k] * A.P1[k] + S.ax[i] * zbx[k];
      qbz[k] = S.Cz[k] * A.P1[k] + S.az[j] * zbz[k];
      cm[k] = S.Cm[k] * A.P1[k];
    }
  Arr psbx(g.size()), psbz(g.size()), tx(g.size()), tz(g.size()), mx(g.size());
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      psbx[k] = A.PSx[k] - d1x(qbx, g, i, j, h);
      psbz[k] = A.PSz[k] - d1z(qbz, g, i, j, h);
      tx[k] = S.ax[i] * psbx[k];
      tz[k] = S.az[j] * psbz[k];
    }
  d2xz(cm, mx, g, h, par);
  Arr lam(g.size()), mu(g.size());
#pragma omp parallel for if (par)
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      lam[k] = A.P0[k] + 2.0 * A.P1[k] + d2x(qbx, g, i, j, h) + d2z(qbz, g, i, j, h) -
               d1x(tx, g, i, j, h) - d1z(tz, g, i, j, h) + dt2 * A.H1[k];
      mu[k] = A.H0[k] + 2.0 * A.H1[k] - mx[k];
    }
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const size_t k = g.idx(i, j);
      A.P0[k] = -A.P1[k];
      A.H0[k] = -A.H1[k];
      A.PSx[k] = S.bx[i] * psbx[k];
      A.PSz[k] = S.bz[j] * psbz[k];
      A.ZEx[k] = S.bx[i] * zbx[k];
      A.ZEz[k] = S.bz[j] * zbz[k];
    }
  A.P1.swap(lam);
  A.H1.swap(mu);
}

void vti_forward_shot(const VtiSetup& S, int s, const double* wav, double* gath, bool par) {
  VtiState st;
  st.zeros(S.g.size());
  const size_t* rec = S.rec.empty() ? nullptr : &S.rec[(size_t)s * S.nrec];
  for (int n = 0; n < S.nt; ++n) {
    vti_step(S, st, S.src[s], wav[n], nullptr, par);
    if (gath)
      for (int r = 0; r < S.nrec; ++r) gath[(size_t)n * S.nrec + r] = st.p1[rec[r]];
  }
}

// Gradient of one shot with checkpoints every k steps: dJ/d(Cx, Cz, Cm) on
// the padded grid, optionally sbar[nt] and the forward gathers.
void vti_gradient_shot(const VtiSetup& S, int s, const double* wav, const double* resid, int k,
                       Arr& gx, Arr& gz, Arr& gm, double* sbar, double* gath, bool par) {
  const Grid2& g = S.g;
  const int nt = S.nt;
  if (k <= 0 || k > nt) k = nt;
  const int nseg = (nt + k - 1) / k;
  const size_t* rec = &S.rec[(size_t)s * S.nrec];
  std::vector<VtiState> ck(nseg);
  VtiState st;
  st.zeros(g.size());
  for (int n = 0; n < nt; ++n) {
    if (n % k == 0) ck[n / k] = st;
    vti_step(S, st, S.src[s], wav[n], nullptr, par);
    if (gath)
      for (int r = 0; r < S.nrec; ++r) gath[(size_t)n * S.nrec + r] = st.p1[rec[r]];
  }
  for (Arr* a : {&gx, &gz, &gm}) a->assign(g.size(), 0.0);
  VtiAdj A;
  A.zeros(g.size());
  std::vector<VtiTrace> seg(k);
  for (VtiTrace& t : seg)
    for (Arr* a : {&t.Bx, &t.Bz, &t.M}) a->assign(g.size(), 0.0);
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int n0 = sg * k, n1 = std::min(nt, n0 + k);
    VtiState w = ck[sg];
    for (int n = n0; n < n1; ++n) vti_step(S, w, S.src[s], wav[n], &seg[n - n0], par);
    for (int n = n1 - 1; n >= n0; --n)
      vti_adj_step(S, A, resid + (size_t)n * S.nrec, rec, S.src[s], seg[n - n0], gx, gz, gm,
                   sbar ? sbar + n : nullptr, par);
  }
}

// dJ/d(vv, v, eta) on the model grid from dJ/d(Cx, Cz, Cm) on the padded grid:
//   Cx = (1+2 eta) v^2 dt^2, Cz = vv^2 dt^2, Cm = 2 eta v^2 vv^2 dt^2;
// pad cells replicate the edge cells' vv and v (their derivatives fold back
// onto those cells) but hold eta = 0, which depends on no model value.
void fold(const VtiSetup& S, const Arr& gx, const Arr& gz, const Arr& gm, double* grad) {
  const Grid2& g = S.g;
  const size_t mn = (size_t)S.nx * S.nz;
  const double dt2 = S.dt * S.dt;
  std::fill(grad, grad + 3 * mn, 0.0);
  for (int j = 0; j < g.NZ; ++j)
    for (int i = 0; i < g.NX; ++i) {
      bool pad = false;
      const size_t m = model_cell(S, i, j, &pad), k = g.idx(i, j);
      const double vv = S.vv[k], vn = S.vn[k], et = S.eta[k];
      grad[m] += gz[k] * 2.0 * vv * dt2 + gm[k] * 4.0 * et * vn * vn * vv * dt2;
      grad[mn + m] += gx[k] * 2.0 * (1.0 + 2.0 * et) * vn * dt2 + gm[k] * 4.0 * et * vn * vv * vv * dt2;
      if (!pad) grad[2 * mn + m] += gx[k] * 2.0 * vn * vn * dt2 + gm[k] * 2.0 * vn * vn * vv * vv * dt2;
    }
}

}  // namespace

extern "C" int orc_vti_forward(const orc_problem* pb, const double* model, const int* src_xz,
                               const double* wavelet, const int* rec_xz, double* gathers) {
  VtiSetup S;
  if (!src_xz || !rec_xz || !wavelet || !gathers) return -1;
  if (vti_setup(pb, model, src_xz, rec_xz, S)) return -1;
  const int nth = default_threads(pb);
  const bool inner = S.nshots == 1;
#pragma omp parallel for schedule(dynamic) num_threads(nth) if (!inner)
  for (int s = 0; s < S.nshots; ++s)
    vti_forward_shot(S, s, wavelet + (size_t)s * S.nt, gathers + (size_t)s * S.nt * S.nrec,
                     inner);
  return 0;
}

extern "C" int orc_vti_gradient(const orc_problem* pb, const double* model, const int* src_xz,
                                const double* wavelet, const int* rec_xz, const double* resid,
                                double* grad, double* grad_wavelet, double* gathers) {
  VtiSetup S;
  if (!src_xz || !rec_xz || !wavelet || !resid || !grad) return -1;
  if (vti_setup(pb, model, src_xz, rec_xz, S)) return -1;
  const int nth = default_threads(pb);
  const bool inner = S.nshots == 1;
  std::vector<Arr> gx(S.nshots), gz(S.nshots), gm(S.nshots);
#pragma omp parallel for schedule(dynamic) num_threads(nth) if (!inner)
  for (int s = 0; s < S.nshots; ++s)
    vti_gradient_shot(S, s, wavelet + (size_t)s * S.nt, resid + (size_t)s * S.nt * S.nrec,
                      pb->ckpt_every, gx[s], gz[s], gm[s],
                      grad_wavelet ? grad_wavelet + (size_t)s * S.nt : nullptr,
                      gathers ? gathers + (size_t)s * S.nt * S.nrec : nullptr, inner);
  // sum over shots in shot order, then the chain rule and the pad fold
  Arr tx(S.g.size(), 0.0), tz(S.g.size(), 0.0), tm(S.g.size(), 0.0);
  for (int s = 0; s < S.nshots; ++s)
    for (size_t k = 0; k < tx.size(); ++k) {
      tx[k] += gx[s][k];
      tz[k] += gz[s][k];
      tm[k] += gm[s][k];
    }
  fold(S, tx, tz, tm, grad);
  return 0;
}
