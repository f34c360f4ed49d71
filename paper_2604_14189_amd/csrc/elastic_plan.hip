// Host-side scheduler of the elastic path: workspace layout, forward time loop
// with checkpoints, and the segment-wise recomputation + reverse sweep.
#include <algorithm>
#include <cstring>
#include <string>

#include "elastic.h"
#include "plan.h"

namespace sweep {

namespace {

constexpr int kCoefPlanes = 13;  // vp vs rho lam mu bx bz mxz cxx_x cxx_z czz_x czz_z smask
constexpr int kStatePlanes = 13; // vx vz txx tzz txz + 8 memory variables
constexpr int kTracePlanes = 5;  // fvx fvz exx ezz exz
constexpr int kAdjPlanes = 21;   // 5 field adjoints + 2 x 8 memory-variable adjoints
constexpr int kGradPlanes = 5;   // lambda mu mu_xz bx bz

size_t take(size_t& off, size_t bytes) {
  const size_t o = off;
  off = align_up(off + bytes);
  return o;
}

template <class T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// Forward taps (offset, weight) of z-derivative `kind` at output row j under a
// free surface: 0 Dz+ of tzz, 1 Dz- of txz, 2 Dz+ of vx, 3 Dz- of vz.
int fwd_taps(int kind, int j, int* off, float* w) {
  const float c1 = 9.0f / 8.0f, c2 = -1.0f / 24.0f;
  switch (kind) {
    case 0:
      if (j == 0) {
        off[0] = 1; w[0] = c1 + c2; off[1] = 0; w[1] = -c1; off[2] = 2; w[2] = c2;
        return 3;
      }
      off[0] = 1; w[0] = c1; off[1] = 0; w[1] = -c1; off[2] = 2; w[2] = c2; off[3] = -1; w[3] = -c2;
      return 4;
    case 1:
      if (j == 0) {
        off[0] = 0; w[0] = 2.0f * c1; off[1] = 1; w[1] = 2.0f * c2;
        return 2;
      }
      if (j == 1) {
        off[0] = 0; w[0] = c1; off[1] = -1; w[1] = -c1 + c2; off[2] = 1; w[2] = c2;
        return 3;
      }
      off[0] = 0; w[0] = c1; off[1] = -1; w[1] = -c1; off[2] = 1; w[2] = c2; off[3] = -2; w[3] = -c2;
      return 4;
    case 2:
      if (j == 0) {
        off[0] = 1; w[0] = 1.0f; off[1] = 0; w[1] = -1.0f;
        return 2;
      }
      off[0] = 1; w[0] = c1; off[1] = 0; w[1] = -c1; off[2] = 2; w[2] = c2; off[3] = -1; w[3] = -c2;
      return 4;
    case 3:
      if (j == 0) return 0;
      if (j == 1) {
        off[0] = 0; w[0] = 1.0f; off[1] = -1; w[1] = -1.0f;
        return 2;
      }
      off[0] = 0; w[0] = c1; off[1] = -1; w[1] = -c1; off[2] = 1; w[2] = c2; off[3] = -2; w[3] = -c2;
      return 4;
  }
  return 0;
}

}  // namespace

// Transposed taps for input rows 0..3: (D^T g)[jin] = sum_jout w(jout, jin) g[jout],
// collected from every output row whose forward taps reach jin.
void el_build_tables(sweep_plan* p) {
  std::memset(p->tt_cnt, 0, sizeof(p->tt_cnt));
  std::memset(p->tt_off, 0, sizeof(p->tt_off));
  std::memset(p->tt_w, 0, sizeof(p->tt_w));
  for (int kind = 0; kind < 4; ++kind)
    for (int jout = 0; jout < std::min(8, p->NZ); ++jout) {
      int off[4];
      float w[4];
      const int n = fwd_taps(kind, jout, off, w);
      for (int q = 0; q < n; ++q) {
        const int jin = jout + off[q];
        if (jin < 0 || jin >= 4 || jin >= p->NZ) continue;
        int& c = p->tt_cnt[kind][jin];
        p->tt_off[kind][jin][c] = jout - jin;
        p->tt_w[kind][jin][c] = w[q];
        ++c;
      }
    }
}

void el_layout(const sweep_plan* p, ElLayout& L) {
  const size_t ns = p->pb.nshots, nr = p->pb.nrec;
  const size_t plane = (size_t)p->NX * p->NZ;
  const size_t f = sizeof(float);
  L.plane = plane;
  size_t off = 0;
  L.coef = take(off, kCoefPlanes * plane * f);
  L.tabx = take(off, 4 * (size_t)p->NX * f);
  L.tabz = take(off, 4 * (size_t)p->NZ * f);
  L.dM = take(off, 2 * (size_t)p->NX * f);
  L.wav = take(off, ns * p->pb.nt * f);
  L.src_cell = take(off, ns * sizeof(int));
  L.rec_cell = take(off, std::max<size_t>(ns * nr, 1) * sizeof(int));
  L.rec_sorted = take(off, std::max<size_t>(ns * nr, 1) * sizeof(int4));
  L.state = take(off, kStatePlanes * ns * plane * f);
  L.fwd_end = off;
  const int k = p->ckpt;
  L.nseg = (p->pb.nt + k - 1) / k;
  // stored segments: the traces of the last keep_b segments, written by the
  // saving forward so that the backward does not recompute those segments;
  // they are never restored, so only the other segments have a checkpoint
  L.nkeep = std::min(std::max(p->tune.keep_b, 0), L.nseg);
  L.ck = take(off, (size_t)(L.nseg - L.nkeep) * kStatePlanes * ns * plane * f);
  L.trace = take(off, (size_t)k * kTracePlanes * ns * plane * f);
  L.adj = take(off, kAdjPlanes * ns * plane * f);
  L.gpart = take(off, kGradPlanes * ns * plane * f);
  L.tot = take(off, kGradPlanes * plane * sizeof(double));
  L.trkeep = take(off, (size_t)L.nkeep * k * kTracePlanes * ns * plane * f);
  L.bwd_end = off;
}

namespace {

bool el_kept(const ElLayout& L, int sg) { return sg >= L.nseg - L.nkeep; }

// Trace plane q of step m of segment sg: its stored block for a stored
// segment, else the one segment buffer that the recomputation fills.
float* el_trace(void* work, const ElLayout& L, size_t nsplane, int k, int sg, int m, int q) {
  if (el_kept(L, sg))
    return at<float>(work, L.trkeep) +
           (((size_t)(sg - (L.nseg - L.nkeep)) * k + m) * kTracePlanes + q) * nsplane;
  return at<float>(work, L.trace) + ((size_t)m * kTracePlanes + q) * nsplane;
}

ElCoef coef_ptrs(const sweep_plan* p, void* work, const ElLayout& L) {
  ElCoef c;
  float* b = at<float>(work, L.coef);
  const size_t pl = L.plane;
  float** planes[kCoefPlanes] = {&c.vp, &c.vs, &c.rho, &c.lam, &c.mu, &c.bx, &c.bz,
                                 &c.mxz, &c.cxx_x, &c.cxx_z, &c.czz_x, &c.czz_z, &c.smask};
  for (int q = 0; q < kCoefPlanes; ++q) *planes[q] = b + q * pl;
  float* tx = at<float>(work, L.tabx);
  c.axi = tx;
  c.bxi = tx + p->NX;
  c.axh = tx + 2 * p->NX;
  c.bxh = tx + 3 * p->NX;
  float* tz = at<float>(work, L.tabz);
  c.azi = tz;
  c.bzi = tz + p->NZ;
  c.azh = tz + 2 * p->NZ;
  c.bzh = tz + 3 * p->NZ;
  float* dm = at<float>(work, L.dM);
  c.dM_dl = dm;
  c.dM_dm = dm + p->NX;
  return c;
}

ElStep step_base(const sweep_plan* p, void* work, const ElLayout& L, const ElCoef& c) {
  ElStep a;
  std::memset(&a, 0, sizeof(a));
  a.NX = p->NX;
  a.NZ = p->NZ;
  a.nt = p->pb.nt;
  a.nrec = p->pb.nrec;
  a.nshots = p->pb.nshots;
  a.fs = p->pb.free_surface;
  a.fluid = p->pb.physics == SWEEP_ACOUSTIC_VD;
  a.dt = (float)p->pb.dt;
  a.w = (float)(p->pb.dt / (p->pb.h * p->pb.h));
  a.ih = (float)(1.0 / p->pb.h);
  a.bx = c.bx;
  a.bz = c.bz;
  a.mxz = c.mxz;
  a.cxx_x = c.cxx_x;
  a.cxx_z = c.cxx_z;
  a.smask = c.smask;
  a.dM_dl = c.dM_dl;
  a.dM_dm = c.dM_dm;
  a.axi = c.axi;
  a.bxi = c.bxi;
  a.axh = c.axh;
  a.bxh = c.bxh;
  a.azi = c.azi;
  a.bzi = c.bzi;
  a.azh = c.azh;
  a.bzh = c.bzh;
  a.src_cell = at<int>(work, L.src_cell);
  a.wavelet = at<float>(work, L.wav);
  a.rec_cell = at<int>(work, L.rec_cell);
  a.rec_sorted = at<int4>(work, L.rec_sorted);
  std::memcpy(a.tt_cnt, p->tt_cnt, sizeof(a.tt_cnt));
  std::memcpy(a.tt_off, p->tt_off, sizeof(a.tt_off));
  std::memcpy(a.tt_w, p->tt_w, sizeof(a.tt_w));
  return a;
}

// points the step at a 13-plane state block (5 fields then 8 memory variables)
void set_state(ElStep& a, float* st, size_t nsplane) {
  a.vx = st;
  a.vz = st + nsplane;
  a.txx = st + 2 * nsplane;
  a.tzz = st + 3 * nsplane;
  a.txz = st + 4 * nsplane;
  for (int q = 0; q < 8; ++q) a.ps[q] = st + (5 + q) * nsplane;
}

}  // namespace

// Workspace checks and the geometry upload (host copies, kept out of a
// captured graph).
int el_forward_prepare(sweep_plan* p, void* work, size_t bytes, int save, hipStream_t s) {
  ElLayout L;
  el_layout(p, L);
  const size_t need = save ? L.bwd_end : L.fwd_end;
  if (!work) {
    set_error("workspace pointer is null");
    return SWEEP_EINVAL;
  }
  if (bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return SWEEP_ENOMEM;
  }
  const sweep_problem& pb = p->pb;
  const size_t ns = pb.nshots;
  SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.src_cell), p->src_cell.data(), ns * sizeof(int),
                           hipMemcpyHostToDevice, s));
  if (pb.nrec > 0) {
    SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.rec_cell), p->rec_cell.data(),
                             p->rec_cell.size() * sizeof(int), hipMemcpyHostToDevice, s));
    SWEEP_HIP(hipMemcpyAsync(at<int4>(work, L.rec_sorted), p->rec_sorted.data(),
                             p->rec_sorted.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  }
  return SWEEP_OK;
}

// The forward's device work (kernels only: it may be captured).
int el_forward_enqueue(sweep_plan* p, const float* model, const float* wavelet, float* gathers,
                       void* work, int save, hipStream_t s) {
  ElLayout L;
  el_layout(p, L);
  const sweep_problem& pb = p->pb;
  const size_t ns = pb.nshots, nsplane = ns * L.plane;
  int rc;
  const ElCoef c = coef_ptrs(p, work, L);
  if ((rc = el_launch_prep(model, c, pb.nx, pb.nz, p->P, pb.free_surface,
                           pb.physics == SWEEP_ACOUSTIC_VD, pb.h, pb.dt, pb.pml_vmax, pb.pml_f0,
                           pb.pml_R, s)))
    return rc;
  if ((rc = launch_copy(at<float>(work, L.wav), wavelet, ns * pb.nt, s))) return rc;
  float* st = at<float>(work, L.state);
  if ((rc = launch_fill(st, kStatePlanes * nsplane, 0.0f, s))) return rc;
  ElStep base = step_base(p, work, L, c);
  set_state(base, st, nsplane);
  base.gathers = gathers;
  const int k = p->ckpt;
  float* ck = at<float>(work, L.ck);
  for (int n = 0; n < pb.nt; ++n) {
    if (save && n % k == 0 && !el_kept(L, n / k))
      if ((rc = launch_copy(ck + (size_t)(n / k) * kStatePlanes * nsplane, st,
                            kStatePlanes * nsplane, s)))
        return rc;
    ElStep a = base;
    a.n = n;
    // steps of a stored segment also write its traces (timed with the
    // recomputation, whose work they do)
    const int sg = n / k;
    const bool keepT = save && el_kept(L, sg);
    if (keepT)
      for (int q = 0; q < kTracePlanes; ++q)
        a.tr[q] = el_trace(work, L, nsplane, k, sg, n - sg * k, q);
    if ((rc = el_launch_fwd(a, s, p->timer.take(keepT ? kRecInt : kFwdInt, -1, -1)))) return rc;
  }
  return SWEEP_OK;
}

void el_mark_saved(sweep_plan* p, void* work, const float* model, int save) {
  p->saved = save != 0;
  p->saved_work = work;
  p->saved_model = model;
  p->saved_rz = p->tune.rz;
}

int el_forward(sweep_plan* p, const float* model, const float* wavelet, float* gathers,
               void* work, size_t bytes, int save, hipStream_t s) {
  int rc = el_forward_prepare(p, work, bytes, save, s);
  if (!rc) rc = el_forward_enqueue(p, model, wavelet, gathers, work, save, s);
  if (!rc) el_mark_saved(p, work, model, save);
  return rc;
}

int el_backward_check(const sweep_plan* p, const void* work, size_t bytes) {
  if (!p->saved || p->saved_work != work) {
    set_error("sweep_backward needs a preceding sweep_forward(save_for_backward=1) on the "
              "same workspace");
    return SWEEP_ESTATE;
  }
  ElLayout L;
  el_layout(p, L);
  if (bytes < L.bwd_end) {
    set_error("workspace too small for backward");
    return SWEEP_ENOMEM;
  }
  return SWEEP_OK;
}

int el_backward(sweep_plan* p, const float* resid, float* grad, void* work, size_t bytes,
                hipStream_t s) {
  const int rc = el_backward_check(p, work, bytes);
  return rc ? rc : el_backward_enqueue(p, resid, grad, work, s);
}

// The backward's device work (kernels only: it may be captured).
int el_backward_enqueue(sweep_plan* p, const float* resid, float* grad, void* work,
                        hipStream_t s) {
  ElLayout L;
  el_layout(p, L);
  const sweep_problem& pb = p->pb;
  const size_t ns = pb.nshots, nsplane = ns * L.plane;
  const int nt = pb.nt, k = p->ckpt;
  int rc;
  const ElCoef c = coef_ptrs(p, work, L);
  float* st = at<float>(work, L.state);
  float* ck = at<float>(work, L.ck);
  float* tr = at<float>(work, L.trace);
  float* adj = at<float>(work, L.adj);
  float* gpart = at<float>(work, L.gpart);
  double* tot = at<double>(work, L.tot);
  if ((rc = launch_fill(adj, kAdjPlanes * nsplane, 0.0f, s))) return rc;
  if ((rc = launch_fill_f64(tot, kGradPlanes * L.plane, 0.0, s))) return rc;
  // the fluid kernels write no mu partials (planes 1 and 2): they fold as zeros
  if (pb.physics == SWEEP_ACOUSTIC_VD &&
      (rc = launch_fill(gpart + nsplane, 2 * nsplane, 0.0f, s)))
    return rc;

  ElStep fbase = step_base(p, work, L, c);
  set_state(fbase, st, nsplane);
  ElStep abase = step_base(p, work, L, c);
  abase.resid = resid;
  abase.vx = adj;
  abase.vz = adj + nsplane;
  abase.txx = adj + 2 * nsplane;
  abase.tzz = adj + 3 * nsplane;
  abase.txz = adj + 4 * nsplane;
  float* psbuf[2] = {adj + 5 * nsplane, adj + 13 * nsplane};
  for (int q = 0; q < kGradPlanes; ++q) abase.g[q] = gpart + q * nsplane;

  for (int sg = L.nseg - 1; sg >= 0; --sg) {
    const int n0 = sg * k, n1 = std::min(nt, n0 + k);
    // a stored segment's traces were written by the forward: nothing to recompute
    if (!el_kept(L, sg) &&
        (rc = launch_copy(st, ck + (size_t)sg * kStatePlanes * nsplane, kStatePlanes * nsplane,
                          s)))
      return rc;
    for (int n = n0; n < n1 && !el_kept(L, sg); ++n) {
      ElStep a = fbase;
      a.n = n;
      for (int q = 0; q < kTracePlanes; ++q)
        a.tr[q] = tr + ((size_t)(n - n0) * kTracePlanes + q) * nsplane;
      if ((rc = el_launch_fwd(a, s, p->timer.take(kRecInt, -1, -1)))) return rc;
    }
    for (int n = n1 - 1; n >= n0; --n) {
      const int it = nt - 1 - n;
      ElStep a = abase;
      a.n = n;
      for (int q = 0; q < 8; ++q) {
        a.ps_in[q] = psbuf[it % 2] + q * nsplane;
        a.ps_out[q] = psbuf[(it + 1) % 2] + q * nsplane;
      }
      for (int q = 0; q < kTracePlanes; ++q)
        a.trc[q] = el_trace(work, L, nsplane, k, sg, n - n0, q);
      a.g_init = (n == n1 - 1);
      if ((rc = el_launch_adj(a, s, p->timer.take(kAdjInt, -1, -1)))) return rc;
    }
    if ((rc = el_launch_fold(tot, gpart, (int)ns, L.plane, s))) return rc;
  }
  return el_launch_finish(tot, c, grad, pb.nx, pb.nz, p->P, pb.free_surface,
                          pb.physics == SWEEP_ACOUSTIC_VD, s);
}

}  // namespace sweep
