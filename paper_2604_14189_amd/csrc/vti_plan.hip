// Host-side scheduler of the pseudo-acoustic VTI path (Sec. 3.3.1, Eq. 5):
// workspace layout, the forward time loop with checkpoints every k steps, and
// the segment-wise recomputation (storing Bx', Bz' and D2x'D2z'G of each step)
// and reverse sweep that accumulate dJ/d(cx, cz, cm), folded into FP64 per
// segment and chained to dJ/d(vv, v, eta) at the end. The last keep_b
// segments are stored instead: the saving forward writes their traces and
// skips their checkpoints, and the backward reverses them without recomputing.
#include <algorithm>
#include <cstring>
#include <string>

#include "plan.h"
#include "vti.h"

namespace sweep {

namespace {

size_t take(size_t& off, size_t bytes) {
  const size_t o = off;
  off = align_up(off + bytes);
  return o;
}

template <class T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

}  // namespace

void vti_layout(const sweep_plan* p, VtiLayout& L) {
  const size_t ns = p->pb.nshots, nr = p->pb.nrec, f = sizeof(float);
  const size_t plane = (size_t)p->NX * p->NZ;
  L.plane = plane;
  L.xs = (size_t)p->NZ * 2 * p->P;
  L.zs = (size_t)2 * p->P * p->NX;
  L.aux_elems = 2 * ns * L.xs + 2 * ns * L.zs;
  size_t off = 0;
  L.ax = take(off, p->NX * f);
  L.bx = take(off, p->NX * f);
  L.az = take(off, p->NZ * f);
  L.bz = take(off, p->NZ * f);
  L.pad = take(off, 3 * plane * f);
  L.cx = take(off, plane * f);
  L.cz = take(off, plane * f);
  L.cm = take(off, plane * f);
  L.wav = take(off, ns * p->pb.nt * f);
  L.src_cell = take(off, ns * sizeof(int));
  L.rec_cell = take(off, std::max<size_t>(ns * nr, 1) * sizeof(int));
  L.rec_off = take(off, (ns * (size_t)p->ntiles + 1) * sizeof(int));
  L.rec_ent = take(off, std::max<size_t>(ns * nr, 1) * sizeof(int2));
  L.tl = take(off, std::max<size_t>(p->ntiles, 1) * sizeof(int));
  for (int i = 0; i < 2; ++i) L.pf[i] = take(off, ns * plane * sizeof(double));
  for (int i = 0; i < 2; ++i) L.gf[i] = take(off, ns * plane * sizeof(double));
  for (int i = 0; i < 2; ++i) L.aux[i] = take(off, L.aux_elems * f);
  L.fwd_end = off;
  const int k = p->ckpt;
  L.nseg = (p->pb.nt + k - 1) / k;
  // in floats: P^n, P^{n-1}, G^n, G^{n-1} (float64), memory variables
  L.slot_elems = 8 * ns * plane + L.aux_elems;
  // stored segments are never restored: only the others have a checkpoint
  L.nkeep = std::min(std::max(p->tune.keep_b, 0), L.nseg);
  L.ck = take(off, (size_t)(L.nseg - L.nkeep) * L.slot_elems * f);
  L.tr = take(off, (size_t)k * 3 * ns * plane * f);
  for (int i = 0; i < 2; ++i) L.lf[i] = take(off, ns * plane * f);
  for (int i = 0; i < 2; ++i) L.mf[i] = take(off, ns * plane * sizeof(double));
  for (int i = 0; i < 2; ++i) L.adjaux[i] = take(off, L.aux_elems * f);
  L.gpart = take(off, 3 * ns * plane * f);
  L.tot = take(off, 3 * plane * sizeof(double));
  L.trkeep = take(off, (size_t)L.nkeep * k * 3 * ns * plane * f);
  L.bwd_end = off;
}

namespace {

bool vti_kept(const VtiLayout& L, int sg) { return sg >= L.nseg - L.nkeep; }

// Trace plane q of step m of segment sg: its stored block for a stored
// segment, else the one segment buffer that the recomputation fills.
float* vti_trace(void* work, const VtiLayout& L, size_t nsplane, int k, int sg, int m, int q) {
  if (vti_kept(L, sg))
    return reinterpret_cast<float*>(static_cast<char*>(work) + L.trkeep) +
           (((size_t)(sg - (L.nseg - L.nkeep)) * k + m) * 3 + q) * nsplane;
  return reinterpret_cast<float*>(static_cast<char*>(work) + L.tr) +
         ((size_t)m * 3 + q) * nsplane;
}

VtiStep vti_base(const sweep_plan* p, void* work, const VtiLayout& L) {
  VtiStep a;
  std::memset(&a, 0, sizeof(a));
  a.NX = p->NX;
  a.NZ = p->NZ;
  a.P = p->P;
  a.nt = p->pb.nt;
  a.nrec = p->pb.nrec;
  a.nshots = p->pb.nshots;
  a.tiles_x = p->tiles_x;
  a.ntiles = p->ntiles;
  a.w = (float)((double)p->pb.dt * p->pb.dt / ((double)p->pb.h * p->pb.h));
  a.cx = at<float>(work, L.cx);
  a.cz = at<float>(work, L.cz);
  a.cm = at<float>(work, L.cm);
  a.ax = at<float>(work, L.ax);
  a.bx = at<float>(work, L.bx);
  a.az = at<float>(work, L.az);
  a.bz = at<float>(work, L.bz);
  a.src_cell = at<int>(work, L.src_cell);
  a.wavelet = at<float>(work, L.wav);
  a.rec_off = at<int>(work, L.rec_off);
  a.rec_ent = at<int2>(work, L.rec_ent);
  a.tl = at<int>(work, L.tl);
  a.n_int = p->vti_nint;
  a.n_pml = p->ntiles - p->vti_nint;
  return a;
}

// The tile list of the step kernels (interior tiles first) on the plan.
void vti_split_tiles(sweep_plan* p) {
  std::vector<int> rest;
  p->vti_tl.clear();
  for (int t = 0; t < p->ntiles; ++t) {
    const int x0 = (t % p->tiles_x) * kTX, z0 = (t / p->tiles_x) * kVtiTZ;
    if (vti_near_strip(x0, z0, p->NX, p->NZ, p->P))
      rest.push_back(t);
    else
      p->vti_tl.push_back(t);
  }
  p->vti_nint = (int)p->vti_tl.size();
  p->vti_tl.insert(p->vti_tl.end(), rest.begin(), rest.end());
}

// the four memory-variable arrays of an aux block: psx, zex, psz, zez
void set_aux(VtiStep& a, float* in, float* out, const VtiLayout& L, size_t ns) {
  const size_t o[4] = {0, ns * L.xs, 2 * ns * L.xs, 2 * ns * L.xs + ns * L.zs};
  a.psx_in = in + o[0];
  a.zex_in = in + o[1];
  a.psz_in = in + o[2];
  a.zez_in = in + o[3];
  a.psx_out = out + o[0];
  a.zex_out = out + o[1];
  a.psz_out = out + o[2];
  a.zez_out = out + o[3];
}

int check_bytes(size_t need, void* work, size_t bytes) {
  if (!work) {
    set_error("workspace pointer is null");
    return SWEEP_EINVAL;
  }
  if (bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes, got " +
              std::to_string(bytes));
    return SWEEP_ENOMEM;
  }
  return SWEEP_OK;
}

// Forward step n from the buffer pair c (P^n in pf[c], P^{n-1} in pf[1-c]);
// tr: the step's trace planes or null.
int vti_fwd_step(sweep_plan* p, void* work, const VtiLayout& L, int n, int c, float* gathers,
                 float* const* tr, hipStream_t s, int cls) {
  const size_t ns = p->pb.nshots;
  VtiStep a = vti_base(p, work, L);
  a.n = n;
  a.pcur = at<double>(work, L.pf[c]);
  a.pprev = at<double>(work, L.pf[1 - c]);
  a.gcur = at<double>(work, L.gf[c]);
  a.gprev = at<double>(work, L.gf[1 - c]);
  set_aux(a, at<float>(work, L.aux[n % 2]), at<float>(work, L.aux[1 - n % 2]), L, ns);
  a.gathers = gathers;
  if (tr)
    for (int q = 0; q < 3; ++q) a.tr[q] = tr[q];
  hipEvent_t* ev = p->timer.take(cls, -1, -1);
  if (ev && ev[0]) SWEEP_HIP(hipEventRecord(ev[0], s));
  const int rc = vti_launch_fwd(a, s);
  if (ev && ev[1]) SWEEP_HIP(hipEventRecord(ev[1], s));
  return rc;
}

}  // namespace

// Workspace checks, the tile lists and the geometry upload (host copies, kept
// out of a captured graph).
int vti_forward_prepare(sweep_plan* p, void* work, size_t bytes, int save, hipStream_t s) {
  VtiLayout L;
  vti_layout(p, L);
  int rc = check_bytes(save ? L.bwd_end : L.fwd_end, work, bytes);
  if (rc) return rc;
  const sweep_problem& pb = p->pb;
  const size_t ns = pb.nshots;
  SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.src_cell), p->src_cell.data(), ns * sizeof(int),
                           hipMemcpyHostToDevice, s));
  if (pb.nrec > 0) {
    SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.rec_cell), p->rec_cell.data(),
                             p->rec_cell.size() * sizeof(int), hipMemcpyHostToDevice, s));
    SWEEP_HIP(hipMemcpyAsync(at<int2>(work, L.rec_ent), p->rec_ent.data(),
                             p->rec_ent.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  }
  SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.rec_off), p->rec_off.data(),
                           p->rec_off.size() * sizeof(int), hipMemcpyHostToDevice, s));
  vti_split_tiles(p);
  SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.tl), p->vti_tl.data(), p->vti_tl.size() * sizeof(int),
                           hipMemcpyHostToDevice, s));
  return SWEEP_OK;
}

// The forward's device work (kernels only: it may be captured).
int vti_forward_enqueue(sweep_plan* p, const float* model, const float* wavelet,
                        float* gathers, void* work, int save, hipStream_t s) {
  VtiLayout L;
  vti_layout(p, L);
  const sweep_problem& pb = p->pb;
  const size_t ns = pb.nshots, nsplane = ns * L.plane;
  int rc;
  if ((rc = ac_launch_tables(at<float>(work, L.ax), at<float>(work, L.bx), at<float>(work, L.az),
                             at<float>(work, L.bz), p->NX, p->NZ, p->P, pb.h, pb.dt, pb.pml_vmax,
                             pb.pml_f0, pb.pml_R, s)))
    return rc;
  if ((rc = vti_launch_prep(model, at<float>(work, L.pad), at<float>(work, L.cx),
                            at<float>(work, L.cz), at<float>(work, L.cm), pb.nx, pb.nz, p->P,
                            pb.h, pb.dt, s)))
    return rc;
  if ((rc = launch_copy(at<float>(work, L.wav), wavelet, ns * pb.nt, s))) return rc;
  for (int i = 0; i < 2; ++i) {
    if ((rc = launch_fill(at<float>(work, L.pf[i]), 2 * nsplane, 0.0f, s))) return rc;
    if ((rc = launch_fill(at<float>(work, L.gf[i]), 2 * nsplane, 0.0f, s))) return rc;
    if ((rc = launch_fill(at<float>(work, L.aux[i]), L.aux_elems, 0.0f, s))) return rc;
  }
  const int k = p->ckpt;
  int c = 0;
  for (int n = 0; n < pb.nt; ++n) {
    if (save && n % k == 0 && !vti_kept(L, n / k)) {
      float* slot = at<float>(work, L.ck) + (size_t)(n / k) * L.slot_elems;
      // P and G as raw bits: two floats per float64 value
      if ((rc = launch_copy(slot, at<float>(work, L.pf[c]), 2 * nsplane, s))) return rc;
      if ((rc = launch_copy(slot + 2 * nsplane, at<float>(work, L.pf[1 - c]), 2 * nsplane, s)))
        return rc;
      if ((rc = launch_copy(slot + 4 * nsplane, at<float>(work, L.gf[c]), 2 * nsplane, s)))
        return rc;
      if ((rc = launch_copy(slot + 6 * nsplane, at<float>(work, L.gf[1 - c]), 2 * nsplane, s)))
        return rc;
      if ((rc = launch_copy(slot + 8 * nsplane, at<float>(work, L.aux[n % 2]), L.aux_elems, s)))
        return rc;
    }
    // steps of a stored segment also write its traces (timed with the
    // recomputation, whose work they do)
    const int sg = n / k;
    if (save && vti_kept(L, sg)) {
      float* tr[3];
      for (int q = 0; q < 3; ++q) tr[q] = vti_trace(work, L, nsplane, k, sg, n - sg * k, q);
      if ((rc = vti_fwd_step(p, work, L, n, c, gathers, tr, s, kRecInt))) return rc;
    } else if ((rc = vti_fwd_step(p, work, L, n, c, gathers, nullptr, s, kFwdInt))) {
      return rc;
    }
    c = 1 - c;
  }
  return SWEEP_OK;
}

void vti_mark_saved(sweep_plan* p, void* work, const float* model, int save) {
  p->saved = save != 0;
  p->saved_work = work;
  p->saved_model = model;
  p->saved_rz = p->tune.rz;
}

int vti_forward(sweep_plan* p, const float* model, const float* wavelet, float* gathers,
                void* work, size_t bytes, int save, hipStream_t s) {
  int rc = vti_forward_prepare(p, work, bytes, save, s);
  if (!rc) rc = vti_forward_enqueue(p, model, wavelet, gathers, work, save, s);
  if (!rc) vti_mark_saved(p, work, model, save);
  return rc;
}

int vti_backward_check(const sweep_plan* p, const void* work, size_t bytes) {
  if (!p->saved || p->saved_work != work) {
    set_error("sweep_backward needs a preceding sweep_forward(save_for_backward=1) on the "
              "same workspace");
    return SWEEP_ESTATE;
  }
  VtiLayout L;
  vti_layout(p, L);
  return check_bytes(L.bwd_end, const_cast<void*>(work), bytes);
}

int vti_backward(sweep_plan* p, const float* resid, float* grad, void* work, size_t bytes,
                 hipStream_t s) {
  const int rc = vti_backward_check(p, work, bytes);
  return rc ? rc : vti_backward_enqueue(p, resid, grad, work, s);
}

// The backward's device work (kernels only: it may be captured).
int vti_backward_enqueue(sweep_plan* p, const float* resid, float* grad, void* work,
                         hipStream_t s) {
  VtiLayout L;
  vti_layout(p, L);
  int rc;
  const sweep_problem& pb = p->pb;
  const int nt = pb.nt, k = p->ckpt;
  const size_t ns = pb.nshots, nsplane = ns * L.plane;
  int ac = 0;
  if ((rc = ac_launch_adj_init(at<float>(work, L.lf[0]), at<float>(work, L.lf[1]), nsplane,
                               at<float>(work, L.adjaux[0]), L.aux_elems,
                               at<int>(work, L.rec_cell), resid, (int)ns, nt, pb.nrec, s)))
    return rc;
  for (int i = 0; i < 2; ++i)
    if ((rc = launch_fill(at<float>(work, L.mf[i]), 2 * nsplane, 0.0f, s))) return rc;
  if ((rc = launch_fill(at<float>(work, L.adjaux[1]), L.aux_elems, 0.0f, s))) return rc;
  if ((rc = launch_fill_f64(at<double>(work, L.tot), 3 * L.plane, 0.0, s))) return rc;
  for (int sg = L.nseg - 1; sg >= 0; --sg) {
    const int n0 = sg * k, n1 = std::min(nt, n0 + k);
    // a stored segment's traces were written by the forward: nothing to recompute
    if (!vti_kept(L, sg)) {
      // restore the state entering step n0 into buffer pair 0 and aux[n0 % 2]
      const float* slot = at<float>(work, L.ck) + (size_t)sg * L.slot_elems;
      if ((rc = launch_copy(at<float>(work, L.pf[0]), slot, 2 * nsplane, s))) return rc;
      if ((rc = launch_copy(at<float>(work, L.pf[1]), slot + 2 * nsplane, 2 * nsplane, s)))
        return rc;
      if ((rc = launch_copy(at<float>(work, L.gf[0]), slot + 4 * nsplane, 2 * nsplane, s)))
        return rc;
      if ((rc = launch_copy(at<float>(work, L.gf[1]), slot + 6 * nsplane, 2 * nsplane, s)))
        return rc;
      if ((rc = launch_copy(at<float>(work, L.aux[n0 % 2]), slot + 8 * nsplane, L.aux_elems, s)))
        return rc;
      int c = 0;
      for (int n = n0; n < n1; ++n) {
        float* tr[3];
        for (int q = 0; q < 3; ++q) tr[q] = vti_trace(work, L, nsplane, k, sg, n - n0, q);
        if ((rc = vti_fwd_step(p, work, L, n, c, nullptr, tr, s, kRecInt))) return rc;
        c = 1 - c;
      }
    }
    for (int n = n1 - 1; n >= n0; --n) {
      const int it = nt - 1 - n;
      VtiStep a = vti_base(p, work, L);
      a.n = n;
      a.resid = resid;
      a.cur = at<float>(work, L.lf[ac]);
      a.prev = at<float>(work, L.lf[1 - ac]);
      a.mcur = at<double>(work, L.mf[ac]);
      a.mprev = at<double>(work, L.mf[1 - ac]);
      set_aux(a, at<float>(work, L.adjaux[it % 2]), at<float>(work, L.adjaux[(it + 1) % 2]), L,
              ns);
      for (int q = 0; q < 3; ++q) a.trc[q] = vti_trace(work, L, nsplane, k, sg, n - n0, q);
      a.g = at<float>(work, L.gpart);
      a.g_init = (n == n1 - 1);
      hipEvent_t* ev = p->timer.take(kAdjInt, -1, -1);
      if (ev && ev[0]) SWEEP_HIP(hipEventRecord(ev[0], s));
      if ((rc = vti_launch_adj(a, s))) return rc;
      if (ev && ev[1]) SWEEP_HIP(hipEventRecord(ev[1], s));
      ac = 1 - ac;
    }
    if ((rc = vti_launch_fold(at<double>(work, L.tot), at<float>(work, L.gpart), (int)ns, L.plane,
                              s)))
      return rc;
  }
  return vti_launch_finish(at<double>(work, L.tot), at<float>(work, L.pad), grad, pb.nx, pb.nz,
                           p->P, pb.dt / pb.h, s);
}

}  // namespace sweep
