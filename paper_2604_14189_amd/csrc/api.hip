// C-ABI entry points (include/sweep.h): plans, workspace layout, and the
// host-side scheduler that enqueues the time loop, the checkpointed
// recomputation and the reverse sweep on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "plan.h"

namespace sweep {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

KernelTimer::~KernelTimer() {
  for (auto& v : ev)
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
}

void KernelTimer::reset() {
  for (int c = 0; c < kNumClasses; ++c) used[c] = 0;
}

hipEvent_t* KernelTimer::take(int ci, int cf) {
  if (!on) return nullptr;
  const int cls[2] = {ci, cf};
  for (int k = 0; k < 2; ++k) {
    if (cls[k] < 0) continue;
    std::vector<hipEvent_t>& v = ev[cls[k]];
    while (v.size() < used[cls[k]] + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      v.push_back(e);
    }
    quad[2 * k] = v[used[cls[k]]];
    quad[2 * k + 1] = v[used[cls[k]] + 1];
    used[cls[k]] += 2;
  }
  return quad;
}

// ------------------------------------------------------------------ layout
namespace {

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  }
};

}  // namespace

// Splits [lo, hi) into pieces of at most 48 cells.
static void add_chunks(std::vector<int2>& v, int lo, int hi) {
  for (int c = lo; c < hi; c += 48) v.push_back(make_int2(c, std::min(48, hi - c)));
}

void ac_build_tiling(sweep_plan* p) {
  const int TZ = 4 * p->tune.rz;
  p->TZ = TZ;
  p->tiles_x = (p->NX + kTX - 1) / kTX;
  p->tiles_z = (p->NZ + TZ - 1) / TZ;
  p->ntiles = p->tiles_x * p->tiles_z;
  const int P = p->P;
  // C-PML bands: cells within P+4 of an edge along each axis (the memory
  // variables live in the outer P cells; their first derivative reaches 4 more)
  p->xchunks.clear();
  p->zchunks.clear();
  if (P > 0) {
    const int xl = std::min(P + 4, p->NX), xr = std::max(p->NX - P - 4, xl);
    add_chunks(p->xchunks, 0, xl);
    add_chunks(p->xchunks, xr, p->NX);
    const int zl = std::min(P + 4, p->NZ), zr = std::max(p->NZ - P - 4, zl);
    add_chunks(p->zchunks, 0, zl);
    add_chunks(p->zchunks, zr, p->NZ);
  }
  // receiver CSR over (shot, tile), entries sorted by (local cell, receiver)
  const int ns = p->pb.nshots, nr = p->pb.nrec;
  p->rec_off.assign((size_t)ns * p->ntiles + 1, 0);
  std::vector<std::pair<int64_t, int>> keys((size_t)ns * nr);
  for (int s = 0; s < ns; ++s)
    for (int r = 0; r < nr; ++r) {
      const int c = p->rec_cell[(size_t)s * nr + r];
      const int gx = c % p->NX, gz = c / p->NX;
      const int tile = (gz / TZ) * p->tiles_x + gx / kTX;
      const int local = (gz % TZ) * kTX + gx % kTX;
      const int64_t key = (((int64_t)s * p->ntiles + tile) << 20) | local;
      keys[(size_t)s * nr + r] = {key, r};
    }
  std::sort(keys.begin(), keys.end());
  p->rec_ent.resize(keys.size());
  for (size_t e = 0; e < keys.size(); ++e) {
    const int64_t st = keys[e].first >> 20;
    p->rec_off[st + 1]++;
    p->rec_ent[e] = make_int2((int)(keys[e].first & 0xFFFFF), keys[e].second);
  }
  for (size_t i = 1; i < p->rec_off.size(); ++i) p->rec_off[i] += p->rec_off[i - 1];
}

// Worst-case tile count (smallest TZ) so the geometry area fits every tuning.
static size_t ac_max_tiles(const sweep_plan* p) {
  return (size_t)((p->NX + kTX - 1) / kTX) * (size_t)((p->NZ + 3) / 4);
}

void ac_layout(const sweep_plan* p, AcLayout& L) {
  const size_t ns = p->pb.nshots, nr = p->pb.nrec;
  const size_t plane = (size_t)p->NX * p->NZ;
  const size_t xs = (size_t)p->NZ * 2 * p->P, zs = (size_t)2 * p->P * p->NX;
  L.plane = plane;
  L.xs = xs;
  L.zs = zs;
  L.aux_elems = 2 * ns * xs + 2 * ns * zs;
  Carver c;
  const size_t f = sizeof(float);
  L.ax = c.take(p->NX * f);
  L.bx = c.take(p->NX * f);
  L.az = c.take(p->NZ * f);
  L.bz = c.take(p->NZ * f);
  L.vpad = c.take(plane * f);
  L.Cs = c.take(plane * f);
  L.wav = c.take(ns * p->pb.nt * f);
  L.src_cell = c.take(ns * sizeof(int));
  L.rec_cell = c.take(ns * nr * sizeof(int));
  L.rec_off = c.take((ns * ac_max_tiles(p) + 1) * sizeof(int));
  L.rec_ent = c.take(std::max<size_t>(ns * nr, 1) * sizeof(int2));
  L.xch = c.take(((size_t)p->NX / 48 + 4) * sizeof(int2));
  L.zch = c.take(((size_t)p->NZ / 48 + 4) * sizeof(int2));
  L.pA = c.take(ns * plane * f);
  L.pB = c.take(ns * plane * f);
  L.aux[0] = c.take(L.aux_elems * f);
  L.aux[1] = c.take(L.aux_elems * f);
  L.fwd_end = c.off;
  const int k = p->ckpt;
  L.nseg = (p->pb.nt + k - 1) / k;
  L.slot_elems = 2 * ns * plane + L.aux_elems;
  L.ck = c.take((size_t)L.nseg * L.slot_elems * f);
  L.Bseg = c.take((size_t)k * ns * plane * f);
  L.lA = c.take(ns * plane * f);
  L.lB = c.take(ns * plane * f);
  L.adjaux[0] = c.take(L.aux_elems * f);
  L.adjaux[1] = c.take(L.aux_elems * f);
  L.gpart = c.take(ns * plane * f);
  L.tot = c.take(plane * sizeof(double));
  L.bwd_end = c.off;
}

}  // namespace sweep

using namespace sweep;

namespace {

template <class T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// Points the six memory-variable arrays of an aux block (psx, zex, psz, zez order).
struct AuxPtr {
  float *psx, *zex, *psz, *zez;
};
AuxPtr aux_ptrs(float* base, const AcLayout& L, size_t ns) {
  AuxPtr a;
  a.psx = base;
  a.zex = base + ns * L.xs;
  a.psz = base + 2 * ns * L.xs;
  a.zez = base + 2 * ns * L.xs + ns * L.zs;
  return a;
}

void set_aux(AcStep& a, const AuxPtr& i, const AuxPtr& o) {
  a.psx_in = i.psx;
  a.zex_in = i.zex;
  a.psz_in = i.psz;
  a.zez_in = i.zez;
  a.psx_out = o.psx;
  a.zex_out = o.zex;
  a.psz_out = o.psz;
  a.zez_out = o.zez;
}

int check_work(const sweep_plan* p, size_t need, void* work, size_t bytes) {
  if (!work) {
    set_error("workspace pointer is null");
    return SWEEP_EINVAL;
  }
  if (bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes, got " +
              std::to_string(bytes));
    return SWEEP_ENOMEM;
  }
  (void)p;
  return SWEEP_OK;
}

AcStep ac_base(const sweep_plan* p, void* work, const AcLayout& L) {
  AcStep a;
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
  a.Cs = at<float>(work, L.Cs);
  a.ax = at<float>(work, L.ax);
  a.bx = at<float>(work, L.bx);
  a.az = at<float>(work, L.az);
  a.bz = at<float>(work, L.bz);
  a.src_cell = at<int>(work, L.src_cell);
  a.rec_off = at<int>(work, L.rec_off);
  a.rec_ent = at<int2>(work, L.rec_ent);
  a.xchunks = at<int2>(work, L.xch);
  a.n_xchunks = (int)p->xchunks.size();
  a.zchunks = at<int2>(work, L.zch);
  a.n_zchunks = (int)p->zchunks.size();
  return a;
}

int ac_upload_geometry(sweep_plan* p, void* work, const AcLayout& L, hipStream_t s) {
  SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.src_cell), p->src_cell.data(),
                           p->src_cell.size() * sizeof(int), hipMemcpyHostToDevice, s));
  if (!p->rec_cell.empty()) {
    SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.rec_cell), p->rec_cell.data(),
                             p->rec_cell.size() * sizeof(int), hipMemcpyHostToDevice, s));
    SWEEP_HIP(hipMemcpyAsync(at<int2>(work, L.rec_ent), p->rec_ent.data(),
                             p->rec_ent.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  }
  SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.rec_off), p->rec_off.data(),
                           p->rec_off.size() * sizeof(int), hipMemcpyHostToDevice, s));
  if (!p->xchunks.empty())
    SWEEP_HIP(hipMemcpyAsync(at<int2>(work, L.xch), p->xchunks.data(),
                             p->xchunks.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  if (!p->zchunks.empty())
    SWEEP_HIP(hipMemcpyAsync(at<int2>(work, L.zch), p->zchunks.data(),
                             p->zchunks.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  return SWEEP_OK;
}

int ac_forward(sweep_plan* p, const float* model, const float* wavelet, float* gathers,
               void* work, size_t bytes, int save, hipStream_t s) {
  AcLayout L;
  ac_layout(p, L);
  int rc = check_work(p, save ? L.bwd_end : L.fwd_end, work, bytes);
  if (rc) return rc;
  if ((rc = ac_upload_geometry(p, work, L, s))) return rc;
  const sweep_problem& pb = p->pb;
  if ((rc = ac_launch_prep(model, at<float>(work, L.vpad), at<float>(work, L.Cs),
                           at<float>(work, L.ax), at<float>(work, L.bx), at<float>(work, L.az),
                           at<float>(work, L.bz), pb.nx, pb.nz, p->P, pb.h, pb.dt, pb.pml_vmax,
                           pb.pml_f0, pb.pml_R, s)))
    return rc;
  const size_t ns = pb.nshots;
  float* wav = at<float>(work, L.wav);
  if ((rc = launch_copy(wav, wavelet, ns * pb.nt, s))) return rc;
  float* pA = at<float>(work, L.pA);
  float* pB = at<float>(work, L.pB);
  float* aux[2] = {at<float>(work, L.aux[0]), at<float>(work, L.aux[1])};
  if ((rc = launch_fill(pA, ns * L.plane, 0.0f, s))) return rc;
  if ((rc = launch_fill(pB, ns * L.plane, 0.0f, s))) return rc;
  if ((rc = launch_fill(aux[0], L.aux_elems, 0.0f, s))) return rc;
  if ((rc = launch_fill(aux[1], L.aux_elems, 0.0f, s))) return rc;

  AcStep base = ac_base(p, work, L);
  base.wavelet = wav;
  base.gathers = gathers;
  const int k = p->ckpt;
  float* ck = at<float>(work, L.ck);
  for (int n = 0; n < pb.nt; ++n) {
    AcStep a = base;
    a.n = n;
    float* cur = (n % 2 == 0) ? pB : pA;
    float* prev = (n % 2 == 0) ? pA : pB;
    a.cur = cur;
    a.prev = prev;
    a.next = prev;
    a.prev_adj = prev;
    set_aux(a, aux_ptrs(aux[n % 2], L, ns), aux_ptrs(aux[(n + 1) % 2], L, ns));
    if (save && n % k == 0) {
      // checkpoint: the state entering step n
      float* slot = ck + (size_t)(n / k) * L.slot_elems;
      if ((rc = launch_copy(slot, cur, ns * L.plane, s))) return rc;
      if ((rc = launch_copy(slot + ns * L.plane, prev, ns * L.plane, s))) return rc;
      if ((rc = launch_copy(slot + 2 * ns * L.plane, aux[n % 2], L.aux_elems, s))) return rc;
    }
    if ((rc = ac_launch_fwd(a, p->tune.rz, s, p->timer.take(kFwdMain, kFwdBand)))) return rc;
  }
  p->saved = save != 0;
  p->saved_work = work;
  p->saved_model = model;
  p->saved_rz = p->tune.rz;
  return SWEEP_OK;
}

int ac_backward(sweep_plan* p, const float* resid, float* grad, void* work, size_t bytes,
                hipStream_t s) {
  if (!p->saved || p->saved_work != work || p->saved_rz != p->tune.rz) {
    set_error("sweep_backward needs a preceding sweep_forward(save_for_backward=1) on the "
              "same workspace and tuning");
    return SWEEP_ESTATE;
  }
  AcLayout L;
  ac_layout(p, L);
  int rc = check_work(p, L.bwd_end, work, bytes);
  if (rc) return rc;
  const sweep_problem& pb = p->pb;
  const size_t ns = pb.nshots;
  const int nt = pb.nt, k = p->ckpt;
  float* pA = at<float>(work, L.pA);
  float* pB = at<float>(work, L.pB);
  float* aux[2] = {at<float>(work, L.aux[0]), at<float>(work, L.aux[1])};
  float* lA = at<float>(work, L.lA);
  float* lB = at<float>(work, L.lB);
  float* adjaux[2] = {at<float>(work, L.adjaux[0]), at<float>(work, L.adjaux[1])};
  float* Bseg = at<float>(work, L.Bseg);
  float* gpart = at<float>(work, L.gpart);
  double* tot = at<double>(work, L.tot);
  float* ck = at<float>(work, L.ck);

  // adjoint state: lambda^{nt} = r_{nt-1} at the receivers (iteration 0 reads lB)
  if ((rc = ac_launch_adj_init(lB, lA, ns * L.plane, adjaux[0], L.aux_elems,
                               at<int>(work, L.rec_cell), resid, (int)ns, nt, pb.nrec, s)))
    return rc;
  if ((rc = launch_fill(adjaux[1], L.aux_elems, 0.0f, s))) return rc;
  if ((rc = launch_fill_f64(tot, L.plane, 0.0, s))) return rc;

  AcStep base = ac_base(p, work, L);
  for (int sg = L.nseg - 1; sg >= 0; --sg) {
    const int n0 = sg * k, n1 = std::min(nt, n0 + k);
    // restore the state entering step n0 and recompute the segment, keeping B^n
    float* slot = ck + (size_t)sg * L.slot_elems;
    if ((rc = launch_copy(pB, slot, ns * L.plane, s))) return rc;
    if ((rc = launch_copy(pA, slot + ns * L.plane, ns * L.plane, s))) return rc;
    if ((rc = launch_copy(aux[0], slot + 2 * ns * L.plane, L.aux_elems, s))) return rc;
    for (int n = n0; n < n1; ++n) {
      const int m = n - n0;
      AcStep a = base;
      a.n = n;
      a.wavelet = at<float>(work, L.wav);
      float* prev = (m % 2 == 0) ? pA : pB;
      a.cur = (m % 2 == 0) ? pB : pA;
      a.prev = prev;
      a.next = prev;
      a.prev_adj = prev;
      set_aux(a, aux_ptrs(aux[m % 2], L, ns), aux_ptrs(aux[(m + 1) % 2], L, ns));
      a.B_out = Bseg + (size_t)m * ns * L.plane;
      if ((rc = ac_launch_fwd(a, p->tune.rz, s, p->timer.take(kRecMain, kRecBand)))) return rc;
    }
    // reverse sweep over the segment
    for (int n = n1 - 1; n >= n0; --n) {
      const int it = nt - 1 - n;
      AcStep a = base;
      a.n = n;
      a.resid = resid;
      float* prev = (it % 2 == 0) ? lA : lB;
      a.cur = (it % 2 == 0) ? lB : lA;
      a.prev = prev;
      a.next = prev;
      a.prev_adj = prev;
      set_aux(a, aux_ptrs(adjaux[it % 2], L, ns), aux_ptrs(adjaux[(it + 1) % 2], L, ns));
      a.B_in = Bseg + (size_t)(n - n0) * ns * L.plane;
      a.g = gpart;
      a.g_init = (n == n1 - 1);
      if ((rc = ac_launch_adj(a, p->tune.rz, s, p->timer.take(kAdjMain, kAdjBand)))) return rc;
    }
    if ((rc = ac_launch_fold(tot, gpart, (int)ns, L.plane, s))) return rc;
  }
  const double scale = 2.0 * (double)pb.dt * pb.dt / ((double)pb.h * pb.h);
  return ac_launch_finish(tot, at<float>(work, L.vpad), grad, pb.nx, pb.nz, p->P, p->NX, scale,
                          s);
}

}  // namespace

// ====================================================================== C-ABI
extern "C" const char* sweep_last_error(void) { return g_last_error.c_str(); }

extern "C" int sweep_plan_create(const sweep_problem* pb, const int32_t* src_xz,
                                 const int32_t* rec_xz, sweep_plan** out) {
  if (!pb || !out || !src_xz || (pb->nrec > 0 && !rec_xz)) {
    set_error("sweep_plan_create: null argument");
    return SWEEP_EINVAL;
  }
  *out = nullptr;
  if (pb->physics != SWEEP_ACOUSTIC && pb->physics != SWEEP_ELASTIC) {
    set_error("unknown physics");
    return SWEEP_EINVAL;
  }
  if (pb->nx < 1 || pb->nz < 1 || pb->pml < 0 || pb->nt < 1 || pb->nshots < 1 || pb->nrec < 0 ||
      !(pb->h > 0) || !(pb->dt > 0) || pb->ckpt_every < 0 || !(pb->pml_R > 0 && pb->pml_R < 1) ||
      !(pb->pml_vmax > 0) || pb->pml_f0 < 0) {
    set_error("sweep_plan_create: invalid sizes or constants");
    return SWEEP_EINVAL;
  }
  if (pb->physics == SWEEP_ACOUSTIC && pb->free_surface) {
    set_error("free_surface is only supported for the elastic physics");
    return SWEEP_EINVAL;
  }
  const double cfl = (double)pb->pml_vmax * pb->dt / pb->h;
  const double limit = pb->physics == SWEEP_ACOUSTIC ? 0.5546 : 0.6061;
  if (cfl > limit) {
    set_error("CFL number " + std::to_string(cfl) + " exceeds the stability limit " +
              std::to_string(limit));
    return SWEEP_ECFL;
  }
  sweep_plan* p = new (std::nothrow) sweep_plan();
  if (!p) {
    set_error("out of host memory");
    return SWEEP_EINVAL;
  }
  p->pb = *pb;
  p->P = pb->pml;
  p->NX = pb->nx + 2 * pb->pml;
  p->NZ = pb->nz + (pb->free_surface ? 1 : 2) * pb->pml;
  if ((long long)p->NX * p->NZ >= (1LL << 31) / 4 || p->NX * 16 + 16 > (1 << 20) * 16) {
    delete p;
    set_error("grid too large");
    return SWEEP_EINVAL;
  }
  p->ckpt = pb->ckpt_every > 0 ? pb->ckpt_every : 50;
  if (p->ckpt > pb->nt) p->ckpt = pb->nt;
  p->src_cell.resize(pb->nshots);
  for (int s = 0; s < pb->nshots; ++s) {
    const int x = src_xz[2 * s], z = src_xz[2 * s + 1];
    if (x < 0 || x >= pb->nx || z < 0 || z >= pb->nz) {
      delete p;
      set_error("source " + std::to_string(s) + " lies outside the model");
      return SWEEP_EINVAL;
    }
    p->src_cell[s] = (z + (pb->free_surface ? 0 : p->P)) * p->NX + x + p->P;
  }
  p->rec_cell.resize((size_t)pb->nshots * pb->nrec);
  for (size_t r = 0; r < p->rec_cell.size(); ++r) {
    const int x = rec_xz[2 * r], z = rec_xz[2 * r + 1];
    if (x < 0 || x >= pb->nx || z < 0 || z >= pb->nz) {
      delete p;
      set_error("receiver " + std::to_string(r) + " lies outside the model");
      return SWEEP_EINVAL;
    }
    p->rec_cell[r] = (z + (pb->free_surface ? 0 : p->P)) * p->NX + x + p->P;
  }
  p->tune.rz = 8;
  p->tune.shots_per_block = 1;
  p->tune.use_graph = 0;
  if (pb->physics == SWEEP_ACOUSTIC) {
    ac_build_tiling(p);
  } else {
    el_build_tables(p);
    p->rec_sorted.resize(p->rec_cell.size());
    for (size_t r = 0; r < p->rec_cell.size(); ++r)
      p->rec_sorted[r] = make_int4((int)(r / pb->nrec), p->rec_cell[r], (int)(r % pb->nrec), 0);
    std::sort(p->rec_sorted.begin(), p->rec_sorted.end(), [](const int4& a, const int4& b) {
      if (a.x != b.x) return a.x < b.x;
      if (a.y != b.y) return a.y < b.y;
      return a.z < b.z;
    });
  }
  *out = p;
  return SWEEP_OK;
}

extern "C" void sweep_plan_destroy(sweep_plan* plan) { delete plan; }

extern "C" int sweep_plan_set_tuning(sweep_plan* p, const sweep_tuning* t) {
  if (!p || !t) {
    set_error("null argument");
    return SWEEP_EINVAL;
  }
  if (!(t->rz == 1 || t->rz == 2 || t->rz == 4 || t->rz == 8) || t->shots_per_block != 1 ||
      (t->use_graph != 0 && t->use_graph != 1)) {
    set_error("unsupported tuning");
    return SWEEP_EINVAL;
  }
  p->tune = *t;
  if (p->pb.physics == SWEEP_ACOUSTIC) ac_build_tiling(p);
  p->saved = false;
  return SWEEP_OK;
}

extern "C" int sweep_plan_get_tuning(const sweep_plan* p, sweep_tuning* t) {
  if (!p || !t) {
    set_error("null argument");
    return SWEEP_EINVAL;
  }
  *t = p->tune;
  return SWEEP_OK;
}

extern "C" size_t sweep_plan_workspace_bytes(const sweep_plan* p, int for_backward) {
  if (!p) return 0;
  if (p->pb.physics == SWEEP_ELASTIC) {
    ElLayout E;
    el_layout(p, E);
    return for_backward ? E.bwd_end : E.fwd_end;
  }
  AcLayout L;
  ac_layout(p, L);
  return for_backward ? L.bwd_end : L.fwd_end;
}

extern "C" int sweep_plan_padded(const sweep_plan* p, int* NX, int* NZ) {
  if (!p || !NX || !NZ) {
    set_error("null argument");
    return SWEEP_EINVAL;
  }
  *NX = p->NX;
  *NZ = p->NZ;
  return SWEEP_OK;
}

extern "C" int sweep_forward(sweep_plan* p, const float* d_model, const float* d_wavelet,
                             float* d_gathers, void* d_work, size_t work_bytes,
                             int save_for_backward, void* stream) {
  if (!p || !d_model || !d_wavelet || (!d_gathers && p->pb.nrec > 0)) {
    set_error("sweep_forward: null argument");
    return SWEEP_EINVAL;
  }
  p->saved = false;
  if (p->pb.physics == SWEEP_ELASTIC)
    return el_forward(p, d_model, d_wavelet, d_gathers, d_work, work_bytes, save_for_backward,
                      (hipStream_t)stream);
  return ac_forward(p, d_model, d_wavelet, d_gathers, d_work, work_bytes, save_for_backward,
                    (hipStream_t)stream);
}

extern "C" int sweep_backward(sweep_plan* p, const float* d_resid, float* d_grad, void* d_work,
                              size_t work_bytes, void* stream) {
  if (!p || !d_resid || !d_grad) {
    set_error("sweep_backward: null argument");
    return SWEEP_EINVAL;
  }
  if (p->pb.physics == SWEEP_ELASTIC)
    return el_backward(p, d_resid, d_grad, d_work, work_bytes, (hipStream_t)stream);
  return ac_backward(p, d_resid, d_grad, d_work, work_bytes, (hipStream_t)stream);
}

extern "C" int sweep_plan_set_profiling(sweep_plan* p, int enable) {
  if (!p) {
    set_error("null plan");
    return SWEEP_EINVAL;
  }
  p->timer.on = enable != 0;
  p->timer.reset();
  return SWEEP_OK;
}

extern "C" int sweep_plan_kernel_time(sweep_plan* p, int kernel_class, int* launches,
                                      double* total_ms) {
  if (!p || !launches || !total_ms || kernel_class < 0 || kernel_class >= kNumClasses) {
    set_error("sweep_plan_kernel_time: bad argument");
    return SWEEP_EINVAL;
  }
  const std::vector<hipEvent_t>& v = p->timer.ev[kernel_class];
  const size_t n = p->timer.used[kernel_class];
  double tot = 0.0;
  for (size_t i = 0; i + 1 < n; i += 2) {
    SWEEP_HIP(hipEventSynchronize(v[i + 1]));
    float ms = 0.0f;
    SWEEP_HIP(hipEventElapsedTime(&ms, v[i], v[i + 1]));
    tot += ms;
  }
  *launches = (int)(n / 2);
  *total_ms = tot;
  return SWEEP_OK;
}
