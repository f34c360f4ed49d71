// C-ABI entry points (include/sweep.h): plans, workspace layout, and the
// host-side scheduler that enqueues the time loop, the checkpointed
// recomputation and the reverse sweep on the caller's stream.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <climits>
#include <fstream>
#include <sstream>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "plan.h"

namespace sweep {

namespace {
thread_local char g_last_error[1024] = "";
}

void set_error_c(const char* msg) noexcept {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg ? msg : "");
}

void set_error(const std::string& msg) { set_error_c(msg.c_str()); }

KernelTimer::~KernelTimer() {
  for (auto& v : ev)
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
}

void KernelTimer::reset() {
  for (int c = 0; c < kNumClasses; ++c) used[c] = 0;
  calls = 0;
}

hipEvent_t* KernelTimer::take(int ci, int cz, int cx) {
  if (!on || (calls++ % period) != 0) return nullptr;
  const int cls[3] = {ci, cz, cx};
  for (int k = 0; k < 3; ++k) {
    six[2 * k] = six[2 * k + 1] = nullptr;
    if (cls[k] < 0) continue;
    std::vector<hipEvent_t>& v = ev[cls[k]];
    while (v.size() < used[cls[k]] + 2) {
      hipEvent_t e;
      // timing only: no system-scope fence, which would write back and
      // invalidate the caches and slow the launch that follows
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      v.push_back(e);
    }
    six[2 * k] = v[used[cls[k]]];
    six[2 * k + 1] = v[used[cls[k]] + 1];
    used[cls[k]] += 2;
  }
  return six;
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

void ac_build_tiling(sweep_plan* p) {
  const int TZ = 4 * p->tune.rz;
  p->TZ = TZ;
  p->tiles_x = (p->NX + kTX - 1) / kTX;
  p->tiles_z = (p->NZ + TZ - 1) / TZ;
  p->ntiles = p->tiles_x * p->tiles_z;
  // Interior tiles: whole tiles with no cell within P+4 of an edge (the memory
  // variables live in the outer P cells; their first derivative reaches 4 more).
  const int m = p->P > 0 ? p->P + 4 : 0;
  int itx0 = (m + kTX - 1) / kTX, itx1 = std::max(p->NX - m, 0) / kTX;
  int itz0 = (m + TZ - 1) / TZ, itz1 = std::max(p->NZ - m, 0) / TZ;
  if (itx1 <= itx0 || itz1 <= itz0) itx0 = itx1 = itz0 = itz1 = 0;
  p->itx0 = itx0;
  p->itx1 = itx1;
  p->itz0 = itz0;
  p->itz1 = itz1;
  p->n_int = (itx1 - itx0) * (itz1 - itz0);
  p->n_pml = p->ntiles - p->n_int;
  p->n_xf = (itx0 + p->tiles_x - itx1) * p->tiles_z;
  p->n_zf = (itx1 - itx0) * (itz0 + p->tiles_z - itz1);
  const int ns = p->pb.nshots, nr = p->pb.nrec;
  // Deep tiles (two steps per pass): interior tiles with no C-PML band cell
  // within 4 cells (the first step is recomputed on a 4-cell ring) and no
  // source or receiver of any shot on the tile or its 4-cell ring. The pass
  // computes values only there: a source adds to p^{n+1} and a residual to
  // lambda^n at its own cell, and a receiver records its own cell, so cells
  // further out (the 8-cell halo is only read) need no injection or recording.
  constexpr int R = 4;
  std::vector<char> near((size_t)p->ntiles, 0);
  auto mark = [&](int c) {
    const int gx = c % p->NX, gz = c / p->NX;
    for (int tz = std::max(0, (gz - R - TZ + 1) / TZ - 1); tz <= (gz + R) / TZ && tz < p->tiles_z; ++tz)
      for (int tx = std::max(0, (gx - R - kTX + 1) / kTX - 1); tx <= (gx + R) / kTX && tx < p->tiles_x;
           ++tx) {
        const int x0 = tx * kTX, z0 = tz * TZ;
        if (gx >= x0 - R && gx < x0 + kTX + R && gz >= z0 - R && gz < z0 + TZ + R)
          near[(size_t)tz * p->tiles_x + tx] = 1;
      }
  };
  for (int c : p->src_cell) mark(c);
  for (int c : p->rec_cell) mark(c);
  p->ilist_all.clear();
  p->ilist_ring.clear();
  p->dlist.clear();
  std::vector<char> deep((size_t)p->ntiles, 0);
  for (int tz = itz0; tz < itz1; ++tz)
    for (int tx = itx0; tx < itx1; ++tx) {
      const int t = tz * p->tiles_x + tx, x0 = tx * kTX, z0 = tz * TZ;
      p->ilist_all.push_back(t);
      const bool clear_band =
          p->P == 0 || (x0 - 4 >= m && x0 + kTX + 4 <= p->NX - m && z0 - 4 >= m && z0 + TZ + 4 <= p->NZ - m);
      // the two-step kernels read an 8-cell halo without bounds checks
      const bool halo_in = x0 >= 8 && x0 + kTX + 8 <= p->NX && z0 >= 8 && z0 + TZ + 8 <= p->NZ;
      deep[t] = clear_band && halo_in && !near[t];
      if (deep[t])
        p->dlist.push_back(t);
      else
        p->ilist_ring.push_back(t);
    }
  // Deep runs: the deep tiles of a tile column that follow each other in z, cut
  // into chunks of about equal length, each marched by one work-group per shot.
  // Chunks hold at least 64 rows (the first 8 rows of p^{n+1} above a chunk are
  // recomputed) and are cut so that chunks x shots reaches about 2048 groups.
  p->drun.clear();
  if (!p->dlist.empty()) {
    const long long want = 2048;
    const int cmin = (64 + TZ - 1) / TZ;
    const int cmax = (int)std::max<long long>(
        cmin, ((long long)p->dlist.size() * std::max(ns, 1) + want - 1) / want);
    for (int tx = itx0; tx < itx1; ++tx)
      for (int tz = itz0; tz < itz1;) {
        if (!deep[(size_t)tz * p->tiles_x + tx]) {
          ++tz;
          continue;
        }
        int e = tz;
        while (e < itz1 && deep[(size_t)e * p->tiles_x + tx]) ++e;
        const int len = e - tz, nch = (len + cmax - 1) / cmax;
        for (int q = 0; q < nch; ++q) {
          const int a0 = tz + len * q / nch, a1 = tz + len * (q + 1) / nch;
          p->drun.push_back(make_int2(tx, a0 | ((a1 - a0) << 16)));
        }
        tz = e;
      }
  }
  // receiver CSR over (shot, tile), entries sorted by (local cell, receiver)
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

void ac_layout(const sweep_plan* p, AcLayout& L, bool keep) {
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
  const size_t nsrc = p->nsrc;
  L.wav = c.take(ns * nsrc * p->pb.nt * f);
  L.src_cell = c.take(ns * nsrc * sizeof(int));
  L.co_off = c.take((ns + 1) * sizeof(int));
  L.co_rec = c.take(std::max<size_t>(p->co_rec.size(), 1) * sizeof(int));
  L.rec_cell = c.take(ns * nr * sizeof(int));
  L.rec_off = c.take((ns * ac_max_tiles(p) + 1) * sizeof(int));
  L.rec_ent = c.take(std::max<size_t>(ns * nr, 1) * sizeof(int2));
  L.tl_cap = ac_max_tiles(p);
  L.tl = c.take(4 * L.tl_cap * sizeof(int));  // interior, ring, runs (int2)
  for (int i = 0; i < 4; ++i) L.pf[i] = c.take(ns * plane * f);
  L.aux[0] = c.take(L.aux_elems * f);
  L.aux[1] = c.take(L.aux_elems * f);
  L.fwd_end = c.off;
  const int k = p->ckpt;
  L.nseg = (p->pb.nt + k - 1) / k;
  L.slot_elems = 2 * ns * plane + L.aux_elems;
  // a stored segment is never recomputed, so only the others need a checkpoint
  L.nkeep = keep ? std::min(std::max(p->tune.keep_b, 0), L.nseg) : 0;
  L.ck = c.take((size_t)(L.nseg - L.nkeep) * L.slot_elems * f);
  // B'^n of a recomputed segment. The backward reverses the stored segments
  // (the last ones) before it recomputes any other, so a plan that stores
  // some recomputes into the first stored segment's slots (set below) and
  // needs no buffer of its own.
  L.Bseg = L.nkeep > 0 ? 0 : c.take((size_t)k * ns * plane * f);
  for (int i = 0; i < 4; ++i) L.lf[i] = c.take(ns * plane * f);
  L.adjaux[0] = c.take(L.aux_elems * f);
  L.adjaux[1] = c.take(L.aux_elems * f);
  L.gpart = c.take(ns * plane * f);
  L.tot = c.take(plane * sizeof(double));
  L.Bkeep = c.take((size_t)L.nkeep * k * ns * plane * f);
  if (L.nkeep > 0) L.Bseg = L.Bkeep;
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
  // encoded shots: the step kernels inject nothing (ac_encode_sources does)
  a.w = p->nsrc > 1 ? 0.0f : (float)((double)p->pb.dt * p->pb.dt / ((double)p->pb.h * p->pb.h));
  a.Cs = at<float>(work, L.Cs);
  a.ax = at<float>(work, L.ax);
  a.bx = at<float>(work, L.bx);
  a.az = at<float>(work, L.az);
  a.bz = at<float>(work, L.bz);
  a.src_cell = at<int>(work, L.src_cell);
  a.rec_off = at<int>(work, L.rec_off);
  a.rec_ent = at<int2>(work, L.rec_ent);
  a.itx0 = p->itx0;
  a.itx1 = p->itx1;
  a.itz0 = p->itz0;
  a.itz1 = p->itz1;
  a.n_int = (int)p->ilist_all.size();
  a.ilist = at<int>(work, L.tl);
  a.drun = reinterpret_cast<const int2*>(at<int>(work, L.tl) + 2 * L.tl_cap);
  a.n_run = 0;
  a.n_pml = p->n_pml;
  a.n_xf = p->n_xf;
  a.n_zf = p->n_zf;
  a.tz = p->TZ;
  a.nsub = p->tune.rz / p->tune.pml_rz;
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
  const std::vector<int>* lists[2] = {&p->ilist_all, &p->ilist_ring};
  for (int q = 0; q < 2; ++q)
    if (!lists[q]->empty())
      SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.tl) + q * L.tl_cap, lists[q]->data(),
                               lists[q]->size() * sizeof(int), hipMemcpyHostToDevice, s));
  if (!p->drun.empty())
    SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.tl) + 2 * L.tl_cap, p->drun.data(),
                             p->drun.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  if (p->nsrc > 1) {
    SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.co_off), p->co_off.data(),
                             p->co_off.size() * sizeof(int), hipMemcpyHostToDevice, s));
    if (!p->co_rec.empty())
      SWEEP_HIP(hipMemcpyAsync(at<int>(work, L.co_rec), p->co_rec.data(),
                               p->co_rec.size() * sizeof(int), hipMemcpyHostToDevice, s));
  }
  return SWEEP_OK;
}

// ---------------------------------------------------------------- forward
// Everything before the time loop: geometry, model preparation, zero state.
int ac_fwd_prologue(sweep_plan* p, const float* model, const float* wavelet, void* work,
                    const AcLayout& L, hipStream_t s) {
  const sweep_problem& pb = p->pb;
  int rc;
  if ((rc = ac_launch_prep(model, at<float>(work, L.vpad), at<float>(work, L.Cs),
                           at<float>(work, L.ax), at<float>(work, L.bx), at<float>(work, L.az),
                           at<float>(work, L.bz), pb.nx, pb.nz, p->P, pb.h, pb.dt, pb.pml_vmax,
                           pb.pml_f0, pb.pml_R, s)))
    return rc;
  const size_t ns = pb.nshots;
  if ((rc = launch_copy(at<float>(work, L.wav), wavelet, ns * p->nsrc * pb.nt, s))) return rc;
  p->frot = Rot();
  if ((rc = launch_fill(at<float>(work, L.pf[p->frot.prev]), ns * L.plane, 0.0f, s))) return rc;
  if ((rc = launch_fill(at<float>(work, L.pf[p->frot.cur]), ns * L.plane, 0.0f, s))) return rc;
  if ((rc = launch_fill(at<float>(work, L.aux[0]), L.aux_elems, 0.0f, s))) return rc;
  if ((rc = launch_fill(at<float>(work, L.aux[1]), L.aux_elems, 0.0f, s))) return rc;
  return SWEEP_OK;
}

// Checkpoint of the state entering forward step n (a multiple of k).
int ac_checkpoint(sweep_plan* p, void* work, const AcLayout& L, int n, hipStream_t s) {
  const size_t ns = p->pb.nshots;
  float* slot = at<float>(work, L.ck) + (size_t)(n / p->ckpt) * L.slot_elems;
  int rc;
  if ((rc = launch_copy(slot, at<float>(work, L.pf[p->frot.cur]), ns * L.plane, s))) return rc;
  if ((rc = launch_copy(slot + ns * L.plane, at<float>(work, L.pf[p->frot.prev]), ns * L.plane, s)))
    return rc;
  return launch_copy(slot + 2 * ns * L.plane, at<float>(work, L.aux[n % 2]), L.aux_elems, s);
}

// One forward-type step n (forward, or recomputation when B_out is given):
// fields (cur, prev) -> next, memory variables aux[par] -> aux[1 - par].
AcStep ac_fwd_single(sweep_plan* p, void* work, const AcLayout& L, int n, int par, int cur,
                     int prev, int next, float* gathers, float* B_out) {
  const size_t ns = p->pb.nshots;
  AcStep a = ac_base(p, work, L);
  a.wavelet = at<float>(work, L.wav);
  a.gathers = gathers;
  a.n = n;
  a.cur = at<float>(work, L.pf[cur]);
  a.prev = at<float>(work, L.pf[prev]);
  a.next = at<float>(work, L.pf[next]);
  float* aux[2] = {at<float>(work, L.aux[0]), at<float>(work, L.aux[1])};
  set_aux(a, aux_ptrs(aux[par], L, ns), aux_ptrs(aux[1 - par], L, ns));
  a.B_out = B_out;
  return a;
}

// Timer events for the launches of one step; a tile set with nothing to launch
// gets no events (they would never be recorded).
hipEvent_t* step_events(sweep_plan* p, const AcStep& a, int ci, int cz, int cx) {
  return p->timer.take(a.n_int > 0 ? ci : -1, a.n_zf > 0 ? cz : -1, a.n_xf > 0 ? cx : -1);
}

// Encoded shots: the sources of step n into p^{n+1} (next) and the receivers
// on source cells recorded again; nothing for one source per shot.
int ac_encode_sources(sweep_plan* p, void* work, const AcLayout& L, int n, float* next,
                      float* gathers, hipStream_t s) {
  if (p->nsrc <= 1) return SWEEP_OK;
  const sweep_problem& pb = p->pb;
  const float w = (float)((double)pb.dt * pb.dt / ((double)pb.h * pb.h));
  return ac_launch_inject_encoded(next, L.plane, at<int>(work, L.src_cell),
                                  at<float>(work, L.wav), p->nsrc, pb.nt, n, w, pb.nshots,
                                  at<int>(work, L.co_off), at<int>(work, L.co_rec),
                                  at<int>(work, L.rec_cell), gathers, pb.nrec, s);
}

// One forward-type step from the plan's rotation; advances it.
int ac_fwd_one(sweep_plan* p, void* work, const AcLayout& L, int n, int par, float* gathers,
               float* B_out, hipStream_t s, int ci, int cz, int cx) {
  Rot& r = p->frot;
  const int o = r.free_buf(0);
  const AcStep a = ac_fwd_single(p, work, L, n, par, r.cur, r.prev, o, gathers, B_out);
  int rc = ac_launch_fwd(a, p->tune.rz, p->tune.pml_rz, s, step_events(p, a, ci, cz, cx));
  if (!rc) rc = ac_encode_sources(p, work, L, n, a.next, gathers, s);
  r.prev = r.cur;
  r.cur = o;
  return rc;
}

// The launches of a step pair: the two-step pass over the deep tiles (d), then
// steps a0 and a1 of the other tiles (interior ring and frame), in that order.
struct StepPair {
  AcStep d, a0, a1;
};

// Forward-type steps n and n+1 from the plan's rotation; advances it.
StepPair ac_fwd_pair(sweep_plan* p, void* work, const AcLayout& L, int n, int par,
                     float* gathers, float* B_out, float* B_out2) {
  Rot& r = p->frot;
  const int o1 = r.free_buf(0), o2 = r.free_buf(1);
  StepPair P;
  P.d = ac_fwd_single(p, work, L, n, par, r.cur, r.prev, o1, gathers, B_out);
  P.d.next2 = at<float>(work, L.pf[o2]);
  P.d.B_out2 = B_out2;
  P.d.n_run = (int)p->drun.size();
  P.a0 = ac_fwd_single(p, work, L, n, par, r.cur, r.prev, o1, gathers, B_out);
  P.a1 = ac_fwd_single(p, work, L, n + 1, 1 - par, o1, r.cur, o2, gathers, B_out2);
  P.a0.ilist = P.a1.ilist = at<int>(work, L.tl) + L.tl_cap;
  P.a0.n_int = P.a1.n_int = (int)p->ilist_ring.size();
  r.prev = o1;
  r.cur = o2;
  return P;
}

// Forward-type steps n and n+1: the deep tiles in one two-step pass, the other
// tiles (interior ring and frame) as two single steps; advances the rotation.
int ac_fwd_two(sweep_plan* p, void* work, const AcLayout& L, int n, int par, float* gathers,
               float* B_out, float* B_out2, hipStream_t s, bool rec) {
  const StepPair P = ac_fwd_pair(p, work, L, n, par, gathers, B_out, B_out2);
  const int rz = p->tune.rz, prz = p->tune.pml_rz;
  int rc;
  if ((rc = ac_launch_deep(P.d, false, s, p->timer.take(rec ? kRecDeep : kFwdDeep, -1, -1))))
    return rc;
  const int ci = rec ? kRecInt : kFwdInt, cz = rec ? kRecZ : kFwdZ, cx = rec ? kRecX : kFwdX;
  if ((rc = ac_launch_fwd(P.a0, rz, prz, s, step_events(p, P.a0, ci, cz, cx)))) return rc;
  if ((rc = ac_encode_sources(p, work, L, n, P.a0.next, gathers, s))) return rc;
  if ((rc = ac_launch_fwd(P.a1, rz, prz, s, step_events(p, P.a1, ci, cz, cx)))) return rc;
  return ac_encode_sources(p, work, L, n + 1, P.a1.next, gathers, s);
}

bool ac_two_steps(const sweep_plan* p) { return p->tune.tblock == 2 && !p->dlist.empty(); }

void ac_mark_saved(sweep_plan* p, void* work, const float* model, int save) {
  p->saved = save != 0;
  p->saved_work = work;
  p->saved_model = model;
  p->saved_rz = p->tune.rz;
}

// B'^n of step n = n0 + m of segment sg: in the stored segments (the last
// L.nkeep, written by the saving forward) or in the segment buffer (written by
// the recomputation)
bool ac_kept(const AcLayout& L, int sg) { return sg >= L.nseg - L.nkeep; }
float* ac_bseg(sweep_plan* p, void* work, const AcLayout& L, int sg, int m) {
  const size_t ns = p->pb.nshots;
  if (ac_kept(L, sg))
    return at<float>(work, L.Bkeep) +
           ((size_t)(sg - (L.nseg - L.nkeep)) * p->ckpt + m) * ns * L.plane;
  return at<float>(work, L.Bseg) + (size_t)m * ns * L.plane;
}

int ac_forward_enqueue(sweep_plan* p, const float* model, const float* wavelet, float* gathers,
                       void* work, const AcLayout& L, int save, hipStream_t s) {
  int rc;
  if ((rc = ac_fwd_prologue(p, model, wavelet, work, L, s))) return rc;
  const int nt = p->pb.nt, k = p->ckpt;
  const bool two = ac_two_steps(p);
  for (int n = 0; n < nt;) {
    if (save && n % k == 0 && !ac_kept(L, n / k) && (rc = ac_checkpoint(p, work, L, n, s)))
      return rc;
    // steps of a stored segment also write B'^n (timed with the recomputation,
    // whose launches they are)
    const int sg = n / k, m = n - sg * k;
    const bool keepB = save && ac_kept(L, sg);
    // a pair never spans a checkpoint (the state entering step n+1 is not formed)
    if (two && n + 1 < nt && (!save || (n + 1) % k != 0)) {
      if ((rc = ac_fwd_two(p, work, L, n, n % 2, gathers,
                           keepB ? ac_bseg(p, work, L, sg, m) : nullptr,
                           keepB ? ac_bseg(p, work, L, sg, m + 1) : nullptr, s, keepB)))
        return rc;
      n += 2;
    } else {
      if ((rc = keepB ? ac_fwd_one(p, work, L, n, n % 2, gathers, ac_bseg(p, work, L, sg, m), s,
                                   kRecInt, kRecZ, kRecX)
                      : ac_fwd_one(p, work, L, n, n % 2, gathers, nullptr, s, kFwdInt, kFwdZ,
                                   kFwdX)))
        return rc;
      n += 1;
    }
  }
  return SWEEP_OK;
}

// ---------------------------------------------------------------- backward
int ac_bwd_prologue(sweep_plan* p, const float* resid, void* work, const AcLayout& L,
                    hipStream_t s) {
  const size_t ns = p->pb.nshots;
  int rc;
  p->arot = Rot();
  if ((rc = ac_launch_adj_init(at<float>(work, L.lf[p->arot.cur]), at<float>(work, L.lf[p->arot.prev]),
                               ns * L.plane, at<float>(work, L.adjaux[0]), L.aux_elems,
                               at<int>(work, L.rec_cell), resid, (int)ns, p->pb.nt, p->pb.nrec,
                               s)))
    return rc;
  if ((rc = launch_fill(at<float>(work, L.adjaux[1]), L.aux_elems, 0.0f, s))) return rc;
  return launch_fill_f64(at<double>(work, L.tot), L.plane, 0.0, s);
}

// restore the state entering segment sg (the first step of the recomputation)
int ac_bwd_restore(sweep_plan* p, void* work, const AcLayout& L, int sg, hipStream_t s) {
  const size_t ns = p->pb.nshots;
  float* slot = at<float>(work, L.ck) + (size_t)sg * L.slot_elems;
  p->frot = Rot();
  int rc;
  if ((rc = launch_copy(at<float>(work, L.pf[p->frot.cur]), slot, ns * L.plane, s))) return rc;
  if ((rc = launch_copy(at<float>(work, L.pf[p->frot.prev]), slot + ns * L.plane, ns * L.plane, s)))
    return rc;
  return launch_copy(at<float>(work, L.aux[0]), slot + 2 * ns * L.plane, L.aux_elems, s);
}


// Reverse of step n inside the segment [n0, n1): fields (cur, prev) -> next,
// adjoint memory variables by the parity of nt - 1 - n.
AcStep ac_adj_single(sweep_plan* p, void* work, const AcLayout& L, const float* resid, int n,
                     int n0, int n1, int cur, int prev, int next) {
  const size_t ns = p->pb.nshots;
  const int it = p->pb.nt - 1 - n;
  AcStep a = ac_base(p, work, L);
  a.n = n;
  a.resid = resid;
  a.cur = at<float>(work, L.lf[cur]);
  a.prev = at<float>(work, L.lf[prev]);
  a.next = at<float>(work, L.lf[next]);
  float* adjaux[2] = {at<float>(work, L.adjaux[0]), at<float>(work, L.adjaux[1])};
  set_aux(a, aux_ptrs(adjaux[it % 2], L, ns), aux_ptrs(adjaux[(it + 1) % 2], L, ns));
  a.B_in = ac_bseg(p, work, L, n0 / p->ckpt, n - n0);
  a.g = at<float>(work, L.gpart);
  a.g_init = (n == n1 - 1);
  return a;
}

int ac_adj_one(sweep_plan* p, void* work, const AcLayout& L, const float* resid, int n, int n0,
               int n1, hipStream_t s) {
  Rot& r = p->arot;
  const int o = r.free_buf(0);
  const AcStep a = ac_adj_single(p, work, L, resid, n, n0, n1, r.cur, r.prev, o);
  const int rc = ac_launch_adj(a, p->tune.rz, p->tune.pml_rz, s, step_events(p, a, kAdjInt, kAdjZ, kAdjX));
  r.prev = r.cur;
  r.cur = o;
  return rc;
}

// Reverse steps n and n-1 (both inside [n0, n1)) from the plan's rotation;
// advances it.
StepPair ac_adj_pair(sweep_plan* p, void* work, const AcLayout& L, const float* resid, int n,
                     int n0, int n1) {
  Rot& r = p->arot;
  const size_t ns = p->pb.nshots;
  const int o1 = r.free_buf(0), o2 = r.free_buf(1);
  StepPair P;
  P.d = ac_adj_single(p, work, L, resid, n, n0, n1, r.cur, r.prev, o1);
  P.d.next2 = at<float>(work, L.lf[o2]);
  P.d.B_in2 = ac_bseg(p, work, L, n0 / p->ckpt, n - 1 - n0);
  P.d.n_run = (int)p->drun.size();
  P.a0 = ac_adj_single(p, work, L, resid, n, n0, n1, r.cur, r.prev, o1);
  P.a1 = ac_adj_single(p, work, L, resid, n - 1, n0, n1, o1, r.cur, o2);
  P.a0.ilist = P.a1.ilist = at<int>(work, L.tl) + L.tl_cap;
  P.a0.n_int = P.a1.n_int = (int)p->ilist_ring.size();
  r.prev = o1;
  r.cur = o2;
  return P;
}

// Reverse steps n and n-1 (both inside [n0, n1)): deep tiles in one pass.
int ac_adj_two(sweep_plan* p, void* work, const AcLayout& L, const float* resid, int n, int n0,
               int n1, hipStream_t s) {
  const StepPair P = ac_adj_pair(p, work, L, resid, n, n0, n1);
  const int rz = p->tune.rz, prz = p->tune.pml_rz;
  int rc;
  if ((rc = ac_launch_deep(P.d, true, s, p->timer.take(kAdjDeep, -1, -1)))) return rc;
  if ((rc = ac_launch_adj(P.a0, rz, prz, s, step_events(p, P.a0, kAdjInt, kAdjZ, kAdjX))))
    return rc;
  return ac_launch_adj(P.a1, rz, prz, s, step_events(p, P.a1, kAdjInt, kAdjZ, kAdjX));
}

int ac_bwd_fold(sweep_plan* p, void* work, const AcLayout& L, hipStream_t s) {
  return ac_launch_fold(at<double>(work, L.tot), at<float>(work, L.gpart), p->pb.nshots, L.plane,
                        s);
}

int ac_bwd_finish(sweep_plan* p, void* work, const AcLayout& L, float* grad, hipStream_t s) {
  const sweep_problem& pb = p->pb;
  const double scale = 2.0 * pb.dt * pb.dt / (pb.h * pb.h);
  return ac_launch_finish(at<double>(work, L.tot), at<float>(work, L.vpad), grad, pb.nx, pb.nz,
                          p->P, p->NX, scale, s);
}

int ac_backward_enqueue(sweep_plan* p, const float* resid, float* grad, void* work,
                        const AcLayout& L, hipStream_t s) {
  const int nt = p->pb.nt, k = p->ckpt;
  const size_t ns = p->pb.nshots;
  const bool two = ac_two_steps(p);
  int rc;
  if ((rc = ac_bwd_prologue(p, resid, work, L, s))) return rc;
  for (int sg = L.nseg - 1; sg >= 0; --sg) {
    const int n0 = sg * k, n1 = std::min(nt, n0 + k);
    // a stored segment was written by the forward: nothing to recompute
    if (!ac_kept(L, sg) && (rc = ac_bwd_restore(p, work, L, sg, s))) return rc;
    for (int m = 0; m < n1 - n0 && !ac_kept(L, sg);) {
      if (two && m + 1 < n1 - n0) {
        if ((rc = ac_fwd_two(p, work, L, n0 + m, m % 2, nullptr, ac_bseg(p, work, L, sg, m),
                             ac_bseg(p, work, L, sg, m + 1), s, true)))
          return rc;
        m += 2;
      } else {
        if ((rc = ac_fwd_one(p, work, L, n0 + m, m % 2, nullptr, ac_bseg(p, work, L, sg, m), s,
                             kRecInt, kRecZ, kRecX)))
          return rc;
        m += 1;
      }
    }
    for (int n = n1 - 1; n >= n0;) {
      if (two && n - 1 >= n0) {
        if ((rc = ac_adj_two(p, work, L, resid, n, n0, n1, s))) return rc;
        n -= 2;
      } else {
        if ((rc = ac_adj_one(p, work, L, resid, n, n0, n1, s))) return rc;
        n -= 1;
      }
    }
    if ((rc = ac_bwd_fold(p, work, L, s))) return rc;
  }
  return ac_bwd_finish(p, work, L, grad, s);
}

// ---------------------------------------------------------------- graphs
// Enqueues `body` on the caller's stream, or (use_graph) captures it once on a
// private stream into a hipGraph keyed by `key` and launches that graph.
template <class F>
int run_maybe_graph(GraphCache& gc, bool use_graph, const std::vector<const void*>& key,
                    hipStream_t s, F body) {
  if (!use_graph) return body(s);
  if (!gc.exec || gc.key != key) {
    if (gc.exec) {
      (void)hipGraphExecDestroy(gc.exec);
      gc.exec = nullptr;
    }
    if (!gc.stream) SWEEP_HIP(hipStreamCreateWithFlags(&gc.stream, hipStreamNonBlocking));
    SWEEP_HIP(hipStreamBeginCapture(gc.stream, hipStreamCaptureModeRelaxed));
    const int rc = body(gc.stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(gc.stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) {
      set_error(std::string("hipStreamEndCapture failed: ") + hipGetErrorString(e));
      return SWEEP_EHIP;
    }
    size_t nn = 0;
    if (hipGraphGetNodes(graph, nullptr, &nn) != hipSuccess) nn = 0;
    const hipError_t e2 = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
      gc.exec = nullptr;
      set_error(std::string("hipGraphInstantiate failed: ") + hipGetErrorString(e2));
      return SWEEP_EHIP;
    }
    gc.key = key;
    gc.nodes = nn;
  }
  SWEEP_HIP(hipGraphLaunch(gc.exec, s));
  return SWEEP_OK;
}

int ac_forward(sweep_plan* p, const float* model, const float* wavelet, float* gathers,
               void* work, size_t bytes, int save, hipStream_t s) {
  AcLayout L;
  ac_layout(p, L);
  int rc = check_work(p, save ? L.bwd_end : L.fwd_end, work, bytes);
  if (rc) return rc;
  if ((rc = ac_upload_geometry(p, work, L, s))) return rc;
  const bool graph = p->tune.use_graph && !p->timer.on;
  const std::vector<const void*> key = {model, wavelet, gathers, work, (const void*)(size_t)save};
  rc = run_maybe_graph(p->gfwd, graph, key, s, [&](hipStream_t st) {
    return ac_forward_enqueue(p, model, wavelet, gathers, work, L, save, st);
  });
  if (rc) return rc;
  ac_mark_saved(p, work, model, save);
  return SWEEP_OK;
}

// Born (tangent-linear) modelling, Eq. 16. The background field p and the
// perturbation dp advance together: the background (two-step passes over the
// deep tiles, as in the forward) stores B'^n in one plane per shot and step,
// and the perturbation step, the same recurrence with no source, adds dCs B'^n
// at every cell and records dp^{n+1} at the receivers. The perturbation state
// lives in the adjoint half of the workspace (its four time-level buffers
// and two memory-variable sets), B'^n in the first slot of the segment
// buffer and dCs in the first plane of the gradient partial.
int ac_born(sweep_plan* p, const float* model, const float* dmodel, const float* wavelet,
            float* dgathers, void* work, size_t bytes, hipStream_t s) {
  AcLayout L;
  ac_layout(p, L, false);
  int rc = check_work(p, L.bwd_end, work, bytes);
  if (rc) return rc;
  if ((rc = ac_upload_geometry(p, work, L, s))) return rc;
  if ((rc = ac_fwd_prologue(p, model, wavelet, work, L, s))) return rc;
  const sweep_problem& pb = p->pb;
  const size_t ns = pb.nshots;
  float* dCs = at<float>(work, L.gpart);
  float* Bn = at<float>(work, L.Bseg);
  if ((rc = ac_launch_born_prep(model, dmodel, dCs, pb.nx, pb.nz, p->P, pb.h, pb.dt, s)))
    return rc;
  Rot br;
  if ((rc = launch_fill(at<float>(work, L.lf[br.prev]), ns * L.plane, 0.0f, s))) return rc;
  if ((rc = launch_fill(at<float>(work, L.lf[br.cur]), ns * L.plane, 0.0f, s))) return rc;
  float* daux[2] = {at<float>(work, L.adjaux[0]), at<float>(work, L.adjaux[1])};
  if ((rc = launch_fill(daux[0], L.aux_elems, 0.0f, s))) return rc;
  if ((rc = launch_fill(daux[1], L.aux_elems, 0.0f, s))) return rc;
  const int rz = p->tune.rz, prz = p->tune.pml_rz;
  // perturbation step n with the background's B'^n in B
  auto dstep = [&](int n, const float* B) {
    const int par = n % 2;
    const int o = br.free_buf(0);
    AcStep d = ac_base(p, work, L);
    d.wavelet = at<float>(work, L.wav);
    d.w = 0.0f;  // no source term in the perturbation
    d.gathers = dgathers;
    d.n = n;
    d.cur = at<float>(work, L.lf[br.cur]);
    d.prev = at<float>(work, L.lf[br.prev]);
    d.next = at<float>(work, L.lf[o]);
    set_aux(d, aux_ptrs(daux[par], L, ns), aux_ptrs(daux[1 - par], L, ns));
    d.bdC = dCs;
    d.bB = B;
    const int r = ac_launch_born(d, rz, prz, s);
    br.prev = br.cur;
    br.cur = o;
    return r;
  };
  // the background takes the plan's two-step passes where it has deep tiles
  // (B'^n and B'^{n+1} in the first two slots of the segment buffer, which
  // holds ckpt >= 2 of them); the perturbation takes single steps
  const bool two = ac_two_steps(p) && p->ckpt >= 2;
  float* Bn2 = Bn + ns * L.plane;
  for (int n = 0; n < pb.nt;) {
    if (two && n + 1 < pb.nt) {
      if ((rc = ac_fwd_two(p, work, L, n, n % 2, nullptr, Bn, Bn2, s, false))) return rc;
      if ((rc = dstep(n, Bn))) return rc;
      if ((rc = dstep(n + 1, Bn2))) return rc;
      n += 2;
    } else {
      if ((rc = ac_fwd_one(p, work, L, n, n % 2, nullptr, Bn, s, -1, -1, -1))) return rc;
      if ((rc = dstep(n, Bn))) return rc;
      n += 1;
    }
  }
  p->saved = false;
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
  const bool graph = p->tune.use_graph && !p->timer.on;
  const std::vector<const void*> key = {resid, grad, work};
  return run_maybe_graph(p->gbwd, graph, key, s, [&](hipStream_t st) {
    return ac_backward_enqueue(p, resid, grad, work, L, st);
  });
}

// ---------------------------------------------------------------- batches
// Several acoustic plans of different grids, shot counts and step counts
// advanced together: every time step is one launch per kernel kind covering
// the tiles of all plans still running (plans stop at their own nt).
int batch_layouts(const sweep_batch* b, int for_backward, std::vector<AcLayout>& L,
                  std::vector<size_t>& off, size_t& total) {
  L.resize(b->plans.size());
  off.resize(b->plans.size());
  total = 0;
  for (size_t q = 0; q < b->plans.size(); ++q) {
    ac_layout(b->plans[q], L[q]);  // with each plan's stored segments
    off[q] = total;
    total = align_up(total + (for_backward ? L[q].bwd_end : L[q].fwd_end));
  }
  return SWEEP_OK;
}

// One batched time-step pair: the two-step passes of the plans that pair
// (deep), then every plan's step n (s0), then step n+1 (s1). Plans that do not
// pair take two single steps; their step n+1 is built only after step n is
// enqueued (`later`), so that a checkpoint can come between the two.
struct BatchPair {
  std::vector<AcStep> deep, s0, s1;
  std::vector<int> later;
  void clear() {
    deep.clear();
    s0.clear();
    s1.clear();
    later.clear();
  }
  void add(const StepPair& P) {
    deep.push_back(P.d);
    s0.push_back(P.a0);
    s1.push_back(P.a1);
  }
};

// Single forward-type step from the plan's rotation (built, not launched).
AcStep fwd_single_rot(sweep_plan* p, void* work, const AcLayout& L, int n, int par,
                      float* gathers, float* B_out) {
  Rot& r = p->frot;
  const int o = r.free_buf(0);
  const AcStep a = ac_fwd_single(p, work, L, n, par, r.cur, r.prev, o, gathers, B_out);
  r.prev = r.cur;
  r.cur = o;
  return a;
}
AcStep adj_single_rot(sweep_plan* p, void* work, const AcLayout& L, const float* resid, int n,
                      int n0, int n1) {
  Rot& r = p->arot;
  const int o = r.free_buf(0);
  const AcStep a = ac_adj_single(p, work, L, resid, n, n0, n1, r.cur, r.prev, o);
  r.prev = r.cur;
  r.cur = o;
  return a;
}

// nmax: stop after that many steps (the autotuner's short runs).
int batch_forward_enqueue(sweep_batch* b, const float* const* models, const float* const* wavs,
                          float* const* gathers, void* work, const std::vector<AcLayout>& L,
                          const std::vector<size_t>& off, int save, hipStream_t s,
                          int nmax = INT_MAX) {
  const int np = (int)b->plans.size();
  int rc, maxnt = 0;
  for (int q = 0; q < np; ++q) {
    if ((rc = ac_fwd_prologue(b->plans[q], models[q], wavs[q], at<char>(work, off[q]), L[q], s)))
      return rc;
    maxnt = std::max(maxnt, b->plans[q]->pb.nt);
  }
  maxnt = std::min(maxnt, nmax);
  BatchPair B;
  for (int n = 0; n < maxnt; n += 2) {
    B.clear();
    for (int q = 0; q < np; ++q) {
      sweep_plan* p = b->plans[q];
      const int nt = p->pb.nt, k = p->ckpt;
      if (n >= nt) continue;
      void* wq = at<char>(work, off[q]);
      const int sg = n / k, m = n - sg * k;
      const bool keepB = save && ac_kept(L[q], sg);
      if (save && n % k == 0 && !keepB && (rc = ac_checkpoint(p, wq, L[q], n, s))) return rc;
      const bool has1 = n + 1 < std::min(nt, maxnt);
      // a pair never spans a checkpoint (the state entering step n+1 is not formed)
      if (ac_two_steps(p) && has1 && (!save || (n + 1) % k != 0)) {
        B.add(ac_fwd_pair(p, wq, L[q], n, n % 2, gathers[q],
                          keepB ? ac_bseg(p, wq, L[q], sg, m) : nullptr,
                          keepB ? ac_bseg(p, wq, L[q], sg, m + 1) : nullptr));
      } else {
        B.s0.push_back(fwd_single_rot(p, wq, L[q], n, n % 2, gathers[q],
                                      keepB ? ac_bseg(p, wq, L[q], sg, m) : nullptr));
        if (has1) B.later.push_back(q);
      }
    }
    if ((rc = ac_launch_deep_batch(B.deep.data(), (int)B.deep.size(), false, s))) return rc;
    if ((rc = ac_launch_fwd_batch(B.s0.data(), (int)B.s0.size(), b->rz, b->prz, s))) return rc;
    for (int q : B.later) {
      sweep_plan* p = b->plans[q];
      void* wq = at<char>(work, off[q]);
      const int sg = (n + 1) / p->ckpt, m = n + 1 - sg * p->ckpt;
      const bool keepB = save && ac_kept(L[q], sg);
      if (save && (n + 1) % p->ckpt == 0 && !keepB &&
          (rc = ac_checkpoint(p, wq, L[q], n + 1, s)))
        return rc;
      B.s1.push_back(fwd_single_rot(p, wq, L[q], n + 1, (n + 1) % 2, gathers[q],
                                    keepB ? ac_bseg(p, wq, L[q], sg, m) : nullptr));
    }
    if (!B.s1.empty() &&
        (rc = ac_launch_fwd_batch(B.s1.data(), (int)B.s1.size(), b->rz, b->prz, s)))
      return rc;
  }
  return SWEEP_OK;
}

// Recompute steps [n0, n1) of every plan (storing B^n) and reverse them, as
// batched step pairs. resids[q] may be null (nothing injected: timing runs).
int batch_segment_enqueue(sweep_batch* b, const float* const* resids, void* work,
                          const std::vector<AcLayout>& L, const std::vector<size_t>& off,
                          const std::vector<int>& n0, const std::vector<int>& n1, int lenmax,
                          hipStream_t s) {
  const int np = (int)b->plans.size();
  int rc;
  BatchPair B;
  // recompute the segments, storing B^n (not those the saving forward stored)
  for (int m = 0; m < lenmax; m += 2) {
    B.clear();
    for (int q = 0; q < np; ++q) {
      const int len = n1[q] - n0[q];
      if (m >= len || ac_kept(L[q], n0[q] / b->plans[q]->ckpt)) continue;
      sweep_plan* p = b->plans[q];
      void* wq = at<char>(work, off[q]);
      const size_t ns = p->pb.nshots;
      if (ac_two_steps(p) && m + 1 < len) {
        const int sg = n0[q] / p->ckpt;
        B.add(ac_fwd_pair(p, wq, L[q], n0[q] + m, m % 2, nullptr, ac_bseg(p, wq, L[q], sg, m),
                          ac_bseg(p, wq, L[q], sg, m + 1)));
      } else {
        B.s0.push_back(fwd_single_rot(p, wq, L[q], n0[q] + m, m % 2, nullptr,
                                      ac_bseg(p, wq, L[q], n0[q] / p->ckpt, m)));
        if (m + 1 < len) B.later.push_back(q);
      }
    }
    if ((rc = ac_launch_deep_batch(B.deep.data(), (int)B.deep.size(), false, s))) return rc;
    if ((rc = ac_launch_fwd_batch(B.s0.data(), (int)B.s0.size(), b->rz, b->prz, s))) return rc;
    for (int q : B.later) {
      sweep_plan* p = b->plans[q];
      void* wq = at<char>(work, off[q]);
      B.s1.push_back(fwd_single_rot(p, wq, L[q], n0[q] + m + 1, (m + 1) % 2, nullptr,
                                    ac_bseg(p, wq, L[q], n0[q] / p->ckpt, m + 1)));
    }
    if (!B.s1.empty() &&
        (rc = ac_launch_fwd_batch(B.s1.data(), (int)B.s1.size(), b->rz, b->prz, s)))
      return rc;
  }
  // reverse steps n1-1 .. n0
  for (int m = 0; m < lenmax; m += 2) {
    B.clear();
    for (int q = 0; q < np; ++q) {
      const int len = n1[q] - n0[q];
      if (m >= len) continue;
      sweep_plan* p = b->plans[q];
      void* wq = at<char>(work, off[q]);
      const int n = n1[q] - 1 - m;
      if (ac_two_steps(p) && m + 1 < len) {
        B.add(ac_adj_pair(p, wq, L[q], resids[q], n, n0[q], n1[q]));
      } else {
        B.s0.push_back(adj_single_rot(p, wq, L[q], resids[q], n, n0[q], n1[q]));
        if (m + 1 < len) B.later.push_back(q);
      }
    }
    if ((rc = ac_launch_deep_batch(B.deep.data(), (int)B.deep.size(), true, s))) return rc;
    if ((rc = ac_launch_adj_batch(B.s0.data(), (int)B.s0.size(), b->rz, b->prz, s))) return rc;
    for (int q : B.later) {
      sweep_plan* p = b->plans[q];
      B.s1.push_back(adj_single_rot(p, at<char>(work, off[q]), L[q], resids[q],
                                    n1[q] - 2 - m, n0[q], n1[q]));
    }
    if (!B.s1.empty() &&
        (rc = ac_launch_adj_batch(B.s1.data(), (int)B.s1.size(), b->rz, b->prz, s)))
      return rc;
  }
  return SWEEP_OK;
}

int batch_backward_enqueue(sweep_batch* b, const float* const* resids, float* const* grads,
                           void* work, const std::vector<AcLayout>& L,
                           const std::vector<size_t>& off, hipStream_t s) {
  const int np = (int)b->plans.size();
  int rc, maxseg = 0;
  for (int q = 0; q < np; ++q) {
    if ((rc = ac_bwd_prologue(b->plans[q], resids[q], at<char>(work, off[q]), L[q], s)))
      return rc;
    maxseg = std::max(maxseg, L[q].nseg);
  }
  std::vector<int> n0(np), n1(np);
  BatchPair B;
  for (int r = 0; r < maxseg; ++r) {
    int lenmax = 0;
    for (int q = 0; q < np; ++q) {
      sweep_plan* p = b->plans[q];
      n0[q] = n1[q] = 0;
      if (r >= L[q].nseg) continue;
      const int sg = L[q].nseg - 1 - r;
      n0[q] = sg * p->ckpt;
      n1[q] = std::min(p->pb.nt, n0[q] + p->ckpt);
      lenmax = std::max(lenmax, n1[q] - n0[q]);
      if (!ac_kept(L[q], sg) && (rc = ac_bwd_restore(p, at<char>(work, off[q]), L[q], sg, s)))
        return rc;
    }
    if ((rc = batch_segment_enqueue(b, resids, work, L, off, n0, n1, lenmax, s))) return rc;
    for (int q = 0; q < np; ++q)
      if (n1[q] > n0[q] && (rc = ac_bwd_fold(b->plans[q], at<char>(work, off[q]), L[q], s)))
        return rc;
  }
  for (int q = 0; q < np; ++q)
    if ((rc = ac_bwd_finish(b->plans[q], at<char>(work, off[q]), L[q], grads[q], s))) return rc;
  return SWEEP_OK;
}

}  // namespace

// ====================================================================== C-ABI
extern "C" const char* sweep_last_error(void) { return g_last_error; }

extern "C" int sweep_plan_create(const sweep_ctx* ctx, const sweep_problem* pb,
                                 const int32_t* src_xz, const int32_t* rec_xz,
                                 sweep_plan** out) try {
  if (!pb || !out || !src_xz || (pb->nrec > 0 && !rec_xz)) {
    set_error("sweep_plan_create: null argument");
    return SWEEP_EINVAL;
  }
  *out = nullptr;
  if (pb->physics != SWEEP_ACOUSTIC && pb->physics != SWEEP_ELASTIC &&
      pb->physics != SWEEP_ACOUSTIC_VD && pb->physics != SWEEP_VTI) {
    set_error("unknown physics");
    return SWEEP_EINVAL;
  }
  if (pb->nx < 1 || pb->nz < 1 || pb->pml < 0 || pb->nt < 1 || pb->nshots < 1 || pb->nrec < 0 ||
      !(pb->h > 0) || !(pb->dt > 0) || pb->ckpt_every < 0 || !(pb->pml_R > 0 && pb->pml_R < 1) ||
      !(pb->pml_vmax > 0) || pb->pml_f0 < 0) {
    set_error("sweep_plan_create: invalid sizes or constants");
    return SWEEP_EINVAL;
  }
  if ((pb->physics == SWEEP_ACOUSTIC || pb->physics == SWEEP_VTI) && pb->free_surface) {
    set_error("free_surface is only supported for the elastic physics");
    return SWEEP_EINVAL;
  }
  const double cfl = (double)pb->pml_vmax * pb->dt / pb->h;
  const double limit =
      pb->physics == SWEEP_ACOUSTIC || pb->physics == SWEEP_VTI ? 0.5546 : 0.6061;
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
  if (ctx) {
    p->device = ctx->device;
    p->arch = ctx->arch;
    p->scratch = ctx->scratch;
  }
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
  if (pb->nsrc < 0 || (pb->nsrc > 1 && pb->physics != SWEEP_ACOUSTIC)) {
    delete p;
    set_error("nsrc must be >= 0, and > 1 only for the acoustic physics");
    return SWEEP_EINVAL;
  }
  p->nsrc = pb->nsrc > 1 ? pb->nsrc : 1;
  p->src_cell.resize((size_t)pb->nshots * p->nsrc);
  for (size_t q = 0; q < p->src_cell.size(); ++q) {
    const int x = src_xz[2 * q], z = src_xz[2 * q + 1];
    if (x < 0 || x >= pb->nx || z < 0 || z >= pb->nz) {
      delete p;
      set_error("source " + std::to_string(q) + " lies outside the model");
      return SWEEP_EINVAL;
    }
    p->src_cell[q] = (z + (pb->free_surface ? 0 : p->P)) * p->NX + x + p->P;
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
  // encoded shots: the receivers that sit on a source cell of their shot
  p->co_off.assign((size_t)pb->nshots + 1, 0);
  p->co_rec.clear();
  if (p->nsrc > 1)
    for (int s = 0; s < pb->nshots; ++s) {
      const int* sc = &p->src_cell[(size_t)s * p->nsrc];
      for (int r = 0; r < pb->nrec; ++r)
        if (std::find(sc, sc + p->nsrc, p->rec_cell[(size_t)s * pb->nrec + r]) != sc + p->nsrc)
          p->co_rec.push_back(r);
      p->co_off[s + 1] = (int)p->co_rec.size();
    }
  p->tune.rz = 8;
  p->tune.pml_rz = 4;
  p->tune.tblock = 2;
  p->tune.use_graph = 0;
  p->tune.keep_b = 0;
  if (pb->physics == SWEEP_VTI) {
    // 64 x 16 tiles: the tile CSR of the receivers is that of rz = 4
    p->tune.rz = 4;
    p->tune.tblock = 1;
    ac_build_tiling(p);
  } else if (pb->physics == SWEEP_ACOUSTIC) {
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
SWEEP_ABI_CATCH("sweep_plan_create")

extern "C" void sweep_plan_destroy(sweep_plan* plan) { delete plan; }

extern "C" int sweep_plan_set_tuning(sweep_plan* p, const sweep_tuning* t) try {
  if (!p || !t) {
    set_error("null argument");
    return SWEEP_EINVAL;
  }
  const bool ok_rz = t->rz == 1 || t->rz == 2 || t->rz == 4 || t->rz == 8;
  const bool ok_prz = (t->pml_rz == 1 || t->pml_rz == 2 || t->pml_rz == 4 || t->pml_rz == 8) &&
                      t->pml_rz <= t->rz;
  if (!ok_rz || !ok_prz || (t->use_graph != 0 && t->use_graph != 1) ||
      (t->tblock != 1 && t->tblock != 2) || t->keep_b < 0) {
    set_error("unsupported tuning");
    return SWEEP_EINVAL;
  }
  if (p->pb.physics == SWEEP_VTI && t->rz != 4) {
    set_error("VTI plans take 64 x 16 tiles (rz 4)");
    return SWEEP_EINVAL;
  }
  p->tune = *t;
  ++p->tune_gen;
  if (p->pb.physics == SWEEP_ACOUSTIC || p->pb.physics == SWEEP_VTI) ac_build_tiling(p);
  p->saved = false;
  p->gfwd.reset();
  p->gbwd.reset();
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_plan_set_tuning")

extern "C" int sweep_plan_get_tuning(const sweep_plan* p, sweep_tuning* t) try {
  if (!p || !t) {
    set_error("null argument");
    return SWEEP_EINVAL;
  }
  *t = p->tune;
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_plan_get_tuning")

extern "C" size_t sweep_plan_workspace_bytes(const sweep_plan* p, int for_backward) try {
  if (!p) return 0;
  if (p->pb.physics == SWEEP_VTI) {
    VtiLayout V;
    vti_layout(p, V);
    return for_backward ? V.bwd_end : V.fwd_end;
  }
  if (p->pb.physics != SWEEP_ACOUSTIC) {
    ElLayout E;
    el_layout(p, E);
    return for_backward ? E.bwd_end : E.fwd_end;
  }
  AcLayout L;
  ac_layout(p, L);
  return for_backward ? L.bwd_end : L.fwd_end;
}
SWEEP_ABI_CATCH_SIZE("sweep_plan_workspace_bytes")

extern "C" int sweep_plan_padded(const sweep_plan* p, int* NX, int* NZ) try {
  if (!p || !NX || !NZ) {
    set_error("null argument");
    return SWEEP_EINVAL;
  }
  *NX = p->NX;
  *NZ = p->NZ;
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_plan_padded")

extern "C" int sweep_plan_tiles(const sweep_plan* p, int* interior_tiles, int* frame_tiles,
                                int* tile_rows, int* rect) try {
  if (!p || !interior_tiles || !frame_tiles || !tile_rows) {
    set_error("null argument");
    return SWEEP_EINVAL;
  }
  if (p->pb.physics != SWEEP_ACOUSTIC) {
    set_error("sweep_plan_tiles: acoustic plans only");
    return SWEEP_EINVAL;
  }
  *interior_tiles = p->n_int;
  *frame_tiles = p->n_pml;
  *tile_rows = p->TZ;
  if (rect) {
    rect[0] = p->itx0;
    rect[1] = p->itx1;
    rect[2] = p->itz0;
    rect[3] = p->itz1;
    rect[4] = p->tune.tblock == 2 ? (int)p->dlist.size() : 0;
  }
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_plan_tiles")

extern "C" int sweep_forward(sweep_plan* p, const float* d_model, const float* d_wavelet,
                             float* d_gathers, void* d_work, size_t work_bytes,
                             int save_for_backward, void* stream) try {
  if (!p || !d_model || !d_wavelet || (!d_gathers && p->pb.nrec > 0)) {
    set_error("sweep_forward: null argument");
    return SWEEP_EINVAL;
  }
  DeviceGuard dg_(p->device);
  if (!dg_.ok) {
    set_error("cannot make the plan's device current");
    return SWEEP_EHIP;
  }
  p->saved = false;
  if (p->pb.physics == SWEEP_ACOUSTIC)
    return ac_forward(p, d_model, d_wavelet, d_gathers, d_work, work_bytes, save_for_backward,
                      (hipStream_t)stream);
  // staggered and VTI plans: host checks and copies, then the device work
  // (eager, or captured once into a graph and replayed), then the saved state
  const bool vti = p->pb.physics == SWEEP_VTI;
  const hipStream_t s = (hipStream_t)stream;
  int rc = vti ? vti_forward_prepare(p, d_work, work_bytes, save_for_backward, s)
               : el_forward_prepare(p, d_work, work_bytes, save_for_backward, s);
  if (rc) return rc;
  const bool graph = p->tune.use_graph && !p->timer.on;
  const std::vector<const void*> key = {d_model, d_wavelet, d_gathers, d_work,
                                        (const void*)(size_t)save_for_backward};
  rc = run_maybe_graph(p->gfwd, graph, key, s, [&](hipStream_t st) {
    return vti ? vti_forward_enqueue(p, d_model, d_wavelet, d_gathers, d_work, save_for_backward,
                                     st)
               : el_forward_enqueue(p, d_model, d_wavelet, d_gathers, d_work, save_for_backward,
                                    st);
  });
  if (rc) return rc;
  if (vti)
    vti_mark_saved(p, d_work, d_model, save_for_backward);
  else
    el_mark_saved(p, d_work, d_model, save_for_backward);
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_forward")

extern "C" int sweep_forward_noalloc(sweep_plan* p, const float* d_model,
                                     const float* d_wavelet, float* d_gathers,
                                     void* stream) try {
  if (!p || !d_model || !d_wavelet || (!d_gathers && p->pb.nrec > 0)) {
    set_error("sweep_forward_noalloc: null argument");
    return SWEEP_EINVAL;
  }
  p->saved = false;
  if (!p->scratch) {
    set_error("sweep_forward_noalloc: the plan was created without a context, so it has no "
              "static device workspace");
    return SWEEP_EINVAL;
  }
  const size_t need = sweep_plan_workspace_bytes(p, 0);
  if (need == 0 || need > kNoAllocScratchBytes) {
    set_error("sweep_forward_noalloc: the plan's forward workspace of " + std::to_string(need) +
              " bytes exceeds the static workspace of " + std::to_string(kNoAllocScratchBytes) +
              " bytes; use sweep_forward with a workspace");
    return SWEEP_EINVAL;
  }
  DeviceGuard dg_(p->device);
  if (!dg_.ok) {
    set_error("cannot make the plan's device current");
    return SWEEP_EHIP;
  }
  // eager launches only (a graph capture would create a stream and graph
  // objects) and no timing events
  const int use_graph = p->tune.use_graph;
  const bool timing = p->timer.on;
  p->tune.use_graph = 0;
  p->timer.on = false;
  hipStream_t s = (hipStream_t)stream;
  const int rc =
      p->pb.physics == SWEEP_VTI
          ? vti_forward(p, d_model, d_wavelet, d_gathers, p->scratch, need, 0, s)
      : p->pb.physics != SWEEP_ACOUSTIC
          ? el_forward(p, d_model, d_wavelet, d_gathers, p->scratch, need, 0, s)
          : ac_forward(p, d_model, d_wavelet, d_gathers, p->scratch, need, 0, s);
  p->tune.use_graph = use_graph;
  p->timer.on = timing;
  p->saved = false;
  return rc;
}
SWEEP_ABI_CATCH("sweep_forward_noalloc")

extern "C" int sweep_born_forward(sweep_plan* p, const float* d_model, const float* d_dmodel,
                                  const float* d_wavelet, float* d_dgathers, void* d_work,
                                  size_t work_bytes, void* stream) try {
  if (!p || !d_model || !d_dmodel || !d_wavelet || (!d_dgathers && p->pb.nrec > 0)) {
    set_error("sweep_born_forward: null argument");
    return SWEEP_EINVAL;
  }
  if (p->pb.physics != SWEEP_ACOUSTIC) {
    set_error("sweep_born_forward: acoustic plans only");
    return SWEEP_EINVAL;
  }
  DeviceGuard dg_(p->device);
  if (!dg_.ok) {
    set_error("cannot make the plan's device current");
    return SWEEP_EHIP;
  }
  p->saved = false;
  return ac_born(p, d_model, d_dmodel, d_wavelet, d_dgathers, d_work, work_bytes,
                 (hipStream_t)stream);
}
SWEEP_ABI_CATCH("sweep_born_forward")

extern "C" int sweep_backward(sweep_plan* p, const float* d_resid, float* d_grad, void* d_work,
                              size_t work_bytes, void* stream) try {
  if (!p || (!d_resid && p->pb.nrec > 0) || !d_grad) {
    set_error("sweep_backward: null argument");
    return SWEEP_EINVAL;
  }
  DeviceGuard dg_(p->device);
  if (!dg_.ok) {
    set_error("cannot make the plan's device current");
    return SWEEP_EHIP;
  }
  if (p->pb.physics == SWEEP_ACOUSTIC)
    return ac_backward(p, d_resid, d_grad, d_work, work_bytes, (hipStream_t)stream);
  const bool vti = p->pb.physics == SWEEP_VTI;
  const int rc = vti ? vti_backward_check(p, d_work, work_bytes)
                     : el_backward_check(p, d_work, work_bytes);
  if (rc) return rc;
  const bool graph = p->tune.use_graph && !p->timer.on;
  const std::vector<const void*> key = {d_resid, d_grad, d_work};
  return run_maybe_graph(p->gbwd, graph, key, (hipStream_t)stream, [&](hipStream_t st) {
    return vti ? vti_backward_enqueue(p, d_resid, d_grad, d_work, st)
               : el_backward_enqueue(p, d_resid, d_grad, d_work, st);
  });
}
SWEEP_ABI_CATCH("sweep_backward")

extern "C" int sweep_plan_set_profiling(sweep_plan* p, int enable) try {
  if (!p) {
    set_error("null plan");
    return SWEEP_EINVAL;
  }
  p->timer.on = enable > 0;
  p->timer.period = enable > 0 ? enable : 1;
  p->timer.reset();
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_plan_set_profiling")

extern "C" int sweep_plan_kernel_time(sweep_plan* p, int kernel_class, int* launches,
                                      double* total_ms) try {
  if (!p || !launches || !total_ms || kernel_class < 0 || kernel_class >= kNumClasses) {
    set_error("sweep_plan_kernel_time: bad argument");
    return SWEEP_EINVAL;
  }
  DeviceGuard dg_(p->device);
  if (!dg_.ok) {
    set_error("cannot make the plan's device current");
    return SWEEP_EHIP;
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
SWEEP_ABI_CATCH("sweep_plan_kernel_time")

// ----------------------------------------------------------------- batch C-ABI
namespace {
// The batch launches one template per (rz, pml_rz) over every plan's tile
// lists, so every member must still have the batch's tiling: a member whose
// tuning changed since (sweep_plan_set_tuning) is refused until the batch is
// re-tuned or re-created.
int batch_check_members(const sweep_batch* b) {
  for (size_t q = 0; q < b->plans.size(); ++q) {
    const sweep_plan* p = b->plans[q];
    if (p->tune.rz != b->rz || p->tune.pml_rz != b->prz) {
      set_error("batch plan " + std::to_string(q) + " has rz/pml_rz " +
                std::to_string(p->tune.rz) + "/" + std::to_string(p->tune.pml_rz) +
                " but the batch was made for " + std::to_string(b->rz) + "/" +
                std::to_string(b->prz) + " (set the same tiling on every plan, or re-create "
                "the batch)");
      return SWEEP_EINVAL;
    }
  }
  return SWEEP_OK;
}
}  // namespace

extern "C" int sweep_batch_create(const sweep_ctx* ctx, sweep_plan* const* plans, int nplans,
                                  sweep_batch** out) try {
  if (!plans || !out || nplans < 1 || nplans > kMaxBatchPlans) {
    set_error("sweep_batch_create: need 1.." + std::to_string(kMaxBatchPlans) + " plans");
    return SWEEP_EINVAL;
  }
  *out = nullptr;
  for (int q = 0; q < nplans; ++q) {
    if (!plans[q] || plans[q]->pb.physics != SWEEP_ACOUSTIC || plans[q]->nsrc > 1) {
      set_error("sweep_batch_create: batches hold acoustic plans with one source per shot");
      return SWEEP_EINVAL;
    }
    if (plans[q]->tune.rz != plans[0]->tune.rz || plans[q]->tune.pml_rz != plans[0]->tune.pml_rz) {
      set_error("sweep_batch_create: all plans of a batch must use the same rz and pml_rz");
      return SWEEP_EINVAL;
    }
    if (plans[q]->device != (ctx ? ctx->device : plans[0]->device)) {
      set_error("sweep_batch_create: all plans of a batch must be bound to the batch's device");
      return SWEEP_EINVAL;
    }
    for (int r = 0; r < q; ++r)
      if (plans[r] == plans[q]) {
        set_error("sweep_batch_create: a plan appears twice");
        return SWEEP_EINVAL;
      }
  }
  sweep_batch* b = new sweep_batch();
  b->plans.assign(plans, plans + nplans);
  b->device = ctx ? ctx->device : plans[0]->device;
  b->rz = plans[0]->tune.rz;
  b->prz = plans[0]->tune.pml_rz;
  *out = b;
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_batch_create")

extern "C" void sweep_batch_destroy(sweep_batch* b) { delete b; }

extern "C" int sweep_batch_set_graph(sweep_batch* b, int use_graph) try {
  if (!b) {
    set_error("null batch");
    return SWEEP_EINVAL;
  }
  b->use_graph = use_graph != 0;
  b->gfwd.reset();
  b->gbwd.reset();
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_batch_set_graph")

extern "C" int sweep_plan_graph_nodes(const sweep_plan* p, size_t* fwd_nodes,
                                      size_t* bwd_nodes) try {
  if (!p || !fwd_nodes || !bwd_nodes) {
    set_error("sweep_plan_graph_nodes: null argument");
    return SWEEP_EINVAL;
  }
  *fwd_nodes = p->gfwd.exec ? p->gfwd.nodes : 0;
  *bwd_nodes = p->gbwd.exec ? p->gbwd.nodes : 0;
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_plan_graph_nodes")

extern "C" int sweep_batch_graph_nodes(const sweep_batch* b, size_t* fwd_nodes,
                                       size_t* bwd_nodes) try {
  if (!b || !fwd_nodes || !bwd_nodes) {
    set_error("sweep_batch_graph_nodes: null argument");
    return SWEEP_EINVAL;
  }
  *fwd_nodes = b->gfwd.exec ? b->gfwd.nodes : 0;
  *bwd_nodes = b->gbwd.exec ? b->gbwd.nodes : 0;
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_batch_graph_nodes")

extern "C" size_t sweep_batch_workspace_bytes(const sweep_batch* b, int for_backward) try {
  if (!b) return 0;
  std::vector<AcLayout> L;
  std::vector<size_t> off;
  size_t total = 0;
  batch_layouts(b, for_backward, L, off, total);
  return total;
}
SWEEP_ABI_CATCH_SIZE("sweep_batch_workspace_bytes")

extern "C" int sweep_batch_forward(sweep_batch* b, const float* const* d_models,
                                   const float* const* d_wavelets, float* const* d_gathers,
                                   void* d_work, size_t work_bytes, int save_for_backward,
                                   void* stream) try {
  if (!b || !d_models || !d_wavelets || !d_gathers || !d_work) {
    set_error("sweep_batch_forward: null argument");
    return SWEEP_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  b->saved = false;
  int rc = batch_check_members(b);
  if (rc) return rc;
  DeviceGuard dg_(b->device);
  if (!dg_.ok) {
    set_error("cannot make the batch's device current");
    return SWEEP_EHIP;
  }
  std::vector<AcLayout> L;
  std::vector<size_t> off;
  size_t total = 0;
  batch_layouts(b, save_for_backward, L, off, total);
  if (work_bytes < total) {
    set_error("workspace too small: need " + std::to_string(total) + " bytes");
    return SWEEP_ENOMEM;
  }
  const int np = (int)b->plans.size();
  // the captured graph holds the plans' tilings and stored-segment layouts:
  // their tuning generations are part of its key
  std::vector<const void*> key = {d_work, (const void*)(size_t)save_for_backward};
  std::vector<unsigned> gen(np);
  for (int q = 0; q < np; ++q) {
    gen[q] = b->plans[q]->tune_gen;
    key.push_back((const void*)(size_t)gen[q]);
  }
  for (int q = 0; q < np; ++q) {
    if (!d_models[q] || !d_wavelets[q] || (!d_gathers[q] && b->plans[q]->pb.nrec > 0)) {
      set_error("sweep_batch_forward: null pointer for plan " + std::to_string(q));
      return SWEEP_EINVAL;
    }
    b->plans[q]->saved = false;
    if ((rc = ac_upload_geometry(b->plans[q], at<char>(d_work, off[q]), L[q], s))) return rc;
    key.push_back(d_models[q]);
    key.push_back(d_wavelets[q]);
    key.push_back(d_gathers[q]);
  }
  rc = run_maybe_graph(b->gfwd, b->use_graph, key, s, [&](hipStream_t st) {
    return batch_forward_enqueue(b, d_models, d_wavelets, d_gathers, d_work, L, off,
                                 save_for_backward, st);
  });
  if (rc) return rc;
  b->saved = save_for_backward != 0;
  b->saved_work = d_work;
  b->saved_gen = gen;
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_batch_forward")

extern "C" int sweep_batch_backward(sweep_batch* b, const float* const* d_resids,
                                    float* const* d_grads, void* d_work, size_t work_bytes,
                                    void* stream) try {
  if (!b || !d_resids || !d_grads || !d_work) {
    set_error("sweep_batch_backward: null argument");
    return SWEEP_EINVAL;
  }
  if (!b->saved || b->saved_work != d_work) {
    set_error("sweep_batch_backward needs a preceding sweep_batch_forward(save_for_backward=1) "
              "on the same workspace");
    return SWEEP_ESTATE;
  }
  for (size_t q = 0; q < b->plans.size(); ++q)
    if (b->plans[q]->tune_gen != b->saved_gen[q]) {
      set_error("sweep_batch_backward: the tuning of plan " + std::to_string(q) +
                " changed after the saving forward (its saved layout no longer holds)");
      return SWEEP_ESTATE;
    }
  int rc0 = batch_check_members(b);
  if (rc0) return rc0;
  DeviceGuard dg_(b->device);
  if (!dg_.ok) {
    set_error("cannot make the batch's device current");
    return SWEEP_EHIP;
  }
  std::vector<AcLayout> L;
  std::vector<size_t> off;
  size_t total = 0;
  batch_layouts(b, 1, L, off, total);
  if (work_bytes < total) {
    set_error("workspace too small");
    return SWEEP_ENOMEM;
  }
  std::vector<const void*> key = {d_work};
  for (size_t q = 0; q < b->plans.size(); ++q) key.push_back((const void*)(size_t)b->saved_gen[q]);
  for (size_t q = 0; q < b->plans.size(); ++q) {
    if ((!d_resids[q] && b->plans[q]->pb.nrec > 0) || !d_grads[q]) {
      set_error("sweep_batch_backward: null pointer for plan " + std::to_string(q));
      return SWEEP_EINVAL;
    }
    key.push_back(d_resids[q]);
    key.push_back(d_grads[q]);
  }
  return run_maybe_graph(b->gbwd, b->use_graph, key, (hipStream_t)stream, [&](hipStream_t st) {
    return batch_backward_enqueue(b, d_resids, d_grads, d_work, L, off, st);
  });
}
SWEEP_ABI_CATCH("sweep_batch_backward")

// ----------------------------------------------------------------- autotuner
// Times every supported (rz, pml_rz, tblock) and keeps the fastest. Results
// are cached as JSON lines, one object per search:
//   {"arch":"gfx950","physics":"acoustic","mode":"plan-forward","shapes":"NXxNZxNSHOTSxP",
//    "rz":8,"pml_rz":4,"tblock":2,"us_per_step":123.4}
// "shapes" lists every plan of a batch (space-separated) and "mode" is
// plan-forward, batch-forward or batch-gradient. A search whose fields up to
// "shapes" match a line takes that line's choice.
namespace {

std::string tune_arch(const sweep_plan* p) {
  if (!p->arch.empty()) return p->arch;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    return std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
  return "unknown";
}

std::string tune_shape(const sweep_plan* p) {
  return std::to_string(p->NX) + "x" + std::to_string(p->NZ) + "x" +
         std::to_string(p->pb.nshots) + "x" + std::to_string(p->pb.pml);
}

// the cache line up to (and with) "shapes"; the tiling choices follow it
std::string tune_key(const sweep_plan* p0, const char* mode, const std::string& shapes) {
  return "{\"arch\":\"" + tune_arch(p0) + "\",\"physics\":\"acoustic\",\"mode\":\"" + mode +
         "\",\"shapes\":\"" + shapes + "\",";
}

// integer field "name": of one cache line (false when absent or malformed)
bool json_int(const std::string& line, const char* name, int& v) {
  const std::string k = std::string("\"") + name + "\":";
  const size_t at = line.find(k);
  if (at == std::string::npos) return false;
  char* end = nullptr;
  const char* b = line.c_str() + at + k.size();
  const long x = std::strtol(b, &end, 10);
  if (end == b) return false;
  v = (int)x;
  return true;
}

bool rz_ok(int v) { return v == 1 || v == 2 || v == 4 || v == 8; }

// the cached choice for `key`, if a well-formed line holds one
bool tune_lookup(const char* path, const std::string& key, int& rz, int& prz, int& tb) {
  if (!path || !*path) return false;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    if (line.compare(0, key.size(), key) != 0) continue;
    const std::string rest = line.substr(key.size());
    if (json_int(rest, "rz", rz) && json_int(rest, "pml_rz", prz) &&
        json_int(rest, "tblock", tb) && rz_ok(rz) && rz_ok(prz) && prz <= rz &&
        (tb == 1 || tb == 2))
      return true;
  }
  return false;
}

void tune_store(const char* path, const std::string& key, int rz, int prz, int tb, double us) {
  if (!path || !*path) return;
  std::ofstream out(path, std::ios::app);
  std::ostringstream os;
  os.precision(6);
  os << key << "\"rz\":" << rz << ",\"pml_rz\":" << prz << ",\"tblock\":" << tb
     << ",\"us_per_step\":" << us << "}\n";
  out << os.str();
}

}  // namespace

extern "C" int sweep_plan_autotune(sweep_plan* p, const float* d_model, const float* d_wavelet,
                                   void* d_work, size_t work_bytes, int steps,
                                   const char* cache_path, void* stream, int* chosen_rz) try {
  if (!p || !d_model || !d_wavelet || !d_work || steps < 1) {
    set_error("sweep_plan_autotune: bad argument");
    return SWEEP_EINVAL;
  }
  DeviceGuard dg_(p->device);
  if (!dg_.ok) {
    set_error("cannot make the plan's device current");
    return SWEEP_EHIP;
  }
  if (p->pb.physics != SWEEP_ACOUSTIC) {  // the elastic kernels have no tile choice
    if (chosen_rz) *chosen_rz = p->tune.rz;
    return SWEEP_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  const std::string key = tune_key(p, "plan-forward", tune_shape(p));
  {
    int rz = 0, prz = 0, tb = 0;
    if (tune_lookup(cache_path, key, rz, prz, tb)) {
      sweep_tuning t = p->tune;
      t.rz = rz;
      t.pml_rz = prz;
      t.tblock = tb;
      const int rc = sweep_plan_set_tuning(p, &t);
      if (rc) return rc;
      if (chosen_rz) *chosen_rz = rz;
      return SWEEP_OK;
    }
  }
  AcLayout L;
  ac_layout(p, L);
  int rc = check_work(p, L.fwd_end, d_work, work_bytes);
  if (rc) return rc;
  const sweep_tuning keep = p->tune;
  const bool timing = p->timer.on;
  p->timer.on = false;
  hipEvent_t e0, e1;
  SWEEP_HIP(hipEventCreate(&e0));
  SWEEP_HIP(hipEventCreate(&e1));
  const int cand[4] = {1, 2, 4, 8};
  int best = keep.rz, best_p = keep.pml_rz, best_t = keep.tblock;
  double best_us = 1e300;
  const int nsteps = std::min(steps, p->pb.nt);
  for (int c : cand) {
    for (int cp : cand) {
     for (int tb = 1; tb <= 2; ++tb) {
      if (cp > c || rc) continue;
      p->tune.rz = c;
      p->tune.pml_rz = cp;
      p->tune.tblock = tb;
      ac_build_tiling(p);
      if (tb == 2 && !ac_two_steps(p)) continue;  // no deep tiles: same as tb = 1
      if ((rc = ac_upload_geometry(p, d_work, L, s))) break;
      for (int rep = 0; rep < 2 && !rc; ++rep) {  // first pass warms up
        rc = ac_fwd_prologue(p, d_model, d_wavelet, d_work, L, s);
        if (rc) break;
        SWEEP_HIP(hipEventRecord(e0, s));
        const bool two = ac_two_steps(p);
        for (int n = 0; n < nsteps && !rc;) {
          if (two && n + 1 < nsteps) {
            rc = ac_fwd_two(p, d_work, L, n, n % 2, nullptr, nullptr, nullptr, s, false);
            n += 2;
          } else {
            rc = ac_fwd_one(p, d_work, L, n, n % 2, nullptr, nullptr, s, kFwdInt, kFwdZ, kFwdX);
            n += 1;
          }
        }
        SWEEP_HIP(hipEventRecord(e1, s));
        SWEEP_HIP(hipEventSynchronize(e1));
      }
      if (rc) break;
      float ms = 0.0f;
      SWEEP_HIP(hipEventElapsedTime(&ms, e0, e1));
      const double us = 1e3 * ms / nsteps;
      if (us < best_us) {
        best_us = us;
        best = c;
        best_p = cp;
        best_t = tb;
      }
     }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->timer.on = timing;
  p->tune = keep;
  if (rc) {
    ac_build_tiling(p);
    return rc;
  }
  sweep_tuning t = keep;
  t.rz = best;
  t.pml_rz = best_p;
  t.tblock = best_t;
  if ((rc = sweep_plan_set_tuning(p, &t))) return rc;
  tune_store(cache_path, key, best, best_p, best_t, best_us);
  if (chosen_rz) *chosen_rz = best;
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_plan_autotune")

extern "C" int sweep_batch_autotune(sweep_batch* b, const float* const* d_models,
                                    const float* const* d_wavelets, void* d_work,
                                    size_t work_bytes, int steps, int for_backward,
                                    const char* cache_path, void* stream, int* chosen) try {
  if (!b || !d_models || !d_wavelets || !d_work || steps < 1) {
    set_error("sweep_batch_autotune: bad argument");
    return SWEEP_EINVAL;
  }
  const int np = (int)b->plans.size();
  for (int q = 0; q < np; ++q)
    if (!d_models[q] || !d_wavelets[q]) {
      set_error("sweep_batch_autotune: null pointer for plan " + std::to_string(q));
      return SWEEP_EINVAL;
    }
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg_(b->device);
  if (!dg_.ok) {
    set_error("cannot make the batch's device current");
    return SWEEP_EHIP;
  }
  std::string shapes;
  for (sweep_plan* p : b->plans) shapes += (shapes.empty() ? "" : " ") + tune_shape(p);
  const std::string key =
      tune_key(b->plans[0], for_backward ? "batch-gradient" : "batch-forward", shapes);
  auto apply = [&](int rz, int prz, int tb) {
    for (sweep_plan* p : b->plans) {
      sweep_tuning t = p->tune;
      t.rz = rz;
      t.pml_rz = prz;
      t.tblock = tb;
      const int rc = sweep_plan_set_tuning(p, &t);
      if (rc) return rc;
    }
    b->rz = rz;
    b->prz = prz;
    b->saved = false;
    b->gfwd.reset();
    b->gbwd.reset();
    if (chosen) {
      chosen[0] = rz;
      chosen[1] = prz;
      chosen[2] = tb;
    }
    return SWEEP_OK;
  };
  {
    int rz = 0, prz = 0, tb = 0;
    if (tune_lookup(cache_path, key, rz, prz, tb)) return apply(rz, prz, tb);
  }
  std::vector<AcLayout> L;
  std::vector<size_t> off;
  size_t total = 0;
  batch_layouts(b, for_backward ? 1 : 0, L, off, total);
  if (work_bytes < total) {
    set_error("workspace too small: need " + std::to_string(total) + " bytes");
    return SWEEP_ENOMEM;
  }
  // the gradient mix: recompute and reverse the first `steps` steps (at most a
  // segment) of every plan after the forward steps; the values are not used
  std::vector<int> n0(np, 0), n1(np, 0);
  std::vector<const float*> noresid(np, nullptr);
  int lenmax = 0;
  for (int q = 0; q < np; ++q) {
    sweep_plan* p = b->plans[q];
    n1[q] = std::min(std::min(steps, p->pb.nt), p->ckpt);
    lenmax = std::max(lenmax, n1[q]);
  }
  std::vector<bool> timing(np);
  for (int q = 0; q < np; ++q) {
    timing[q] = b->plans[q]->timer.on;
    b->plans[q]->timer.on = false;
  }
  std::vector<float*> nogathers(np, nullptr);
  hipEvent_t e0, e1;
  SWEEP_HIP(hipEventCreate(&e0));
  SWEEP_HIP(hipEventCreate(&e1));
  const int cand[4] = {1, 2, 4, 8};
  int best[3] = {b->rz, b->prz, b->plans[0]->tune.tblock};
  double best_us = 1e300;
  int rc = SWEEP_OK;
  for (int c : cand)
    for (int cp : cand)
      for (int tb = 1; tb <= 2 && !rc; ++tb) {
        if (cp > c) continue;
        if ((rc = apply(c, cp, tb))) break;
        bool deep = false;
        for (sweep_plan* p : b->plans) deep = deep || ac_two_steps(p);
        if (tb == 2 && !deep) continue;  // no deep tiles: the same as tblock = 1
        for (int q = 0; q < np && !rc; ++q)
          rc = ac_upload_geometry(b->plans[q], at<char>(d_work, off[q]), L[q], s);
        for (int rep = 0; rep < 2 && !rc; ++rep) {  // the first pass warms up
          if ((rc = hipEventRecord(e0, s) == hipSuccess ? SWEEP_OK : SWEEP_EHIP)) break;
          rc = batch_forward_enqueue(b, d_models, d_wavelets, nogathers.data(), d_work, L, off, 0,
                                     s, steps);
          for (int q = 0; q < np && !rc && for_backward; ++q) {
            sweep_plan* p = b->plans[q];
            void* wq = at<char>(d_work, off[q]);
            p->arot = Rot();
            for (int k = 0; k < 2 && !rc; ++k)
              rc = launch_fill(at<float>(wq, L[q].adjaux[k]), L[q].aux_elems, 0.0f, s);
            for (int k = 0; k < 4 && !rc; ++k)
              rc = launch_fill(at<float>(wq, L[q].lf[k]), p->pb.nshots * L[q].plane, 0.0f, s);
            if (!rc) rc = ac_bwd_restore(p, wq, L[q], 0, s);
          }
          if (!rc && for_backward)
            rc = batch_segment_enqueue(b, noresid.data(), d_work, L, off, n0, n1, lenmax, s);
          if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
            rc = SWEEP_EHIP;
        }
        if (rc) break;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = SWEEP_EHIP;
          break;
        }
        if (ms < best_us) {
          best_us = ms;
          best[0] = c;
          best[1] = cp;
          best[2] = tb;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int q = 0; q < np; ++q) b->plans[q]->timer.on = timing[q];
  if (rc) {
    if (rc == SWEEP_EHIP) set_error("sweep_batch_autotune: HIP error while timing");
    return rc;
  }
  if ((rc = apply(best[0], best[1], best[2]))) return rc;
  tune_store(cache_path, key, best[0], best[1], best[2], 1e3 * best_us / steps);
  return SWEEP_OK;
}
SWEEP_ABI_CATCH("sweep_batch_autotune")
