// Host-side plan object and workspace layout (not part of the C-ABI).
#pragma once

#include <string>
#include <vector>

#include "internal.h"

// Workspace layout of an acoustic plan (byte offsets into the caller's buffer).
namespace sweep {
struct AcLayout {
  size_t plane, xs, zs, aux_elems;
  size_t ax, bx, az, bz, vpad, Cs, wav, src_cell, rec_cell, rec_off, rec_ent;
  size_t co_off, co_rec;  // encoded shots: receivers on source cells (CSR per shot)
  size_t tl, tl_cap;  // tile lists (all interior, ring, deep), tl_cap ints each
  size_t pf[4], aux[2];  // forward field buffers (rotated), C-PML memory variables
  size_t fwd_end;
  int nseg;
  size_t slot_elems;
  size_t ck, Bseg, lf[4], adjaux[2], gpart, tot;
  int nkeep;    // checkpoint segments (the last ones) whose B'^n the forward stores
  size_t Bkeep;  // their B'^n: [nkeep][k][nshots][NZ][NX]
  size_t bwd_end;
};

// Which of the four field buffers hold the current and the previous field; a
// step writes a free buffer, so no kernel overwrites values a neighbouring
// tile may still read.
struct Rot {
  int cur = 1, prev = 0;
  int free_buf(int k) const {
    int f[2], c = 0;
    for (int i = 0; i < 4; ++i)
      if (i != cur && i != prev) f[c++] = i;
    return f[k];
  }
};
}  // namespace sweep

// Optional per-launch timing of the step kernels (hipEvent pairs recorded on the
// caller's stream around every launch of a kernel class).
namespace sweep {
// Acoustic: interior-tile kernel, z-frame and x-frame C-PML kernels of the
// forward, adjoint and recompute; elastic: one class per pass (Int slots).
enum KernelClass {
  kFwdInt = 0,
  kFwdZ = 1,
  kFwdX = 2,
  kAdjInt = 3,
  kAdjZ = 4,
  kAdjX = 5,
  kRecInt = 6,
  kRecZ = 7,
  kRecX = 8,
  kFwdDeep = 9,   // two-step passes over the deep tiles
  kAdjDeep = 10,
  kRecDeep = 11,
  kNumClasses = 12
};
struct KernelTimer {
  bool on = false;
  int period = 1;     // time the launches of every period-th step
  long long calls = 0;
  std::vector<hipEvent_t> ev[kNumClasses];  // start, stop, start, stop, ...
  size_t used[kNumClasses] = {};
  ~KernelTimer();
  void reset();
  // Six events: start/stop pairs for the classes (ci, cz, cx) of one step's
  // interior, z-frame and x-frame launches (negative: not timed, its pair is
  // null), or null when timing is off.
  hipEvent_t* take(int ci, int cz, int cx);
  hipEvent_t six[6];
};
}  // namespace sweep

namespace sweep {
struct ElLayout {
  size_t plane;
  size_t coef, tabx, tabz, dM, wav, src_cell, rec_cell, rec_sorted, state;
  size_t fwd_end;
  int nseg;
  size_t ck, trace, adj, gpart, tot;
  int nkeep;      // checkpoint segments (the last ones) whose traces the forward stores
  size_t trkeep;  // their traces: [nkeep][k][5][nshots][NZ][NX]
  size_t bwd_end;
};
}  // namespace sweep

namespace sweep {
// Pseudo-acoustic VTI plan: fields P and G = F / dt^2 (both float64), two
// buffers each (the new level overwriting the oldest), C-PML strips as in the
// acoustic layout.
struct VtiLayout {
  size_t plane, xs, zs, aux_elems;
  size_t ax, bx, az, bz, pad, cx, cz, cm, wav, src_cell, rec_cell, rec_off, rec_ent;
  size_t tl;  // tile list: the interior tiles, then the others (ntiles ints)
  size_t pf[2], gf[2], aux[2];
  size_t fwd_end;
  int nseg;
  size_t slot_elems;  // checkpoint (floats): P^n, P^{n-1}, G^n, G^{n-1} (2 each), memory variables
  size_t ck, tr, lf[2], mf[2], adjaux[2], gpart, tot;
  int nkeep;      // checkpoint segments (the last ones) whose traces the forward stores
  size_t trkeep;  // their traces: [nkeep][k][3][nshots][NZ][NX]
  size_t bwd_end;
};
}  // namespace sweep

namespace sweep {
// An instantiated hipGraph of a forward or backward call, reused while the
// pointers it was captured with are unchanged.
struct GraphCache {
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
  std::vector<const void*> key;
  size_t nodes = 0;  // nodes (kernel launches) of the captured graph
  ~GraphCache() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (stream) (void)hipStreamDestroy(stream);
  }
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    key.clear();
    nodes = 0;
  }
};
}  // namespace sweep

// A library context: the HIP device its plans and batches run on.
struct sweep_ctx {
  int device = 0;
  std::string arch;        // gcnArchName without feature suffixes, e.g. "gfx950"
  void* scratch = nullptr;  // device address of the static workspace on `device`
};

struct sweep_plan {
  sweep_problem pb;
  sweep_tuning tune;
  int device = -1;  // the context's device (-1: the device current at each call)
  std::string arch;  // the context's arch ("": queried at each autotune)
  void* scratch = nullptr;  // the context's static device workspace (null: no context)
  // incremented by every tuning change; a batch refuses a backward (or the
  // replay of a captured graph) after a member plan's tuning changed
  unsigned tune_gen = 0;
  int P = 0, NX = 0, NZ = 0, ckpt = 50;
  std::vector<int> src_cell;  // [nshots][nsrc] padded linear index
  int nsrc = 1;               // sources per shot (> 1: encoded shots, acoustic)
  std::vector<int> co_off, co_rec;  // receivers on source cells, CSR per shot
  std::vector<int> rec_cell;  // [nshots][nrec] padded linear index
  // tiling for the current tuning
  int TZ = 0, tiles_x = 0, tiles_z = 0, ntiles = 0;
  // interior rectangle of tiles without C-PML cells (tile coordinates)
  int itx0 = 0, itx1 = 0, itz0 = 0, itz1 = 0, n_int = 0, n_pml = 0, n_xf = 0, n_zf = 0;
  // interior tiles; those advanced two steps per pass (deep) and the others
  std::vector<int> ilist_all, ilist_ring, dlist;
  std::vector<int2> drun;  // deep tiles as chunks of tile-column runs
  sweep::Rot frot, arot;  // forward / adjoint buffer rotation
  // elastic: receivers sorted by (shot, cell, r) for deterministic injection,
  // and the transposed z-taps of the first rows under a free surface
  std::vector<int4> rec_sorted;
  int tt_cnt[4][4];
  int tt_off[4][4][8];
  float tt_w[4][4][8];
  std::vector<int> rec_off;
  std::vector<int2> rec_ent;
  // VTI: the 64 x 16 tiles with no C-PML strip within 4 cells, then the
  // others, and how many of the first kind (set by each forward)
  std::vector<int> vti_tl;
  int vti_nint = 0;
  // state of the last forward
  bool saved = false;
  const void* saved_work = nullptr;
  const float* saved_model = nullptr;
  int saved_rz = 0;
  sweep::KernelTimer timer;
  sweep::GraphCache gfwd, gbwd;
};

namespace sweep {
void ac_build_tiling(sweep_plan* p);
// keep: include the stored B'^n segments of tune.keep_b (single plans; a batch
// layout and Born modelling use none)
void ac_layout(const sweep_plan* p, AcLayout& L, bool keep = true);
void el_layout(const sweep_plan* p, ElLayout& L);
void el_build_tables(sweep_plan* p);
// Forward and backward of the staggered (elastic, variable-density) and VTI
// plans. Each is also split for graph capture: *_prepare / *_backward_check
// (workspace checks and host-to-device geometry copies, not captured), then
// *_enqueue (kernels only, which a graph may capture and replay), then
// *_mark_saved (the plan's saved-forward state).
int el_forward(sweep_plan* p, const float* model, const float* wavelet, float* gathers,
               void* work, size_t bytes, int save, hipStream_t s);
int el_backward(sweep_plan* p, const float* resid, float* grad, void* work, size_t bytes,
                hipStream_t s);
int el_forward_prepare(sweep_plan* p, void* work, size_t bytes, int save, hipStream_t s);
int el_forward_enqueue(sweep_plan* p, const float* model, const float* wavelet, float* gathers,
                       void* work, int save, hipStream_t s);
void el_mark_saved(sweep_plan* p, void* work, const float* model, int save);
int el_backward_check(const sweep_plan* p, const void* work, size_t bytes);
int el_backward_enqueue(sweep_plan* p, const float* resid, float* grad, void* work,
                        hipStream_t s);
void vti_layout(const sweep_plan* p, VtiLayout& L);
int vti_forward(sweep_plan* p, const float* model, const float* wavelet, float* gathers,
                void* work, size_t bytes, int save, hipStream_t s);
int vti_backward(sweep_plan* p, const float* resid, float* grad, void* work, size_t bytes,
                 hipStream_t s);
int vti_forward_prepare(sweep_plan* p, void* work, size_t bytes, int save, hipStream_t s);
int vti_forward_enqueue(sweep_plan* p, const float* model, const float* wavelet,
                        float* gathers, void* work, int save, hipStream_t s);
void vti_mark_saved(sweep_plan* p, void* work, const float* model, int save);
int vti_backward_check(const sweep_plan* p, const void* work, size_t bytes);
int vti_backward_enqueue(sweep_plan* p, const float* resid, float* grad, void* work,
                         hipStream_t s);
}  // namespace sweep

struct sweep_batch {
  std::vector<sweep_plan*> plans;  // owned by the caller
  int device = -1;                 // the plans' device (-1: current at each call)
  int rz = 8, prz = 2;
  bool use_graph = false;
  bool saved = false;
  const void* saved_work = nullptr;
  std::vector<unsigned> saved_gen;  // the plans' tuning generations at the saving forward
  sweep::GraphCache gfwd, gbwd;
};
