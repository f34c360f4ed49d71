// Internal declarations shared by the library's translation units.
// Host code and kernels for gfx950; nothing here crosses the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "sweep.h"

namespace sweep {

// ------------------------------------------------------------------ errors
// The message of the last error on the calling thread. set_error_c never
// throws (it copies into a fixed thread-local buffer), so the ABI's catch
// clauses can call it.
void set_error(const std::string& msg);
void set_error_c(const char* msg) noexcept;

// Catch clauses closing the function-try-block of every extern "C" entry
// point, so that no C++ exception crosses the ABI: host allocation failure is
// reported as SWEEP_ENOMEM, anything else as SWEEP_EINVAL; entry points that
// return a size report 0.
#define SWEEP_ABI_CATCH(fn)                                              \
  catch (const std::bad_alloc&) {                                        \
    ::sweep::set_error_c(fn ": out of host memory");                    \
    return SWEEP_ENOMEM;                                                 \
  }                                                                      \
  catch (...) {                                                          \
    ::sweep::set_error_c(fn ": unexpected C++ exception");              \
    return SWEEP_EINVAL;                                                 \
  }
#define SWEEP_ABI_CATCH_SIZE(fn)                                         \
  catch (...) {                                                          \
    ::sweep::set_error_c(fn ": unexpected C++ exception");              \
    return 0;                                                            \
  }
#define SWEEP_ABI_CATCH_VOID(fn) \
  catch (...) {                  \
    ::sweep::set_error_c(fn ": unexpected C++ exception"); \
  }

// Makes `dev` the current HIP device for the lifetime of the guard and
// restores the previous one afterwards; dev < 0 leaves the current device.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (dev < 0) return;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) {
      ok = false;
      return;
    }
    if (cur == dev) return;
    if (hipSetDevice(dev) != hipSuccess) {
      ok = false;
      return;
    }
    prev = cur;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;
};
#define SWEEP_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ::sweep::set_error(std::string(#call) + " failed: " + hipGetErrorString(e_));  \
      return SWEEP_EHIP;                                                             \
    }                                                                                \
  } while (0)

// Work-group shape used by every stencil kernel: one wave64 row of 64 columns,
// four rows of waves (256 threads). A tile is 64 columns by TZ rows.
constexpr int kTX = 64;
constexpr int kThreads = 256;

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Work-groups of one launch are dealt to the 8 XCDs round-robin by flat index,
// and each XCD has its own L2. xcd_spread renumbers the flat index f of n so
// that every XCD receives one contiguous run of the logical block order
// (consecutive tiles of a shot, then the next shot): tiles that share halo
// cache lines then run under the same L2. It is a bijection of [0, n).
__device__ __forceinline__ int xcd_spread(int f, int n) {
  const int x = f & 7, k = f >> 3;
  const int q = n >> 3, r = n & 7;
  return x * q + min(x, r) + k;
}

// f[i] for a base f that is the same for the whole work-group (a per-shot
// plane, a model plane, a memory-variable strip) and a 32-bit lane index i.
// Plans hold fewer than 2^29 cells per plane, so the byte offset (4 or 8 bytes
// per cell) fits in 32 bits; formed there, it lets the access take the
// scalar-base addressing form (32-bit lane offset, 64-bit base in scalar
// registers) instead of a 64-bit address computed in every lane.
template <class T>
__device__ __forceinline__ T& u32at(T* f, unsigned i) {
  using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return *reinterpret_cast<T*>(reinterpret_cast<C*>(f) + i * (unsigned)sizeof(T));
}

// Guarded load through u32at: the caller passes an index that is valid (0
// where !ok), so every lane loads and the value is selected afterwards (a
// guarded load written as a branch must complete before the other path writes
// its register, which serialises a sequence of them).
__device__ __forceinline__ float ldz32(const float* f, unsigned i, bool ok) {
  const float v = u32at(f, i);
  return ok ? v : 0.0f;
}

// ------------------------------------------------------------------ acoustic
// Device-side view of one time step of the acoustic recurrence (all shots of one
// plan). Fields are [shot][NZ][NX]; x-strip memory variables [shot][NZ][2P]
// (columns [0,P) then [NX-P,NX)); z-strip ones [shot][2P][NX].
struct AcStep {
  int NX, NZ, P, nt, nrec, nshots;
  int n;          // time step being taken (forward) or reversed (adjoint)
  int tiles_x;    // tile columns in the global tiling
  int ntiles;     // tiles in the global tiling (receiver CSR stride)
  float w;        // (dt/h)^2, source scale
  const float* Cs;   // (v dt / h)^2, [NZ][NX]
  const float* ax;   // C-PML a, b along x [NX] and z [NZ]
  const float* bx;
  const float* az;
  const float* bz;
  // forward: p^n (cur), p^{n-1} (prev), p^{n+1} (next)
  // adjoint: lambda^{n+1} (cur), lambda^{n+2} (prev), lambda^n (next)
  // A pass of two steps over the deep tiles also writes p^{n+2} / lambda^{n-1}
  // to next2. The kernels read prev and write next at a tile's own cells only.
  const float* cur;
  const float* prev;
  float* next;
  float* next2;
  // memory variables: read *_in (time n-1), write *_out (time n)
  const float* psx_in;
  float* psx_out;
  const float* zex_in;
  float* zex_out;
  const float* psz_in;
  float* psz_out;
  const float* zez_in;
  float* zez_out;
  // sources / receivers
  const int* src_cell;    // [nshots] padded linear index
  const float* wavelet;   // [nshots][nt]
  const int* rec_off;     // [nshots * ntiles + 1] CSR over (shot, tile)
  const int2* rec_ent;    // (local cell index in tile, receiver index)
  float* gathers;         // forward: [nshots][nt][nrec] output, or null
  const float* resid;     // adjoint: [nshots][nt][nrec] injected at step n-1
  // forward extras
  float* B_out;           // [nshots][NZ][NX] Laplacian term B'^n, or null
  float* B_out2;          // B'^{n+1} (two-step pass), or null
  // adjoint extras
  const float* B_in;      // B'^n of this step
  const float* B_in2;     // B'^{n-1} (two-step pass)
  float* g;               // [nshots][NZ][NX] gradient partial
  int g_init;             // 1: g = P1 B (first step of a segment), 0: g += P1 B
  // tiles: the interior rectangle [itx0, itx1) x [itz0, itz1) of tile
  // coordinates holds the n_int tiles without C-PML cells; the other n_pml
  // tiles (the frame) take the PML kernel
  int itx0, itx1, itz0, itz1;
  int n_int, n_pml;
  const int* ilist;  // the n_int tiles the interior kernel takes
  // runs of a two-step pass: (tile column, first tile row | tile rows << 16)
  const int2* drun;
  int n_run;
  int n_xf, n_zf;  // frame tiles: left/right columns (x frame), above/below (z frame)
  int tz;    // rows of a tile
  int nsub;  // PML work-groups per frame tile (each takes tz / nsub rows)
  // Born (tangent-linear) step, Eq. 16: p^{n+1} += dCs * bB at every cell
  // (last, so the other fields keep their kernel-argument offsets)
  const float* bdC;       // [NZ][NX] dCs = 2 v dv (dt/h)^2
  const float* bB;        // [nshots][NZ][NX] background B'^n
};

// Static device workspace of sweep_forward_noalloc (per GPU): the largest
// forward workspace it accepts.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
// Device address of that workspace on `device` (current); set up once per
// device by the first context created on it (ctx.hip).
int scratch_address(int device, void** out);

// Several plans of different shapes advanced by one launch per kernel kind.
// A launch carries the step descriptors of up to kPlansPerLaunch plans in its
// kernel arguments; a batch of more plans takes one launch per group of them.
constexpr int kPlansPerLaunch = 8;
constexpr int kMaxBatchPlans = 4096;
struct AcBatch {
  int nplans;
  int base[kPlansPerLaunch + 1];  // first flat block of each plan in this launch
  AcStep step[kPlansPerLaunch];
};

// Launchers (acoustic.hip). Tiles are 64 x 4 rz; the interior kernel keeps rz rows
// per thread, the PML kernel prz (prz <= rz, a frame tile split into rz / prz pieces).
int ac_launch_prep(const float* v, float* vpad, float* Cs, float* ax, float* bx, float* az,
                   float* bz, int nx, int nz, int P, double h, double dt, double vmax,
                   double f0, double R, hipStream_t s);
// C-PML tables a, b along x (NX) and z (NZ) of an acoustic-type padded grid.
int ac_launch_tables(float* ax, float* bx, float* az, float* bz, int NX, int NZ, int P,
                     double h, double dt, double vmax, double f0, double R, hipStream_t s);
int ac_launch_fwd(const AcStep& a, int rz, int prz, hipStream_t s, hipEvent_t* ev);
int ac_launch_adj(const AcStep& a, int rz, int prz, hipStream_t s, hipEvent_t* ev);
// Born perturbation step (a.bdC, a.bB set; single steps over all tile sets)
// and its model perturbation dCs[NZ][NX] from v, dv [nz][nx].
int ac_launch_born(const AcStep& a, int rz, int prz, hipStream_t s);
// Encoded shots: adds the nsrc sources of every shot to p^{n+1} (next) after
// step n and records again the receivers on source cells (gathers may be null).
int ac_launch_inject_encoded(float* next, size_t plane, const int* src_cell, const float* wav,
                             int nsrc, int nt, int n, float w, int nshots, const int* co_off,
                             const int* co_rec, const int* rec_cell, float* gathers, int nrec,
                             hipStream_t s);
int ac_launch_born_prep(const float* v, const float* dv, float* dCs, int nx, int nz, int P,
                        double h, double dt, hipStream_t s);
int ac_launch_fwd_batch(const AcStep* steps, int n, int rz, int prz, hipStream_t s);
// Two steps over the deep runs (a.drun): forward n and n+1, or adjoint n and n-1.
int ac_launch_deep(const AcStep& a, bool adj, hipStream_t s, hipEvent_t* ev);
// The same for several plans in one launch (steps[q].n_run == 0: no pass).
int ac_launch_deep_batch(const AcStep* steps, int n, bool adj, hipStream_t s);
int ac_launch_adj_batch(const AcStep* steps, int n, int rz, int prz, hipStream_t s);
int ac_launch_adj_init(float* lam_cur, float* lam_prev, size_t plane_elems, float* aux,
                       size_t aux_elems, const int* rec_cell, const float* resid, int nshots,
                       int nt, int nrec, hipStream_t s);
int ac_launch_fold(double* tot, const float* gpart, int nshots, size_t plane, hipStream_t s);
int ac_launch_finish(const double* tot, const float* vpad, float* grad, int nx, int nz, int P,
                     int NX, double scale, hipStream_t s);

// Generic helpers (util.hip).
int launch_fill(float* p, size_t n, float v, hipStream_t s);
int launch_fill_f64(double* p, size_t n, double v, hipStream_t s);
int launch_copy(float* dst, const float* src, size_t n, hipStream_t s);

}  // namespace sweep
