/*
 * libsweep: MI355X (gfx950) HIP implementation of the SWEEP hot path
 * (arXiv 2604.14189): the 2-D finite-difference time loop, its exact adjoint and
 * the resulting full-waveform-inversion gradients, for the constant-density
 * acoustic equation (Sec. 3.1.2, Eq. 2) and the isotropic elastic
 * velocity-stress system (Sec. 3.5, Eq. 12); plus the Fourier-feature MLP
 * velocity model the paper's neural-network workflow calls for (Sec. 1).
 *
 * The split follows the paper's Propagator / Source / Receiver modules
 * (Sec. 2.1): a plan fixes the grid, time axis, absorbing pad, sources and
 * receivers ("shapes are inferred from the model"); forward() runs the whole
 * time loop for every shot and returns shot gathers; backward() runs the
 * adjoint and returns d(loss)/d(model) for a given d(loss)/d(gathers).
 * Batch modelling (Sec. 2.2): every call advances all shots of a plan, and the
 * batch API advances several plans of uneven size, in one kernel per step.
 *
 * Conventions for every call
 *  - Fields and models are float32, row-major [z][x] with x contiguous
 *    (x = horizontal, z = depth). Source / receiver positions are integer cell
 *    indices (x, z) of the model grid.
 *  - All pointers named d_* are DEVICE pointers owned by the caller; the library
 *    never allocates, frees or keeps them beyond the call. Host pointers are
 *    read during the call only.
 *  - `stream` is a hipStream_t passed as void*; every call only enqueues work on
 *    it and returns without synchronising (except where stated).
 *  - Return value: SWEEP_OK (0) or a negative error code; sweep_last_error()
 *    gives a message for the calling thread. No C++ exception crosses the ABI.
 *  - Calls on one plan are not thread-safe; different plans are independent.
 *  - Plans and batches created with a context run on the context's device:
 *    each call makes that device current and restores the caller's device
 *    before returning. Without a context (NULL) they run on the device current
 *    at each call. The MLP, Adam and misfit calls run on the current device.
 */
#ifndef SWEEP_H
#define SWEEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWEEP_OK 0
#define SWEEP_EINVAL (-1) /* bad shape, position outside the model, nt < 1, ... */
#define SWEEP_EHIP (-2)   /* a HIP runtime call failed; the message names it */
#define SWEEP_ENOMEM (-3) /* the workspace passed is smaller than required, or host
                             memory ran out inside the call */
#define SWEEP_ECFL (-4)   /* pml_vmax * dt / h exceeds the scheme's stability limit */
#define SWEEP_ESTATE (-5) /* call out of order (e.g. backward without a saved forward) */

#define SWEEP_ACOUSTIC 0 /* Eq. 2: 2nd order in time, 8th order in space, C-PML */
#define SWEEP_ELASTIC 1  /* Eq. 12: staggered velocity-stress, 4th order, C-PML */
/* Eq. 1: first-order variable-density acoustic (particle velocity and
 * pressure). Computed by the SWEEP_ELASTIC scheme with shear modulus 0: the
 * two normal stresses then both equal -p and the shear stress stays 0, which
 * is the first-order acoustic system on the same staggered grid. The step
 * kernels run their fluid variants, which leave out the shear stress and its
 * terms (all products with mu = 0): the same results, fewer bytes. Model
 * (vp, rho), gathers (vx, vz), gradients (vp, rho); free_surface = 1 is the
 * pressure-release top. */
#define SWEEP_ACOUSTIC_VD 2
/* Eq. 5: pseudo-acoustic wave equation of VTI media, P_tt = (1 + 2 eta) v^2 P_xx
 * + vv^2 P_zz - 2 eta v^2 vv^2 F_xxzz with P = F_tt (v the NMO velocity, vv the
 * vertical velocity, eta >= 0 the anisotropy parameter). Both fields advance by
 * the leapfrog of the acoustic scheme with its 8th-order operators (F_xxzz as
 * D2x D2z F) and per-axis C-PML; the pad replicates vv and v and holds
 * eta = 0 (an elliptic absorbing layer). Model (vv, v, eta), gathers P,
 * gradients (vv, v, eta). pml_vmax must be at least the fastest horizontal
 * speed v sqrt(1 + 2 eta) (the Courant limit is the acoustic one); eta < 0 is
 * not supported (the scheme's two modes would not stay real). 64 x 16 tiles,
 * single steps: tuning.rz must stay 4. The source
 * should sit where eta = 0, as the formulation asks (the paper's figure shows
 * the artificial mode it otherwise excites). */
#define SWEEP_VTI 3

/* Problem description. The padded grid adds `pml` absorbing cells on each side
 * (and none on top when free_surface = 1, elastic only); the model is
 * replicated from its edge cells into the pad. */
typedef struct {
  int physics;      /* SWEEP_ACOUSTIC, SWEEP_ELASTIC, SWEEP_ACOUSTIC_VD or SWEEP_VTI */
  int nx, nz;       /* model grid (cells) */
  int pml;          /* absorbing pad width (cells), >= 0 */
  int free_surface; /* elastic: 1 = traction-free top row (acoustic_vd: p = 0
                       there); acoustic: must be 0 */
  double h;         /* grid spacing dx = dz (m) */
  double dt;        /* time step (s) */
  int nt;           /* time steps */
  double pml_vmax;  /* velocity of the damping profile (m/s); fixed, not differentiated */
  double pml_f0;    /* C-PML frequency (Hz), usually the source peak frequency */
  double pml_R;     /* target reflection coefficient, e.g. 1e-3 */
  int ckpt_every;   /* checkpoint interval k (steps) for backward(); 0 = default 50 */
  int nshots;       /* shots advanced together */
  int nrec;         /* receivers per shot */
  int nsrc;         /* sources per shot, 0 or 1 = one. Acoustic only: > 1 makes
                       every shot an encoded shot (source encoding, Sec. 1: one
                       simulation of several sources, each with its own wavelet,
                       e.g. one shot's wavelet times a random sign). Source k of
                       a shot adds its term after the update, in the order k = 0
                       .. nsrc-1. Plans with nsrc > 1 do not join batches */
} sweep_problem;

/* Tile / launch choices (what the autotuner searches). Results are bitwise
 * independent of every field here. */
typedef struct {
  int rz;          /* acoustic tiles are 64 x 4 rz cells; rows per thread of the
                      interior kernel: 1, 2, 4 or 8 (default 8) */
  int pml_rz;      /* rows per thread of the C-PML (frame-tile) kernels, <= rz: a
                      frame tile is split into rz / pml_rz work-groups (default 4) */
  int use_graph;   /* 1 = capture each forward/backward time loop as a hipGraph
                      (every physics; the geometry upload and the state checks
                      stay outside it). A graph is captured on the first call
                      with given pointers (model, wavelets, gathers, workspace,
                      save flag; residuals, gradient, workspace) and replayed
                      by the next ones; a tuning change drops it. Calls with
                      profiling on run eagerly */
  int tblock;      /* acoustic: 2 = advance the deep interior tiles (no C-PML cell
                      within 4 cells, no source or receiver within 4, an 8-cell halo
                      inside the grid) two time steps per pass, marching down runs of
                      them; 1 = one step per pass (default 2). In a batch each
                      plan follows its own setting */
  int keep_b;      /* every physics; in a batch each plan its own count: the
                      saving forward stores what the backward needs of the last
                      keep_b checkpoint segments in the workspace, and backward()
                      reverses those segments without recomputing them (the
                      same bits). Acoustic: B'^n, and a stored segment needs no
                      checkpoint, so each one costs ckpt_every * nshots * NX *
                      NZ * 4 workspace bytes less its checkpoint slot (2 *
                      nshots * NX * NZ fields plus the C-PML memory variables,
                      4 bytes each); with any stored, the recomputed segments
                      write B'^n into the first stored segment's slots (free
                      by then), so the recomputation's own buffer of the same
                      size is dropped. Elastic and variable-density acoustic: the
                      five trace planes of each step, ckpt_every * 5 * nshots *
                      NX * NZ * 4 bytes per segment. VTI: the three trace
                      planes of each step (Bx', Bz', D2x'D2z'G), ckpt_every * 3
                      * nshots * NX * NZ * 4 bytes per segment, less its
                      checkpoint slot (P^n, P^{n-1}, G^n, G^{n-1} in float64 and
                      the C-PML memory variables). Elastic, variable-density and
                      VTI stored segments need no checkpoint either.
                      sweep_plan_workspace_bytes includes this. 0 = recompute
                      every segment (default) */
} sweep_tuning;

typedef struct sweep_plan sweep_plan;
typedef struct sweep_ctx sweep_ctx;

/* Message describing the last error on the calling thread ("" if none). */
const char* sweep_last_error(void);

/* Library context for HIP device `hip_device` (0 .. device count - 1): plans
 * and batches created with it are bound to that device (Sec. 2.3 places one
 * model replica per device; on one GPU a context is that device). Queries the
 * device's properties; allocates no device memory. SWEEP_EINVAL for a device
 * outside the range, SWEEP_EHIP if the runtime cannot be reached. The context
 * must outlive the plans and batches created with it. */
int sweep_ctx_create(sweep_ctx** out, int hip_device);
void sweep_ctx_destroy(sweep_ctx* ctx);
/* The context's device (-1 for NULL). */
int sweep_ctx_device(const sweep_ctx* ctx);

/* Create a plan on the context's device (ctx may be NULL: the plan then runs
 * on whatever device is current at each call). src_xz: host [nshots][nsrc][2] ([nshots][2] for one source);
 * rec_xz: host [nshots][nrec][2] (model-grid cells, x then z); the wavelets of
 * sweep_forward are then [nshots][nsrc][nt]. The arrays are copied. Fails with SWEEP_EINVAL on
 * inconsistent sizes or positions outside the model, SWEEP_ECFL when
 * pml_vmax*dt/h exceeds 0.5546 (acoustic, 8th order) or 0.6061 (elastic, 4th).
 * Does not touch the GPU. */
int sweep_plan_create(const sweep_ctx* ctx, const sweep_problem* pb, const int32_t* src_xz,
                      const int32_t* rec_xz, sweep_plan** out);
void sweep_plan_destroy(sweep_plan* plan);

/* Select tile / launch choices (validated; SWEEP_EINVAL if unsupported). Every
 * call discards the plan's saved forward state, and a batch holding the plan
 * refuses its backward (SWEEP_ESTATE) until its next saving forward. */
int sweep_plan_set_tuning(sweep_plan* plan, const sweep_tuning* t);
int sweep_plan_get_tuning(const sweep_plan* plan, sweep_tuning* t);

/* Autotuner: runs `steps` forward steps of this plan for every supported tile
 * choice (rz and pml_rz in 1, 2, 4, 8 with pml_rz <= rz) and time-blocking
 * depth (tblock 1 or 2; 2 only where the tiling has deep tiles), keeps the
 * fastest and stores it in the plan; `cache_path` (may be NULL) is a file of
 * previous results, one JSON object per line:
 *   {"arch":"gfx950","physics":"acoustic","mode":"plan-forward",
 *    "shapes":"NXxNZxNSHOTSxPML","rz":8,"pml_rz":4,"tblock":2,"us_per_step":...}
 * keyed by everything up to and including "shapes" (GPU arch, physics, mode,
 * padded NX and NZ, nshots, pad width), read first and appended to. Elastic,
 * variable-density and VTI plans have no choice to make and return at once.
 * Synchronises `stream`. d_work needs the forward-only
 * workspace. Results never depend on the choice (bitwise). *chosen_rz (may be
 * NULL) receives the selected value. */
int sweep_plan_autotune(sweep_plan* plan, const float* d_model, const float* d_wavelet,
                        void* d_work, size_t work_bytes, int steps, const char* cache_path,
                        void* stream, int* chosen_rz);

/* Device workspace the caller must provide: for_backward = 0 for a forward-only
 * call, 1 for forward(save_for_backward=1) followed by backward(). */
size_t sweep_plan_workspace_bytes(const sweep_plan* plan, int for_backward);

/* Padded grid size of the plan (NX, NZ). */
int sweep_plan_padded(const sweep_plan* plan, int* NX, int* NZ);

/* Acoustic tiling under the current tuning: the padded grid is cut into tiles
 * of 64 columns x tile_rows rows. The interior tiles hold no C-PML cell (no
 * cell within pml + 4 of an edge) and form the rectangle of tile columns
 * [rect[0], rect[1]) x tile rows [rect[2], rect[3]) (all zero when empty);
 * they are advanced by the interior kernel (16 bytes per cell-update forward).
 * rect[4] receives how many of them are deep (no C-PML cell within 4 cells,
 * no source or receiver within 4, their 8-cell halo inside the grid) and
 * advance two steps per pass when tuning.tblock = 2 (0 when tblock = 1). The frame_tiles others are advanced
 * by the C-PML kernels: the z frame (the rectangle's columns above and below
 * it) and the x frame (all other tile columns). rect (5 ints) may be NULL.
 * EINVAL for an elastic plan or a null pointer. */
int sweep_plan_tiles(const sweep_plan* plan, int* interior_tiles, int* frame_tiles,
                     int* tile_rows, int* rect);

/* Forward modelling of every shot.
 *   d_model   [nparam][nz][nx]: acoustic vp (nparam 1); elastic vp, vs, rho (3);
 *             acoustic_vd vp, rho (2); vti vv, v, eta (3)
 *   d_wavelet [nshots][nt]: source time function, sample n injected at step n
 *   d_gathers [nshots][nt][nrec][ncomp] out: acoustic and vti p (ncomp 1) at step n+1;
 *             elastic (vx, vz) (ncomp 2)
 *   d_work    workspace of at least sweep_plan_workspace_bytes(plan, save) bytes
 *   save_for_backward: 1 stores checkpoints every ckpt_every steps in d_work
 * Acoustic: the padded-grid recurrence is p^{n+1} = 2p^n - p^{n-1} + (v dt)^2 B^n
 * + (dt/h)^2 s_n at the source, where B^n is the 8th-order Laplacian with C-PML
 * memory terms (the step function of Sec. 2.1 in the interior). */
int sweep_forward(sweep_plan* plan, const float* d_model, const float* d_wavelet,
                  float* d_gathers, void* d_work, size_t work_bytes, int save_for_backward,
                  void* stream);

/* Forward modelling that allocates nothing, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, harnesses
 * that forbid allocation): sweep_forward(plan, d_model, d_wavelet, d_gathers,
 * work, bytes, save_for_backward = 0, stream) with the workspace taken from a
 * static device array of the library (32 MiB per GPU the library runs on,
 * reserved when the library is loaded and held until the process ends)
 * instead of a caller buffer. The caller still passes the inputs and the
 * gathers (layouts as in sweep_forward). The plan must have been created
 * with a context (SWEEP_EINVAL otherwise) and its forward-only workspace
 * (sweep_plan_workspace_bytes(plan, 0)) must fit in 32 MiB (SWEEP_EINVAL
 * otherwise; a 240 x 240 padded grid with 1 shot and 1000 steps needs 1.6 MiB). Launches
 * are eager (tuning.use_graph is ignored) and untimed; no state is left for
 * sweep_backward. Every call on a GPU uses that GPU's one array: calls that
 * overlap on one GPU (other streams or threads) race and must be serialised
 * by the caller; each call writes every part of the array it reads first. */
int sweep_forward_noalloc(sweep_plan* plan, const float* d_model, const float* d_wavelet,
                          float* d_gathers, void* stream);

/* Born (tangent-linear) modelling of every shot, Eq. 16 (acoustic plans only):
 *   d_dgathers = (d gathers / d vp) . d_dmodel
 *   d_model, d_dmodel [nz][nx]: background vp and its perturbation dvp
 *   d_wavelet  [nshots][nt] as in sweep_forward
 *   d_dgathers [nshots][nt][nrec] out: the perturbation dp at step n+1
 *   d_work     workspace of at least sweep_plan_workspace_bytes(plan, 1) bytes
 * The background recurrence of sweep_forward runs with a perturbation field dp
 * that obeys the same recurrence (C-PML included) without the source and with
 * dC B^n added at every cell, dC = 2 vp dvp dt^2 (dvp edge-replicated into the
 * pad like vp). Its transpose is sweep_backward: the adjoint of Born modelling
 * (the migration / least-squares RTM image) is the model gradient for the
 * residual given. Single steps only (the tuning's tblock is not used). Leaves
 * no state for sweep_backward (a following backward needs a new forward).
 * Errors: SWEEP_EINVAL (null pointer, elastic plan), SWEEP_ENOMEM (workspace
 * too small), SWEEP_EHIP. All pointers are caller-owned device memory. */
int sweep_born_forward(sweep_plan* plan, const float* d_model, const float* d_dmodel,
                       const float* d_wavelet, float* d_dgathers, void* d_work,
                       size_t work_bytes, void* stream);

/* Adjoint: given d_resid = dJ/d(gathers) (layout of d_gathers; may be null
 * when nrec = 0, and the gradient is then zero), writes
 * d_grad [nparam][nz][nx] = dJ/d(model) summed over shots. Requires the
 * preceding sweep_forward(save_for_backward = 1) on the same plan, model and
 * workspace (SWEEP_ESTATE otherwise). The result is the exact transpose of the
 * forward recurrence (dot-product test of Sec. 1), evaluated by recomputing each
 * checkpoint segment and sweeping it backwards. */
int sweep_backward(sweep_plan* plan, const float* d_resid, float* d_grad, void* d_work,
                   size_t work_bytes, void* stream);

/* Kernel timing for measurement tools. When enabled, every launch of the step
 * kernels is bracketed by a pair of hipEvents recorded on the call's stream
 * (the events add a few microseconds per launch). Acoustic classes, for the
 * forward (0-2), the adjoint (3-5) and the segment recompute that also stores
 * B^n (6-8): interior-tile kernel, z-frame C-PML kernel, x-frame C-PML kernel;
 * with tuning.tblock = 2 the two-step passes over the deep tiles are classes 9
 * (forward), 10 (adjoint) and 11 (recompute), and the interior classes then
 * time the remaining interior tiles. An elastic plan times each whole step
 * (both of its kernels) in classes 0, 3 and 6.
 * enable: 0 off; n >= 1 times the launches of every n-th step (n = 1: all); a
 * step pair of a two-step pass counts as three launch groups (deep pass, step
 * n, step n+1).
 * sweep_plan_set_profiling resets the counters; sweep_plan_kernel_time waits for
 * the recorded events and returns the number of timed launches and their summed
 * duration in milliseconds since the reset. */
int sweep_plan_set_profiling(sweep_plan* plan, int enable);
/* Number of nodes of the plan's captured forward and backward graphs
 * (tuning.use_graph = 1; each node one kernel launch of the time loop; 0 when
 * nothing is captured). */
int sweep_plan_graph_nodes(const sweep_plan* plan, size_t* fwd_nodes, size_t* bwd_nodes);
int sweep_plan_kernel_time(sweep_plan* plan, int kernel_class, int* launches, double* total_ms);

/* ---- batches: several acoustic plans of different grids / shots / nt ----
 * Batch modelling of different models (Sec. 2.2): every time step of every
 * plan in the batch is advanced by one launch per kernel kind (plans whose nt
 * is reached drop out), so k launches serve all of them instead of one set per
 * plan. Results are bitwise identical to running each plan alone. The plans
 * stay owned by the caller and must outlive the batch; they must be distinct,
 * bound to the batch's device (ctx, or the first plan's when ctx is NULL) and
 * share the same rz and pml_rz tuning, which they must keep: forward and
 * backward return SWEEP_EINVAL when a member's rz or pml_rz no longer matches
 * the batch's, and backward returns SWEEP_ESTATE when any member's tuning
 * changed after the saving forward. 1 .. 4096 plans; each launch carries up to
 * 8 of them, so a batch of n plans takes ceil(n / 8) launches per kernel kind
 * and step. With use_graph = 1 the whole forward (and
 * the whole backward) is captured once as a hipGraph and replayed while the
 * pointers passed and the plans' tunings are unchanged. Pointer arrays are
 * host arrays of device pointers, one per plan; the workspace is carved into
 * one region per plan. */
typedef struct sweep_batch sweep_batch;
int sweep_batch_create(const sweep_ctx* ctx, sweep_plan* const* plans, int nplans,
                       sweep_batch** out);
void sweep_batch_destroy(sweep_batch* batch);
int sweep_batch_set_graph(sweep_batch* batch, int use_graph);
/* Number of nodes of the captured forward and backward graphs (each node is
 * one kernel launch of the batch's time loop; 0 when nothing is captured), so
 * that a caller can see how many launches one graph launch replaces. */
int sweep_batch_graph_nodes(const sweep_batch* batch, size_t* fwd_nodes, size_t* bwd_nodes);
size_t sweep_batch_workspace_bytes(const sweep_batch* batch, int for_backward);
int sweep_batch_forward(sweep_batch* batch, const float* const* d_models,
                        const float* const* d_wavelets, float* const* d_gathers, void* d_work,
                        size_t work_bytes, int save_for_backward, void* stream);
int sweep_batch_backward(sweep_batch* batch, const float* const* d_resids, float* const* d_grads,
                         void* d_work, size_t work_bytes, void* stream);

/* Batch autotuner: for every tile choice (rz, pml_rz as for sweep_plan_autotune)
 * and time-blocking depth (tblock 1 or 2; 2 only where some plan has deep
 * tiles) it times `steps` batched forward steps (nothing recorded, no
 * checkpoints) and, with for_backward = 1, the recomputation and reversal of
 * the first `steps` steps too (at most one checkpoint segment, no residual),
 * which is the step mix of a gradient; it sets the fastest on every plan of
 * the batch. `cache_path` (may be NULL) is the JSON-lines file of
 * sweep_plan_autotune, with "mode" batch-forward or batch-gradient and
 * "shapes" every plan's NXxNZxNSHOTSxPML (space-separated, in batch order),
 * read first and appended to. Synchronises `stream`; d_work needs the batch's workspace
 * for_backward. Results never depend on the choice (bitwise); the fields of the
 * workspace hold no result afterwards. chosen (3 ints: rz, pml_rz, tblock; may
 * be NULL) receives it. */
int sweep_batch_autotune(sweep_batch* batch, const float* const* d_models,
                         const float* const* d_wavelets, void* d_work, size_t work_bytes,
                         int steps, int for_backward, const char* cache_path, void* stream,
                         int* chosen);

/* L2 misfit of FWI (Sec. 1: the inversion fits the data in the least-squares
 * sense): d_resid[i] = d_pred[i] - d_obs[i] and *d_J = 0.5 * sum resid^2
 * (float64, device), with no time-step weight. d_resid is the dJ/d(gathers)
 * that sweep_backward takes. n elements of any layout (the gathers of one
 * plan: nshots * nt * nrec * ncomp). Deterministic two-stage reduction (fixed
 * contiguous chunks per block, then a fixed tree): the same n gives the same
 * bits. d_scratch (caller-owned device memory) must hold
 * sweep_l2_misfit_scratch_bytes(n) bytes of float64 partial sums. d_resid may
 * alias d_pred. SWEEP_EINVAL for a null pointer. */
size_t sweep_l2_misfit_scratch_bytes(size_t n);
int sweep_l2_misfit(const float* d_pred, const float* d_obs, float* d_resid, double* d_J,
                    size_t n, void* d_scratch, void* stream);

/* ---- MLP velocity model (neural-network velocity representation, Sec. 1) ----
 * v(x) = vmin + vscale * sigmoid(f(gamma(x))), gamma(x) = [cos 2 pi B x, sin 2 pi B x]
 * with 64 random frequencies B [64][2] and x = (i/(nx-1), j/(nz-1)) for model cell
 * (i, j) (point index m = j nx + i); f: 128 -> 256 -> 256 -> 256 -> 256 -> 1 with ReLU.
 * theta: float32 parameter vector of sweep_mlp_param_count() entries, in the order
 * W1 [256][128], b1 [256], W2 [256][256], b2, W3, b3, W4, b4, w5 [256], b5 [1]
 * (matrices stored out x in). Matrix products run on bf16 MFMA with float32
 * accumulation: features, weights (the pack made by sweep_mlp_cast),
 * hidden activations and back-propagated pre-activation gradients are
 * bfloat16 (round to nearest even); everything else is float32.
 * Device buffers: d_feats [npoints][128] bf16, d_wpack sweep_mlp_pack_count()
 * uint16, d_v / d_dv [npoints] float32, d_grad like theta. d_work holds the
 * forward activations that sweep_mlp_backward needs (same d_work, same npoints).
 * Its layout is public so that callers can inspect the bf16 intermediates:
 * with A(x) = x rounded up to a multiple of 256 bytes and S = npoints*256*2,
 * H1..H4 (hidden activations) at 0, S, 2S, 3S; y (float32 pre-sigmoid output)
 * at A(4S); after sweep_mlp_backward, dZ1..dZ4 (gradients with respect to the
 * hidden pre-activations) at A(A(4S) + 4 npoints) + l S, l = 0..3; every block
 * row-major [npoints][256].
 * All reductions are split over fixed row chunks and summed in a fixed order:
 * the results are deterministic. */
size_t sweep_mlp_param_count(void);
size_t sweep_mlp_pack_count(void);
size_t sweep_mlp_workspace_bytes(int npoints);
int sweep_mlp_encode(const float* d_B, int nx, int nz, uint16_t* d_feats, void* stream);
int sweep_mlp_cast(const float* d_theta, uint16_t* d_wpack, void* stream);
int sweep_mlp_forward(const uint16_t* d_wpack, const float* d_theta, const uint16_t* d_feats,
                      int npoints, float vmin, float vscale, float* d_v, void* d_work,
                      size_t work_bytes, void* stream);
int sweep_mlp_backward(const uint16_t* d_wpack, const uint16_t* d_feats, int npoints, float vscale,
                       const float* d_dv, float* d_grad, void* d_work, size_t work_bytes,
                       void* stream);

/* Adam (Kingma & Ba 2015) on n float32 parameters, step t >= 1 (bias-corrected):
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; theta -= lr m^ / (sqrt(v^) + eps). */
int sweep_adam_step(float* d_theta, float* d_m, float* d_v, const float* d_g, size_t n, float lr,
                    float b1, float b2, float eps, int t, void* stream);

#ifdef __cplusplus
}
#endif
#endif
