/*
 * FP64 CPU oracle for the SWEEP hot path (arXiv 2604.14189).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link or
 * call this library: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it. It shares no code, header, table or helper with the HIP
 * library; the two meet only through seeded inputs that neither side generates.
 *
 * What it computes (the paper gives the PDEs; the discretisation is the reading
 * written out in oracle/README.md and mirrored by the GPU kernels):
 *   - constant-density acoustic wave equation, second order in time (Sec. 3.1.2,
 *     Eq. 2), advanced with the leapfrog update of the step function shown in
 *     Sec. 2.1; 8th-order centred space stencil; C-PML absorbing pad;
 *   - its exact discrete adjoint (the dot-product test of Sec. 1 holds to
 *     rounding), the model gradient of an L2 misfit, and the Born
 *     (tangent-linear) operator of Eq. 16;
 *   - isotropic elastic velocity-stress system (Sec. 3.5, Eq. 12) on a staggered
 *     grid, 4th order in space, C-PML, free surface; its adjoint and gradients;
 *   - the pseudo-acoustic wave equation of VTI media (Sec. 3.3.1, Eq. 5) with
 *     the acoustic scheme's operators and pad, its adjoint and gradients.
 *
 * Everything is double precision, plain loops, no blocking, no fusion. OpenMP is
 * used only over independent shots (or over rows when there is a single shot).
 * Return value of every entry point: 0 on success, -1 on invalid arguments.
 */
#ifndef SWEEP_ORACLE_H
#define SWEEP_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Problem description shared by the acoustic and elastic oracle calls.
 * Model grid nx (horizontal, x) by nz (depth, z); fields are stored [z][x]
 * row-major with x contiguous.  The padded grid adds `pml` cells on every side
 * (on the top only when free_surface == 0). */
typedef struct {
  int nx, nz;         /* model grid */
  int pml;            /* absorbing pad width in cells */
  int free_surface;   /* elastic only: 1 = traction-free top row, no top pad */
  double h;           /* grid spacing dx = dz (m) */
  double dt;          /* time step (s) */
  int nt;             /* number of time steps */
  double pml_vmax;    /* velocity used for the damping profile (m/s) */
  double pml_f0;      /* frequency used for the C-PML alpha term (Hz) */
  double pml_R;       /* target reflection coefficient */
  int nshots;         /* number of shots */
  int nrec;           /* receivers per shot */
  int ckpt_every;     /* gradient: checkpoint interval in steps (0 = store all) */
  int nthreads;       /* OpenMP threads (<= 0: library default) */
} orc_problem;

/* ---- building blocks exported so the tests can pin them directly ---- */

/* C-PML profile along one padded axis of length n with lo_pad / hi_pad pad
 * cells at its two ends (lo_pad = 0 for an axis whose low side is a free
 * surface), evaluated at positions i + shift (shift 0 for integer nodes, 0.5
 * for staggered half nodes). Writes the recursion coefficients a[n], b[n]. */
int orc_pml_profile(int n, int lo_pad, int hi_pad, double shift, double h, double dt,
                    double vmax, double f0, double R, double* a, double* b);

/* 8th-order second derivative and first derivative along a 1-D zero-padded
 * array f[n] (values beyond the ends are zero). */
int orc_d2_1d(const double* f, int n, double h, double* out);
int orc_d1_1d(const double* f, int n, double h, double* out);

/* ---- acoustic (Eq. 2) ---- */

/* Forward modelling. v[nz][nx] (m/s); src_xz[nshots][2] and rec_xz[nshots][nrec][2]
 * are model-grid cell indices (x, z); wavelet[nshots][nt]; gathers out
 * [nshots][nt][nrec] with gathers[s][n][r] = p^{n+1} at receiver r. */
int orc_ac_forward(const orc_problem* pb, const double* v, const int* src_xz,
                   const double* wavelet, const int* rec_xz, double* gathers);

/* Single-shot full wavefield history: snaps[nt][NZ][NX] = p^{n+1} on the padded
 * grid (NX = nx + 2 pml, NZ = nz + 2 pml). Uses pb->nshots = 1 semantics. */
int orc_ac_wavefield(const orc_problem* pb, const double* v, const int* src_xz,
                     const double* wavelet, double* snaps);

/* Adjoint / gradient. Given resid[nshots][nt][nrec] = dJ/d(gathers), returns
 * grad_v[nz][nx] = dJ/dv summed over shots, optionally grad_wavelet[nshots][nt]
 * = dJ/d(wavelet) (pass NULL to skip) and the forward gathers (NULL to skip). */
int orc_ac_gradient(const orc_problem* pb, const double* v, const int* src_xz,
                    const double* wavelet, const int* rec_xz, const double* resid,
                    double* grad_v, double* grad_wavelet, double* gathers);

/* Encoded shots (source encoding: nsrc sources in one simulation):
 * src_xz[nshots][nsrc][2], wavelet[nshots][nsrc][nt]; source k adds
 * (dt^2/h^2) wavelet[s][k][n] at its cell after step n, in the order k = 0 ..
 * nsrc-1. Gathers and grad_v as in orc_ac_forward / orc_ac_gradient. */
int orc_ac_forward_encoded(const orc_problem* pb, int nsrc, const double* v, const int* src_xz,
                           const double* wavelet, const int* rec_xz, double* gathers);
int orc_ac_gradient_encoded(const orc_problem* pb, int nsrc, const double* v, const int* src_xz,
                            const double* wavelet, const int* rec_xz, const double* resid,
                            double* grad_v);

/* Born / tangent-linear modelling (Eq. 16): dgathers = (d gathers / d v) . dv. */
int orc_ac_born(const orc_problem* pb, const double* v, const double* dv,
                const int* src_xz, const double* wavelet, const int* rec_xz,
                double* dgathers);

/* ---- elastic (Eq. 12) ---- */

/* model = [3][nz][nx] holding vp, vs, rho. Explosive source (added to both normal
 * stresses). gathers[nshots][nt][nrec][2] = (vx, vz) at the receiver nodes. */
int orc_el_forward(const orc_problem* pb, const double* model, const int* src_xz,
                   const double* wavelet, const int* rec_xz, double* gathers);

/* Single-shot snapshots of the five fields after each full step:
 * snaps[nt][5][NZ][NX] in the order vx, vz, txx, tzz, txz. */
int orc_el_wavefield(const orc_problem* pb, const double* model, const int* src_xz,
                     const double* wavelet, double* snaps);

/* grad[3][nz][nx] = dJ/d(vp, vs, rho); grad_wavelet / gathers optional. */
int orc_el_gradient(const orc_problem* pb, const double* model, const int* src_xz,
                    const double* wavelet, const int* rec_xz, const double* resid,
                    double* grad, double* grad_wavelet, double* gathers);

/* Tangent-linear elastic modelling with respect to (vp, vs, rho). */
int orc_el_born(const orc_problem* pb, const double* model, const double* dmodel,
                const int* src_xz, const double* wavelet, const int* rec_xz,
                double* dgathers);

/* ---- pseudo-acoustic VTI (Sec. 3.3.1, Eq. 5) ---- */

/* model = [3][nz][nx] holding vv (vertical P velocity), v (NMO velocity) and
 * eta >= 0 (anisotropy); free_surface must be 0. The pad replicates vv and v
 * from the edge cells and holds eta = 0. wavelet[nshots][nt]; gathers
 * [nshots][nt][nrec] = P^{n+1} at the receivers. The scheme (both fields by
 * leapfrog, F_xxzz = D2x D2z F) is written out in vti.cpp. */
int orc_vti_forward(const orc_problem* pb, const double* model, const int* src_xz,
                    const double* wavelet, const int* rec_xz, double* gathers);

/* grad[3][nz][nx] = dJ/d(vv, v, eta); grad_wavelet / gathers optional. */
int orc_vti_gradient(const orc_problem* pb, const double* model, const int* src_xz,
                     const double* wavelet, const int* rec_xz, const double* resid,
                     double* grad, double* grad_wavelet, double* gathers);

#ifdef __cplusplus
}
#endif
#endif
