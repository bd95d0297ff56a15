/*
 * lbe_csf.h -- C ABI of liblbe_csf.so: the fused time step of the continuous-
 * surface-force (CSF) lattice Boltzmann method for thermocapillary flow
 * (L. Zheng, S. Zheng, Q. Zhai, arXiv:1412.6238), for AMD MI355X (gfx950).
 *
 * One step advances three coupled D2Q9 lattices on an nx x ny grid:
 *   f     flow, with the CSF interface force        (Sec. II, Eqs. 6-9)
 *   g     Cahn-Hilliard order parameter c          (Sec. II, Eqs. 12-16)
 *   hbar  temperature                               (Sec. III, Eqs. 22-26)
 * coupled through the chemical potential mu = mu0(c) - eps^2 lap c, the
 * linear surface tension sigma(T) = sigma0 - sigmaT (T - Tref) (Eq. 5, with
 * sigmaT = -d sigma / dT) and the force
 *   F = kcap sigma mu grad c + eps alpha (|grad c|^2 grad sigma
 *       - (grad c . grad sigma) grad c) + rho a             (Eqs. 3-4),
 * whose capillary part may instead take the curvature form of Eq. 4
 * (csf_form = 1).  With two densities (rho2) rho = rho(c) and the density
 * terms of Eqs. 6 and 9 and Sec. III enter.
 *
 * Grid: sites (i, j), x = i + 1/2, y = j + 1/2, index j * nx + i (x fastest).
 * x is periodic.  With walls_y = 1 no-slip walls sit halfway, at y = 0 and
 * y = ny, with fixed wall temperatures (the paper's test problems, Sec. IV);
 * with walls_y = 0 y is periodic too.
 *
 * State contract: the library holds F_n, the post-streaming (pre-collision)
 * distributions at step n; one step is F_{n+1} = Stream(Collide(F_n)).
 * F_0 is the equilibrium of the initial fields (u = 0, p = p0).
 *
 * Memory: the library never allocates device memory.  The caller provides
 * one device workspace (size from lbe_csf_workspace_size) and every input and
 * output array; all are borrowed, none is freed by the library, and they must
 * stay valid while the handle uses them (the workspace for the handle's life,
 * inputs of lbe_csf_create only during that call).  All device work is
 * enqueued on the stream given at creation (a hipStream_t; NULL is the null
 * stream).  Calls that return host values synchronise that stream.
 *
 * Errors: every int-returning call returns LBE_CSF_OK (0) or a negative
 * lbe_csf_status; a message for the last failure is available from
 * lbe_csf_last_error.  No C++ exception crosses the ABI.  A handle is not
 * thread-safe: serialise calls on one handle.
 */
#ifndef LBE_CSF_H
#define LBE_CSF_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define LBE_CSF_API __attribute__((visibility("default")))
#else
#define LBE_CSF_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBE_CSF_OK = 0,
  LBE_CSF_EINVAL = -1,       /* invalid argument or parameter             */
  LBE_CSF_ENOMEM = -2,       /* workspace smaller than required           */
  LBE_CSF_EDEVICE = -3,      /* a HIP runtime error (see last_error)      */
  LBE_CSF_ENOTRECORDED = -4, /* backward without a recorded forward run   */
  LBE_CSF_ENONFINITE = -5    /* a diagnostic pass found NaN or Inf        */
} lbe_csf_status;

typedef enum {
  LBE_CSF_FP64 = 0,     /* distributions stored and evolved in FP64            */
  LBE_CSF_FP32_DEV = 1  /* FP32 deviations from the rest-weight equilibrium:
                           f - w p0, g, hbar - w rho cv T_ref(y) with the
                           linear reference T_ref = T_shift + T_grad y (g_0
                           in FP64; FP64 sums for the diagnostics)          */
} lbe_csf_precision;

/* Parameters (plain data; lattice units, dt = dx = 1, cs^2 = 1/3). */
typedef struct {
  int32_t nx, ny;        /* grid, each >= 3                                   */
  int32_t walls_y;       /* 1: halfway walls at y = 0, ny; 0: periodic y      */
  int32_t precision;     /* lbe_csf_precision                                 */
  double rho, cv;        /* uniform density and specific heat, > 0            */
  double tau_f[2];       /* flow relaxation time at c = 0 and c = 1, > 1/2;
                            viscosity eta = rho (tau_f - 1/2) / 3 (Sec. II)   */
  double tau_T[2];       /* thermal relaxation time tau_h + 1/2, > 1/2;
                            conductivity lambda = rho cv (tau_T - 1/2) / 3    */
  double tau_g;          /* Cahn-Hilliard relaxation time, > 1/2              */
  double mobility;       /* M = Gamma (tau_g - 1/2) (Eq. 16), > 0             */
  double width;          /* interface width W: the planar profile is
                            c = 1/2 + 1/2 tanh(z / W), so eps = W sqrt(beta/2) */
  double beta;           /* double-well coefficient, E0 = beta c^2 (1-c)^2    */
  double sigma0, sigmaT, Tref; /* sigma = sigma0 - sigmaT (T - Tref)           */
  double force[2];       /* body acceleration a (adds rho a to F)             */
  double p0;             /* pressure of the initial state                     */
  double T_shift;        /* FP32_DEV: the hbar deviations refer to the linear  */
  double T_grad;         /* temperature T_ref(y) = T_shift + T_grad y (a
                            background close to the expected field, such as
                            the conduction profile between the walls, keeps
                            the stored deviations and their rounding small);
                            must be 0 with walls_y = 0 (not periodic)        */
  int32_t diag_every;    /* > 0: diagnostics of every diag_every-th state
                            during lbe_csf_step (kept on the device, fetched
                            by lbe_csf_diag_history); 0: none               */
  int32_t csf_form;      /* capillary part of the CSF force (Eq. 4):
                            0: potential form kcap sigma mu grad c (exact on
                               the equilibrium profile);
                            1: curvature form -sigma (div n) n delta as
                               printed, with n = grad c/|grad c| and
                               delta = eps alpha |grad c|^2, evaluated as
                               -sigma eps alpha (t.H.t) grad c (t the unit
                               tangent, H the nine-point Hessian of c)      */
  double rho2;           /* density of the c = 1 fluid; rho above is that of
                            the c = 0 fluid.  0 (or rho2 == rho): one
                            density.  Two densities (both precisions; no
                            adjoint) make rho(c) = rho + c (rho2 - rho) and
                            bring in the density terms of Eq. 6, the
                            pressure p = sum f + (1/2) u.grad(rho cs^2) of
                            Eq. 9 (an extra pass per step and an FP64
                            plane of workspace) and F-bar of Sec. III.  The
                            FP32 form keeps its hbar deviations relative to
                            w rho cv (T_shift + T_grad y) with the rho of
                            the c = 0 fluid                               */
} lbe_csf_params;

/* Global diagnostics of a state F_n (FP64 sums; u_r of Sec. IV C). */
typedef struct {
  int64_t step;          /* n                                                 */
  double mass;           /* sum c                                             */
  double energy;         /* sum rho cv T                                      */
  double sum_cy;         /* sum c y                                           */
  double sum_cx;         /* sum c x (meaningful without x wrap-around)        */
  double mass_thr;       /* sum of c over sites with c >= 1/2                 */
  double sum_cuy_thr;    /* sum of c u_y over sites with c >= 1/2             */
  double centroid_y;     /* sum_cy / mass                                     */
  double u_r;            /* sum_cuy_thr / mass_thr (migration velocity)       */
  int64_t n_nonfinite;   /* sites where c, T, p or u is NaN or Inf            */
} lbe_csf_diag;

typedef struct lbe_csf lbe_csf; /* opaque host object */

/* Bytes of device workspace needed for these parameters.  record_steps > 0
 * reserves room for lbe_csf_backward after a recorded run of that many steps
 * (ceil(sqrt(N)) spaced checkpoints plus one segment of replay states).
 * Two densities add one FP64 plane of nx*ny (the pressure of Eq. 9).
 * Errors: EINVAL for invalid parameters or NULL bytes. */
LBE_CSF_API int lbe_csf_workspace_size(const lbe_csf_params *params, int64_t record_steps,
                           size_t *bytes);

/* Create a handle and write F_0 (the equilibrium of the initial fields).
 * workspace: device memory of at least workspace_size bytes, 256-byte aligned.
 * stream: hipStream_t the handle enqueues on.
 * phi0, T0: device FP64 arrays of nx*ny (phi = 2c - 1, c = 1 in fluid 2).
 * Twall_bot, Twall_top: device FP64 arrays of nx, the wall temperatures at
 * y = 0 and y = ny per column (copied into the workspace; ignored, may be
 * NULL, when walls_y = 0).  Record capacity for backward is the record_steps
 * the workspace was sized with (passed again here).
 * Errors: EINVAL (parameters, NULL pointers, misaligned workspace), ENOMEM
 * (workspace too small), EDEVICE. */
LBE_CSF_API int lbe_csf_create(const lbe_csf_params *params, void *workspace, size_t bytes,
                   int64_t record_steps, void *stream, const double *phi0,
                   const double *T0, const double *Twall_bot,
                   const double *Twall_top, lbe_csf **out);

/* Advance nsteps >= 0 steps.  record = 1 keeps ceil(sqrt(N)) checkpoints of
 * this run for lbe_csf_backward (the run must start at the handle's current
 * state and N = nsteps <= record_steps; the adjoint covers both force
 * forms with one density, so record = 1 is EINVAL with two densities);
 * record = 0 discards any record.  With two densities every
 * step is two launches: the pressure of Eq. 9, then the step.
 * With diag_every > 0 the diagnostics of F_n for every n divisible by
 * diag_every in [start, start + nsteps) are computed inside the step kernel
 * and this call synchronises once at its end to check them: ENONFINITE if any
 * state had a non-finite site.  Errors: EINVAL, EDEVICE, ENONFINITE. */
LBE_CSF_API int lbe_csf_step(lbe_csf *h, int64_t nsteps, int32_t record);

/* Macroscopic fields of the current state into caller device FP64 arrays of
 * nx*ny (any may be NULL): phi = 2c - 1, u (Eq. 9 with the force), p, T. */
LBE_CSF_API int lbe_csf_fields(lbe_csf *h, double *phi, double *ux, double *uy, double *p,
                   double *T);

/* Diagnostics of the current state (synchronises the stream). */
LBE_CSF_API int lbe_csf_diagnostics(lbe_csf *h, lbe_csf_diag *out);

/* The diagnostics of lbe_csf_diagnostics, computed without any device memory
 * beyond the handle's state: for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The per-block partial sums and the record live in a static device array
 * of the library (one per GPU, about 0.9 MB, held until the process ends):
 * at most 16384 blocks per diagnostic launch, else EINVAL with a message.
 * Calls on one GPU share that array: calls that overlap on one GPU (from
 * other threads or streams) race and must be serialised by the caller.
 * Makes the handle's device current for the call and restores the caller's.
 * Synchronises the stream.  Errors: EINVAL, EDEVICE. */
LBE_CSF_API int lbe_csf_diagnostics_noalloc(lbe_csf *h, lbe_csf_diag *out);

/* Copy up to max records taken during lbe_csf_step (oldest first, the device
 * keeps the last 4096) into host out; *count receives the number copied.
 * Clears the history.  Synchronises the stream. */
LBE_CSF_API int lbe_csf_diag_history(lbe_csf *h, lbe_csf_diag *out, int32_t max,
                         int32_t *count);

/* Copy the current state F_n to / from a caller device FP64 array laid out
 * [27][ny][nx]: f_0..8, g_0..8, hbar_0..8 with the D2Q9 order
 * (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
 * In FP32_DEV the values are converted (rounded to FP32 deviations on set).
 * set_state leaves the step counter unchanged and drops any record. */
LBE_CSF_API int lbe_csf_get_state(lbe_csf *h, double *F);
LBE_CSF_API int lbe_csf_set_state(lbe_csf *h, const double *F);

/* Number of steps taken since creation (host value, no synchronisation). */
LBE_CSF_API int64_t lbe_csf_step_count(const lbe_csf *h);

/* Gradient of J = sum_x c_N(x) dJdc(x) (for the centroid objective
 * dJdc = (y - J)/sum c) through the recorded run of N steps (Sec. II-III step
 * transposed), by reverse sweeps over checkpoint segments with recomputation.
 * dJ_dc: device FP64 nx*ny seed on c of the final state F_N.
 * dJ_dsigmaT: host FP64 scalar (output).
 * dJ_dTwall: device FP64 2*nx (output: bottom then top wall), through the wall
 *   rules and the temperature ghosts; may be NULL.
 * dJ_dF0: device FP64 [27][ny][nx] (output: the adjoint of F_0), may be NULL.
 * dJ_dT0: device FP64 nx*ny (output: the adjoint of the initial temperature
 *   field through the initial equilibrium), may be NULL.
 * Errors: ENOTRECORDED if the last lbe_csf_step was not recorded (or the state
 * changed since), EINVAL, EDEVICE. */
LBE_CSF_API int lbe_csf_backward(lbe_csf *h, const double *dJ_dc, double *dJ_dsigmaT,
                     double *dJ_dTwall, double *dJ_dF0, double *dJ_dT0);

/* Release the host object (device memory is the caller's). */
LBE_CSF_API void lbe_csf_destroy(lbe_csf *h);

LBE_CSF_API const char *lbe_csf_strerror(int status);
LBE_CSF_API const char *lbe_csf_last_error(const lbe_csf *h);

#ifdef __cplusplus
}
#endif
#endif /* LBE_CSF_H */
