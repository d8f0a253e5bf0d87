/*
 * osscir.h -- C ABI of the MI355X (gfx950) library for one-step spectral-CT
 * image reconstruction (OSSCIR) by MOCCA with diagonal or m-block-diagonal
 * step preconditioning (Sidky, Barber, Gilat-Schmidt, Pan, arXiv 1801.06263).
 *
 * Problem (Sec. II): given measured counts c_{w,l} in W energy windows along
 * rays l, normalised window responses s_{w,i}, incident counts N_w, material
 * attenuation mu_{m,i} and the scan geometry (which fixes the projection
 * X_{l,k}), recover material maps f_{k,m} by minimising
 * D_TPL(c, chat(f)) with the softexp counts model (Eq. finalModel).
 *
 * Conventions shared by every call
 *  - Image arrays are [n_ch][n][n] float32, x fastest; pixel (ix, iy) is
 *    centred at ((ix-(n-1)/2) h, (iy-(n-1)/2) h), h = pixel_cm.
 *  - Sinogram arrays are [n_ch][n_views][n_bins] float32, bin fastest; ray
 *    l = v*n_bins + d; L = n_views*n_bins.
 *  - Every data pointer argument is a DEVICE pointer owned by the caller
 *    (allocated on the device the plan was created on), unless documented
 *    "host".  The library allocates device memory only inside
 *    osscir_plan_create (its constant tables, ray geometry and a 32 (n+8)^2-byte
 *    image scratch used by osscir_forward_project), freed in
 *    osscir_plan_destroy, and inside the batch calls (osscir_batch_*: slot
 *    table, work lists, per-tile sums, the tuner's snapshot), freed in
 *    osscir_batch_destroy.  Apart from a batch's bound slots it keeps no
 *    pointer to caller memory after a call returns.
 *  - Calls that take a stream enqueue their work asynchronously on it (NULL =
 *    the null stream) and return without synchronising.  Only
 *    osscir_plan_create and osscir_plan_destroy synchronise.
 *  - Return codes: OSSCIR_OK (0), OSSCIR_EINVAL (-1: null pointer, bad size,
 *    unsupported material/window count), OSSCIR_EDEVICE (-2: a HIP call or
 *    launch failed), OSSCIR_ENOMEM (-3), OSSCIR_ESTATE (-4: workspace too
 *    small).  osscir_last_error() returns the calling thread's last message.
 *  - A plan may be used from one host thread and one stream at a time
 *    (osscir_forward_project uses the plan's scratch; the iteration calls use
 *    the caller's workspace); different plans are independent.  Results are deterministic: no floating-point atomics, fixed
 *    accumulation order.
 */
#ifndef OSSCIR_H
#define OSSCIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OSSCIR_OK 0
#define OSSCIR_EINVAL (-1)
#define OSSCIR_EDEVICE (-2)
#define OSSCIR_ENOMEM (-3)
#define OSSCIR_ESTATE (-4)

#define OSSCIR_PRECOND_DIAG 0   /* diagonal SPC (Pock-Chambolle), Sec. II "Step lengths" */
#define OSSCIR_PRECOND_BLOCK 1  /* m-block-diagonal SPC, Sec. II "A m-block diagonal SPC" */

#define OSSCIR_CURV_WINDOW 0    /* local quadratic curvature diag(c_l) */
#define OSSCIR_CURV_CLIP 1      /* per-ray Hessian with negative curvature removed */

typedef struct osscir_plan_s *osscir_plan;
typedef void *osscir_stream; /* a hipStream_t */

/* Fan-beam scan with a flat detector.  View v has source angle
 * beta_v = view0_rad + arc_rad * v / n_views, source at sid_cm (cos, sin),
 * detector centre at -(sdd_cm - sid_cm)(cos, sin), detector axis
 * (-sin, cos), bin d centred at (d - (n_bins-1)/2) * bin_cm.  The ray of
 * (v, d) joins the source to the bin centre; X_{l,k} is its chord length (cm)
 * inside pixel k.  Limits: 1 <= n <= 4096, 1 <= n_views, 1 <= n_bins,
 * n_views * n_bins < 2^31, 0 < pixel_cm, sid_cm > n*pixel_cm/sqrt(2),
 * sdd_cm > sid_cm. */
typedef struct {
  int32_t n;
  double pixel_cm;
  int32_t n_views, n_bins;
  double sid_cm, sdd_cm, bin_cm;
  double view0_rad, arc_rad;
} osscir_geometry;

/* Spectral tables of Eq. (fullModel), HOST pointers, copied at plan creation:
 * mu [n_mat][n_energy] (cm^-1 per unit material fraction) and n_resp sets of
 * window responses s [n_resp][n_win][n_energy] (each row >= 0 and summing
 * to 1) with incident photons per ray n0 [n_resp][n_win].  n_resp = 0 or 1:
 * one response shared by every ray; n_resp = n_bins: one per detector bin d
 * (the same in every view), the calibrated per-pixel spectra of Sec. III.
 * n0_ray (optional, NULL = none): incident photons of every ray and window,
 * [n_views][n_bins][n_win], the N_{w,l} of Eq. (fullModel) in full (for
 * instance a tube current that varies with the view); it replaces n0 for
 * every ray, with either kind of response.
 * Supported: n_mat = 3, n_win = 4, 1 <= n_energy <= 512. */
typedef struct {
  int32_t n_mat, n_win, n_energy;
  const double *mu;
  const double *s;
  const double *n0;
  int32_t n_resp;
  const double *n0_ray;
} osscir_spectral;

/* Step-size ratio lambda > 0 (Sec. II: "a step size ratio parameter that must
 * be tuned"), preconditioner and curvature choice, and whether the per-ray
 * tail (3x3 eigen-clip, 4x4 dual solve) runs in FP64 (fp64_small = 1) or FP32
 * (0; the 3x3 Gram inverse of the clipped-curvature dual step is FP64 in both,
 * which keeps the FP32 tail within 1e-3 of the FP64 oracle's maps).
 * Projection weights, line integrals and energy sums are FP32 in both cases;
 * back-projection sums over views and the per-pixel 3x3 solve are always
 * FP64 (the 3x3 step blocks are ill-conditioned). */
typedef struct {
  double lambda;
  int32_t precond;
  int32_t curvature;
  int32_t fp64_small;
} osscir_params;

/* Iteration state, all DEVICE pointers owned by the caller.
 *   f    [3][n][n]        f_n, updated in place to f_{n+1}
 *   fbar [3][n][n]        extrapolated point fbar_n (the expansion point),
 *                         updated in place to 2 f_{n+1} - f_n
 *   y    [4][V][D]        dual variable, updated in place
 *   c    [4][V][D]        measured counts (read only)
 *   work, work_bytes      scratch of at least osscir_workspace_bytes() */
typedef struct {
  float *f;
  float *fbar;
  float *y;
  const float *c;
  void *work;
  size_t work_bytes;
} osscir_state;

/* Build a plan: validates the inputs, allocates the device tables on the
 * current device, builds the per-ray line parameters in FP64 and stores them
 * as FP32, and computes rho_l = (X 1)_l with the library's own projector.
 * Synchronises.  *out is set to NULL on failure. */
int osscir_plan_create(const osscir_geometry *geom, const osscir_spectral *spec, osscir_plan *out);
int osscir_plan_destroy(osscir_plan plan);

/* How the spectral step of an iteration forms its per-ray energy sums (the
 * window sums, Jacobian rows and curvature sums over the energy bins of
 * Eq. finalModel and the Hessian of Sec. II): matrix_cores = 1 runs them as a
 * dense FP32 contraction of the response table with the softexp values of
 * 64 rays on the matrix cores (the default wherever it applies: one shared
 * response table within 64 KB of LDS, i.e. n_resp <= 1 and n_energy <= 336);
 * 0 sums them per ray with vector FMAs in energy order.  Both are FP32 and
 * meet the same bars against the FP64 oracle; their roundings differ.  Takes
 * effect for the plan's later calls and for batch slots bound afterwards.
 * EINVAL if matrix_cores = 1 where it does not apply. */
int osscir_plan_set_energy_sums(osscir_plan plan, int32_t matrix_cores);

/* Bytes of device scratch osscir_mocca_iterate, osscir_dtpl and the step
 * calls need (host out-parameter). */
int osscir_workspace_bytes(osscir_plan plan, size_t *bytes);

/* rho_l = sum_k X_{l,k} (cm), the chord of each ray through the image square:
 * copies the plan's [L] array into rho (device). */
int osscir_ray_lengths(osscir_plan plan, float *rho, osscir_stream stream);

/* Host only, no device work: the per-view sources and per-ray line
 * parameters a plan of this geometry evaluates X with (Sec. II, Eq. fullModel:
 * X_{l,k} is the chord of ray l in pixel k).  In pixel index coordinates
 * (pixel (ix, iy) centred at (ix, iy)) the chord is
 *   clamp(kappa a - |kappa n . (S_v - (ix, iy))|, 0, hmax)   (cm)
 * with n the ray's unit normal, a = (|n_x| + |n_y|) / 2, kappa =
 * pixel_cm / |n_x n_y| and hmax = pixel_cm / max(|n_x|, |n_y|).  A ray
 * within 2^-23 of an image axis (exactly parallel at views whose angle is a
 * multiple of pi/2) is turned about its source to that tilt, toward the +
 * side of its minor axis: a line lying exactly on a pixel edge is counted
 * once, in the pixel on its + side.
 * Outputs (HOST): rays [L][6] = kappa n_x, kappa n_y (the FP64 values the
 * kernels use), kappa a, hmax, kappa (their FP32 values), 0; src [n_views][2]
 * = the source (FP64).  EINVAL on a geometry osscir_plan_create rejects. */
int osscir_ray_table(const osscir_geometry *geom, double *rays, double *src);

/* Forward projection p_{c,l} = sum_k X_{l,k} f_{c,k} (Eq. fullModel's
 * X f) of n_ch >= 1 channels: f [n_ch][n][n] -> p [n_ch][V][D].  Ray-driven;
 * p is fully overwritten. */
int osscir_forward_project(osscir_plan plan, const float *f, int32_t n_ch, float *p, osscir_stream stream);

/* Back-projection b_{c,k} = sum_l X_{l,k} q_{c,l}, the exact transpose of
 * osscir_forward_project (the same FP32 weight for every (ray, pixel) pair):
 * q [n_ch][V][D] -> b [n_ch][n][n], fully overwritten; deterministic
 * pixel-driven gather in fixed view order. */
int osscir_back_project(osscir_plan plan, const float *q, int32_t n_ch, float *b, osscir_stream stream);

/* Per-ray spectral model at material line integrals p [3][V][D] with counts
 * c [4][V][D] (Sec. II): chat_{w,l} = N_w sum_i s_{w,i} softexp(-z_{l,i}),
 * z = sum_m mu_{m,i} p_{m,l}; r = c - chat; G_l[w][m] = sum_i A_{wl,li} mu_{m,i}
 * (so that K_{wl,mk} = G_l[w][m] X_{l,k}); H_l the p-space Hessian
 * -mu diag(B^T r) mu^T + G^T diag(chat + r) G; and H_l^+ (negative
 * eigenvalues set to zero).  Outputs (device, each may be NULL to skip):
 * chat, r [4][L]; G [12][L] (index w*3+m); H, Hplus [6][L] (upper triangle
 * 00,01,02,11,12,22).  fp64_small selects the precision of the eigen-clip. */
int osscir_spectral_model(osscir_plan plan, const float *p, const float *c, float *chat, float *r, float *G,
                          float *H, float *Hplus, int32_t fp64_small, osscir_stream stream);

/* Block-diagonal SPC step lengths at G [12][L] (Sec. II):
 *   sigma_{w,l} = 1 / (lambda sum_k sqrt(sum_m K^2)) = 1 / (lambda rho_l |G_l[w]|),
 *   (T^-1)_k    = (1/lambda) sum_{w,l} K_{.,mk} K_{.,m'k} / |K_{.,k}|
 *               = (1/lambda) sum_l X_{l,k} S_l,  S_l = sum_w G_l[w]^T G_l[w] / |G_l[w]|.
 * Outputs: sigma [4][L] (0 for rays with rho_l = 0), tinv [6][n][n] (upper
 * triangle of each 3x3 block).  Needs work. */
int osscir_block_spc_steps(osscir_plan plan, const float *G, double lambda, float *sigma, float *tinv,
                           void *work, size_t work_bytes, osscir_stream stream);

/* Diagonal SPC step lengths (Sec. II):
 *   sigma_{w,l} = (1/lambda) / sum_{mk} |K| = 1 / (lambda rho_l sum_m |G_l[w][m]|),
 *   T_{mk}      = lambda / sum_{wl} |K|    = lambda / sum_l X_{l,k} sum_w |G_l[w][m]|.
 * Outputs sigma [4][L], tau [3][n][n].  Needs work. */
int osscir_diag_spc_steps(osscir_plan plan, const float *G, double lambda, float *sigma, float *tau, void *work,
                          size_t work_bytes, osscir_stream stream);

/* n_iter MOCCA iterations (CPPD steps on the local convex quadratic with
 * expansion point fbar_n, one inner iteration per expansion point):
 *   y_{n+1}    = prox_{Sigma Q*}(y_n + Sigma K fbar_n) = y_n + Sigma (Sigma + D_l)^-1 (r_l - y_n)
 *   f_{n+1}    = f_n - T K^T y_{n+1}
 *   fbar_{n+1} = 2 f_{n+1} - f_n
 * with K, Sigma, T, r, D_l evaluated at fbar_n.  Rays with rho_l = 0 are
 * masked (y = 0).  If dtpl is not NULL it is a DEVICE array of n_iter doubles
 * receiving D_TPL(c, chat(f_{n+1})) after each iteration (an extra forward
 * projection per iteration).  Two to three kernel launches per iteration,
 * no host synchronisation. */
int osscir_mocca_iterate(osscir_plan plan, const osscir_params *params, osscir_state *state, int32_t n_iter,
                         double *dtpl, osscir_stream stream);

/* MOCCA with nested loops (Sec. III: with a single inner iteration per
 * expansion point MOCCA can diverge; nested inner and outer loops are the
 * remedy the paper sets aside for speed).
 * n_outer expansion points, each f0 = fbar at the start of its outer
 * iteration; n_inner CPPD steps on the fixed convex quadratic Q(K(f0) f),
 * with K, Sigma, T, r, D_l and u0 = K(f0) f0 all formed at f0:
 *   y_{j+1}    = prox_{Sigma Q*}(y_j + Sigma K(f0) fbar_j)
 *              = y_j + Sigma (Sigma + D_l)^-1 (r_l + D_l K(f0) (fbar_j - f0) - y_j)
 *   f_{j+1}    = f_j - T K(f0)^T y_{j+1},   fbar_{j+1} = 2 f_{j+1} - f_j.
 * The first inner step of every outer iteration is the osscir_mocca_iterate
 * step, so n_inner = 1 gives osscir_mocca_iterate's results bit for bit.
 * p0: DEVICE [3][V][D] floats, caller-owned scratch; on return it holds
 * X f0 of the last expansion point.  dtpl as in osscir_mocca_iterate, with
 * n_outer * n_inner entries (one per inner step).  EINVAL if n_outer < 0,
 * n_inner < 1, n_outer * n_inner overflows int32, or p0 is NULL. */
int osscir_mocca_iterate_nested(osscir_plan plan, const osscir_params *params, osscir_state *state,
                                int32_t n_outer, int32_t n_inner, float *p0, double *dtpl, osscir_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): exactly
 * osscir_mocca_iterate (same kernels, same results bit for bit) on the state
 * buffers f, fbar, y (updated in place) and c, with the workspace taken
 * from a static device array of 64 MiB that the library holds on every
 * device it runs on until the process ends (enough for the 512^2,
 * 720 x 1024 scan, which needs 50.5 MiB).  Calls no allocating routine.
 * EINVAL if the plan's workspace (osscir_workspace_bytes) exceeds 64 MiB.
 * Every call on one device shares that device's array and leaves the last
 * call's contents in it (each call writes all it reads first): calls that
 * overlap on one device race, so issue them on one stream, or order them. */
int osscir_mocca_iterate_noalloc(osscir_plan plan, const osscir_params *params, float *f, float *fbar, float *y,
                                 const float *c, int32_t n_iter, double *dtpl, osscir_stream stream);

/* One stage of a MOCCA iteration, exactly as osscir_mocca_iterate runs it:
 *   stage 0  forward projection p = X fbar into the workspace
 *   stage 1  spectral model, step lengths and dual step (reads p, updates y)
 *   stage 2  back-projection fused with the primal step (updates f, fbar)
 * Running stages 0, 1, 2 in order equals one call of osscir_mocca_iterate
 * with n_iter = 1 and dtpl = NULL.  For callers that time or interleave the
 * stages. */
int osscir_mocca_stage(osscir_plan plan, const osscir_params *params, osscir_state *state, int32_t stage,
                       osscir_stream stream);

/* nnz[l] = number of pixels with X_{l,k} > 0 (the FP32 weights the library
 * uses), int32 DEVICE array [V][D]. */
int osscir_ray_nnz(osscir_plan plan, int32_t *nnz, osscir_stream stream);

/* D_TPL(c, chat(f)) of Eq. (DTPL) at maps f [3][n][n], accumulated in FP64
 * in a fixed order, written to the DEVICE double *out.  Needs work. */
int osscir_dtpl(osscir_plan plan, const float *f, const float *c, double *out, void *work, size_t work_bytes,
                osscir_stream stream);

/* mu-preconditioning (Sec. I; Sec. II "Step lengths"): MOCCA with diagonal
 * SPC in a material basis that is orthonormal in energy.  The paper defers
 * the transform to its Ref. Barber2016b; this library reads it as
 * Gram-Schmidt of the attenuation rows mu_m(E_i), in material order, under
 * the inner product <u, v> = sum_i w_i u_i v_i, w_i = (1/n_win) sum_w s_{w,i}.
 * Outputs (HOST arrays): B [3][3] row-major, lower triangular, and
 * mu_out [3][n_energy] = B mu with <mu_out_j, mu_out_k> = delta_jk.  A plan
 * built with mu_out in place of mu and run with OSSCIR_PRECOND_DIAG iterates
 * the coefficients g of the new basis; the maps are f = B^T g (and
 * g = B^-T f), applied with osscir_material_transform.  EINVAL if the rows
 * are dependent under the weights or the responses are per detector bin
 * (n_resp > 1).  Host only, no device work. */
int osscir_mu_pc_basis(const osscir_spectral *spec, double *B, double *mu_out);

/* out[j][k] = sum_m M[j][m] in[m][k] for 3-channel maps of n_pixels pixels
 * (DEVICE in, out, FP32; M a HOST 3x3 row-major matrix applied in FP64; in
 * place allowed): the change of material basis of mu-preconditioning. */
int osscir_material_transform(const double *M, const float *in, float *out, int32_t n_pixels,
                              osscir_stream stream);

/* ------------------------------------------------------------------------
 * Batched iterations: many independent scans ("slots", each with its own
 * plan, state and lambda) advanced together, one launch per stage for the
 * whole batch (forward projection, spectral model + dual step,
 * back-projection + primal step, end-of-iteration bookkeeping).  Each slot
 * follows exactly the trajectory osscir_mocca_iterate gives its scan alone
 * (bit for bit, whatever the other slots and the launch configuration); its
 * iteration is the one of Sec. II, unchanged.
 *
 * A slot stops by itself once it has run max_iter iterations (if > 0) or
 * once the relative change ||f_{n+1} - f_n||_2 / ||f_{n+1}||_2 (FP64, over
 * the three maps) is <= tol (if > 0); a stopped slot keeps its last iterate
 * and costs nothing further.  A slot whose maps stop being finite (a NaN or
 * an infinity in f, from non-finite inputs or a diverging step) stops after
 * that iteration with OSSCIR_SLOT_FAILED, the other slots unaffected.  A batch is used from one host thread, with one
 * stream for all its calls.  Batch calls synchronise where stated.
 * ------------------------------------------------------------------------ */
typedef struct osscir_batch_s *osscir_batch;

#define OSSCIR_SLOT_EMPTY 0
#define OSSCIR_SLOT_RUNNING 1
#define OSSCIR_SLOT_DONE 2
#define OSSCIR_SLOT_FAILED 3

typedef struct {
  int32_t state;      /* OSSCIR_SLOT_* */
  int32_t iters;      /* iterations run since the slot was bound */
  double rel_change;  /* relative change of f in the last iteration */
} osscir_slot_status;

/* Launch configuration of the batched kernels (results do not depend on it):
 * rays per workgroup of the forward and spectral kernels (64, 128 or 256),
 * workgroups of each kernel (a multiple of 8, 8..65536; each workgroup walks
 * its XCD's share of the work list), and whether work is split over the 8
 * XCDs in contiguous cost-balanced ranges (1) or dealt round-robin (0). */
typedef struct {
  int32_t fp_rays, fp_wgs, fp_xcd;
  int32_t spec_rays, spec_wgs, spec_xcd;
  int32_t bp_wgs, bp_xcd;
} osscir_batch_config;

/* Create a batch of up to max_slots (1..256) slots on the current device.
 * modes supplies precond, curvature and fp64_small for every slot (its lambda
 * is ignored).  *out is NULL on failure. */
int osscir_batch_create(const osscir_params *modes, int32_t max_slots, osscir_batch *out);
/* Synchronises the device and frees the batch (not the plans or states). */
int osscir_batch_destroy(osscir_batch batch);

/* Bytes of device scratch a batch slot of this plan needs (host
 * out-parameter): the iteration workspace without the region where the
 * single-scan back-projection of a scan with few 16 x 16 tiles leaves its
 * per-part sums (the batched kernels form the same sums in registers), so at
 * most osscir_workspace_bytes. */
int osscir_batch_workspace_bytes(osscir_plan plan, size_t *bytes);

/* Bind scan `plan` with caller state `state` (as for osscir_mocca_iterate,
 * with work_bytes >= osscir_batch_workspace_bytes; its buffers must stay
 * allocated until the slot is cleared or rebound) and
 * step ratio lambda to slot `slot`, replacing what was bound there, with the
 * stopping rule (max_iter, tol).  Enqueues the packing of state->fbar on
 * stream; the slot starts running with the next osscir_batch_iterate.  The
 * plan must outlive the binding. */
int osscir_batch_set_slot(osscir_batch batch, int32_t slot, osscir_plan plan, const osscir_state *state,
                          double lambda, int32_t max_iter, double tol, osscir_stream stream);
/* osscir_batch_set_slot for MOCCA with nested loops (as
 * osscir_mocca_iterate_nested): n_inner steps per expansion point, the
 * expansion point re-taken at fbar every n_inner steps counted from binding;
 * iters, max_iter and the relative change count inner steps.  p0: DEVICE
 * [3][V][D] floats of caller memory that the slot uses while bound
 * (X f0 of its current expansion point); ignored when n_inner = 1, which is
 * osscir_batch_set_slot.  A slot computes bit for bit what
 * osscir_mocca_iterate_nested computes for its scan.  EINVAL if n_inner < 1
 * or (n_inner > 1 and p0 is NULL). */
int osscir_batch_set_slot_nested(osscir_batch batch, int32_t slot, osscir_plan plan, const osscir_state *state,
                                 double lambda, int32_t max_iter, double tol, int32_t n_inner, float *p0,
                                 osscir_stream stream);
/* Unbind a slot (state becomes OSSCIR_SLOT_EMPTY). */
int osscir_batch_clear_slot(osscir_batch batch, int32_t slot);

/* n_iter batched iterations of every running slot.  use_graph = 1 replays a
 * captured HIP graph of one iteration (captured on first use and again after
 * the work lists outgrow their buffers or the configuration changes);
 * 0 launches the kernels directly.  Asynchronous, except that it may wait for
 * its own earlier uploads before refilling the host staging buffers. */
int osscir_batch_iterate(osscir_batch batch, int32_t n_iter, int32_t use_graph, osscir_stream stream);

/* Status of every slot into the HOST array out[max_slots].  Synchronises the
 * stream. */
int osscir_batch_status(osscir_batch batch, osscir_slot_status *out, osscir_stream stream);

int osscir_batch_get_config(osscir_batch batch, osscir_batch_config *cfg);
int osscir_batch_set_config(osscir_batch batch, const osscir_batch_config *cfg);

/* Autotuner: times candidate configurations of each stage on the bound
 * slots (iters_per_trial timed iterations after one warm-up per candidate),
 * keeps the fastest per stage, and restores every slot's f, fbar, y and
 * status afterwards, so tuning leaves the trajectories unchanged.
 * Synchronises.  The chosen configuration is returned in *cfg (may be
 * NULL). */
int osscir_batch_tune(osscir_batch batch, int32_t iters_per_trial, osscir_batch_config *cfg, osscir_stream stream);

/* Thread-local description of the last error ("" if none). */
const char *osscir_last_error(void);

/* Library version string. */
const char *osscir_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OSSCIR_H */
