/*
 * gpair.h -- C ABI of the GPAIR direct-evaluation operators on MI355X (gfx950).
 *
 * GPAIR (Gaussian-kernel-based ultrafast 3D photoacoustic iterative
 * reconstruction, arXiv 2602.03893) represents the initial pressure as a sum of
 * isotropic Gaussian kernels (Methods, "Gaussian-kernel-based distribution for
 * the continuous source discretization", first two equations) and models the
 * pressure each kernel produces at a point detector in closed form, Eq.
 * (single_forward): p = A/(2r) * d * exp(-d^2/(2 sigma^2)), d = r - v t, kept
 * only inside the window |d| <= n_sigma * sigma (the "3 sigma principle" stated
 * right after that equation).  This library evaluates that sum directly for
 * every kernel, sensor and in-window sample (the "straightforward approach" the
 * paper describes at the start of the "Adaptive supersampling alignment"
 * subsection), with a per-kernel width sigma_k, and its exact transpose.
 *
 * Conventions shared by every entry point
 *  - Units are SI: metres, seconds, metres per second.
 *  - "device" pointers are HIP device memory owned by the caller (for instance
 *    torch tensors); "host" pointers are ordinary host memory owned by the
 *    caller.  The library never allocates or frees device memory: the caller
 *    supplies every device buffer, workspaces included.
 *  - Traces are float32, row-major [n_sensors][n_samples] (time contiguous).
 *    Sample n of every sensor is taken at time t0 + n*dt.
 *  - Kernel arrays (A, sigma, gA, gsigma) are float32 [n_kernels] in the
 *    caller's kernel order (the order of cx/cy/cz at plan creation).
 *  - Work is enqueued on the given HIP stream (NULL = the legacy default
 *    stream).  Calls return once the work is enqueued; device faults surface at
 *    the caller's next synchronisation.  Arguments are validated on the host
 *    before anything is launched: on a negative status nothing was launched and
 *    no output was touched.  No C++ exception crosses this boundary.
 *  - A plan is immutable after creation, but its workspace holds per-call
 *    scratch (per-kernel coefficient records): calls that use one plan must be
 *    ordered on one stream; concurrent calls on one plan race.
 *  - Outputs are overwritten, never accumulated into.
 */
#ifndef GPAIR_H
#define GPAIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPAIR_ABI_VERSION 2

/* Identical to hipStream_t. */
typedef struct ihipStream_t *gpair_stream;

typedef enum gpair_status {
  GPAIR_OK = 0,
  GPAIR_NOT_CONVERGED = 1,     /* solver: iteration cap reached before tol  */
  GPAIR_ERR_INVALID_ARG = -1,  /* null pointer, bad size, bad scalar        */
  GPAIR_ERR_NEAR_FIELD = -2,   /* a kernel lies closer than 10*sigma_max to
                                  a sensor: the dropped incoming-wave term
                                  of the two-term pressure is not negligible */
  GPAIR_ERR_NONFINITE = -3,    /* NaN/Inf met (geometry, or solver state)   */
  GPAIR_ERR_HIP = -4,          /* a HIP runtime call or launch failed        */
  GPAIR_ERR_WORKSPACE = -5,    /* workspace null, too small or misaligned    */
  GPAIR_ERR_SIGMA_RANGE = -6   /* a sigma_k outside (0, sigma_max] was seen  */
} gpair_status;

/* Human-readable name of a status; never NULL. */
const char *gpair_status_string(gpair_status st);

/* GPAIR_ABI_VERSION of the built library. */
int gpair_abi_version(void);

/* ------------------------------------------------------------------------ */
/* a0. Plan: geometry, spatial tiling, workspace                              */
/* ------------------------------------------------------------------------ */

/*
 * Acquisition geometry and operator constants.
 *  cx, cy, cz   host float32 [n_kernels]: kernel centres c_k (the voxel
 *               centres r_i of the source model).  Any point cloud is allowed;
 *               a regular grid tiles best.
 *  sensors      host float32 [n_sensors][3]: point-detector positions s_j.
 *  n_samples    samples per trace N_t; sample n is at t0 + n*dt.
 *  dt, t0       sampling interval (> 0) and time of sample 0.  Kept in double
 *               because r - v t must be resolved to ~1e-11 m at r ~ 4e-2 m.
 *  c_sound      speed of sound v (> 0).
 *  n_sigma      window half-width in units of sigma (> 0; 3 in the paper).
 *  sigma_max    upper bound of every sigma_k passed later (> 0).  It sizes
 *               the per-tile time segments; a larger sigma_k is an error.
 *  fwd_tile     most kernels per forward workgroup, 0 = automatic, else a
 *               power of two in [64, 8192].
 *  adj_tile     most kernels per adjoint workgroup, 0 = automatic (256),
 *               else 64, 128 or 256.
 *  fwd_waves    waves per forward workgroup (they split a tile's kernels and
 *               share one trace segment), 0 = automatic (4), else 1, 2, 4
 *               or 8.
 */
typedef struct gpair_geometry {
  int64_t n_kernels;
  const float *cx;
  const float *cy;
  const float *cz;
  int32_t n_sensors;
  const float *sensors;
  int32_t n_samples;
  double dt;
  double t0;
  double c_sound;
  double n_sigma;
  double sigma_max;
  int32_t fwd_tile;
  int32_t adj_tile;
  int32_t fwd_waves;
  int32_t deterministic;  /* != 0: bitwise reproducible forward (gpair_forward, gpair_forward_aniso) */
} gpair_geometry;

typedef struct gpair_plan_s *gpair_plan;

/* Read-only description of a plan (for tests, tuning and reports). */
typedef struct gpair_plan_info {
  int64_t n_kernels;
  int32_t n_sensors;
  int32_t n_samples;
  int32_t fwd_tile;          /* kernels per forward workgroup              */
  int32_t adj_tile;          /* kernels per adjoint workgroup              */
  int32_t fwd_waves;         /* waves per forward workgroup                */
  int64_t fwd_tiles;         /* number of forward tiles                    */
  int64_t adj_tiles;         /* number of adjoint tiles                    */
  int32_t fwd_segment;       /* samples in a forward LDS trace segment     */
  int32_t adj_segment;       /* samples in an adjoint LDS residual segment */
  int32_t max_taps;          /* taps per pair at sigma_max                 */
  double max_tile_radius;    /* largest tile bounding radius (m)           */
  double min_distance;       /* lower bound of the kernel-sensor distances */
  size_t workspace_bytes;
} gpair_plan_info;

/*
 * Validate g and tile the kernels into compact spatial tiles (aligned blocks
 * of the kernel lattice in Morton order; quantised positions for a point
 * cloud).  Host-only: g and its host arrays are read during the call and not
 * retained.  The plan must then be bound to a device workspace
 * (gpair_plan_bind_workspace) before any operator call.
 * Errors: INVALID_ARG, NONFINITE (geometry), NEAR_FIELD.  On error *out is
 * set to NULL.
 */
gpair_status gpair_plan_create(const gpair_geometry *g, gpair_plan *out);

/* Bytes of device workspace the plan needs.  Errors: INVALID_ARG. */
gpair_status gpair_plan_workspace_size(gpair_plan p, size_t *bytes);

/*
 * Upload the plan's tables (float64 sensors and centres, tile bounding
 * spheres, kernel permutation) into the caller's device workspace
 * (>= gpair_plan_workspace_size bytes, 256-byte aligned).  The workspace must
 * outlive every later call on the plan and must not be shared with another
 * plan.  Synchronous with respect to `stream`.  May be called again to move
 * the plan to another workspace.  Errors: INVALID_ARG, WORKSPACE, HIP.
 */
gpair_status gpair_plan_bind_workspace(gpair_plan p, void *workspace,
                                       size_t workspace_bytes,
                                       gpair_stream stream);

/* Release the host-side plan object (the workspace stays the caller's). */
void gpair_plan_destroy(gpair_plan p);

/* Fill *info.  Errors: INVALID_ARG. */
gpair_status gpair_plan_get_info(gpair_plan p, gpair_plan_info *info);

/*
 * The binning invariant the operators rely on (no LDS index is clamped): for
 * a tile with bounding sphere (c_t, rho_t) and a sensor s, the segment starts
 * at sample nb = floor((|s - c_t| - rho_t)/(v dt) - t0/dt - h_max) - 1, and
 * every member's window, with the up to two masked padding taps of the
 * unrolled tap loops, lies in slots [0, segment) of it.  gpair_plan_create
 * proves this per (tile, sensor) from the sphere bounds and refuses the
 * geometry (INVALID_ARG) if the margins do not hold.  This host-only call
 * checks it pair by pair instead, for every member of every forward
 * (which = 0) or adjoint (which = 1) tile and every sensor, at the widest
 * admitted window: *min_first = the smallest first-tap slot (>= 0 when the
 * invariant holds) and *max_last = the largest slot touched (<= the
 * segment length - 1).  Cost O(n_kernels * n_sensors) on the host threads.
 * Errors: INVALID_ARG.
 */
gpair_status gpair_plan_tiling_slots(gpair_plan p, int32_t which, int64_t *min_first,
                                     int64_t *max_last);

/*
 * The float32 window filter of the direct operators (see gpair_forward):
 * *float64_blocks = the number of adjoint tiles whose pairs are all decided
 * in float64 because a sensor is too close for the filter's error bound
 * (within 4 tile radii, or a radius too large for the guard), and
 * *max_steps = the most fixed-point steps any other tile runs for its
 * distance offsets.  Host-only.  Errors: INVALID_ARG.
 */
gpair_status gpair_plan_filter_stats(gpair_plan p, int64_t *float64_blocks, int32_t *max_steps);

/* ------------------------------------------------------------------------ */
/* a1 + a2. Forward operator                                                  */
/* ------------------------------------------------------------------------ */

/*
 * y = A(x): for every sensor j and sample n,
 *   y_j[n] = sum_k [ |d| <= n_sigma*sigma_k ] * A_k/(2 r_jk) * d
 *            * exp(-d^2 / (2 sigma_k^2)),   d = r_jk - v (t0 + n dt),
 * i.e. Eq. (single_forward) summed over the kernels by linearity of the wave
 * equation, with the window of the "3 sigma principle" (inclusive) and
 * samples outside [0, n_samples) dropped.  Window membership is the float64
 * decision (a float32 filter with a guard, and float64 for the pairs within
 * the guard of a window edge); taps are evaluated in float32.  The
 * partial sum of each group of nearby kernels (a tile) at a sensor is carried
 * in 32-bit fixed point whose unit is 2^-30 of a bound on that sum
 * (sum_k |A_k| sigma_max e^{-1/2} / (2 r_min)), then added to y in float32
 * (float atomics: the last bits of y depend on the order of the tiles).  With
 * the plan's `deterministic` set, each tile sum is instead rounded to a
 * global 64-bit fixed-point unit (2^-62 of a bound on every sample) and added
 * with integer atomics, so y is bitwise reproducible run to run.
 *  A      device float32 [n_kernels]  amplitudes A_k (any sign).
 *  sigma  device float32 [n_kernels]  widths sigma_k in (0, sigma_max].
 *  y      device float32 [n_sensors][n_samples], overwritten.
 * A sigma_k outside (0, sigma_max] is clamped into range for that kernel and
 * counted (see gpair_sigma_violations); the call still returns GPAIR_OK.
 * Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_forward(gpair_plan p, const float *A, const float *sigma,
                           float *y, gpair_stream stream);

/* ------------------------------------------------------------------------ */
/* a3. Adjoint operator (gradient with respect to A and sigma)                */
/* ------------------------------------------------------------------------ */

/*
 * The exact transpose of gpair_forward (the transposition principle of the
 * "Adjoint Operator" subsection, applied to the direct sum) and the
 * sigma-derivative of Eq. (single_forward):
 *   gA_k     = sum_j sum_{n in W_jk} delta_j[n] * d * e / (2 r_jk)
 *   gsigma_k = sum_j sum_{n in W_jk} delta_j[n] * A_k * d^3 * e
 *                                    / (2 r_jk sigma_k^3)
 * with e = exp(-d^2/(2 sigma_k^2)) and W_jk the same window as the forward.
 * For a loss L(y) with dL/dy = delta these are dL/dA_k and dL/dsigma_k (the
 * window indicator is locally constant in sigma, so it has no derivative).
 *  A       device float32 [n_kernels]; read only when gsigma != NULL (may
 *          then be NULL otherwise).
 *  sigma   device float32 [n_kernels].
 *  delta   device float32 [n_sensors][n_samples].
 *  gA      device float32 [n_kernels], overwritten.
 *  gsigma  device float32 [n_kernels], overwritten, or NULL to skip.
 * Sums over sensors are carried in float64.  Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_adjoint(gpair_plan p, const float *A, const float *sigma,
                           const float *delta, float *gA, float *gsigma,
                           gpair_stream stream);

/*
 * gpair_adjoint plus the gradient with respect to the kernel centres
 * (learnable centres, named as future work in the paper's Discussion): the
 * derivative of Eq. (single_forward) through r = |s_j - c_k| at fixed window
 * membership,
 *   gc_k = sum_j (c_k - s_j)/r * sum_{n in W} delta_j[n] A_k e/(2r)
 *          (1 - d^2/sigma_k^2 - d/r),
 * the same a.e. derivative as the sigma-gradient.  The plan's geometry (its
 * tiling and tile spheres) stays that of plan creation: centres that move
 * are taken up by creating a plan with the new centres.
 *  A        device float32 [n_kernels] (required).
 *  gcentres device float32 [n_kernels][3] (x, y, z), overwritten.
 *  gA, gsigma as gpair_adjoint (gsigma may be NULL).
 * Sums over sensors are carried in float64.  Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_adjoint_centres(gpair_plan p, const float *A, const float *sigma,
                                   const float *delta, float *gA, float *gsigma,
                                   float *gcentres, gpair_stream stream);

/*
 * The same operators in two steps, for callers that apply the forward and
 * the adjoint to the same (A, sigma), as one iteration of Algorithm 2 does:
 * gpair_prepare builds the per-kernel coefficients from (A, sigma) (A may be
 * NULL: zero amplitudes), and the _prepared calls use the coefficients of the
 * last direct-operator call that built them on this plan (gpair_prepare,
 * gpair_forward, gpair_adjoint, gpair_adjoint_centres).  A gsigma request
 * needs coefficients built with A.  An ASSA call on the plan overwrites the
 * coefficients: a _prepared call after it, or before any build, returns
 * INVALID_ARG.  Same results, bit for bit, as gpair_forward / gpair_adjoint.
 * Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_prepare(gpair_plan p, const float *A, const float *sigma,
                           gpair_stream stream);
gpair_status gpair_forward_prepared(gpair_plan p, float *y, gpair_stream stream);
gpair_status gpair_adjoint_prepared(gpair_plan p, const float *delta, float *gA,
                                    float *gsigma, gpair_stream stream);

/*
 * Anisotropic kernels (learnable anisotropic Gaussians, the other half of the
 * future work named in the paper's Discussion).  Kernel k has initial
 * pressure A_k exp(-(x - c_k)^T Sigma_k^-1 (x - c_k) / 2) with a symmetric
 * positive definite covariance Sigma_k.  Far-field reading: the detector's
 * sphere is flat across the kernel (the step that keeps only the outgoing
 * term of Eq. (single_forward)), so Eq. (pa_wave) integrates the kernel's
 * marginal along n = (s_j - c_k)/r and gives
 *   p = A_k sqrt(det Sigma_k)/sigma_n^3 * d/(2r) * exp(-d^2/(2 sigma_n^2)),
 *   sigma_n^2 = n^T Sigma_k n, d = r - v t, inside |d| <= n_sigma sigma_n,
 * which is Eq. (single_forward) exactly when Sigma_k = sigma^2 I; its
 * relative error against the full sphere integral falls like sigma/r (about
 * 2e-3 at 40 mm for axes up to 0.1 mm).
 *  A       device float32 [n_kernels] (gpair_adjoint_aniso reads it only when
 *          gsigma6 != NULL; it may then be NULL otherwise).
 *  sigma6  device float32 [6][n_kernels] (structure of arrays): the entries
 *          xx, yy, zz, xy, xz, yz of Sigma_k in m^2.  A covariance that is not
 *          positive definite or whose largest eigenvalue exceeds sigma_max^2
 *          is replaced by sigma_max^2 I for that kernel and counted (see
 *          gpair_sigma_violations); the call still returns GPAIR_OK.
 *  y       device float32 [n_sensors][n_samples], overwritten (forward; with
 *          the plan's `deterministic` option the tile sums go through the same
 *          64-bit integer flush as gpair_forward's, so y is bitwise
 *          reproducible).
 *  delta   device float32 [n_sensors][n_samples] (adjoint).
 *  gA      device float32 [n_kernels], overwritten: the transpose of the
 *          forward applied to delta.
 *  gsigma6 device float32 [6][n_kernels], overwritten, or NULL to skip: the
 *          gradient of <forward, delta> with respect to the six parameters at
 *          fixed windows, dp/dSigma = p [Sigma^-1/2 + (d^2/(2 sigma_n^4) -
 *          3/(2 sigma_n^2)) n n^T], an off-diagonal parameter carrying both
 *          symmetric entries (twice the matrix entry).
 * Each pair's window is decided in float64; sums over sensors are carried in
 * float64.  These calls overwrite the direct operators' per-kernel
 * coefficients (a _prepared call after them returns INVALID_ARG).
 * Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_forward_aniso(gpair_plan p, const float *A, const float *sigma6, float *y,
                                 gpair_stream stream);
gpair_status gpair_adjoint_aniso(gpair_plan p, const float *A, const float *sigma6,
                                 const float *delta, float *gA, float *gsigma6,
                                 gpair_stream stream);

/*
 * gpair_adjoint_aniso plus the gradient with respect to the kernel centres at
 * fixed windows: with u = s_j - c_k, n = u/r and the pressure p above,
 *   gc_k = -sum_j sum_{n in W} delta_j[n] (dp/dr n + dp/d(sigma_n^2) (2/r)
 *          (Sigma_k n - sigma_n^2 n)),
 *   dp/dr (sigma_n held) = A sqrt(det)/sigma_n^3 e/(2r) (1 - d^2/sigma_n^2 - d/r),
 *   dp/d(sigma_n^2) = p (d^2/(2 sigma_n^4) - 3/(2 sigma_n^2)),
 * which is gpair_adjoint_centres' gradient when Sigma_k = sigma^2 I.  The
 * plan's tiling stays that of plan creation (centres that move are taken up
 * by a new plan).
 *  A        device float32 [n_kernels] (required).
 *  gcentres device float32 [n_kernels][3] (x, y, z), overwritten.
 *  gA, gsigma6 as gpair_adjoint_aniso (gsigma6 may be NULL).
 * Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_adjoint_aniso_centres(gpair_plan p, const float *A, const float *sigma6,
                                         const float *delta, float *gA, float *gsigma6,
                                         float *gcentres, gpair_stream stream);

/*
 * Synchronise `stream` and return in *count how many sigma_k values outside
 * (0, sigma_max] (and anisotropic covariances outside the admitted set) the
 * operators have met since the plan was created (each forward/adjoint call
 * adds its count).  Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_sigma_violations(gpair_plan p, int64_t *count,
                                    gpair_stream stream);

/* ------------------------------------------------------------------------ */
/* a4. Residual and norms                                                     */
/* ------------------------------------------------------------------------ */

/*
 * delta = scale * (y - b) over the plan's n_sensors*n_samples samples, and
 * norms[0] = sum (y - b)^2, norms[1] = sum b^2, both float64 summed in a fixed
 * order (bitwise reproducible).  The residual of Algorithm 2 ("Loss
 * Calculation" and the trace gradient y - b) with the caller's scale.
 *  y, b    device float32 [n_sensors][n_samples].
 *  delta   device float32, same shape, overwritten; may alias y; may be NULL
 *          (norms only).
 *  norms   device float64 [2], overwritten.
 * Uses the plan workspace for partial sums.  Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_residual(gpair_plan p, const float *y, const float *b,
                            float scale, float *delta, double *norms,
                            gpair_stream stream);

/* ------------------------------------------------------------------------ */
/* a5. Parameter updates                                                      */
/* ------------------------------------------------------------------------ */

/*
 * Projected gradient step x <- min(hi, max(lo, x - step * g)) over n
 * elements ("hard clipping" projection named in the "Nonnegative
 * parameterization constraint" subsection, with lo = 0, hi = +inf for A >= 0).
 *  x  device float32 [n], updated in place;  g  device float32 [n].
 * Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_pgd_update(int64_t n, float *x, const float *g, float step,
                              float lo, float hi, gpair_stream stream);

/*
 * One Adam step (the optimiser of the "Optimization formulation and
 * algorithm" subsection; Kingma and Ba's update with bias correction) on n
 * elements, followed by the projection x <- min(hi, max(lo, x)):
 *   g' = grad_scale * g;  m = b1 m + (1-b1) g';  v = b2 v + (1-b2) g'^2;
 *   x -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 *  x, m, v  device float32 [n], updated in place (m, v start at zero);
 *  g        device float32 [n];  t  1-based step count.
 * Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_adam_update(int64_t n, float *x, const float *g, float *m,
                               float *v, float grad_scale, float lr,
                               float beta1, float beta2, float eps, int32_t t,
                               float lo, float hi, gpair_stream stream);

/* ------------------------------------------------------------------------ */
/* a8 (last step). Least-squares rescale of a warm start, with fallback        */
/* ------------------------------------------------------------------------ */

typedef struct gpair_warm_report {
  double c_star;     /* the scale applied (0 when the start fell back)        */
  double rho;        /* ||A(c* x) - b|| / ||b|| (1 when it fell back)         */
  int32_t fell_back; /* 1: A was set to zero (the zero start, rho = 1)        */
  int32_t pad;
} gpair_warm_report;

/*
 * Rescale a candidate start x (for instance a learned or back-projected
 * image) by the least-squares factor c* = max(0, <A x, b> / ||A x||^2), the
 * scale that minimises ||A(c x) - b|| over c >= 0, so that the rescaled start
 * is never worse than the zero start (rho(0) = 1).  When c* = 0 or the
 * rescaled relative residual is not below 1 the start is replaced by zero.
 * The relative residual rho is the one of Algorithm 2's loss.
 *  A         device float32 [n_kernels]: x on entry, c* x (or 0) on return.
 *  sigma     device float32 [n_kernels].
 *  b         device float32 [n_sensors][n_samples], ||b|| > 0.
 *  y_scratch device float32 [n_sensors][n_samples]: receives A x.
 *  report    host, filled on success.
 * Synchronises `stream` (the fallback is decided on the host).  Errors:
 * INVALID_ARG (also for b = 0), NONFINITE (a non-finite dot product; A is
 * then left unchanged), HIP.
 */
gpair_status gpair_warm_rescale(gpair_plan p, float *A, const float *sigma, const float *b,
                                float *y_scratch, gpair_warm_report *report,
                                gpair_stream stream);

/* ------------------------------------------------------------------------ */
/* a6. Iterative reconstruction driver                                        */
/* ------------------------------------------------------------------------ */

#define GPAIR_SOLVE_PGD 0
#define GPAIR_SOLVE_ADAM 1

/*
 * Options of gpair_solve.  The loss is 0.5*||A(x) - b||^2 / ||b||^2 (the data
 * term of the paper's objective up to a constant factor, so that Adam sees
 * scale-free gradients); PGD uses 0.5*||A(x) - b||^2 with step `step`.
 *  method        GPAIR_SOLVE_PGD or GPAIR_SOLVE_ADAM.
 *  max_iters     iteration cap (>= 0).
 *  tol           stop when ||A(x) - b|| / ||b|| <= tol (0 disables).
 *  step          PGD step size (e.g. 1 / ||A^T A||).
 *  lr_A, lr_sigma, beta1, beta2, eps   Adam hyper-parameters.
 *  learn_sigma   non-zero: also update sigma (Adam only).
 *  sigma_lo, sigma_hi   clamp of sigma after each update (sigma_hi <=
 *                the plan's sigma_max).
 *  a_lo, a_hi    clamp of A after each update (a_lo = 0 gives A >= 0).
 *  check_every   read the residual back to the host every this many
 *                iterations (>= 1); the stop test runs only then.
 * The rest of the paper's objective (Algorithm 2 in full; all off when zero):
 *  npc           non-zero: the non-negativity parameterisation x = (z +
 *                npc_eps)^2 with Adam on the latent z (Adam only; A then
 *                holds z on entry and x = (z + npc_eps)^2 on return, and
 *                a_lo / a_hi are not used).
 *  reg_lambda, reg_beta, reg_eps   the vessel continuity regulariser (see
 *                gpair_vcr) added to the loss as reg_lambda * R_VCR(x), on the
 *                kernel lattice grid_nx x grid_ny x grid_nz (caller order, x
 *                fastest; the product must equal n_kernels).
 *  lr_min, cawr_T0, cawr_Tmult   cawr_T0 > 0: the learning rate of A (or z)
 *                follows gpair_cawr_rate(t, lr_min, lr_A, cawr_T0, cawr_Tmult).
 */
typedef struct gpair_solve_opts {
  int32_t method;
  int32_t max_iters;
  double tol;
  double step;
  double lr_A;
  double lr_sigma;
  double beta1;
  double beta2;
  double eps;
  int32_t learn_sigma;
  double sigma_lo;
  double sigma_hi;
  double a_lo;
  double a_hi;
  int32_t check_every;
  int32_t npc;
  double npc_eps;
  double reg_lambda;
  double reg_beta;
  double reg_eps;
  int32_t grid_nx;
  int32_t grid_ny;
  int32_t grid_nz;
  double lr_min;
  int32_t cawr_T0;
  int32_t cawr_Tmult;
} gpair_solve_opts;

/*
 * Report of gpair_solve (host memory).
 *  history   host float64 [max_iters + 1] or NULL: relative residual before
 *            each iteration (entry i = rho(x_i)) and after the last one, for
 *            the iterations at which it was read (others are set to -1).
 */
typedef struct gpair_solve_report {
  int32_t iters;
  double rel_residual;
  double seconds;
  int32_t converged;
  double *history;
} gpair_solve_report;

/* Device workspace bytes gpair_solve needs for (p, o). */
gpair_status gpair_solve_workspace_size(gpair_plan p,
                                        const gpair_solve_opts *o,
                                        size_t *bytes);

/*
 * Algorithm 2: from the caller's start, repeat [NPC map ->] forward ->
 * residual -> adjoint [-> + lambda grad R_VCR -> NPC chain rule] -> update
 * (with the [CAWR] rate) until rho <= tol or max_iters; the bracketed steps
 * run when the options enable them.  One host synchronisation every
 * check_every iterations.
 *  b       device float32 [n_sensors][n_samples]  measured traces.
 *  A       device float32 [n_kernels]  in: start, out: result.
 *  sigma   device float32 [n_kernels]  in/out (updated iff learn_sigma).
 *  workspace  device, >= gpair_solve_workspace_size bytes, 256-B aligned.
 *  r       host report (filled on GPAIR_OK and GPAIR_NOT_CONVERGED).
 * Returns GPAIR_OK when converged, GPAIR_NOT_CONVERGED at the cap,
 * GPAIR_ERR_NONFINITE if the residual became NaN/Inf (A, sigma then hold the
 * last finite-checked state's successor), or another error.
 */
gpair_status gpair_solve(gpair_plan p, const float *b, float *A, float *sigma,
                         const gpair_solve_opts *o, void *workspace,
                         size_t workspace_bytes, gpair_solve_report *r,
                         gpair_stream stream);

/* ------------------------------------------------------------------------ */
/* f1. ASSA operators (adaptive supersampling alignment)                      */
/* ------------------------------------------------------------------------ */

/*
 * The paper's own discretisation of the forward model (Methods, "Adaptive
 * supersampling alignment for the differentiable model operator", and its
 * Algorithm for the forward and adjoint operators): one kernel width sigma
 * shared by all kernels, times of flight snapped to an alpha-times finer time
 * grid, one shared convolution kernel h, decimation back to the sampling grid.
 * It approximates gpair_forward with a constant sigma (the snapping moves each
 * pulse by at most half a fine step); it is not bit-identical to it.
 *
 * Grid ("Adaptive Grid Parameters" equation), with the window n_sigma of the
 * plan as the "3" of the paper:
 *   n_half = ceil(n_sigma sigma / (v dt))   (taken with a relative tolerance
 *            of 1e-9, so that exact integers are not pushed up by rounding)
 *   alpha  = max(1, ceil(12 / n_half))      (N_min = 25 taps at least)
 *   K      = alpha * n_half,  fine step dt_up = dt / alpha,
 *   fine grid of n_fine = alpha * n_samples points, point k at t0 + k dt_up.
 */
typedef struct gpair_assa_grid {
  int32_t n_half; /* kernel half-width in samples                       */
  int32_t alpha;  /* upsampling factor                                  */
  int32_t K;      /* kernel half-width in fine samples (alpha * n_half) */
  int32_t n_fine; /* alpha * n_samples                                  */
  int32_t fwd_segment; /* fine samples per forward LDS segment          */
  int32_t fwd_passes;  /* passes of the forward over a tile's time shell
                          (1 unless the shell exceeds the LDS budget)   */
  int32_t adj_segment; /* fine samples per adjoint LDS stage row        */
  int32_t adj_stage_sensors; /* sensors staged per adjoint LDS refill   */
} gpair_assa_grid;

/*
 * Grid parameters and segment sizes for `sigma`.  sigma must be finite and in
 * (0, sigma_max] of the plan (the far-field check of the plan assumes it).
 * Errors: SIGMA_RANGE; INVALID_ARG when K > 120 (n_half > 120) or the fine
 * indices of the geometry exceed 1e9.
 */
gpair_status gpair_assa_grid_params(gpair_plan p, double sigma, gpair_assa_grid *out);

/*
 * Bytes of the device work buffer gpair_assa_adjoint needs for `sigma`
 * (the convolved residual, float32 [n_sensors][alpha n_samples]).
 * Errors: as gpair_assa_grid_params.
 */
gpair_status gpair_assa_workspace_size(gpair_plan p, double sigma, size_t *bytes);

/*
 * y = S(h * P_up(x)):
 *   P_up: for each kernel-sensor pair, k_ij = floor((r_ij / v - t0) alpha/dt
 *         + 1/2) (float64), and x_i / r_ij is added to z_j[k_ij]; pairs with
 *         k_ij outside [0, n_fine) are dropped;
 *   h:    h[m] = (1/2) d exp(-d^2 / (2 sigma^2)), d = -v m dt_up, m = -K..K
 *         (normalisation 1/2: a pulse whose time of flight is on the fine
 *         grid gives exactly the samples of Eq. (single_forward));
 *   S:    y_j[n] = (h * z_j)[alpha n], n in [0, n_samples).
 *  x      device float32 [n_kernels], any sign.
 *  sigma  the shared kernel width (m).
 *  y      device float32 [n_sensors][n_samples], overwritten.
 * Impulses accumulate in float32 (LDS), h and the convolution are float32.
 * Errors: INVALID_ARG, SIGMA_RANGE, HIP.
 */
gpair_status gpair_assa_forward(gpair_plan p, const float *x, double sigma, float *y,
                                gpair_stream stream);

/*
 * The exact transpose of gpair_assa_forward (the "Adjoint Operator"
 * subsection): zero-filling delta onto the fine grid, correlation with h
 * (convolution with the reversed kernel), back-projection
 *   g_i = sum_j delta_conv_j[k_ij] / r_ij      (pairs with k_ij in range).
 *  delta  device float32 [n_sensors][n_samples].
 *  g      device float32 [n_kernels], overwritten.
 *  work   device buffer of at least gpair_assa_workspace_size bytes, owned by
 *         the caller, 256-byte aligned; its contents are scratch.
 * Sums over sensors are carried in float64.
 * Errors: INVALID_ARG, SIGMA_RANGE, WORKSPACE (work too small), HIP.
 */
gpair_status gpair_assa_adjoint(gpair_plan p, double sigma, const float *delta, float *g,
                                void *work, size_t work_bytes, gpair_stream stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc):
 * gpair_assa_adjoint without the work argument.  The convolved residual is
 * kept in a fixed device array of this library instead,
 * gpair_assa_static_scratch_bytes() bytes (64 MiB, enough for
 * n_sensors * alpha * n_samples <= 16,777,216: the paper-scale shape needs
 * 12,582,912), which each GPU holds from the first call on it until the
 * process ends.  The plan's device must be current.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (several streams or
 * threads) race, so serialise them.  The call itself allocates nothing.
 *  delta, g  as gpair_assa_adjoint (g overwritten).
 * Errors: INVALID_ARG, SIGMA_RANGE, WORKSPACE (the residual would not fit the
 * array; nothing is launched), HIP.
 */
gpair_status gpair_assa_adjoint_static(gpair_plan p, double sigma, const float *delta, float *g,
                                       gpair_stream stream);
size_t gpair_assa_static_scratch_bytes(void);

/* ------------------------------------------------------------------------ */
/* f2. The paper's full objective: NPC, VCR, CAWR                             */
/* ------------------------------------------------------------------------ */

/*
 * Non-negativity parameterisation ("Nonnegative parameterization
 * constraint"): x = (z + eps)^2 elementwise (the paper's eps = 1e-8).
 *  z, x   device float32 [n]; x may alias z.  Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_npc_map(int64_t n, const float *z, double eps, float *x,
                           gpair_stream stream);

/*
 * Its chain rule: gz = gx * 2 (z + eps) elementwise.
 *  z, gx, gz  device float32 [n]; gz may alias gx.  Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_npc_grad(int64_t n, const float *z, const float *gx, double eps,
                            float *gz, gpair_stream stream);

/* Device work bytes of gpair_vcr on an nx x ny x nz volume.  INVALID_ARG. */
gpair_status gpair_vcr_workspace_size(int32_t nx, int32_t ny, int32_t nz, size_t *bytes);

/*
 * Vessel continuity regulariser ("Vessel continuity regularization"):
 *   R_VCR(x) = R_H(x) + beta R_TV(x),
 *   R_H  = sum_i sqrt( sum_{p,q in {x,y,z}} (D_pq x_i)^2 + eps ),
 *   R_TV = sum_i sqrt( sum_{d} (D_d x_i)^2 + eps ),
 * on a volume stored [nz][ny][nx] (x fastest: the caller's kernel order of a
 * lattice plan), unit spacing, with D_d x_i = x[i+e_d] - x[i],
 * D_pp x_i = x[i+e_p] - 2 x[i] + x[i-e_p], D_pq x_i = x[i+e_p+e_q] - x[i+e_p]
 * - x[i+e_q] + x[i] (p != q; D_pq = D_qp, so each mixed term counts twice) and
 * every difference whose stencil leaves the volume taken as 0.
 *  x      device float32 [nz][ny][nx].
 *  grad   device float32 [nz][ny][nx] or NULL: grad += lambda * dR_VCR/dx.
 *  value  device float64 [1] or NULL: R_VCR(x), summed in a fixed order.
 *  work   device, >= gpair_vcr_workspace_size bytes, 256-byte aligned.
 * Differences and norms are float64, the normalised terms float32.
 * Errors: INVALID_ARG, WORKSPACE, HIP.
 */
gpair_status gpair_vcr(int32_t nx, int32_t ny, int32_t nz, const float *x, double beta,
                       double eps, double lambda, float *grad, double *value, void *work,
                       size_t work_bytes, gpair_stream stream);

/*
 * Cosine annealing with warm restarts ("Optimization formulation and
 * algorithm"), host only: eta_t = eta_min + (eta_max - eta_min)(1 + cos(pi
 * T_cur / T_i)) / 2 for iteration t >= 0, where period i has length
 * T0 * Tmult^i and T_cur counts iterations since the period began (the cited
 * SGDR schedule; for Tmult = 1 exactly the printed formula with
 * T_cur = t mod T0).  Errors: INVALID_ARG (t < 0, T0 < 1, Tmult < 1,
 * non-finite rates).
 */
gpair_status gpair_cawr_rate(int64_t t, double eta_min, double eta_max, int64_t T0,
                             int32_t Tmult, double *rate);

/* ------------------------------------------------------------------------ */
/* Kernel timing (measurement support)                                        */
/* ------------------------------------------------------------------------ */

#define GPAIR_TIMER_FORWARD 0 /* main forward kernel of the last forward  */
#define GPAIR_TIMER_ADJOINT 1 /* main adjoint kernel of the last adjoint  */
#define GPAIR_TIMER_ASSA_FORWARD 2 /* the ASSA forward kernel             */
#define GPAIR_TIMER_ASSA_ADJOINT 3 /* the ASSA back-projection kernel     */
#define GPAIR_TIMER_KINDS 4

#define GPAIR_TIMER_SLOTS 64   /* launches remembered per kind              */

/*
 * Issue-rate probe of one vector instruction (the ceilings the operators'
 * roofline is stated against): blocks x 256 threads, each running 8
 * independent dependency chains of `iters` x 8 steps of
 *   kind 0: float32 FMA (v_fma_f32)      kind 1: float64 FMA (v_fma_f64)
 *   kind 2: float32 exp2 (v_exp_f32)     kind 3: float32 1/sqrt (v_rsq_f32)
 *   kind 4: float64 1/sqrt (v_rsq_f64)
 * then one float per thread written to out (device float32 [blocks * 256];
 * its value is meaningless).  *per_wave (host) receives the number of probed
 * instructions each wave issues; divide waves x per_wave by the kernel's time.
 * Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_peak_probe(int32_t kind, int32_t blocks, int32_t iters, float *out,
                              int64_t *per_wave, gpair_stream stream);

/*
 * enable != 0: record a pair of HIP events around the main kernel of each
 * later forward/adjoint call, on the call's stream (the events are created
 * here, once per plan).  Errors: INVALID_ARG, HIP.
 */
gpair_status gpair_plan_set_timing(gpair_plan p, int enable);

/*
 * Durations (ms) of the main kernel of the most recent calls of kind `which`
 * recorded since timing was enabled or since the previous read (at most
 * GPAIR_TIMER_SLOTS, oldest first).  Synchronises on the last recorded event.
 * Writes min(count, capacity) values to ms (host float32 [capacity]) and the
 * number available to *count, then forgets them.
 * Errors: INVALID_ARG (timing off), HIP.
 */
gpair_status gpair_plan_kernel_times(gpair_plan p, int which, float *ms,
                                     int32_t capacity, int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* GPAIR_H */
