/*
 * celmi.h -- C ABI of the MI355X (gfx950) library for the variational objective of
 * Regier et al., "Approximate Inference for Constructing Astronomical Catalogs from
 * Images" (arXiv 1803.00113).
 *
 * The library evaluates, for a catalog of S light sources observed in N images, the
 * evidence lower bound (ELBO) of Section 4.2 (equation elbo) and its gradient, takes
 * trust-region Newton steps on per-source parameter blocks (Section 4.3) and runs block
 * coordinate ascent over non-overlapping sources (Sections 4.3-4.4).
 *
 * Conventions
 *  - Every function returns a cel_status (0 = CEL_OK, < 0 = error, > 0 = information).
 *    Arguments are validated on the host before anything is enqueued; on error nothing
 *    is launched and no output is written.  cel_strerror() names a status.
 *  - "DEVICE" pointers are HIP device memory on the context's device, owned by the
 *    caller and never retained past the call's stream work.  "HOST" pointers are read
 *    during the call only.
 *  - Calls are asynchronous on the given stream (0 = the null stream).  Outputs are valid
 *    once the caller synchronises that stream.  cel_elbo_eval and cel_elbo_grad allocate
 *    nothing (their scratch is made by cel_prepare and owned by the plan); the Hessian,
 *    Newton, sweep and likelihood calls allocate their own scratch at their first call on
 *    a plan; cel_elbo_grad_static never allocates.
 *  - A context and its plans are not thread-safe; use one per host thread.
 *  - Results are deterministic: a fixed plan and inputs give bitwise-identical outputs,
 *    independent of launch configuration and of which other sources share a launch.
 *
 * Parameters of source s (theta[s*32 + k], float64, unconstrained coordinates):
 *   0-1   u: position (reference pixel frame; image n sees pixel = A_n u + b_n)
 *   2     logit(a): a = q(star), Section 4.1 (eq0)
 *   3,4   mean of log r given galaxy / star
 *   5,6   log variance of log r given galaxy / star
 *   7-10  colour means given galaxy;   11-14 colour means given star
 *   15-18 log colour variances given galaxy; 19-22 given star
 *   23    galaxy angle (radians) | 24 log half-light radius (pixels)
 *   25    logit(e_profile) (weight of the de Vaucouleurs profile) | 26 logit(e_axis)
 *   27-31 unused: read as given, gradient written as 0
 * Colours are c_k = ln(l_{k+1} / l_k) over bands u,g,r,i,z; the reference flux r is the
 * r band (index 2).
 */
#ifndef CELMI_H
#define CELMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cel_status;
#define CEL_OK 0
#define CEL_EINVAL (-1)        /* invalid argument (null pointer, bad size, bad table)   */
#define CEL_ENOMEM (-2)        /* device or pinned host allocation failed (cel_prepare)  */
#define CEL_EHIP (-3)          /* a HIP runtime call failed                              */
#define CEL_EUNSUPPORTED (-4)  /* a size beyond the library's compiled limits            */
#define CEL_ESCRATCH (-5)      /* cel_elbo_grad_static: scratch need beyond the static
                                  buffer (CEL_STATIC_SCRATCH_BYTES)                     */

/* per-source status written by cel_newton_step / cel_sweep */
#define CEL_ST_SKIPPED 0       /* not selected by the mask                               */
#define CEL_ST_ACCEPTED 1      /* trust-region step accepted                             */
#define CEL_ST_REJECTED 2      /* step rejected, radius shrunk                           */
#define CEL_ST_CONVERGED 3     /* convergence test met, theta unchanged                  */
#define CEL_ST_NONFINITE 4     /* objective or gradient not finite, theta unchanged      */

/* conditions found on the device, accumulated per context (cel_last_device_error) */
#define CEL_DEVERR_NONFINITE_OBJECTIVE 1  /* some L_s evaluated to a non-finite value      */
#define CEL_DEVERR_NONFINITE_STEP 2       /* a Newton step met non-finite theta, gradient
                                             or Hessian (that source: CEL_ST_NONFINITE)  */
#define CEL_DEVERR_NONFINITE_HESSIAN 4    /* cel_elbo_hessian produced a non-finite entry  */
#define CEL_DEVERR_BAD_INDEX 8            /* cel_psf_fit met an image index out of range
                                             (that fit's output rows are NaN)              */

#define CEL_N_THETA 32
#define CEL_N_PARAM 27
#define CEL_Z_N 16             /* point values per source (cel_loglik)                   */
#define CEL_MAX_PSF 4
#define CEL_MAX_PROFILE 8
#define CEL_N_COLOUR_COMPONENTS 8
#define CEL_MAX_EIGEN 4        /* PSF eigen-images per image (cel_psf_fit)                */
#define CEL_PSF_MAX_SIDE 63    /* knots per side of a PSF eigen-image                     */

/* One image (Section 2.2, Table 3): band, PSF as a Gaussian mixture in pixels (Section
 * 2.2.3), linear WCS, calibration and a sky knot grid (Section 2.2.1). */
typedef struct {
  int32_t band;                 /* 0..4 = u,g,r,i,z                                     */
  int32_t H, W;                 /* rows, cols                                           */
  int32_t n_psf;                /* 1..CEL_MAX_PSF                                       */
  double psf[CEL_MAX_PSF][6];   /* weight, mean_x, mean_y, cov_xx, cov_xy, cov_yy       */
  double A[2][2];               /* pixel (x=col, y=row) = A u + b                       */
  double b[2];
  double iota;                  /* expected counts per unit flux (> 0)                  */
  int32_t sky_qh, sky_qw;       /* knot grid rows, cols (>= 1), spanning the corners    */
  int64_t sky_off;              /* offset of the row-major knot grid in sky_knots       */
} cel_image;

/* The active pixels of one source in one image: a rectangle of pixel centres
 * cols x0..x0+w-1, rows y0..y0+h-1, stored row-major at pixels[pix_off...]. */
typedef struct {
  int32_t src, img, x0, y0, w, h;
  int64_t pix_off;
} cel_patch;

/* Prior hyperparameters (Section 2.1, Table 2).  Type index 0 = galaxy, 1 = star. */
typedef struct {
  double star_prob;                                  /* A in (0,1)                      */
  double r[2][2];                                    /* mean, variance of log r         */
  double c_w[2][CEL_N_COLOUR_COMPONENTS];            /* colour GMM weights (sum 1)      */
  double c_mean[2][CEL_N_COLOUR_COMPONENTS][4];
  double c_cov[2][CEL_N_COLOUR_COMPONENTS][4][4];    /* symmetric positive definite     */
  double radius[2];                                  /* mean, variance of log radius    */
  double profile[2];                                 /* Beta parameters (> 0)           */
  double axis[2];                                    /* Beta parameters (> 0)           */
} cel_prior;

/* Galaxy profile mixtures (Section 2.1.2, equation hsi): sum_j alpha_j N(0, tau_j Sigma). */
typedef struct {
  int32_t n_exp, n_dev;                              /* 1..CEL_MAX_PROFILE each          */
  double exp_alpha[CEL_MAX_PROFILE], exp_tau[CEL_MAX_PROFILE];
  double dev_alpha[CEL_MAX_PROFILE], dev_tau[CEL_MAX_PROFILE];
} cel_profiles;

/* A problem.  Tables are HOST memory (copied by cel_prepare); pixels are DEVICE memory
 * holding integer-valued counts >= 0 (float32).  Patches must be sorted by (src, img),
 * have at most one patch per (src, img), lie inside their image, have w, h >= 1 and
 * w*h <= 2^22, and not overlap in `pixels`. */
typedef struct {
  int32_t n_sources, n_images, n_patches;
  const cel_image* images;       /* HOST [n_images]                                     */
  const double* sky_knots;       /* HOST [n_sky_knots]                                  */
  int64_t n_sky_knots;
  const cel_patch* patches;      /* HOST [n_patches]                                    */
  const float* pixels;           /* DEVICE [n_pixels]; read only inside cel_prepare     */
  int64_t n_pixels;
  const cel_prior* prior;        /* HOST                                                */
  const cel_profiles* profiles;  /* HOST                                                */
  const double* patch_psf;       /* HOST [n_patches][CEL_MAX_PSF][6] or NULL: the PSF
                                    mixture of each patch (a spatially varying PSF,
                                    Section 2.2.2, e.g. from cel_psf_fit), in the layout
                                    of cel_image.psf with the n_psf components of the
                                    patch's image; NULL = every patch uses its image's   */
} cel_problem;

typedef struct {
  int32_t pixels_per_lane;       /* 1, 2 or 4; 0 = default                              */
  int32_t chunk_pixels;          /* pixels per work item (multiple of 64); 0 = default  */
  int32_t pixel_fp64;            /* 1: evaluate pixels in float64 instead of float32     */
  int32_t hessian_fp64;          /* 1: Newton steps from the float64 pixel path          */
  int32_t hessian_fd;            /* 1: pixel Hessian by central differences of the
                                    gradient (54 variants); 0 (default): analytic       */
  double fd_step;                /* central-difference step of the Hessian; 0 = 1e-2 with
                                    float32 gradients, 1e-3 with float64 ones             */
  double radius0, radius_max, eta, gtol, ftol, radius_min;   /* trust region (0 = default) */
  int32_t timing;                /* 1: record HIP events around each phase (see below)  */
  int32_t map_pixels_per_lane;   /* neighbour moment maps: 1, 2, 4 (default; 0 in the
                                    struct = default) or 8 pixels per lane 64 apart, values
                                    directly; -1: runs of 8 pixels along a row, values by
                                    recurrence                                           */
} cel_options;

typedef struct cel_ctx cel_ctx;
typedef struct cel_plan cel_plan;

const char* cel_strerror(cel_status s);

/* Create a context on HIP device `hip_device`.  opt may be NULL (defaults).  Plans made
 * from a context must be freed before it is destroyed. */
cel_status cel_create(cel_ctx** out, int32_t hip_device, const cel_options* opt);
void cel_destroy(cel_ctx* ctx);

/* Conditions the kernels of this context's plans found since the last call (a bitwise OR
 * of CEL_DEVERR_*; 0 = none), then cleared.  Device-detected conditions never abort a
 * batch: the affected sources carry their own status.  Call after synchronising the
 * streams the work ran on; the read itself is a synchronous copy.  code: HOST int32. */
cel_status cel_last_device_error(cel_ctx* ctx, int32_t* code);

/* Validate a problem and build a plan: patch overlap lists, the source overlap graph and
 * its greedy colouring (ascending id, smallest free colour), work items sorted by cost,
 * and device copies of the tables; reads the pixels once (on `stream`, synchronised
 * before return) to form per-pixel (count, sky) pairs and the per-patch data constants
 * sum(x log x - x - log x!).  Owns all scratch of later calls.  Synchronous.
 * CEL_EUNSUPPORTED beyond the compiled limits: 2^20 images, image width 2^20, 2^24 patches,
 * 2^22 pixels per patch, 2^30 work items, 4 PSF components, 8 + 8 profile components. */
cel_status cel_prepare(cel_ctx* ctx, const cel_problem* prob, cel_plan** out, void* stream);
void cel_plan_free(cel_plan* plan);

/* Add a problem's sources, images and patches to a plan (a serving loop admitting a region
 * request into its resident set).  The part's ids follow the plan's: source s of the part
 * becomes n_sources + s, and so on for images and patches; its patches refer to its own
 * images, so no source of the part overlaps one already in the plan.  part->pixels is
 * DEVICE memory read during the call.  The cost depends on the part only (amortised: the
 * plan's device arrays grow by doubling): the part is validated and prepared on its own
 * (as cel_prepare) and spliced in; results for sources already in the plan are unchanged
 * bit for bit.  The part must share the plan's prior and profile tables (CEL_EINVAL
 * otherwise); per-patch PSFs are not supported here (CEL_EUNSUPPORTED).  Captured sweep
 * graphs of the plan are dropped.  Synchronous; the plan must not be in use meanwhile. */
cel_status cel_plan_append(cel_ctx* ctx, cel_plan* plan, const cel_problem* part, void* stream);

/* Plan facts.  colours: HOST [n_sources] or NULL; returns counts via out-pointers (any may
 * be NULL): active pixels, colour classes, work items, and the device bytes the plan holds
 * now (its tables, pixels and the scratch of the calls made so far). */
cel_status cel_plan_info(const cel_plan* plan, int64_t* n_units, int32_t* n_colours, int32_t* colours,
                         int64_t* n_work_items, int64_t* device_bytes);

/* ELBO (Section 4.2, equation elbo).  theta: DEVICE float64 [S*32].
 * elbo_total: DEVICE float64 [1] -- every pixel of the union of patches once, minus
 *   every source's KL.
 * elbo_local: DEVICE float64 [S] or NULL -- L_s = sum over the pixels of s's patches of
 *   the expected log-likelihood term (with every source's light) minus KL_s; its
 *   gradient in theta_s equals that of the total. */
cel_status cel_elbo_eval(cel_ctx* ctx, const cel_plan* plan, const double* theta, double* elbo_total,
                         double* elbo_local, void* stream);

/* ELBO and its gradient in the unconstrained coordinates: grad DEVICE float64 [S*32]
 * (entries 27-31 written 0).  elbo_total / elbo_local as above (either may be NULL). */
cel_status cel_elbo_grad(cel_ctx* ctx, const cel_plan* plan, const double* theta, double* elbo_total,
                         double* elbo_local, double* grad, void* stream);

/* For callers that cannot allocate device memory at call time (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cel_elbo_grad with its
 * per-call scratch (component tables, neighbour moment maps, slot rows, per-source sums)
 * in one static device buffer of CEL_STATIC_SCRATCH_BYTES per device, held from the
 * library's first cel_create on that device until the process ends, instead of the plan's
 * own blocks.  It calls no allocating routine.  Same kernels and launch order as
 * cel_elbo_grad, so the outputs are bitwise identical.  Arguments as cel_elbo_grad.
 * Need in bytes (each part rounded up to 256): n_patches x 6016 (float64 pixels: 12032)
 * + active pixels x 8 (16) + work items x 128 + sources x 272; CEL_ESCRATCH beyond the
 * buffer (the 1000-source batched workload of 1.7e7 pixels needs 204 MB).  All calls on
 * one device share the buffer: calls that overlap in time on one device (several streams,
 * several host threads, several contexts) race and must be serialised by the caller; a
 * call's outputs are complete once its stream is synchronised. */
#define CEL_STATIC_SCRATCH_BYTES ((int64_t)256 << 20)
cel_status cel_elbo_grad_static(cel_ctx* ctx, const cel_plan* plan, const double* theta, double* elbo_total,
                                double* elbo_local, double* grad, void* stream);

/* Same as cel_elbo_grad, one launch sequence per source ("plain" form, for comparison
 * with the batched form).  Slower by design; identical results. */
cel_status cel_elbo_grad_plain(cel_ctx* ctx, const cel_plan* plan, const double* theta, double* elbo_total,
                               double* elbo_local, double* grad, void* stream);

/* Per-source Hessians of L_s in the unconstrained coordinates, every other source fixed
 * (the dense Newton Hessian of Section 4.3; also what a Laplace approximation needs).
 * Exact (analytic) in both the pixel and the KL parts.  mask: HOST uint8 [S] or NULL
 * (all sources).  hess: DEVICE float64 [S][27][27] out (rows of unmasked sources left
 * untouched); grad: DEVICE float64 [S][32] out or NULL; elbo_local: DEVICE [S] or NULL. */
cel_status cel_elbo_hessian(cel_ctx* ctx, const cel_plan* plan, const double* theta, const uint8_t* mask,
                            double* hess, double* grad, double* elbo_local, void* stream);

/* One trust-region Newton step (Section 4.3) on every source with mask[s] != 0 (HOST
 * uint8 [S], NULL = all), all from the same iterate.  Masked sources must be pairwise
 * non-overlapping (checked against the plan: CEL_EINVAL otherwise); with the exact Hessian
 * they are stepped as one batch whatever their colour classes.  Hessian exact (as
 * cel_elbo_hessian), or with options.hessian_fd by central differences of the gradient
 * (pixel part; the KL part is always exact); the subproblem is solved
 * exactly (eigen-decomposition, boundary multiplier by a safeguarded secular-equation
 * iteration, hard case completed along the lowest eigenvector).
 * theta: DEVICE [S*32] in/out; radius: DEVICE float64 [S] in/out (trust radii);
 * step_status: DEVICE int32 [S] out (CEL_ST_*); elbo_local: DEVICE float64 [S] out or
 * NULL (L_s at the returned theta, NaN for skipped sources). */
cel_status cel_newton_step(cel_ctx* ctx, const cel_plan* plan, double* theta, double* radius,
                           const uint8_t* mask, int32_t* step_status, double* elbo_local, void* stream);

typedef struct {
  int32_t n_sweeps;              /* block coordinate ascent passes (default 3)           */
  int32_t max_newton_iters;      /* per colour class per sweep (default 50)              */
  int32_t use_graph;             /* 1: replay a captured HIP graph per colour class      */
  int32_t start_colour;          /* resume: first pass starts at this colour class; 0 =
                                    a fresh pass (radii reset, statuses cleared)         */
  int32_t max_classes;           /* stop after this many colour classes (0 = no limit)  */
} cel_sweep_opts;

typedef struct {
  double elbo_total;             /* at the returned theta                                */
  int32_t n_colours;
  int64_t n_newton_steps;        /* batched steps taken                                  */
  double seconds;                /* wall time of the call                                */
  int32_t sweeps_done;           /* passes completed by this call                        */
  int32_t next_colour;           /* cursor: the colour class a resumed call starts at
                                    (0 when the last pass was completed)                 */
} cel_sweep_report;

/* Block coordinate ascent (Sections 4.3-4.4): for each sweep and each colour class in
 * ascending colour, Newton steps on the whole class (all members at once: they do not
 * overlap) until every member has converged or max_newton_iters steps were taken.  The
 * trust radius of every source starts at radius0 at each sweep.  theta DEVICE in/out;
 * radius DEVICE float64 [S] in/out; status DEVICE int32 [S] in/out (last status per
 * source); report HOST (filled after an internal stream synchronisation).
 * Checkpoint / resume: with max_classes = k the call stops after k colour classes and
 * reports the cursor; (theta, radius, status) and a second call with start_colour =
 * next_colour and n_sweeps = the passes still due (the interrupted one included) continue
 * exactly as one uninterrupted call.  opts NULL: defaults.  CEL_EINVAL if start_colour is
 * outside [0, n_colours) (n_colours > 0) or a count is negative. */
cel_status cel_sweep(cel_ctx* ctx, const cel_plan* plan, double* theta, double* radius, int32_t* status,
                     const cel_sweep_opts* opts, cel_sweep_report* report, void* stream);

/* A spatially varying PSF (Section 2.2.2, Table 1): for each image, n_eigen principal
 * images ("eigen-images") of side x side knots centred on a light source (knot (i, j) at
 * the offset (j - c, i - c) pixels, c = (side - 1) / 2), and loadings that vary smoothly
 * over the image: the loading of eigen-image e at pixel position (x, y) of image n is
 * sum_t coef[n][e][t] m_t with m = (1, u, v, u^2, u v, v^2), u = x / W_n, v = y / H_n.
 * The PSF at (x, y) is sum_e loading_e eigen_e, negative values clipped to zero. */
typedef struct {
  int32_t n_images;
  int32_t n_eigen;               /* 1..CEL_MAX_EIGEN                                     */
  int32_t side;                  /* odd, 3..CEL_PSF_MAX_SIDE                             */
  const double* eigen;           /* DEVICE [n_images][n_eigen][side][side]               */
  const double* coef;            /* DEVICE [n_images][n_eigen][6]                        */
  const double* size;            /* DEVICE [n_images][2]: W, H of each image (pixels)    */
} cel_psf_model;

/* The PSF as a Gaussian mixture (Section 2.2.3: a mixture of bivariate normals keeps a
 * galaxy's convolution with the PSF analytic) at n_fits positions: fit f takes the PSF of
 * image fit_img[f] (DEVICE int32 [n_fits]) at pixel position fit_xy[f] (DEVICE float64
 * [n_fits][2], x = column, y = row) and fits an n_comp-component mixture (1..CEL_MAX_PSF)
 * to its knot values by n_iter expectation-maximisation iterations with the knot values as
 * weights, from a start made of the image's moments (every component at the centroid,
 * component k's covariance the second central moment times 2^(k - (n_comp-1)/2), equal
 * weights); a component whose weight falls to 1e-12 of the total or below keeps its
 * parameters.  out: DEVICE float64 [n_fits][CEL_MAX_PSF][6], rows (weight, mean_x, mean_y,
 * cov_xx, cov_xy, cov_yy) as cel_image.psf with means as offsets from (x, y) and weights
 * summing to one; rows n_comp.. zero.  All arithmetic float64; one workgroup per fit;
 * deterministic.  A fit whose image index is out of range gets NaN rows and sets
 * CEL_DEVERR_BAD_INDEX.  The result feeds cel_problem.patch_psf (the fit at the centre
 * of each patch).  Asynchronous on `stream`; allocates nothing.
 * CEL_EINVAL: null pointers with n_fits > 0, bad sizes; CEL_EUNSUPPORTED beyond the limits. */
cel_status cel_psf_fit(cel_ctx* ctx, const cel_psf_model* model, int32_t n_fits, const int32_t* fit_img,
                       const double* fit_xy, int32_t n_comp, int32_t n_iter, double* out, void* stream);

/* Measurement: with options.timing = 1, every ELBO / gradient evaluation records HIP events
 * on the caller's stream around its phases.  This returns the summed device milliseconds
 * since the last reset -- ms[0] component tables, ms[1] neighbour moment maps, ms[2] pixel
 * kernel, ms[3] finalisation and total (ms: HOST double[4]) -- and the number of
 * evaluations recorded (it synchronises on the recorded events).  reset != 0 clears the
 * record.  CEL_EINVAL if timing was not enabled. */
cel_status cel_phase_times(cel_plan* plan, double* ms, int64_t* n_calls, int32_t reset);

/* Exact Poisson log-likelihood at point values of the latent variables, batched over
 * candidates: the quantity that the annealed importance sampler and slice sampling of the
 * paper's MCMC procedure evaluate (Section 3, equation eqzs: source s is sampled with its
 * neighbours' latent variables z_{-s} held fixed; Section 3.1: the target
 * pi(w_s) = p(x | w_s, a_s, z_{-s}) p(w_s | a_s), whose likelihood factor this is).
 *   ll[c][s] = sum over the active pixels of source s's patches of
 *              x log(lambda) - lambda - log(x!),
 *   lambda   = sky + sum over the sources t whose patch covers the pixel of l_t f_t
 *              (Section 2.2.3), with source s at z_cand[c][s] and every other source at
 *              z_fixed[t].
 * Pixels outside source s's patches do not depend on z_s and are left out.
 * Point values z[s*16 + k] (float64):
 *   0-1  u (reference pixel frame)        | 2  type: 1 star, 0 galaxy (nonzero = star)
 *   3    log r (reference-band flux)      | 4-7 colours c_1..c_4 (as in theta)
 *   8    galaxy angle (radians)           | 9  log half-light radius (pixels)
 *   10   profile weight e_profile, [0, 1] | 11 axis ratio e_axis, (0, 1]
 *   12-15 unused
 * z_fixed: DEVICE [S][16].  z_cand: DEVICE [n_cand][S][16] (rows of unselected sources are
 * not read).  mask: HOST uint8 [S], selected sources (NULL = all); selected sources may
 * overlap (each candidate sees the others at z_fixed).  ll: DEVICE float64 [n_cand][S] out;
 * rows of unselected sources are not written; a candidate outside the support (profile
 * weight or axis ratio out of range, a non-finite value) gets -infinity.
 * Cost: the neighbour maps at z_fixed once, then one ELBO-only pixel pass per candidate over
 * the selected sources' pixels (candidates are batched 56 at a time; the pass takes 4 pixels
 * per lane whatever the plan's pixels-per-lane setting).  Pixel precision as
 * the context's pixel_fp64 option; sums in FP64.  Asynchronous on `stream`; uses the plan's
 * scratch (no two calls on one plan may overlap).
 * CEL_EINVAL: null pointers, n_cand < 0.  CEL_ENOMEM: scratch allocation failed. */
cel_status cel_loglik(cel_ctx* ctx, const cel_plan* plan, const double* z_fixed, int32_t n_cand,
                      const double* z_cand, const uint8_t* mask, double* ll, void* stream);

/* Options of cel_mcmc_step (Section 3).  Defaults of the paper's runs: n_temps = T = 200,
 * n_runs = N' = 25, n_post = B' = 25. */
typedef struct {
  int32_t n_temps;               /* T: annealing temperatures (>= 1)                     */
  int32_t n_runs;                /* N': runs per source type (1..28)                     */
  int32_t n_post;                /* B': slice-sampling sweeps at the target per run (>= 1) */
  int32_t max_step_out;          /* m: the stepping-out interval grows at most m-1 times  */
  int32_t max_shrink;            /* shrinkage draws before an update keeps its point      */
  const double* gamma;           /* HOST [n_temps + 1]: gamma_0 = 0 < ... < gamma_T = 1   */
  double width[CEL_Z_N];         /* slice width per point coordinate (layout of cel_loglik) */
  double box;                    /* half-width (pixels) of the position's uniform prior
                                    around z_fixed's position                            */
  uint64_t seed;                 /* first word of the random generator's key              */
} cel_mcmc_opts;

typedef struct {
  int64_t rounds;                /* lockstep rounds of candidate evaluations              */
  int64_t n_chains;              /* 2 n_runs per selected source                          */
  int64_t evaluations;           /* candidate log targets evaluated by the chains         */
  int64_t candidate_pixels;      /* sum over evaluations of the source's active pixels    */
} cel_mcmc_report;

/* One MCMC update of every selected source (Section 3, equation eqzs: each source sampled
 * from p(z_s | x, z_-s) with every other source at z_fixed; selected sources that do not
 * overlap are conditionally independent, so a colour class updated at once equals updating
 * its members in turn).  Per source and type a (0 galaxy, 1 star): n_runs annealed
 * importance sampling runs (Section 3.1) from the start points z_init (draws from the prior
 * pi_0 = p(w | a), made by the caller) through pi_t = p(w | a) p(x | w, a, z_-s)^gamma_t,
 * each transition one slice-sampling-within-Gibbs sweep over the type's coordinates (u,
 * log r, colours; a galaxy also angle, log radius, profile weight, axis ratio; univariate
 * slice sampling with stepping out and shrinkage), the run's log weight
 * sum_t (gamma_t - gamma_{t-1}) log p(x | w^(t-1)); then n_post further sweeps at the target
 * (Section 3.2), each leaving one sample.  p(a = 1 | x, z_-s) by Bayes' rule from the prior
 * probability of a star and the mean weights; a type is drawn from it, then one of its
 * n_runs x n_post samples uniformly.  Likelihood as cel_loglik (exact Poisson, pixels of
 * the source's patches), prior as cel_log_prior plus the position's uniform prior on the
 * box (a constant, left out); the angle is periodic (an accepted angle is mapped to
 * [0, pi)).  Random numbers: Philox4x64-10 with key (seed, key) at counters fixed by
 * (chain, sweep, coordinate, draw), so results do not depend on launch configuration.
 * z_fixed: DEVICE [S][16]; mask: HOST uint8 [S] (NULL = all); z_init: DEVICE
 * [2][n_runs][S][16] (type 0 rows first); z_out: DEVICE [S][16] (the new point of each
 * selected source); p_star: DEVICE [S]; log_evidence: DEVICE [S][2] (log of the mean
 * weight per type); samples: DEVICE [S][2][n_runs][n_post][16] or NULL; rhat: DEVICE
 * [S][2][16] or NULL: the potential scale reduction factor of the n_runs chains of n_post
 * samples per type and coordinate (Gelman and Rubin 1992, the criterion Section 3.2
 * monitors the chains by: with chain means m_j, their mean g and chain variances v_j of
 * divisor n_post - 1, B = n_post / (n_runs - 1) sum_j (m_j - g)^2, W = mean_j v_j,
 * R = sqrt(((n_post - 1) / n_post W + B / n_post) / W); NaN for a coordinate no chain
 * moves or when n_runs or n_post is 1, +infinity when only the chains' values differ);
 * rows of unselected sources untouched.  report: HOST or NULL.  Pixel precision as the context's
 * pixel_fp64 option.  Synchronous (the host polls the chains every 16 rounds).  Allocates
 * its scratch on the plan at first use.
 * CEL_EINVAL: null pointers, bad options (gamma NULL, n_runs > 28, negative widths). */
cel_status cel_mcmc_step(cel_ctx* ctx, const cel_plan* plan, const double* z_fixed, const uint8_t* mask,
                         const double* z_init, const cel_mcmc_opts* opts, uint64_t key, double* z_out,
                         double* p_star, double* log_evidence, double* samples, double* rhat,
                         cel_mcmc_report* report, void* stream);

/* Log prior density log p(w | a) of n point values (the start distribution pi_0 of the
 * annealed importance sampler, Section 3.1; the priors of Section 2.1), over the point
 * layout's coordinates (see cel_loglik): log r ~ normal(prior mean, variance of the type),
 * colours ~ the type's Gaussian mixture, and for a galaxy (z[2] == 0) log radius ~ normal,
 * profile weight and axis ratio ~ beta, angle ~ uniform on [0, pi) radians.  The position's
 * uniform prior is a constant and left out, as is the type's prior p(a).  Together with
 * cel_loglik this gives the annealed target log pi_t = log p(w | a) + gamma_t ll.
 * z: DEVICE float64 [n][16]; out: DEVICE float64 [n]; -infinity outside the support (as in
 * cel_loglik).  Uses the plan's prior tables only; asynchronous on `stream`.
 * CEL_EINVAL: null pointers with n > 0, n < 0. */
cel_status cel_log_prior(cel_ctx* ctx, const cel_plan* plan, int64_t n, const double* z, double* out, void* stream);

/* Candidate launch settings for cel_tune.  A count of 0 keeps the plan's current value of
 * that setting; a NULL space means the defaults: work items of 256, 512, 1024 and 2048
 * pixels; 1, 2 and 4 pixels per lane in the pixel pass; 1, 2, 4, 8 pixels per lane and the
 * row-run variant (-1) in the moment-map pass.  Values as in cel_options. */
typedef struct cel_tune_space {
  int32_t n_chunk;
  int32_t chunk_pixels[8];
  int32_t n_pixels_per_lane;
  int32_t pixels_per_lane[4];
  int32_t n_map;
  int32_t map_pixels_per_lane[6];
} cel_tune_space;

/* The settings cel_tune kept, and the time of one ELBO-and-gradient evaluation with them
 * (the least of the timed calls). */
typedef struct cel_tuning {
  int32_t chunk_pixels;
  int32_t pixels_per_lane;
  int32_t map_pixels_per_lane;
  int32_t n_timed;            /* settings timed */
  double ms_per_eval;
} cel_tuning;

/* Launch tuning of the evaluation (the paper's thread-level execution study and its remark
 * that sources of varying size make SIMD across sources hard), kept per plan.  After 40
 * untimed evaluations (the device's clocks settle), times the ELBO-and-gradient evaluation
 * at theta over the work-item size and the pixel pass's pixels per lane together, then over
 * the moment-map variants at the chosen pair: every setting in two passes through all
 * candidates, each time one warm-up and five timed calls, the least time counting, on
 * `stream`, synchronised.  The fastest setting replaces the plan's current one when that is
 * no candidate or is slower by more than 5 % (settings closer than that trade places from
 * run to run): a new work-item size re-cuts the plan's work items
 * (item tables, launch orders, per-colour lists and the scratch sized by the item count,
 * as cel_prepare would have cut them with that chunk_pixels).  Later evaluations, Newton
 * steps, sweeps, samplers and appends of the plan use the settings; captured sweep graphs
 * are dropped.  A tuned plan gives, bit for bit, the outputs of a plan prepared on a
 * context created with the kept settings; different settings sum partial results in
 * different groupings (last-bit differences).  theta: DEVICE [S][32].  space: HOST, may be
 * NULL.  out: HOST, may be NULL.  Writes no caller buffer but out; the plan's internal
 * scratch holds the last timed evaluation.  CEL_EINVAL: a candidate outside cel_options'
 * ranges or a count beyond its array.  On an error other than CEL_EINVAL the plan may only
 * be freed. */
cel_status cel_tune(cel_ctx* ctx, cel_plan* plan, const double* theta, const cel_tune_space* space,
                    cel_tuning* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CELMI_H */
