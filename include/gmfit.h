/*
 * gmfit.h -- C ABI of libgmfit.so: batched Levenberg-Marquardt fitting of
 * parametric 2D galaxy light profiles on an AMD Instinct MI355X (gfx950).
 *
 * The fitting problem is the one of Chen, de Souza et al., "galmoss"
 * (arXiv:2404.07780), Sec. 2: per galaxy a start vector p = {p_G, p_L}, a data
 * image D, a sigma image, a mask and a PSF image; a model image is built from
 * radial profiles, convolved with the PSF, a flat sky is added, and chi^2 with
 * the mask is minimised.  Outputs are the fitted parameters, model images and
 * covariance errors (Sec. 5.2).  The paper fits by gradient descent; this
 * library fits by Levenberg-Marquardt (named in Sec. 5.1 as the alternative).
 *
 * Conventions shared by every entry point
 *  - Pixel (row i, column j) of an H x W cutout has centre
 *    (x, y) = (j + 0.5, H - i - 0.5): y grows upwards (Appendix C grid).
 *    Images are row-major FP32.
 *  - Parameters are FP64 in natural units: pixels for centres and scales,
 *    magnitudes (zero point gm_model.m0), position angles in degrees measured
 *    from +x towards +y, counts per pixel for sky and amplitudes.
 *  - A batch is ragged: galaxy g owns pixels [img_off[g], img_off[g] + h*w) of
 *    data/sigma/omega/model_out and a K x K PSF (K odd) at psf[psf_off[g]].
 *    Size metadata (h, w, img_off, psf_k, psf_off) lives in HOST memory; pixel,
 *    PSF, parameter and result arrays live in DEVICE memory owned by the caller.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = default
 *    stream) and returns 0 (GM_OK) or a negative GM_E* code; per-galaxy outcomes
 *    never fail a call.  On an error return nothing has been enqueued, except
 *    GM_EHIP, which reports a failed HIP call.
 *  - One gm_ctx per host thread; calls on one context are serialised by the
 *    caller.  The context owns a grow-only device workspace, reused across calls.
 */
#ifndef GMFIT_H
#define GMFIT_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GM_OK = 0,
    GM_EINVAL = -1,       /* bad argument: sizes, even K, unknown profile, p out of range */
    GM_EHIP = -2,         /* a HIP runtime call failed */
    GM_ENOMEM = -3,       /* workspace allocation failed */
    GM_EUNSUPPORTED = -4  /* valid model that no compiled kernel covers */
};

/* Per-galaxy fit status (gm_fit_batch status_out). */
enum {
    GM_ST_CONVERGED = 0,  /* Gauss-Newton step below step_tol in units of the covariance errors */
    GM_ST_MAXITER = 1,    /* max_iter trials used */
    GM_ST_STALLED = 2,    /* damping exceeded 1e9 */
    GM_ST_NONFINITE = 3,  /* chi^2 at the start vector is not finite */
    GM_ST_TEAM_TIMEOUT = 4 /* a fit shared by several workgroups lost a member (gm_schedule.team):
                              a wait passed its limit; the parameters are the last accepted point */
};

/* Profile types (Sec. 4): natural parameter slots of each, in order
 *   GM_SERSIC   x0 y0 mag r_e n q pa B      Sec. 4.1, eqs. (sersic-intensity), (sersicLtot);
 *               B: boxiness of eq. (r) (0 = ellipse; the generalised radius
 *               (|X|^(B+2) + |Y/q|^(B+2))^(1/(B+2)) and r_box of eq. (rbox)
 *               otherwise), fitted within [-0.9, 2]; a model whose B is free
 *               or fixed at a value other than 0 runs for a single Sersic with
 *               a flat sky (or none) only
 *   GM_EXPDISK  x0 y0 mag r_s q pa          Sec. 4.2.1, eqs. (expdisk_I), (expdiskI0)
 *   GM_FERRER   x0 y0 mag r_out q pa a b    Sec. 4.2.2 (a, b fixed)
 *   GM_KING     x0 y0 I0 r_c r_t q pa alpha Sec. 4.2.3 (alpha fixed)
 *   GM_GAUSSIAN x0 y0 I0 fwhm q pa          Sec. 4.2.4
 *   GM_MOFFAT   x0 y0 mag fwhm q pa beta    Sec. 4.2.5 (beta fixed)
 *   GM_SKY      sky                         Sec. 4.2.6, added after convolution
 *   GM_SKYPLANE sky kx ky                   Appendix D, eq. (new_sky_I): the tilted-plane
 *               sky + kx (x - W/2) + ky (y - H/2) about the cutout's centre, added after
 *               convolution (compiled with a single Sersic; other models GM_EUNSUPPORTED)
 * Every profile other than the Sersic has boxiness 0 (r_box = 1, eq. (rbox)). */
enum { GM_SERSIC = 1, GM_EXPDISK, GM_FERRER, GM_KING, GM_GAUSSIAN, GM_MOFFAT, GM_SKY, GM_SKYPLANE };

typedef struct {
    int32_t type;             /* GM_SERSIC ... GM_SKY */
    int32_t convolve;         /* 1: convolved with the PSF; 0: point source / sky (Appendix C) */
    int32_t param_index[8];   /* slot -> column of the galaxy's parameter vector, -1 = fixed;
                                 one column in several slots ties them (shared centre) */
    double fixed[8];          /* value of every fixed slot (shape constants always fixed) */
} gm_component;

typedef struct {
    int32_t n_comp;           /* 1..4 */
    gm_component comp[4];
    int32_t p;                /* length of each galaxy's parameter vector, 1..16 */
    double m0;                /* magnitude zero point (22.5 in the paper's examples) */
    int32_t oversample;       /* sub-samples per pixel side in the central window (10), 1..16; 1 = off */
    int32_t os_window;        /* side of the central window in pixels (5); 0, or odd and <= 5 */
} gm_model;

typedef struct {
    int32_t n_gal;
    const int32_t *h, *w;     /* HOST [n_gal] cutout sizes, 1..1024 */
    const int64_t *img_off;   /* HOST [n_gal] pixel offsets into data/sigma/omega/model_out */
    const int32_t *psf_k;     /* HOST [n_gal] odd PSF side */
    const int64_t *psf_off;   /* HOST [n_gal] offsets into psf */
    const float *data;        /* DEVICE pixels D */
    const float *sigma;       /* DEVICE pixels sigma (> 0 and finite to be used) */
    const uint8_t *omega;     /* DEVICE pixels mask, 1 = use (Sec. 5.1 Omega); NULL = all used */
    const float *psf;         /* DEVICE PSF kernels, used as given (not renormalised) */
} gm_batch;

typedef struct {
    int32_t max_iter;         /* trials per galaxy (100) */
    double lambda0;           /* initial damping (1e-3) */
    double step_tol;          /* stop when max_k |GN step_k| / sigma_k < step_tol (1e-4) */
    const int32_t *active;    /* DEVICE [n_gal] or NULL: galaxies with active[g] == 0 are
                                 skipped and their outputs left untouched */
    int32_t proposal_max_iter;  /* gm_fit_learned: trials of the LM from the learned start
                                   before the fallback (0 = max_iter) */
    double *err_out;          /* DEVICE [n_gal][p] or NULL: covariance errors at the fit, the
                                 values gm_param_errors gives at the fitted (canonical)
                                 parameters, from the normal matrix of the last accepted
                                 evaluation (no extra evaluation).  Where a component with
                                 a fixed scale is put in canonical form, they are the
                                 errors of the fitted model in the canonical variables. */
} gm_fit_opts;

typedef struct gm_ctx gm_ctx;

/* Create a context on HIP device `hip_device`.  Returns GM_EINVAL for a bad
 * device, GM_EHIP if the device cannot be used. */
int gm_create(gm_ctx **out, int hip_device);
/* Release the context and its workspace (waits for its work to finish). */
void gm_destroy(gm_ctx *ctx);
/* Static text for a GM_* return code. */
const char *gm_error_string(int code);

/* Model image (Sec. 2): M = PSF (x) sum(convolved components)
 * + sum(unconvolved components) + sky, with zero padding and "same" size,
 * at params [n_gal][p] (device).  model_out: device FP32 at img_off. */
int gm_model_image(gm_ctx *ctx, const gm_model *model, const gm_batch *batch,
                   const double *params, float *model_out, void *stream);

/* Jacobian dM/dp_k of the model image for every column k of the parameter
 * vector (natural units: per px, per mag, per degree, ...).  jac_out: device
 * FP32, galaxy g's [p][h][w] block starts at p * img_off[g]. */
int gm_jacobian(gm_ctx *ctx, const gm_model *model, const gm_batch *batch,
                const double *params, float *jac_out, void *stream);

/* Launch schedule of the fitting and error kernels (their workgroup shapes
 * are fixed: 256 threads on 32 x 32 output tiles):
 *   plane_groups -- how many groups the light and derivative planes of one
 *     model evaluation are split into, each group evaluated and convolved in
 *     one pass through LDS (fewer groups: less re-evaluation of the profile,
 *     more LDS per workgroup); 0 = the library's default;
 *   wg_per_cu -- persistent workgroups per compute unit, at most as many as
 *     are resident; 0 = as many as are resident;
 *   team -- workgroups per fit (the paper's Sec. 7 notes that small batches
 *     leave the GPU idle): the G workgroups of a fit share each model
 *     evaluation, tile by tile, and the leader adds their FP64 partial sums
 *     in a fixed order before the LM step (results then differ from one
 *     workgroup's in the last bits of the sums, the fit itself is the same
 *     method).  0 = automatic: when a launch has fewer fits than resident
 *     workgroups, each fit gets min(32, resident / fits, its tiles); 1 = one
 *     workgroup per fit; k > 1 = min(k, tiles) workgroups for every fit of at
 *     least team_min_tiles 32 x 32 tiles, one for the others;
 *   team_min_tiles -- see team (0 = 1);
 *   team_wait_us -- bound of every wait between the workgroups of a team, in
 *     microseconds (0 = 20 s); a fit whose team passes it ends with
 *     GM_ST_TEAM_TIMEOUT (the waits always end: a team's workgroups are
 *     resident together). */
typedef struct {
    int32_t plane_groups;
    int32_t wg_per_cu;
    int32_t team;
    int32_t team_min_tiles;
    int32_t team_wait_us;
} gm_schedule;

/* Use `sched` for models of the same family as `model` whose batches have
 * PSF side psf_k (0: any side without a schedule of its own).  GM_EUNSUPPORTED
 * if the family has no compiled variant with that many plane groups; a
 * variant whose LDS does not fit a batch's PSF side falls back to the default. */
int gm_set_schedule(gm_ctx *ctx, const gm_model *model, int32_t psf_k, const gm_schedule *sched);

/* The plane-group counts compiled for the family of `model` that fit LDS at
 * PSF side psf_k (odd), preferred first: up to cap into plane_groups_out, the
 * total count into n_out.  Needs no device. */
int gm_schedule_options(const gm_model *model, int32_t psf_k, int32_t *plane_groups_out, int32_t cap,
                        int32_t *n_out);

/* Adjoint of gm_model_image (the vector-Jacobian product used by gradient-based
 * fitters such as the paper's, Sec. 5.1): grad_params_out[g][c] =
 * sum over pixels of dM/dp_c (natural units, as gm_jacobian) times
 * grad_image at the same pixel.  grad_image: device FP32 in the image layout;
 * grad_params_out: device [n_gal][p] (columns of fixed slots are 0). */
int gm_model_vjp(gm_ctx *ctx, const gm_model *model, const gm_batch *batch,
                 const double *params, const float *grad_image, double *grad_params_out,
                 void *stream);

/* Moment-based start vector (replaces the SExtractor start values of Sec. 3):
 * border-frame sky, flux-weighted centroid and second moments of the pixels
 * 3 sigma above it.  params_out: device [n_gal][p]; moments_out (nullable):
 * device [n_gal][6] = {x_c - W/2, y_c - H/2, mag, ln r, q, theta_rad}. */
int gm_default_guess(gm_ctx *ctx, const gm_model *model, const gm_batch *batch,
                     double *params_out, double *moments_out, void *stream);

/* Levenberg-Marquardt fit of every galaxy from params_inout (device
 * [n_gal][p], natural units), minimising chi^2 = sum Omega (D - M)^2 / sigma^2
 * (Sec. 5.1, eq. (chinu)).  On return params_inout holds the fit in canonical
 * form (q <= 1, PA in [0, 180)), chi2_out [n_gal] its chi^2, niter_out the
 * trials used, status_out a GM_ST_* code (all device arrays). */
int gm_fit_batch(gm_ctx *ctx, const gm_model *model, const gm_batch *batch,
                 const gm_fit_opts *opts, double *params_inout, double *chi2_out,
                 int32_t *niter_out, int32_t *status_out, void *stream);

/* gm_fit_batch for callers that cannot allocate (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels,
 * one workgroup per fit (gm_schedule.team does not apply), with results bit
 * for bit those of gm_fit_batch under team = 1, and the per-call device
 * metadata (sizes, fit order, work-queue counter) in a fixed device array of
 * the library (about 4 MB per GPU, held until the process ends) instead of
 * the context's grow-only workspace.  No hipMalloc, hipFree or host pinned allocation is made; the
 * host size arrays of the batch are copied to the device with
 * hipMemcpyAsync on `stream` (pageable source: the runtime has copied it
 * when the call returns).  The context must exist (gm_create, which resolves
 * the array on its device).  Galaxies are fitted in index order rather than
 * largest first (same per-galaxy results, other load balance).  At most
 * GM_NOALLOC_MAX_GAL galaxies (GM_EINVAL beyond).  Every call on one GPU uses
 * that GPU's array: calls that overlap in time on one GPU (other streams,
 * other contexts, other host threads) race and must be serialised by the
 * caller; stream-ordered calls on one stream are safe. */
#define GM_NOALLOC_MAX_GAL 65536
int gm_fit_batch_noalloc(gm_ctx *ctx, const gm_model *model, const gm_batch *batch,
                         const gm_fit_opts *opts, double *params_inout, double *chi2_out,
                         int32_t *niter_out, int32_t *status_out, void *stream);

/* Covariance errors sigma_p = sqrt(diag (J^T W J)^-1), W = Omega / sigma^2
 * (Sec. 5.2), unscaled, in natural units at params (device [n_gal][p]).
 * err_out: device [n_gal][p]; cov_out (nullable): device [n_gal][p][p].
 * A galaxy whose J^T W J is not positive definite gets NaN errors. */
int gm_param_errors(gm_ctx *ctx, const gm_model *model, const gm_batch *batch,
                    const double *params, double *err_out, double *cov_out, void *stream);

/* The paper's own fitter (Sec. 5.1: gradient descent; Adam in its examples)
 * on the same model evaluation: Adam (Kingma and Ba 2015) on chi^2 in the LM
 * variables (ln of scales and of n, radians for PA), gradient -2 J^T W r,
 * `steps` steps of rate lr with bias-corrected moments (beta1, beta2, eps),
 * the iterate clamped to the LM bounds after each step, fixed slots
 * untouched; no convergence test.  params_inout as for gm_fit_batch
 * (canonical form on return); chi2_out: chi^2 at the final parameters;
 * status_out: GM_ST_MAXITER (all steps taken) or GM_ST_NONFINITE. */
typedef struct {
    int32_t steps;            /* Adam steps per galaxy (the paper's examples: 1000) */
    double lr, beta1, beta2, eps;
} gm_adam_opts;

int gm_fit_adam(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_adam_opts *opts,
                double *params_inout, double *chi2_out, int32_t *status_out, void *stream);

/* Bootstrap errors (Sec. 5.2: each galaxy image resampled with replacement,
 * typically 100 times, and refitted; sigma^2 = (1/M) sum (m_i - mean)^2).
 * The resampling of the pixels with replacement is taken in its limit for
 * many pixels, independent Poisson(1) pixel weights (the Poisson bootstrap).  Replica r of galaxy g multiplies
 * every pixel weight Omega / sigma^2 by w ~ Poisson(1): w = the number of
 * thresholds T_k <= x, T_k = floor(2^32 F(k)) for k = 0..11 with
 * F(k) = e^-1 sum_{j<=k} 1/j! summed in that order in FP64, x the word
 * (pixel mod 4) of Philox4x32-10 (Salmon et al. 2011) keyed by (seed low
 * word, seed high word) with counter {pixel / 4, g, r, 1} (pixel: row-major
 * index in the cutout).  Every replica is fitted by LM from params (device
 * [n_gal][p], normally the fit) with opts (opts->active and err_out are
 * ignored).  err_out (device [n_gal][p]): sigma with sigma^2 = (1/M) sum
 * (p_r - mean)^2 over the M replicas that end GM_ST_CONVERGED (Sec. 5.2),
 * position angles as differences from params wrapped into (-90, 90]; NaN
 * with fewer than two.  rep_params_out
 * (nullable, device [n_gal][n_boot][p]), rep_status_out and rep_niter_out
 * (nullable, device [n_gal][n_boot]) receive the replica fits.  2 <= n_boot, n_gal n_boot <=
 * 2^30; the replicas share the galaxies' pixels (nothing is copied). */
int gm_bootstrap(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_fit_opts *opts,
                 const double *params, int32_t n_boot, uint64_t seed, double *err_out,
                 double *rep_params_out, int32_t *rep_status_out, int32_t *rep_niter_out,
                 void *stream);

/* ------------------------------------------------------------------------
 * Learned proposal.  The paper motivates learned parameter estimators
 * (Sec. 1) and names the hand-chosen initial parameters as a limitation of
 * its fitter (Sec. 7); it fixes no network, so what follows is this
 * library's design.
 *
 * Features (1056 per galaxy, BF16): with the image moments of
 * gm_default_guess (sky0, F0, centroid x_c y_c, m_g, r0, q0, theta0) and
 * F0' = max(F0, 1), 1024 area-weighted cells -- cell (a, b) covers rows
 * [a H/32, (a+1) H/32) and columns [b W/32, (b+1) W/32); its value is the mean
 * of D - sky0 over its usable area times the cell area H W / 1024, scaled by
 * 32 / F0' (0 if nothing is usable) -- then (x_c - W/2)/2, (y_c - H/2)/2,
 * (m_g - 14)/2, ln r0 - 1.5, e0 cos 2 theta0, e0 sin 2 theta0 with
 * e0 = (1 - q0)/(1 + q0), then 26 zeros.
 *
 * Targets (the first 7 outputs; the rest are 0) of a single Sersic + sky:
 * x0 - x_c, y0 - y_c, (mag - m_g)/0.5, (ln re - 1.7)/0.6, (ln n - 0.6)/0.6,
 * e cos 2 pa / 0.3, e sin 2 pa / 0.3 with e = (1 - q)/(1 + q).  Decoding
 * inverts them with e capped at 0.9 and sky = sky0; a proposal is valid when
 * finite and inside the LM bounds (0 <= x0 <= W, 0 <= y0 <= H,
 * 0.1 <= re <= 2 max(H, W), 0.2 <= n <= 10).
 *
 * Network: n_hidden layers of `hidden` units with the exact-erf GELU, then a
 * linear layer of out_dim outputs of which the first n_out enter the loss.
 * Parameters are one flat FP32 vector, layer by layer W_l [out][in]
 * (row-major) then b_l [out]; products use the BF16 copy of the weights, BF16
 * activations and FP32 accumulation.  Loss: the mean over rows and the n_out
 * used outputs of the squared error.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t in_dim;           /* 1056 for the proposal; multiples of 8 throughout */
    int32_t hidden;           /* 512 */
    int32_t n_hidden;         /* 3 (1..16) */
    int32_t out_dim;          /* 16 */
    int32_t n_out;            /* 7 outputs enter the loss and the decoding */
    float *params;            /* DEVICE FP32 master parameters (gm_mlp_param_count) */
    uint16_t *params_bf16;    /* DEVICE BF16 copy, same layout, 16-byte aligned */
    float *grad;              /* DEVICE gradient, same layout (training only) */
    float *adam_m, *adam_v;   /* DEVICE AdamW moments, same layout (training only) */
} gm_mlp;

typedef struct {
    double lr, beta1, beta2, eps, weight_decay;
} gm_adamw;

/* Number of parameters of the network's sizes, -1 if they are invalid. */
int64_t gm_mlp_param_count(const gm_mlp *mlp);

/* params_bf16 <- BF16(params), round to nearest even. */
int gm_mlp_sync(gm_ctx *ctx, const gm_mlp *mlp, void *stream);

/* out [n][out_dim] (device FP32) for x [n][ldx] (device BF16, ldx >= in_dim,
 * a multiple of 8, 16-byte aligned). */
int gm_mlp_forward(gm_ctx *ctx, const gm_mlp *mlp, int32_t n, const uint16_t *x, int64_t ldx,
                   float *out, void *stream);

/* Gradient of the loss over rows[0..n) of x and targets (device; rows NULL =
 * the first n rows, else every entry must index a row of both x and targets;
 * targets [.][out_dim] FP32) into mlp->grad; loss_out (device FP64, nullable)
 * receives the loss. */
int gm_mlp_backward(gm_ctx *ctx, const gm_mlp *mlp, int32_t n, const uint16_t *x, int64_t ldx,
                    const int32_t *rows, const float *targets, double *loss_out, void *stream);

/* One AdamW step (Loshchilov and Hutter: decoupled weight decay, bias-corrected
 * moments; step counts from 1) from mlp->grad; refreshes params_bf16. */
int gm_mlp_adamw(gm_ctx *ctx, const gm_mlp *mlp, int64_t step, const gm_adamw *opt, void *stream);

/* gm_mlp_backward then gm_mlp_adamw. */
int gm_mlp_train_step(gm_ctx *ctx, const gm_mlp *mlp, int32_t n, const uint16_t *x, int64_t ldx,
                      const int32_t *rows, const float *targets, int64_t step, const gm_adamw *opt,
                      double *loss_out, void *stream);

/* One product of the dense layers' matrix-core kernels in FP32, without the
 * layer epilogues (bias, GELU): C [m][n] (device FP32, pitch ldc >= n)
 * = op(A) op(B) summed over k, from BF16 operands (device, every row
 * 16-byte aligned, pitches multiples of 8):
 *   GM_GEMM_NT  C = A B^T, A [m][lda >= k], B [n][ldb >= k], k a multiple
 *               of 8: the forward product X W^T; a_rows (nullable, device
 *               int32 [m]) takes row a_rows[i] of A as row i (the mini-batch
 *               gather);
 *   GM_GEMM_NN  C = A B,   A [m][lda >= k] (k a multiple of 8, a_rows as
 *               for NT), B [k][ldb >= n] (n a multiple of 8): the backward
 *               product dZ W;
 *   GM_GEMM_TN  C = A^T B, A [k][lda >= m], B [k][ldb >= n] (m and n
 *               multiples of 8); b_rows (nullable, device int32 [k]) takes
 *               row b_rows[i] of B as row i: the weight gradient dZ^T X,
 *               computed in K splits whose partial sums are added in a fixed
 *               order (results do not depend on timing).
 * Unused row maps must be NULL; GM_EINVAL otherwise and for sizes or
 * pitches out of these rules.  Used by gm_mlp_forward, gm_mlp_backward and
 * the tests of the products. */
enum { GM_GEMM_NT = 0, GM_GEMM_NN = 1, GM_GEMM_TN = 2 };
int gm_mlp_gemm(gm_ctx *ctx, int32_t op, int32_t m, int32_t n, int32_t k, const uint16_t *a, int64_t lda,
                const int32_t *a_rows, const uint16_t *b, int64_t ldb, const int32_t *b_rows, float *c,
                int64_t ldc, void *stream);

/* Features of every galaxy: x_out [n_gal][ldx] BF16 (device, ldx >= 1056, a
 * multiple of 8); moments_out (device, nullable) [n_gal][8] =
 * {sky0, F0, x_c, y_c, m_g, r0, q0, theta0_rad}.  Any model (m0 is used). */
int gm_features(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, uint16_t *x_out,
                int64_t ldx, double *moments_out, void *stream);

/* Targets [n_gal][out_dim] (device FP32) of the truths (device [n_gal][p]) of
 * a single-Sersic + sky model whose 8 slots are all columns (else
 * GM_EUNSUPPORTED); moments from gm_features. */
int gm_proposal_targets(gm_ctx *ctx, const gm_model *model, const gm_batch *batch,
                        const double *truth, const double *moments, float *targets_out,
                        int32_t out_dim, void *stream);

/* Decode network outputs [n_gal][out_dim] into start vectors params_out
 * [n_gal][p] and valid_out [n_gal] (1 = usable), same model restriction. */
int gm_proposal_decode(gm_ctx *ctx, const gm_model *model, const gm_batch *batch,
                       const float *out, int32_t out_dim, const double *moments,
                       double *params_out, int32_t *valid_out, void *stream);

/* LM from the network's proposal with the moment-based guess as fallback:
 * galaxies whose proposal is invalid, or whose LM from it does not end
 * GM_ST_CONVERGED within opts->proposal_max_iter trials, are refitted from
 * gm_default_guess (with opts->max_iter trials) by the same workgroup of the
 * same launch; their reported result is the refit and niter_out counts the
 * trials of both fits.  fallback_out (device, nullable) [n_gal]: 0 = fitted
 * from the proposal, 1 = proposal invalid, 2 = LM from the proposal did not
 * converge (refitted).  events (nullable): four hipEvent_t recorded on the
 * stream before the moment guess, before and after the LM launch, and at the
 * end (profiling).  opts->active is ignored.  Same model restriction as
 * gm_proposal_decode. */
int gm_fit_learned(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_mlp *mlp,
                   const gm_fit_opts *opts, double *params_out, double *chi2_out,
                   int32_t *niter_out, int32_t *status_out, int32_t *fallback_out,
                   void *const *events, void *stream);

/* Training images: data_out = F unit + sky + sigma z per galaxy, with unit a
 * noiseless unit-flux model image (device FP32 at img_off, host sizes),
 * F = snr sigma / max(unit) so that snr is the peak signal-to-noise ratio,
 * and z standard normal from Philox4x32-10 (Salmon et al. 2011) keyed by
 * seed, counter {pixel/4, first_index + g (64 bit), 0}, Box-Muller on word
 * pairs.  sigma_out (nullable) is filled with sigma; mag_out (nullable)
 * [g * mag_stride] = m0 - 2.5 log10 F.  snr, sky: device [n_gal] FP64. */
int gm_synth_noise(gm_ctx *ctx, int32_t n_gal, const int32_t *h, const int32_t *w,
                   const int64_t *img_off, const float *unit, const double *snr, const double *sky,
                   float sigma, double m0, uint64_t seed, int64_t first_index, float *data_out,
                   float *sigma_out, double *mag_out, int32_t mag_stride, void *stream);

/* ------------------------------------------------------------------------
 * Captured plans.  A plan records one call sequence on a fixed batch into a
 * HIP graph: the host work of the calls (model matching, schedule choice,
 * size metadata, the cost order of the work queue) is done once, at
 * creation, into device memory the plan owns, and every gm_plan_launch
 * replays only the kernels -- it allocates nothing and copies nothing from
 * the host.  The plan keeps every device pointer it was given (pixels, PSFs,
 * start vectors, network weights, outputs): the caller keeps those buffers
 * alive until gm_plan_destroy and may change their contents between
 * launches; the host size metadata is read at creation only.  A plan uses
 * the schedule its context had at creation.  Launches of one plan must be
 * ordered (one stream, or synchronised): they share the plan's workspace.
 * The kernels and arithmetic are those of the eager calls, so a launch gives
 * the same results bit for bit.  On failure *out is NULL and nothing stays
 * allocated.  Creation synchronises with the device; n_gal must be >= 1.
 * ---------------------------------------------------------------------- */
typedef struct gm_plan gm_plan;

/* params_out <- start (device [n_gal][p]; NULL: the moment-based guess of
 * gm_default_guess), then gm_fit_batch with the covariance errors at the fit
 * in err_out (nullable; gm_fit_opts.err_out is ignored).  timing != 0: the
 * plan records four events of its own as graph nodes -- before the start,
 * before and after the LM launch, at the end -- read with gm_plan_elapsed. */
int gm_plan_fit(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_fit_opts *opts,
                const double *start, double *params_out, double *chi2_out, int32_t *niter_out,
                int32_t *status_out, double *err_out, int32_t timing, gm_plan **out);

/* gm_fit_learned with the covariance errors at the fit in err_out (nullable;
 * gm_fit_opts.err_out is ignored).  timing != 0: four events as those of
 * gm_fit_learned, read with gm_plan_elapsed. */
int gm_plan_fit_learned(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_mlp *mlp,
                        const gm_fit_opts *opts, double *params_out, double *chi2_out,
                        int32_t *niter_out, int32_t *status_out, int32_t *fallback_out,
                        double *err_out, int32_t timing, gm_plan **out);

/* Replays the plan on `stream` (asynchronous). */
int gm_plan_launch(gm_plan *plan, void *stream);

/* Milliseconds between the plan's consecutive timing events in its latest
 * launch (ms_out[3]); waits for that launch's last event.  GM_EINVAL if the
 * plan was made without timing or has not been launched. */
int gm_plan_elapsed(gm_plan *plan, float *ms_out);

/* Waits for the device, then frees the plan (NULL is ignored). */
void gm_plan_destroy(gm_plan *plan);

#ifdef __cplusplus
}
#endif
#endif
