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
    GM_ST_NONFINITE = 3   /* chi^2 at the start vector is not finite */
};

/* Profile types (Sec. 4): natural parameter slots of each, in order
 *   GM_SERSIC   x0 y0 mag r_e n q pa        Sec. 4.1, eqs. (sersic-intensity), (sersicLtot)
 *   GM_EXPDISK  x0 y0 mag r_s q pa          Sec. 4.2.1, eqs. (expdisk_I), (expdiskI0)
 *   GM_FERRER   x0 y0 mag r_out q pa a b    Sec. 4.2.2 (a, b fixed)
 *   GM_KING     x0 y0 I0 r_c r_t q pa alpha Sec. 4.2.3 (alpha fixed)
 *   GM_GAUSSIAN x0 y0 I0 fwhm q pa          Sec. 4.2.4
 *   GM_MOFFAT   x0 y0 mag fwhm q pa beta    Sec. 4.2.5 (beta fixed)
 *   GM_SKY      sky                         Sec. 4.2.6, added after convolution
 * Boxiness is 0 (r_box = 1, eq. (rbox)). */
enum { GM_SERSIC = 1, GM_EXPDISK, GM_FERRER, GM_KING, GM_GAUSSIAN, GM_MOFFAT, GM_SKY };

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
    int32_t oversample;       /* sub-samples per pixel side in the central window (10); 1 = off */
    int32_t os_window;        /* side of the central window in pixels (5); odd, <= 7 */
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

/* Covariance errors sigma_p = sqrt(diag (J^T W J)^-1), W = Omega / sigma^2
 * (Sec. 5.2), unscaled, in natural units at params (device [n_gal][p]).
 * err_out: device [n_gal][p]; cov_out (nullable): device [n_gal][p][p].
 * A galaxy whose J^T W J is not positive definite gets NaN errors. */
int gm_param_errors(gm_ctx *ctx, const gm_model *model, const gm_batch *batch,
                    const double *params, double *err_out, double *cov_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif
