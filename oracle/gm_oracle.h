/*
 * gm_oracle.h -- FP64 CPU oracle for batched galaxy-profile fitting.
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product library.
 */
#ifndef GM_ORACLE_H
#define GM_ORACLE_H
#include <stdint.h>

#define ORC_MAX_COMP 4
#define ORC_MAX_SLOTS 8
#define ORC_MAX_P 16

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ESINGULAR = -3 };
enum { ORC_SERSIC = 1, ORC_EXPDISK, ORC_FERRER, ORC_KING, ORC_GAUSSIAN, ORC_MOFFAT, ORC_SKY, ORC_SKYPLANE };
enum { ORC_ST_CONVERGED = 0, ORC_ST_MAXITER = 1, ORC_ST_STALLED = 2, ORC_ST_NONFINITE = 3 };

/* One component.  Natural slots per type (PA in degrees):
 *   SERSIC   x0 y0 mag r_e n q pa box    (box: B of eq. (r); 0 = ellipse)
 *   EXPDISK  x0 y0 mag r_s q pa
 *   FERRER   x0 y0 mag r_out q pa a b          (a, b fixed or free)
 *   KING     x0 y0 I0 r_c r_t q pa alpha       (alpha fixed or free)
 *   GAUSSIAN x0 y0 I0 fwhm q pa
 *   MOFFAT   x0 y0 mag fwhm q pa beta          (beta always fixed)
 *   SKY      sky
 *   SKYPLANE sky kx ky: the tilted-plane sky of Appendix D, eq. (new_sky_I),
 *            I = sky + kx (x - W/2) + ky (y - H/2) about the cutout's
 *            geometric centre (pixel grid of Appendix C, y up); unconvolved
 * idx[s] is the column of the galaxy's parameter vector that holds slot s,
 * or -1 if the slot is fixed at fixed[s]; a column shared by several slots
 * ties them. */
typedef struct {
    int32_t type, convolve;
    int32_t idx[ORC_MAX_SLOTS];
    double fixed[ORC_MAX_SLOTS];
} orc_comp;

typedef struct {
    int32_t ncomp;
    orc_comp comp[ORC_MAX_COMP];
    int32_t p;
    double m0;               /* magnitude zero point */
    int32_t oversample;      /* sub-samples per pixel side (10); <= 1 disables */
    int32_t os_window;       /* side of the oversampled window in pixels (5) */
} orc_model;

typedef struct {
    int32_t max_iter;
    double lambda0, step_tol;
} orc_lm_opts;

/* Adam (Kingma and Ba 2015) on chi^2: steps, learning rate, moment decays, eps. */
typedef struct {
    int32_t steps;
    double lr, beta1, beta2, eps;
} orc_adam_opts;

double orc_digamma(double x);
double orc_gammainc_p(double a, double x);
double orc_dgammainc_p_da(double a, double x);
double orc_sersic_b(double n);
double orc_sersic_db(double n);
int orc_slot_kind(int type, int slot);
int orc_validate(const orc_model *m);
void orc_convolve(int h, int w, const double *in, int k, const double *psf, double *out);
void orc_canonicalise(const orc_model *m, double *params);
int orc_profile_point(const orc_model *m, int comp, const double *params, double x, double y,
                      double *I, double *dI);
int orc_model_image(const orc_model *m, int h, int w, const float *psf, int k,
                    const double *params, double *out);
int orc_jacobian(const orc_model *m, int h, int w, const float *psf, int k,
                 const double *params, double *jac);
int orc_fit(const orc_model *m, int h, int w, const float *data, const float *sigma,
            const uint8_t *omega, const float *psf, int k, const orc_lm_opts *o,
            double *params, double *chi2, int *niter, int *status);
int orc_fit_adam(const orc_model *m, int h, int w, const float *data, const float *sigma,
                 const uint8_t *omega, const float *psf, int k, const orc_adam_opts *o,
                 double *params, double *chi2, int *status);
int orc_fit_adam_batch(const orc_model *m, int n_gal, const int32_t *h, const int32_t *w,
                       const int64_t *img_off, const float *data, const float *sigma,
                       const uint8_t *omega, const int32_t *psf_k, const int64_t *psf_off,
                       const float *psf, const orc_adam_opts *o, double *params, double *chi2,
                       int32_t *status, int nthreads);
int orc_param_errors(const orc_model *m, int h, int w, const float *data, const float *sigma,
                     const uint8_t *omega, const float *psf, int k, const double *params,
                     double *err, double *cov);
void orc_moments(int h, int w, const float *data, const float *sigma, const uint8_t *omega, double m0,
                 double *out);
int orc_default_guess(const orc_model *m, int h, int w, const float *data, const float *sigma,
                      const uint8_t *omega, double *params, double *mom);
int orc_fit_batch(const orc_model *m, int n_gal, const int32_t *h, const int32_t *w,
                  const int64_t *img_off, const float *data, const float *sigma,
                  const uint8_t *omega, const int32_t *psf_k, const int64_t *psf_off,
                  const float *psf, const orc_lm_opts *o, double *params, double *chi2,
                  int32_t *niter, int32_t *status, int nthreads);
#endif
