/*
 * gm_oracle.c -- plain, slow FP64 CPU oracle for batched Levenberg-Marquardt
 * fitting of parametric 2D galaxy light profiles (Chen, de Souza et al.,
 * "galmoss", arXiv:2404.07780).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header or table with the
 * HIP path.
 *
 * Everything is double precision and written for readability: every pixel of
 * every derivative image is materialised, the convolution is the four-nested
 * loop of its definition, and the normal equations are summed pixel by pixel.
 *
 * What each part follows (paper section / equation):
 *   - pixel grid: Appendix C (grid built from linspace(0.5, W-0.5) in x and
 *     linspace(H-0.5, 0.5) in y, so y grows upwards);
 *   - elliptical radius: Sec. 4.1, eqs. (r), (rmaj), (rmin) with boxiness B=0;
 *     coordinates are rotated before squaring (absolute values vanish at B=0);
 *   - Sersic profile and its magnitude normalisation: Sec. 4.1, eqs.
 *     (sersic-intensity), (sersicLtot), (rbox) with r_box = 1 at B = 0;
 *     nu_n solves the half-light condition P(2n, nu_n) = 1/2;
 *   - exponential disk: Sec. 4.2.1, eqs. (expdisk_I), (expdiskI0);
 *   - modified Ferrer: Sec. 4.2.2, eqs. (ferrer_I), (ferrerI0), zero beyond r_out;
 *   - empirical King: Sec. 4.2.3, eq. (BE_S), read with the two terms of the
 *     second bracket swapped so that I(0) = I0 and I(r_t) = 0, zero beyond r_t;
 *   - Gaussian: Sec. 4.2.4, eq. (gaussion_I), FWHM = 2 sqrt(2 ln 2) sigma;
 *   - Moffat: Sec. 4.2.5, eqs. (moffat_I), (moffat_rd), (moffatI0);
 *   - flat sky: Sec. 4.2.6, eq. (sky_I), added after the convolution (Sec. 2);
 *   - PSF convolution with zero padding and "same" output size: Sec. 2 and
 *     Appendix C (written here as a true convolution; point sources and sky are
 *     not convolved);
 *   - chi^2 with mask and sigma: Sec. 5.1, eq. (chinu);
 *   - covariance errors sqrt(diag (J^T W J)^-1): Sec. 5.2;
 *   - Levenberg-Marquardt: the paper names it (Sec. 5.1, Sec. 5.2) but fixes no
 *     constants; the textbook damped Gauss-Newton scheme of Levenberg (1944)
 *     and Marquardt (1963) is used with the constants listed at orc_fit().
 * The x10 sub-pixel oversampling in the central 5x5 pixels is not in the paper;
 * its rule is stated at oversample_window().
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "gm_oracle.h"

#define ORC_PI 3.14159265358979323846
#define ORC_LN10 2.30258509299404568402

/* ------------------------------------------------------------------------ */
/* Special functions                                                        */
/* ------------------------------------------------------------------------ */

/* Digamma psi(x) for x > 0: shift upwards with psi(x) = psi(x+1) - 1/x until
 * x >= 10, then the asymptotic (Stirling) series with Bernoulli numbers
 * B2..B14.  Truncation error at x = 10 is below 1e-16. */
double orc_digamma(double x)
{
    double acc = 0.0;
    while (x < 10.0) {
        acc -= 1.0 / x;
        x += 1.0;
    }
    double x2 = 1.0 / (x * x);
    double series = x2 * (1.0 / 12.0
                  - x2 * (1.0 / 120.0
                  - x2 * (1.0 / 252.0
                  - x2 * (1.0 / 240.0
                  - x2 * (1.0 / 132.0
                  - x2 * (691.0 / 32760.0
                  - x2 * (1.0 / 12.0)))))));
    return acc + log(x) - 0.5 / x - series;
}

/* Regularised lower incomplete gamma P(a, x) = gamma(a, x) / Gamma(a).
 * For x < a + 1 the power series
 *     P = x^a e^-x / Gamma(a+1) * sum_k x^k / ((a+1)(a+2)...(a+k));
 * otherwise 1 - Q with Q from its continued fraction (modified Lentz). */
double orc_gammainc_p(double a, double x)
{
    if (x <= 0.0)
        return 0.0;
    double lpre = a * log(x) - x - lgamma(a);
    if (x < a + 1.0) {
        double term = 1.0 / a, sum = term;
        for (int k = 1; k < 100000; ++k) {
            term *= x / (a + k);
            sum += term;
            if (fabs(term) < fabs(sum) * 1e-17)
                break;
        }
        return sum * exp(lpre);
    }
    /* Q(a,x) = e^-x x^a / Gamma(a) * 1/(x+1-a- 1(1-a)/(x+3-a- 2(2-a)/(x+5-a- ...))) */
    const double tiny = 1e-300;
    double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 100000; ++i) {
        double an = -i * (i - a);
        b += 2.0;
        d = an * d + b;
        if (fabs(d) < tiny) d = tiny;
        c = b + an / c;
        if (fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        double del = d * c;
        h *= del;
        if (fabs(del - 1.0) < 1e-17)
            break;
    }
    return 1.0 - exp(lpre) * h;
}

/* dP(a, x)/da from the series P(a,x) = e^-x sum_k x^(a+k) / Gamma(a+k+1):
 *     dP/da = e^-x sum_k x^(a+k) [ln x - psi(a+k+1)] / Gamma(a+k+1),
 * with psi(a+k+1) = psi(a+1) + sum_{j=1..k} 1/(a+j). */
double orc_dgammainc_p_da(double a, double x)
{
    if (x <= 0.0)
        return 0.0;
    double lx = log(x), psi = orc_digamma(a + 1.0), sum = 0.0;
    for (int k = 0; k < 100000; ++k) {
        if (k > 0)
            psi += 1.0 / (a + k);
        double t = exp((a + k) * lx - x - lgamma(a + k + 1.0));
        sum += t * (lx - psi);
        if (k > x + 5.0 && t < 1e-18)
            break;
    }
    return sum;
}

/* nu_n (the b_n of the Sersic law): the half-light condition
 * P(2n, b) = 1/2 (Sec. 4.1: the inverse gamma CDF at one half), solved by
 * Newton's method safeguarded by bisection, to |db| < 1e-14 b. */
double orc_sersic_b(double n)
{
    double a = 2.0 * n;
    double lo = 0.0, hi = a + 20.0;
    double b = a - 1.0 / 3.0 + 4.0 / (405.0 * n);
    if (!(b > lo && b < hi))
        b = 0.5 * a;
    for (int it = 0; it < 200; ++it) {
        double f = orc_gammainc_p(a, b) - 0.5;
        if (f > 0.0) hi = b; else lo = b;
        double fp = exp((a - 1.0) * log(b) - b - lgamma(a));
        double nb = b - f / fp;
        if (!(nb > lo && nb < hi))
            nb = 0.5 * (lo + hi);
        double step = fabs(nb - b);
        b = nb;
        if (step < 1e-14 * b)
            break;
    }
    return b;
}

/* db/dn from implicit differentiation of P(2n, b(n)) = 1/2:
 *     2 dP/da + dP/dx * b' = 0,  dP/dx = b^(a-1) e^-b / Gamma(a). */
double orc_sersic_db(double n)
{
    double a = 2.0 * n, b = orc_sersic_b(n);
    double dpdx = exp((a - 1.0) * log(b) - b - lgamma(a));
    return -2.0 * orc_dgammainc_p_da(a, b) / dpdx;
}

/* ------------------------------------------------------------------------ */
/* Parameter slots                                                          */
/* ------------------------------------------------------------------------ */

/* Kind of each natural parameter slot of each profile type.  The LM works on
 * u: identity for centres, magnitudes, amplitudes, axis ratio and sky; the
 * natural log for every positive scale and for the Sersic index; radians for
 * the position angle (the paper's `log=True` / `angle=True` flags,
 * Appendix A, extended to the other scales). */
enum { K_NONE = 0, K_X0, K_Y0, K_MAG, K_AMP, K_SCALE, K_N, K_Q, K_PA, K_SKY, K_SHAPE, K_SKYGRAD, K_BOX,
       K_FA, K_FB, K_KAL };

static const int slot_kind[9][ORC_MAX_SLOTS] = {
    /* 0 unused */ {0},
    /* SERSIC   */ {K_X0, K_Y0, K_MAG, K_SCALE, K_N, K_Q, K_PA, K_BOX},
    /* EXPDISK  */ {K_X0, K_Y0, K_MAG, K_SCALE, K_Q, K_PA, K_NONE, K_NONE},
    /* FERRER   */ {K_X0, K_Y0, K_MAG, K_SCALE, K_Q, K_PA, K_FA, K_FB},
    /* KING     */ {K_X0, K_Y0, K_AMP, K_SCALE, K_SCALE, K_Q, K_PA, K_KAL},
    /* GAUSSIAN */ {K_X0, K_Y0, K_AMP, K_SCALE, K_Q, K_PA, K_NONE, K_NONE},
    /* MOFFAT   */ {K_X0, K_Y0, K_MAG, K_SCALE, K_Q, K_PA, K_SHAPE, K_NONE},
    /* SKY      */ {K_SKY, K_NONE, K_NONE, K_NONE, K_NONE, K_NONE, K_NONE, K_NONE},
    /* SKYPLANE */ {K_SKY, K_SKYGRAD, K_SKYGRAD, K_NONE, K_NONE, K_NONE, K_NONE, K_NONE},
};

int orc_slot_kind(int type, int slot)
{
    if (type < 1 || type > 8 || slot < 0 || slot >= ORC_MAX_SLOTS)
        return -1;
    return slot_kind[type][slot];
}

/* Kind of parameter column k (the first slot that maps to it). */
static int column_kind(const orc_model *m, int k)
{
    for (int c = 0; c < m->ncomp; ++c)
        for (int s = 0; s < ORC_MAX_SLOTS; ++s)
            if (m->comp[c].idx[s] == k)
                return slot_kind[m->comp[c].type][s];
    return K_NONE;
}

int orc_validate(const orc_model *m)
{
    if (m->ncomp < 1 || m->ncomp > ORC_MAX_COMP || m->p < 1 || m->p > ORC_MAX_P)
        return ORC_EINVAL;
    int seen[ORC_MAX_P] = {0};
    for (int c = 0; c < m->ncomp; ++c) {
        const orc_comp *cp = &m->comp[c];
        if (cp->type < ORC_SERSIC || cp->type > ORC_SKYPLANE)
            return ORC_EINVAL;
        if ((cp->type == ORC_SKY || cp->type == ORC_SKYPLANE) && cp->convolve)
            return ORC_EINVAL;
        for (int s = 0; s < ORC_MAX_SLOTS; ++s) {
            int kind = slot_kind[cp->type][s], k = cp->idx[s];
            if (kind == K_NONE) {
                if (k >= 0) return ORC_EINVAL;
                continue;
            }
            if (k < 0) continue;
            if (k >= m->p || kind == K_SHAPE) return ORC_EINVAL;
            int ck = column_kind(m, k);
            if (ck != kind) return ORC_EINVAL; /* tied slots must be of one kind */
            seen[k] = 1;
        }
    }
    for (int k = 0; k < m->p; ++k)
        if (!seen[k]) return ORC_EINVAL;
    return ORC_OK;
}

/* natural value of every slot of component c */
static void comp_values(const orc_model *m, int c, const double *params, double *v)
{
    const orc_comp *cp = &m->comp[c];
    for (int s = 0; s < ORC_MAX_SLOTS; ++s)
        v[s] = cp->idx[s] >= 0 ? params[cp->idx[s]] : cp->fixed[s];
}

/* natural -> LM variable and back, per column kind (Ferrer a and King alpha,
 * positive shape exponents, through their log like the scales) */
static double to_u(int kind, double p)
{
    switch (kind) {
    case K_SCALE: case K_N: case K_FA: case K_KAL: return log(p);
    case K_PA: return p * ORC_PI / 180.0;
    default: return p;
    }
}
static double from_u(int kind, double u)
{
    switch (kind) {
    case K_SCALE: case K_N: case K_FA: case K_KAL: return exp(u);
    case K_PA: return u * 180.0 / ORC_PI;
    default: return u;
    }
}
/* d(natural)/d(u) */
static double dp_du(int kind, double p)
{
    switch (kind) {
    case K_SCALE: case K_N: case K_FA: case K_KAL: return p;
    case K_PA: return 180.0 / ORC_PI;
    default: return 1.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Profiles at one point                                                    */
/* ------------------------------------------------------------------------ */

/* Per-component scalars that do not depend on the pixel. */
typedef struct {
    int type;
    double v[ORC_MAX_SLOTS];     /* natural slot values */
    double cth, sth, q;          /* orientation (theta in radians) */
    double lnamp;                /* log of the amplitude factor */
    /* Sersic */
    double n, b, db, re;
    /* others */
    double scale, scale2, a_f, b_f, alpha, beta, rd;
    double kA, dkA_dlnrc, dkA_dlnrt;   /* King: T^(-1/alpha) and derivatives */
    double kT;                         /* King: T = 1 + (r_t / r_c)^2 */
    double fc2;                        /* Ferrer: 1 + 2 / (2 - b) */
    double xc, yc;               /* plane sky: the cutout's geometric centre */
    double cbox, dlrbox;         /* Sersic: exponent c = B + 2 of eq. (r), d ln r_box / dc */
} comp_prep;

static void prep_component(const orc_model *m, int c, const double *params, comp_prep *cp)
{
    memset(cp, 0, sizeof *cp);
    cp->type = m->comp[c].type;
    comp_values(m, c, params, cp->v);
    double *v = cp->v;
    if (cp->type == ORC_SKY || cp->type == ORC_SKYPLANE)
        return;
    double th = v[5] * ORC_PI / 180.0;  /* PA slot is 5 for all but Sersic */
    double q = v[4];
    if (cp->type == ORC_SERSIC) { th = v[6] * ORC_PI / 180.0; q = v[5]; }
    if (cp->type == ORC_KING)   { th = v[6] * ORC_PI / 180.0; q = v[5]; }
    cp->cth = cos(th);
    cp->sth = sin(th);
    cp->q = q;
    double lnF = -0.4 * ORC_LN10 * (v[2] - m->m0);  /* ln 10^(-0.4(m-m0)) */
    switch (cp->type) {
    case ORC_SERSIC: {
        double re = v[3], n = v[4], c = v[7] + 2.0;
        cp->re = re; cp->n = n;
        cp->b = orc_sersic_b(n);
        cp->db = orc_sersic_db(n);
        /* eq. (rbox): r_box = pi c / (2 beta(1/c, 1/c)), c = B + 2, beta(a, a) =
         * Gamma(a)^2 / Gamma(2a); d ln r_box / dc = 1/c + 2 (psi(1/c) - psi(2/c)) / c^2 */
        double lnrbox = log(ORC_PI * c / 2.0) - (2.0 * lgamma(1.0 / c) - lgamma(2.0 / c));
        cp->cbox = c;
        cp->dlrbox = 1.0 / c + 2.0 * (orc_digamma(1.0 / c) - orc_digamma(2.0 / c)) / (c * c);
        /* eq. (sersicLtot): I_e = r_box F b^(2n) / (2 pi q re^2 n Gamma(2n) e^b) */
        cp->lnamp = lnF + lnrbox + 2.0 * n * log(cp->b) - log(2.0 * ORC_PI * q * re * re * n) - lgamma(2.0 * n)
                    - cp->b;
        break;
    }
    case ORC_EXPDISK: {
        double rs = v[3];
        cp->scale = rs;
        cp->lnamp = lnF - log(2.0 * ORC_PI * q * rs * rs);   /* I0 = F / (2 pi q rs^2) */
        break;
    }
    case ORC_FERRER: {
        double rout = v[3], a = v[6], bb = v[7];
        cp->scale = rout; cp->a_f = a; cp->b_f = bb;
        double c2 = 1.0 + 2.0 / (2.0 - bb);
        double lbeta = lgamma(a) + lgamma(c2) - lgamma(a + c2);
        cp->fc2 = c2;
        /* I0 = F / (pi q rout^2 a beta(a, 1 + 2/(2-b))) */
        cp->lnamp = lnF - log(ORC_PI * q * rout * rout * a) - lbeta;
        break;
    }
    case ORC_KING: {
        double rc = v[3], rt = v[4], al = v[7];
        cp->scale = rc; cp->scale2 = rt; cp->alpha = al;
        double T = 1.0 + (rt / rc) * (rt / rc);
        cp->kT = T;
        cp->kA = pow(T, -1.0 / al);
        /* dA/dln rc = 2 A (T-1) / (alpha T);  dA/dln rt = -2 A (T-1) / (alpha T) */
        cp->dkA_dlnrc = 2.0 * cp->kA * (T - 1.0) / (al * T);
        cp->dkA_dlnrt = -cp->dkA_dlnrc;
        break;
    }
    case ORC_GAUSSIAN: {
        cp->scale = v[3] / (2.0 * sqrt(2.0 * log(2.0)));     /* sigma from FWHM */
        break;
    }
    case ORC_MOFFAT: {
        double fwhm = v[3], be = v[6];
        cp->beta = be;
        cp->rd = fwhm / (2.0 * sqrt(pow(2.0, 1.0 / be) - 1.0));
        /* I0 = (beta - 1) F / (pi q rd^2) */
        cp->lnamp = lnF + log(be - 1.0) - log(ORC_PI * q * cp->rd * cp->rd);
        break;
    }
    }
}

/* Value I and derivatives dI[s] = dI/du_s (u_s the LM variable of slot s) of
 * one component at the point (x, y).  Slots of kind K_SHAPE get 0. */
static void comp_point(const comp_prep *cp, double x, double y, double *I, double *dI)
{
    for (int s = 0; s < ORC_MAX_SLOTS; ++s) dI[s] = 0.0;
    if (cp->type == ORC_SKY) {
        *I = cp->v[0];
        dI[0] = 1.0;
        return;
    }
    if (cp->type == ORC_SKYPLANE) {         /* Appendix D, eq. (new_sky_I) */
        *I = cp->v[0] + cp->v[1] * (x - cp->xc) + cp->v[2] * (y - cp->yc);
        dI[0] = 1.0;
        dI[1] = x - cp->xc;
        dI[2] = y - cp->yc;
        return;
    }
    /* rotate into the component frame (Sec. 4.1) */
    double dx = x - cp->v[0], dy = y - cp->v[1];
    double X = cp->cth * dx + cp->sth * dy;
    double Y = -cp->sth * dx + cp->cth * dy;
    double q = cp->q;
    double r2, floored = 0.0, dr2_dx0, dr2_dy0, dr2_dth, dr2_dq, dr2_dc = 0.0;
    if (cp->type == ORC_SERSIC) {
        /* eq. (r) with boxiness: r = (|X|^c + |Y/q|^c)^(1/c), c = B + 2 */
        double c = cp->cbox, ax = fabs(X), ay = fabs(Y) / q;
        double A = pow(ax, c), Bq = pow(ay, c), S = A + Bq;
        r2 = pow(S, 2.0 / c);
        if (r2 < 1e-12) {
            r2 = 1e-12; floored = 1.0;
            dr2_dx0 = dr2_dy0 = dr2_dth = dr2_dq = 0.0;
        } else {
            /* d ln r / dX = A / (S X), d ln r / dY = Bq / (S Y) (0 on the axes, c > 1) */
            double lx = X != 0.0 ? A / (S * X) : 0.0, ly = Y != 0.0 ? Bq / (S * Y) : 0.0;
            dr2_dx0 = 2.0 * r2 * (-cp->cth * lx + cp->sth * ly);
            dr2_dy0 = 2.0 * r2 * (-cp->sth * lx - cp->cth * ly);
            dr2_dth = 2.0 * r2 * (Y * lx - X * ly);
            dr2_dq = 2.0 * r2 * (-Bq / (q * S));
            double tA = ax > 0.0 ? A * log(ax) : 0.0, tB = ay > 0.0 ? Bq * log(ay) : 0.0;
            dr2_dc = 2.0 * r2 * (-log(S) / (c * c) + (tA + tB) / (c * S));
        }
    } else {
        double r2raw = X * X + Y * Y / (q * q);
        r2 = r2raw;
        if (r2 < 1e-12) { r2 = 1e-12; floored = 1.0; }
        /* d r^2 / d(x0, y0, theta, q); zero where the cusp floor is active */
        double g = 1.0 - floored;
        dr2_dx0 = g * (-2.0 * X * cp->cth + 2.0 * Y * cp->sth / (q * q));
        dr2_dy0 = g * (-2.0 * X * cp->sth - 2.0 * Y * cp->cth / (q * q));
        dr2_dth = g * (2.0 * X * Y * (1.0 - 1.0 / (q * q)));
        dr2_dq  = g * (-2.0 * Y * Y / (q * q * q));
    }

    double val = 0.0, dl_dr2 = 0.0, dl_dq_direct = 0.0;
    int sq = 4, spa = 5;    /* slots of q and PA */
    switch (cp->type) {
    case ORC_SERSIC: {
        sq = 5; spa = 6;
        double n = cp->n, b = cp->b, db = cp->db, re = cp->re;
        double L = log(r2 / (re * re));
        double z = exp(L / (2.0 * n));           /* (r / re)^(1/n) */
        double lnI = cp->lnamp - b * (z - 1.0);
        val = exp(lnI);
        dl_dr2 = -b * z / (2.0 * n * r2);
        dl_dq_direct = -1.0 / q;
        dI[2] = -0.4 * ORC_LN10 * val;                          /* m */
        dI[3] = val * (-2.0 + b * z / n);                        /* ln re */
        double dl_dn = 2.0 * log(b) + 2.0 * n * db / b - 1.0 / n
                     - 2.0 * orc_digamma(2.0 * n) - db * z
                     + b * z * L / (2.0 * n * n);
        dI[4] = val * n * dl_dn;                                 /* ln n */
        dI[7] = val * (cp->dlrbox + dl_dr2 * dr2_dc);            /* B */
        break;
    }
    case ORC_EXPDISK: {
        double rs = cp->scale, r = sqrt(r2);
        val = exp(cp->lnamp - r / rs);
        dl_dr2 = -1.0 / (2.0 * r * rs);
        dl_dq_direct = -1.0 / q;
        dI[2] = -0.4 * ORC_LN10 * val;
        dI[3] = val * (-2.0 + r / rs);                           /* ln rs */
        break;
    }
    case ORC_FERRER: {
        double rout = cp->scale, a = cp->a_f, e = 2.0 - cp->b_f;
        double lnu = 0.5 * e * log(r2 / (rout * rout));     /* ln (r/rout)^(2-b) */
        if (lnu >= 0.0) { val = 0.0; break; }
        double u = exp(lnu), omu = -expm1(lnu);             /* 1 - u */
        val = exp(cp->lnamp + a * log(omu));
        dl_dr2 = -a * e * u / (2.0 * r2 * omu);
        dl_dq_direct = -1.0 / q;
        dI[2] = -0.4 * ORC_LN10 * val;
        dI[3] = val * (-2.0 + a * e * u / omu);                  /* ln rout */
        /* a (as ln a): d ln I / da = ln(1 - u) - 1/a - (psi(a) - psi(a + c2)), the last two
         * from I0 = F / (pi q rout^2 a beta(a, c2)); b: u = (r/rout)^(2-b) gives
         * d ln(1 - u) / db = (u / (1 - u)) ln(r / rout), and dc2/db = 2 / (2 - b)^2 */
        double c2 = cp->fc2, lnr_ro = lnu / e;
        dI[6] = val * a * (log(omu) - 1.0 / a - (orc_digamma(a) - orc_digamma(a + c2)));
        dI[7] = val * (a * u / omu * lnr_ro - (orc_digamma(c2) - orc_digamma(a + c2)) * 2.0 / (e * e));
        break;
    }
    case ORC_KING: {
        double rc = cp->scale, rt = cp->scale2, al = cp->alpha, A = cp->kA;
        if (r2 >= rt * rt) { val = 0.0; sq = 5; spa = 6; break; }
        sq = 5; spa = 6;
        double s = 1.0 + r2 / (rc * rc);
        double S = pow(s, -1.0 / al);
        double Dd = S - A;
        double shape = pow(Dd / (1.0 - A), al);          /* I / I0 */
        double I0 = cp->v[2];
        val = I0 * shape;
        dl_dr2 = -S / (s * rc * rc * Dd);
        double dS_dlnrc = 2.0 * S * (s - 1.0) / (al * s);
        dI[2] = shape;                                           /* I0 */
        dI[3] = val * (al * cp->dkA_dlnrc / (1.0 - A) + al * (dS_dlnrc - cp->dkA_dlnrc) / Dd);
        dI[4] = val * (al * cp->dkA_dlnrt / (1.0 - A) - al * cp->dkA_dlnrt / Dd);
        /* alpha (as ln alpha): ln(I/I0) = alpha [ln(S - A) - ln(1 - A)] with
         * dS/dalpha = S ln s / alpha^2 and dA/dalpha = A ln T / alpha^2 */
        double dS_da = S * log(s) / (al * al), dA_da = A * log(cp->kT) / (al * al);
        dI[7] = val * al * (log(Dd / (1.0 - A)) + al * ((dS_da - dA_da) / Dd + dA_da / (1.0 - A)));
        break;
    }
    case ORC_GAUSSIAN: {
        double sg = cp->scale, I0 = cp->v[2];
        double shape = exp(-r2 / (2.0 * sg * sg));
        val = I0 * shape;
        dl_dr2 = -1.0 / (2.0 * sg * sg);
        dI[2] = shape;                                           /* I0 */
        dI[3] = val * r2 / (sg * sg);                            /* ln FWHM */
        break;
    }
    case ORC_MOFFAT: {
        double rd = cp->rd, be = cp->beta;
        val = exp(cp->lnamp - be * log1p(r2 / (rd * rd)));
        dl_dr2 = -be / (rd * rd + r2);
        dl_dq_direct = -1.0 / q;
        dI[2] = -0.4 * ORC_LN10 * val;
        dI[3] = val * (-2.0 + 2.0 * be * r2 / (rd * rd + r2));   /* ln FWHM */
        break;
    }
    }
    *I = val;
    if (val == 0.0) {
        for (int s = 0; s < ORC_MAX_SLOTS; ++s) dI[s] = 0.0;
        return;
    }
    dI[0] = val * dl_dr2 * dr2_dx0;
    dI[1] = val * dl_dr2 * dr2_dy0;
    dI[sq] = val * (dl_dr2 * dr2_dq + dl_dq_direct);
    dI[spa] = val * dl_dr2 * dr2_dth;
}

/* Value and LM-variable derivatives of component `comp` at one point. */
int orc_profile_point(const orc_model *m, int comp, const double *params, double x, double y,
                      double *I, double *dI)
{
    if (orc_validate(m) || comp < 0 || comp >= m->ncomp)
        return ORC_EINVAL;
    comp_prep cp;
    double tmp[ORC_MAX_SLOTS];
    prep_component(m, comp, params, &cp);
    comp_point(&cp, x, y, I, dI ? dI : tmp);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Images                                                                   */
/* ------------------------------------------------------------------------ */

/* Oversampling window of a radial component (not in the paper): the 5x5
 * pixels around the pixel that holds the centre, jc = floor(x0),
 * ic = floor(H - y0), rows ic-2..ic+2 and columns jc-2..jc+2 clipped to the
 * cutout.  Inside it a pixel's value is the mean of the profile over the
 * f x f sub-pixel centres (j + (s+0.5)/f, H - i - (t+0.5)/f); outside it the
 * profile is sampled at the pixel centre. */
static void oversample_window(const orc_model *m, const comp_prep *cp, int h, int w,
                              int *i0, int *i1, int *j0, int *j1)
{
    *i0 = 1; *i1 = 0; *j0 = 1; *j1 = 0;         /* empty */
    if (cp->type == ORC_SKY || cp->type == ORC_SKYPLANE || m->oversample <= 1 || m->os_window <= 0)
        return;
    int half = m->os_window / 2;
    double jcd = floor(cp->v[0]), icd = floor((double)h - cp->v[1]);
    if (!(fabs(jcd) < 1e9 && fabs(icd) < 1e9))
        return;
    int jc = (int)jcd, ic = (int)icd;
    *i0 = ic - half < 0 ? 0 : ic - half;
    *i1 = ic + half > h - 1 ? h - 1 : ic + half;
    *j0 = jc - half < 0 ? 0 : jc - half;
    *j1 = jc + half > w - 1 ? w - 1 : jc + half;
}

/* Sum of the selected components (convolve flag == want_conv) as an image,
 * and the derivative of that sum with respect to every LM column
 * (der may be NULL). */
static void render_planes(const orc_model *m, const comp_prep *cps, int h, int w, int want_conv,
                          double *val, double *der)
{
    int p = m->p, npix = h * w;
    memset(val, 0, sizeof(double) * npix);
    if (der) memset(der, 0, sizeof(double) * (size_t)p * npix);
    int f = m->oversample > 1 ? m->oversample : 1;
    for (int c = 0; c < m->ncomp; ++c) {
        if ((m->comp[c].convolve != 0) != (want_conv != 0))
            continue;
        const comp_prep *cp = &cps[c];
        int wi0, wi1, wj0, wj1;
        oversample_window(m, cp, h, w, &wi0, &wi1, &wj0, &wj1);
        for (int i = 0; i < h; ++i) {
            for (int j = 0; j < w; ++j) {
                double I = 0.0, dI[ORC_MAX_SLOTS] = {0};
                if (i >= wi0 && i <= wi1 && j >= wj0 && j <= wj1) {
                    double t_dI[ORC_MAX_SLOTS];
                    for (int t = 0; t < f; ++t) {
                        for (int s = 0; s < f; ++s) {
                            double x = j + (s + 0.5) / f;
                            double y = (double)h - i - (t + 0.5) / f;
                            double tI;
                            comp_point(cp, x, y, &tI, t_dI);
                            I += tI;
                            for (int k = 0; k < ORC_MAX_SLOTS; ++k) dI[k] += t_dI[k];
                        }
                    }
                    I /= (double)(f * f);
                    for (int k = 0; k < ORC_MAX_SLOTS; ++k) dI[k] /= (double)(f * f);
                } else {
                    comp_point(cp, j + 0.5, (double)h - i - 0.5, &I, dI);
                }
                val[i * w + j] += I;
                if (der)
                    for (int s = 0; s < ORC_MAX_SLOTS; ++s) {
                        int k = m->comp[c].idx[s];
                        if (k >= 0 && slot_kind[cp->type][s] != K_SHAPE)
                            der[(size_t)k * npix + i * w + j] += dI[s];
                    }
            }
        }
    }
}

/* True 2D convolution with zero padding and output of the input's size:
 * out[i,j] = sum_{u,v} psf[u,v] in[i-(u-c), j-(v-c)], c = (K-1)/2. */
void orc_convolve(int h, int w, const double *in, int k, const double *psf, double *out)
{
    int c = (k - 1) / 2;
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            double acc = 0.0;
            for (int u = 0; u < k; ++u) {
                int ii = i - (u - c);
                if (ii < 0 || ii >= h) continue;
                for (int v = 0; v < k; ++v) {
                    int jj = j - (v - c);
                    if (jj < 0 || jj >= w) continue;
                    acc += psf[u * k + v] * in[ii * w + jj];
                }
            }
            out[i * w + j] = acc;
        }
}

/* Model image M and, if jac != NULL, its derivatives with respect to the LM
 * variables u (jac[k][pix]).  M = PSF (x) sum_conv I + sum_unconv I + sky. */
static int model_and_jacobian_u(const orc_model *m, int h, int w, const double *psf, int k,
                                const double *params, double *model, double *jac)
{
    int p = m->p, npix = h * w;
    comp_prep cps[ORC_MAX_COMP];
    for (int c = 0; c < m->ncomp; ++c) {
        prep_component(m, c, params, &cps[c]);
        cps[c].xc = 0.5 * w;
        cps[c].yc = 0.5 * h;
    }
    double *val = malloc(sizeof(double) * npix);
    double *tmp = malloc(sizeof(double) * npix);
    double *der = jac ? malloc(sizeof(double) * (size_t)p * npix) : NULL;
    if (!val || !tmp || (jac && !der)) {
        free(val); free(tmp); free(der);
        return ORC_ENOMEM;
    }
    /* convolved part */
    render_planes(m, cps, h, w, 1, val, der);
    orc_convolve(h, w, val, k, psf, model);
    if (jac)
        for (int kk = 0; kk < p; ++kk)
            orc_convolve(h, w, der + (size_t)kk * npix, k, psf, jac + (size_t)kk * npix);
    /* unconvolved part (point sources, sky) */
    render_planes(m, cps, h, w, 0, val, der);
    for (int i = 0; i < npix; ++i) model[i] += val[i];
    if (jac)
        for (size_t i = 0; i < (size_t)p * npix; ++i) jac[i] += der[i];
    free(val); free(tmp); free(der);
    return ORC_OK;
}

static double *psf_to_double(const float *psf, int k)
{
    double *d = malloc(sizeof(double) * k * k);
    if (d)
        for (int i = 0; i < k * k; ++i) d[i] = psf[i];
    return d;
}

int orc_model_image(const orc_model *m, int h, int w, const float *psf, int k,
                    const double *params, double *out)
{
    if (orc_validate(m) || h < 1 || w < 1 || k < 1 || (k & 1) == 0)
        return ORC_EINVAL;
    double *ps = psf_to_double(psf, k);
    if (!ps) return ORC_ENOMEM;
    int rc = model_and_jacobian_u(m, h, w, ps, k, params, out, NULL);
    free(ps);
    return rc;
}

int orc_jacobian(const orc_model *m, int h, int w, const float *psf, int k,
                 const double *params, double *jac)
{
    if (orc_validate(m) || h < 1 || w < 1 || k < 1 || (k & 1) == 0)
        return ORC_EINVAL;
    int npix = h * w;
    double *ps = psf_to_double(psf, k);
    double *model = malloc(sizeof(double) * npix);
    if (!ps || !model) { free(ps); free(model); return ORC_ENOMEM; }
    int rc = model_and_jacobian_u(m, h, w, ps, k, params, model, jac);
    /* chain rule to natural parameters: dM/dp = dM/du * du/dp */
    for (int kk = 0; kk < m->p && rc == ORC_OK; ++kk) {
        double s = 1.0 / dp_du(column_kind(m, kk), params[kk]);
        for (int i = 0; i < npix; ++i) jac[(size_t)kk * npix + i] *= s;
    }
    free(ps); free(model);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Normal equations                                                         */
/* ------------------------------------------------------------------------ */

/* Pixel weight w = Omega / sigma^2 (Sec. 5.1); unusable pixels (mask 0,
 * sigma <= 0 or non-finite, non-finite data) get weight 0. */
static double pixel_weight(const float *data, const float *sigma, const uint8_t *omega, int i)
{
    if (omega && omega[i] == 0) return 0.0;
    double s = sigma[i], d = data[i];
    if (!(s > 0.0) || !isfinite(s) || !isfinite(d)) return 0.0;
    return 1.0 / (s * s);
}

typedef struct {
    const orc_model *m;
    int h, w, k;
    const float *data, *sigma;
    const uint8_t *omega;
    const double *psf;
    double *model, *jac;   /* scratch: npix, p*npix */
} fit_ctx;

/* chi^2 = sum w r^2, g = J^T W r, A = J^T W J at parameters params (natural). */
static int normal_equations(fit_ctx *fc, const double *params, double *chi2, double *g, double *A)
{
    const orc_model *m = fc->m;
    int p = m->p, npix = fc->h * fc->w;
    int rc = model_and_jacobian_u(m, fc->h, fc->w, fc->psf, fc->k, params, fc->model, fc->jac);
    if (rc) return rc;
    double c2 = 0.0;
    for (int a = 0; a < p; ++a) {
        g[a] = 0.0;
        for (int b = 0; b < p; ++b) A[a * p + b] = 0.0;
    }
    for (int i = 0; i < npix; ++i) {
        double wgt = pixel_weight(fc->data, fc->sigma, fc->omega, i);
        if (wgt == 0.0) continue;
        double r = (double)fc->data[i] - fc->model[i];
        c2 += wgt * r * r;
        for (int a = 0; a < p; ++a) {
            double ja = fc->jac[(size_t)a * npix + i];
            g[a] += wgt * ja * r;
            for (int b = 0; b <= a; ++b)
                A[a * p + b] += wgt * ja * fc->jac[(size_t)b * npix + i];
        }
    }
    for (int a = 0; a < p; ++a)
        for (int b = a + 1; b < p; ++b) A[a * p + b] = A[b * p + a];
    *chi2 = c2;
    return ORC_OK;
}

/* Cholesky factorisation L L^T = M (lower triangle in L); returns 0 if M is
 * positive definite. */
static int cholesky(int p, const double *M, double *L)
{
    for (int i = 0; i < p * p; ++i) L[i] = 0.0;
    for (int j = 0; j < p; ++j) {
        double d = M[j * p + j];
        for (int k = 0; k < j; ++k) d -= L[j * p + k] * L[j * p + k];
        if (!(d > 0.0) || !isfinite(d)) return -1;
        L[j * p + j] = sqrt(d);
        for (int i = j + 1; i < p; ++i) {
            double s = M[i * p + j];
            for (int k = 0; k < j; ++k) s -= L[i * p + k] * L[j * p + k];
            L[i * p + j] = s / L[j * p + j];
        }
    }
    return 0;
}

static void chol_solve(int p, const double *L, const double *b, double *x)
{
    double y[ORC_MAX_P];
    for (int i = 0; i < p; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * p + k] * y[k];
        y[i] = s / L[i * p + i];
    }
    for (int i = p - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < p; ++k) s -= L[k * p + i] * x[k];
        x[i] = s / L[i * p + i];
    }
}

/* inverse of a PD matrix from its Cholesky factor, column by column */
static void chol_inverse(int p, const double *L, double *inv)
{
    double e[ORC_MAX_P], col[ORC_MAX_P];
    for (int j = 0; j < p; ++j) {
        for (int i = 0; i < p; ++i) e[i] = (i == j);
        chol_solve(p, L, e, col);
        for (int i = 0; i < p; ++i) inv[i * p + j] = col[i];
    }
}

/* Bounds of the LM variables, applied after every trial step (natural units
 * converted to u): centres inside the cutout, positive scales in
 * [0.1, 2 max(H, W)] px, Sersic index in [0.2, 10], axis ratio in
 * [0.05, 20] (q > 1 is allowed during the fit and canonicalised at the end),
 * boxiness B in [-0.9, 2] (c = B + 2 in [1.1, 4]), Ferrer a in [0.1, 10] and
 * b in [-1, 1.95], King alpha in [0.5, 10]. */
static void clamp_u(const orc_model *m, int h, int w, double *u)
{
    double big = 2.0 * (h > w ? h : w);
    for (int k = 0; k < m->p; ++k) {
        int kind = column_kind(m, k);
        double lo = -INFINITY, hi = INFINITY;
        switch (kind) {
        case K_X0: lo = 0.0; hi = w; break;
        case K_Y0: lo = 0.0; hi = h; break;
        case K_SCALE: lo = log(0.1); hi = log(big); break;
        case K_N: lo = log(0.2); hi = log(10.0); break;
        case K_Q: lo = 0.05; hi = 20.0; break;
        case K_BOX: lo = -0.9; hi = 2.0; break;
        case K_FA: lo = log(0.1); hi = log(10.0); break;
        case K_FB: lo = -1.0; hi = 1.95; break;
        case K_KAL: lo = log(0.5); hi = log(10.0); break;
        default: break;
        }
        if (u[k] < lo) u[k] = lo;
        if (u[k] > hi) u[k] = hi;
    }
}

static void u_to_params(const orc_model *m, const double *u, double *params)
{
    for (int k = 0; k < m->p; ++k) params[k] = from_u(column_kind(m, k), u[k]);
}

/* Canonical form of each component (Z17 reading): if q > 1 then q <- 1/q,
 * every scale of the component <- scale * q_old and PA <- PA + 90 deg; PA is
 * then wrapped into [0, 180) deg.  The model image is unchanged. */
void orc_canonicalise(const orc_model *m, double *params)
{
    for (int c = 0; c < m->ncomp; ++c) {
        const orc_comp *cp = &m->comp[c];
        int sq = -1, spa = -1;
        for (int s = 0; s < ORC_MAX_SLOTS; ++s) {
            int kind = slot_kind[cp->type][s];
            if (kind == K_Q) sq = s;
            if (kind == K_PA) spa = s;
        }
        if (sq < 0) continue;
        int kq = cp->idx[sq], kpa = cp->idx[spa];
        if (kq >= 0 && kpa >= 0 && params[kq] > 1.0) {
            double qo = params[kq];
            params[kq] = 1.0 / qo;
            for (int s = 0; s < ORC_MAX_SLOTS; ++s)
                if (slot_kind[cp->type][s] == K_SCALE && cp->idx[s] >= 0)
                    params[cp->idx[s]] *= qo;
            params[kpa] += 90.0;
        }
        if (kpa >= 0) {
            double pa = fmod(params[kpa], 180.0);
            if (pa < 0.0) pa += 180.0;
            if (pa >= 180.0) pa -= 180.0;
            params[kpa] = pa;
        }
    }
}

/* Levenberg-Marquardt for one galaxy.  The paper names the method
 * (Sec. 5.1) without constants; the scheme and constants are:
 *  - start: (chi2, g, A) at u0; lambda = lambda0 (1e-3); chi2 non-finite ->
 *    NONFINITE;
 *  - damping: D = diag(max(A_kk, 1e-12 max_l A_ll)) of the current accepted A
 *    (Marquardt's scaling);
 *  - each trial: solve (A + lambda D) delta = g by Cholesky; if it is not
 *    positive definite, lambda <- 10 lambda and the trial is spent;
 *  - stop test at every accepted state, before any step from it: with
 *    sigma_k = sqrt([A^-1]_kk), the undamped Gauss-Newton step A^-1 g must
 *    satisfy max_k |step_k| / sigma_k < step_tol (1e-4) -> CONVERGED; while A is
 *    not positive definite the damped step is tested instead against
 *    sigma_k = 1/sqrt(D_kk).  The step count reported is the number of trials;
 *  - u' = clamp(u + delta), one evaluation; accept if chi2' is finite and
 *    chi2' < chi2, then lambda <- max(lambda/10, 1e-9); else lambda <- 10 lambda,
 *    and lambda > 1e9 -> STALLED;
 *  - max_iter (100) trials -> MAXITER;
 *  - finally every component is put in canonical form. */
int orc_fit(const orc_model *m, int h, int w, const float *data, const float *sigma,
            const uint8_t *omega, const float *psf, int k, const orc_lm_opts *o,
            double *params, double *chi2_out, int *niter_out, int *status_out)
{
    if (orc_validate(m) || h < 1 || w < 1 || k < 1 || (k & 1) == 0)
        return ORC_EINVAL;
    int p = m->p, npix = h * w;
    int max_iter = o ? o->max_iter : 100;
    double lambda = o ? o->lambda0 : 1e-3, tol = o ? o->step_tol : 1e-4;
    fit_ctx fc = {m, h, w, k, data, sigma, omega, NULL, NULL, NULL};
    fc.psf = psf_to_double(psf, k);
    fc.model = malloc(sizeof(double) * npix);
    fc.jac = malloc(sizeof(double) * (size_t)p * npix);
    if (!fc.psf || !fc.model || !fc.jac) {
        free((void *)fc.psf); free(fc.model); free(fc.jac);
        return ORC_ENOMEM;
    }
    double u[ORC_MAX_P], ut[ORC_MAX_P], pt[ORC_MAX_P];
    double A[ORC_MAX_P * ORC_MAX_P], g[ORC_MAX_P], At[ORC_MAX_P * ORC_MAX_P], gt[ORC_MAX_P];
    double Mx[ORC_MAX_P * ORC_MAX_P], L[ORC_MAX_P * ORC_MAX_P], Ainv[ORC_MAX_P * ORC_MAX_P];
    double D[ORC_MAX_P], sig[ORC_MAX_P], delta[ORC_MAX_P];
    for (int a = 0; a < p; ++a) u[a] = to_u(column_kind(m, a), params[a]);
    clamp_u(m, h, w, u);
    u_to_params(m, u, pt);
    double chi2;
    int status = ORC_ST_MAXITER, t = 0;
    normal_equations(&fc, pt, &chi2, g, A);
    if (!isfinite(chi2)) {
        status = ORC_ST_NONFINITE;
        goto done;
    }
    int fresh = 1;   /* A changed: recompute D, sigma and the stop test */
    int a_pd = 0;
    for (t = 1; t <= max_iter; ++t) {
        if (fresh) {
            double amax = 0.0;
            for (int a = 0; a < p; ++a) if (A[a * p + a] > amax) amax = A[a * p + a];
            for (int a = 0; a < p; ++a) {
                double d = A[a * p + a];
                D[a] = d > 1e-12 * amax ? d : 1e-12 * amax;
            }
            a_pd = cholesky(p, A, L) == 0;
            if (a_pd) {
                chol_inverse(p, L, Ainv);
                for (int a = 0; a < p; ++a) sig[a] = sqrt(Ainv[a * p + a]);
                /* stop test on the undamped Gauss-Newton step A^-1 g */
                chol_solve(p, L, g, delta);
                double smax = 0.0;
                for (int a = 0; a < p; ++a) {
                    double s = fabs(delta[a]) / sig[a];
                    if (!(s <= smax)) smax = s;     /* NaN-propagating max */
                }
                if (smax < tol) {
                    status = ORC_ST_CONVERGED;
                    t -= 1;
                    break;
                }
            } else {
                for (int a = 0; a < p; ++a) sig[a] = 1.0 / sqrt(D[a]);
            }
            fresh = 0;
        }
        for (int a = 0; a < p; ++a)
            for (int b = 0; b < p; ++b)
                Mx[a * p + b] = A[a * p + b] + (a == b ? lambda * D[a] : 0.0);
        if (cholesky(p, Mx, L) != 0) {
            lambda *= 10.0;
            if (lambda > 1e9) { status = ORC_ST_STALLED; break; }
            continue;
        }
        chol_solve(p, L, g, delta);
        if (!a_pd) {
            /* no covariance yet: stop test on the damped step */
            double smax = 0.0;
            for (int a = 0; a < p; ++a) {
                double s = fabs(delta[a]) / sig[a];
                if (!(s <= smax)) smax = s;
            }
            if (smax < tol) {
                status = ORC_ST_CONVERGED;
                t -= 1;
                break;
            }
        }
        for (int a = 0; a < p; ++a) ut[a] = u[a] + delta[a];
        clamp_u(m, h, w, ut);
        u_to_params(m, ut, pt);
        double chi2t;
        normal_equations(&fc, pt, &chi2t, gt, At);
        if (isfinite(chi2t) && chi2t < chi2) {
            memcpy(u, ut, sizeof(double) * p);
            memcpy(g, gt, sizeof(double) * p);
            memcpy(A, At, sizeof(double) * p * p);
            chi2 = chi2t;
            lambda = lambda / 10.0 > 1e-9 ? lambda / 10.0 : 1e-9;
            fresh = 1;
        } else {
            lambda *= 10.0;
            if (lambda > 1e9) { status = ORC_ST_STALLED; break; }
        }
    }
    if (t > max_iter) t = max_iter;
done:
    u_to_params(m, u, params);
    orc_canonicalise(m, params);
    if (chi2_out) *chi2_out = chi2;
    if (niter_out) *niter_out = t;
    if (status_out) *status_out = status;
    free((void *)fc.psf); free(fc.model); free(fc.jac);
    return ORC_OK;
}

/* Gradient descent with Adam, the paper's own fitter (Sec. 5.1: gradient
 * descent through pytorch's adaptive optimisers; its examples run 1000
 * iterations).  The loss is chi^2 (Sec. 5.1) and the variables are the LM
 * variables u (ln of scales and n, PA in radians, the rest as given), so the
 * gradient is d chi^2/du = -2 J^T W r.  Adam's update (Kingma and Ba 2015,
 * Algorithm 1): m <- b1 m + (1-b1) grad, v <- b2 v + (1-b2) grad^2,
 * u <- u - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), then the LM bounds.
 * All `steps` steps are taken (no convergence test); chi^2 is evaluated once
 * more at the final u; the result is put in canonical form.  Status MAXITER,
 * or NONFINITE as soon as chi^2 is not finite (u is then the last finite
 * iterate's successor, as taken). */
int orc_fit_adam(const orc_model *m, int h, int w, const float *data, const float *sigma,
                 const uint8_t *omega, const float *psf, int k, const orc_adam_opts *o,
                 double *params, double *chi2_out, int *status_out)
{
    if (orc_validate(m) || h < 1 || w < 1 || k < 1 || (k & 1) == 0 || !o || o->steps < 0)
        return ORC_EINVAL;
    int p = m->p, npix = h * w;
    fit_ctx fc = {m, h, w, k, data, sigma, omega, NULL, NULL, NULL};
    fc.psf = psf_to_double(psf, k);
    fc.model = malloc(sizeof(double) * npix);
    fc.jac = malloc(sizeof(double) * (size_t)p * npix);
    if (!fc.psf || !fc.model || !fc.jac) {
        free((void *)fc.psf); free(fc.model); free(fc.jac);
        return ORC_ENOMEM;
    }
    double u[ORC_MAX_P], pt[ORC_MAX_P], g[ORC_MAX_P], A[ORC_MAX_P * ORC_MAX_P];
    double m1[ORC_MAX_P] = {0}, m2[ORC_MAX_P] = {0};
    for (int a = 0; a < p; ++a) u[a] = to_u(column_kind(m, a), params[a]);
    clamp_u(m, h, w, u);
    double chi2 = 0.0;
    int status = ORC_ST_MAXITER;
    for (int t = 1; t <= o->steps; ++t) {
        u_to_params(m, u, pt);
        normal_equations(&fc, pt, &chi2, g, A);
        if (!isfinite(chi2)) { status = ORC_ST_NONFINITE; break; }
        double c1 = 1.0 - pow(o->beta1, t), c2 = 1.0 - pow(o->beta2, t);
        for (int a = 0; a < p; ++a) {
            double grad = -2.0 * g[a];
            m1[a] = o->beta1 * m1[a] + (1.0 - o->beta1) * grad;
            m2[a] = o->beta2 * m2[a] + (1.0 - o->beta2) * grad * grad;
            u[a] -= o->lr * (m1[a] / c1) / (sqrt(m2[a] / c2) + o->eps);
        }
        clamp_u(m, h, w, u);
    }
    if (status == ORC_ST_MAXITER) {
        u_to_params(m, u, pt);
        normal_equations(&fc, pt, &chi2, g, A);
        if (!isfinite(chi2)) status = ORC_ST_NONFINITE;
    }
    u_to_params(m, u, params);
    orc_canonicalise(m, params);
    if (chi2_out) *chi2_out = chi2;
    if (status_out) *status_out = status;
    free((void *)fc.psf); free(fc.model); free(fc.jac);
    return ORC_OK;
}

/* sigma_p = sqrt(diag (J^T W J)^-1) in natural units (Sec. 5.2), unscaled,
 * at the given parameters; cov (nullable) is the full natural-unit
 * covariance.  Returns ORC_ESINGULAR (errors NaN) if J^T W J is not PD. */
int orc_param_errors(const orc_model *m, int h, int w, const float *data, const float *sigma,
                     const uint8_t *omega, const float *psf, int k, const double *params,
                     double *err, double *cov)
{
    if (orc_validate(m) || h < 1 || w < 1 || k < 1 || (k & 1) == 0)
        return ORC_EINVAL;
    int p = m->p, npix = h * w;
    fit_ctx fc = {m, h, w, k, data, sigma, omega, NULL, NULL, NULL};
    fc.psf = psf_to_double(psf, k);
    fc.model = malloc(sizeof(double) * npix);
    fc.jac = malloc(sizeof(double) * (size_t)p * npix);
    if (!fc.psf || !fc.model || !fc.jac) {
        free((void *)fc.psf); free(fc.model); free(fc.jac);
        return ORC_ENOMEM;
    }
    double A[ORC_MAX_P * ORC_MAX_P], g[ORC_MAX_P], L[ORC_MAX_P * ORC_MAX_P], Ainv[ORC_MAX_P * ORC_MAX_P];
    double chi2;
    normal_equations(&fc, params, &chi2, g, A);
    int rc = ORC_OK;
    if (cholesky(p, A, L) != 0) {
        for (int a = 0; a < p; ++a) err[a] = NAN;
        if (cov) for (int a = 0; a < p * p; ++a) cov[a] = NAN;
        rc = ORC_ESINGULAR;
    } else {
        chol_inverse(p, L, Ainv);
        for (int a = 0; a < p; ++a) {
            double sa = dp_du(column_kind(m, a), params[a]);
            err[a] = sqrt(Ainv[a * p + a]) * fabs(sa);
            if (cov)
                for (int b = 0; b < p; ++b)
                    cov[a * p + b] = sa * Ainv[a * p + b] * dp_du(column_kind(m, b), params[b]);
        }
    }
    free((void *)fc.psf); free(fc.model); free(fc.jac);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Default initial guess from image moments                                 */
/* ------------------------------------------------------------------------ */

/* Image moments (the source-extraction step the paper delegates to an
 * external detector, replaced here by plain moments):
 *   sky0 = mean of the usable pixels in the 2-px outer frame;
 *   S = usable pixels with D - sky0 > 3 sigma;
 *   F0 = sum over S of D - sky0; (xc, yc) its flux-weighted centroid;
 *   central second moments over S, eigenvalues l+ >= l-;
 *   q0 = clamp(sqrt(l-/l+), 0.1, 1), th0 = atan2(2 Mxy, Mxx - Myy) / 2 (rad),
 *   r0 = clamp(1.1774 sqrt(l+), 1, W/4), m_g = m0 - 2.5 log10 max(F0, 1e-3);
 *   fewer than 5 pixels in S (or F0 <= 0): cutout centre, r0 = 3, q0 = 1,
 *   th0 = 0; peak = max over S of D - sky0 (1 when S is empty).
 * out[9] = {sky0, F0, xc, yc, m_g, r0, q0, th0, peak}. */
void orc_moments(int h, int w, const float *data, const float *sigma, const uint8_t *omega, double m0,
                 double *out)
{
    /* 1. border sky */
    double ssum = 0.0; long scount = 0;
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            if (!(i < 2 || i >= h - 2 || j < 2 || j >= w - 2)) continue;
            int ix = i * w + j;
            if (pixel_weight(data, sigma, omega, ix) == 0.0) continue;
            ssum += data[ix];
            scount++;
        }
    double sky0 = scount ? ssum / scount : 0.0;
    /* 2-3. moments over S */
    double F0 = 0.0, sx = 0.0, sy = 0.0, peak = 0.0;
    long ns = 0;
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            int ix = i * w + j;
            if (pixel_weight(data, sigma, omega, ix) == 0.0) continue;
            double dp = (double)data[ix] - sky0;
            if (!(dp > 3.0 * (double)sigma[ix])) continue;
            double x = j + 0.5, y = (double)h - i - 0.5;
            F0 += dp; sx += dp * x; sy += dp * y; ns++;
            if (dp > peak) peak = dp;
        }
    double xc = 0.5 * w, yc = 0.5 * h, r0 = 3.0, q0 = 1.0, th0 = 0.0;
    if (ns >= 5 && F0 > 0.0) {
        xc = sx / F0; yc = sy / F0;
        double mxx = 0.0, myy = 0.0, mxy = 0.0;
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < w; ++j) {
                int ix = i * w + j;
                if (pixel_weight(data, sigma, omega, ix) == 0.0) continue;
                double dp = (double)data[ix] - sky0;
                if (!(dp > 3.0 * (double)sigma[ix])) continue;
                double dx = j + 0.5 - xc, dy = (double)h - i - 0.5 - yc;
                mxx += dp * dx * dx; myy += dp * dy * dy; mxy += dp * dx * dy;
            }
        mxx /= F0; myy /= F0; mxy /= F0;
        double tr = 0.5 * (mxx + myy), dd = sqrt(0.25 * (mxx - myy) * (mxx - myy) + mxy * mxy);
        double lp = tr + dd, lm = tr - dd;
        if (lm < 0.0) lm = 0.0;
        q0 = lp > 0.0 ? sqrt(lm / lp) : 1.0;
        if (q0 < 0.1) q0 = 0.1;
        if (q0 > 1.0) q0 = 1.0;
        th0 = 0.5 * atan2(2.0 * mxy, mxx - myy);
        r0 = 1.1774 * sqrt(lp > 0.0 ? lp : 0.0);
        if (r0 < 1.0) r0 = 1.0;
        if (r0 > 0.25 * w) r0 = 0.25 * w;
    }
    out[0] = sky0; out[1] = F0; out[2] = xc; out[3] = yc;
    out[4] = m0 - 2.5 * log10(F0 > 1e-3 ? F0 : 1e-3);
    out[5] = r0; out[6] = q0; out[7] = th0; out[8] = peak > 0.0 ? peak : 1.0;
}

/* The paper takes start values from SExtractor (Sec. 3, Appendix A); this
 * build derives them from image moments instead:
 *  1. sky0 = mean of the usable pixels in the 2-px outer frame;
 *  2. S = usable pixels with D - sky0 > 3 sigma;
 *  3. F0 = sum_S (D - sky0); flux-weighted centroid and central second
 *     moments over S; lambda+- their eigenvalues;
 *  4. q0 = clamp(sqrt(lambda-/lambda+), 0.1, 1),
 *     theta0 = atan2(2 Mxy, Mxx - Myy) / 2, r0 = clamp(1.1774 sqrt(lambda+), 1, W/4),
 *     m_g = m0 - 2.5 log10 max(F0, 1e-3);
 *  5. fewer than 5 pixels in S: centre of the cutout, r0 = 3, q0 = 1, theta0 = 0.
 * mom (nullable) receives {x_c - W/2, y_c - H/2, m_g, ln r0, q0, theta0}.
 * Per component (flux split evenly over the components that carry a
 * magnitude or amplitude): Sersic n = 2 alone, n = 4 and r_e = r0/2 with
 * another radial component; exponential disk r_s = r0 / 1.678347; Ferrer
 * r_out = r0; King r_c = r0/2, r_t = 4 r0, I0 = peak; Gaussian FWHM = r0,
 * I0 = peak; Moffat FWHM = r0; q and PA from the moments where free. */
int orc_default_guess(const orc_model *m, int h, int w, const float *data, const float *sigma,
                      const uint8_t *omega, double *params, double *mom)
{
    if (orc_validate(m)) return ORC_EINVAL;
    double mo[9];
    orc_moments(h, w, data, sigma, omega, m->m0, mo);
    const double sky0 = mo[0], xc = mo[2], yc = mo[3], mg = mo[4], r0 = mo[5], q0 = mo[6], th0 = mo[7];
    const double peak = mo[8];
    double pa0 = th0 * 180.0 / ORC_PI;
    if (pa0 < 0.0) pa0 += 180.0;
    if (mom) {
        mom[0] = xc - 0.5 * w; mom[1] = yc - 0.5 * h; mom[2] = mg;
        mom[3] = log(r0); mom[4] = q0; mom[5] = th0;
    }
    int nflux = 0, nrad = 0;
    for (int c = 0; c < m->ncomp; ++c) {
        if (m->comp[c].type == ORC_SKY || m->comp[c].type == ORC_SKYPLANE) continue;
        nrad++;
        if (m->comp[c].idx[2] >= 0) nflux++;
    }
    if (nflux < 1) nflux = 1;
    double msplit = mg + 2.5 * log10((double)nflux);
    double pk = peak > 0.0 ? peak : 1.0;
    for (int c = 0; c < m->ncomp; ++c) {
        const orc_comp *cp = &m->comp[c];
        double v[ORC_MAX_SLOTS] = {0};
        switch (cp->type) {
        case ORC_SERSIC:
            v[0] = xc; v[1] = yc; v[2] = msplit;
            v[3] = nrad > 1 ? 0.5 * r0 : r0; v[4] = nrad > 1 ? 4.0 : 2.0; v[5] = q0; v[6] = pa0;
            break;
        case ORC_EXPDISK:
            v[0] = xc; v[1] = yc; v[2] = msplit; v[3] = r0 / 1.678347; v[4] = q0; v[5] = pa0;
            break;
        case ORC_FERRER:    /* free a, b start at the values printed in Appendix C */
            v[0] = xc; v[1] = yc; v[2] = msplit; v[3] = r0; v[4] = q0; v[5] = pa0; v[6] = 0.5; v[7] = 1.9;
            break;
        case ORC_KING:
            v[0] = xc; v[1] = yc; v[2] = pk; v[3] = 0.5 * r0; v[4] = 4.0 * r0; v[5] = q0; v[6] = pa0; v[7] = 2.0;
            break;
        case ORC_GAUSSIAN:
            v[0] = xc; v[1] = yc; v[2] = pk; v[3] = r0; v[4] = q0; v[5] = pa0;
            break;
        case ORC_MOFFAT:
            v[0] = xc; v[1] = yc; v[2] = msplit; v[3] = r0; v[4] = q0; v[5] = pa0;
            break;
        case ORC_SKY:
            v[0] = sky0;
            break;
        case ORC_SKYPLANE:
            v[0] = sky0; v[1] = 0.0; v[2] = 0.0;
            break;
        }
        /* the first component to claim a column sets it (tied centres) */
        for (int s = 0; s < ORC_MAX_SLOTS; ++s) {
            int kk = cp->idx[s];
            if (kk < 0) continue;
            int claimed = 0;
            for (int c2 = 0; c2 < c; ++c2)
                for (int s2 = 0; s2 < ORC_MAX_SLOTS; ++s2)
                    if (m->comp[c2].idx[s2] == kk) claimed = 1;
            if (!claimed) params[kk] = v[s];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Batch driver: one worker per thread over a shared galaxy counter         */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_model *m;
    int n_gal;
    const int32_t *h, *w;
    const int64_t *img_off;
    const float *data, *sigma;
    const uint8_t *omega;
    const int32_t *psf_k;
    const int64_t *psf_off;
    const float *psf;
    const orc_lm_opts *o;
    double *params, *chi2;
    int32_t *niter, *status;
    volatile long next;
    const orc_adam_opts *adam;   /* non-NULL: Adam instead of LM */
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *b = arg;
    for (;;) {
        long gi = __sync_fetch_and_add(&b->next, 1);
        if (gi >= b->n_gal) break;
        int64_t off = b->img_off[gi];
        int nit = 0, st = 0;
        double c2 = 0.0;
        if (b->adam) {
            orc_fit_adam(b->m, b->h[gi], b->w[gi], b->data + off, b->sigma + off,
                         b->omega ? b->omega + off : NULL, b->psf + b->psf_off[gi], b->psf_k[gi], b->adam,
                         b->params + (size_t)gi * b->m->p, &c2, &st);
        } else {
            orc_fit(b->m, b->h[gi], b->w[gi], b->data + off, b->sigma + off,
                    b->omega ? b->omega + off : NULL, b->psf + b->psf_off[gi], b->psf_k[gi], b->o,
                    b->params + (size_t)gi * b->m->p, &c2, &nit, &st);
            b->niter[gi] = nit;
        }
        b->chi2[gi] = c2;
        b->status[gi] = st;
    }
    return NULL;
}

static int run_batch(batch_job *job, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int i = 0; i < nthreads; ++i)
        if (pthread_create(&th[i], NULL, batch_worker, job) == 0) started++;
        else break;
    if (started == 0) batch_worker(job);
    for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
    return ORC_OK;
}

int orc_fit_batch(const orc_model *m, int n_gal, const int32_t *h, const int32_t *w,
                  const int64_t *img_off, const float *data, const float *sigma,
                  const uint8_t *omega, const int32_t *psf_k, const int64_t *psf_off,
                  const float *psf, const orc_lm_opts *o, double *params, double *chi2,
                  int32_t *niter, int32_t *status, int nthreads)
{
    if (orc_validate(m)) return ORC_EINVAL;
    batch_job job = {m, n_gal, h, w, img_off, data, sigma, omega, psf_k, psf_off, psf, o,
                     params, chi2, niter, status, 0, NULL};
    return run_batch(&job, nthreads);
}

int orc_fit_adam_batch(const orc_model *m, int n_gal, const int32_t *h, const int32_t *w,
                       const int64_t *img_off, const float *data, const float *sigma,
                       const uint8_t *omega, const int32_t *psf_k, const int64_t *psf_off,
                       const float *psf, const orc_adam_opts *o, double *params, double *chi2,
                       int32_t *status, int nthreads)
{
    if (orc_validate(m) || !o || o->steps < 0) return ORC_EINVAL;
    batch_job job = {m, n_gal, h, w, img_off, data, sigma, omega, psf_k, psf_off, psf, NULL,
                     params, chi2, NULL, status, 0, o};
    return run_batch(&job, nthreads);
}

