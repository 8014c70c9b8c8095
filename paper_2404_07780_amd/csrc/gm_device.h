// gm_device.h -- device-side numerics of libgmfit: FP64 special functions for
// the per-galaxy scalar prologue, FP32 profile values and derivatives at one
// point, and the model families the kernels are compiled for.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gm {

constexpr double kLn10 = 2.302585092994045684;
constexpr double kLn2 = 0.693147180559945309;
constexpr double kLog2e = 1.442695040888963407;
constexpr double kPi = 3.141592653589793238;
constexpr float kDMag = -0.921034037197618f;   // d ln F / d m = -0.4 ln 10

// Kinds of LM variables: centres, magnitudes, amplitudes, axis ratio and sky
// are used as they are; positive scales and the Sersic index through their
// natural log; position angles in radians (degrees at the interface).
enum Kind : int { KX0 = 1, KY0, KMAG, KAMP, KSCALE, KN, KQ, KPA, KSKY };

__host__ __device__ inline double nat_to_u(int kind, double p)
{
    if (kind == KSCALE || kind == KN) return log(p);
    if (kind == KPA) return p * (kPi / 180.0);
    return p;
}
__host__ __device__ inline double u_to_nat(int kind, double u)
{
    if (kind == KSCALE || kind == KN) return exp(u);
    if (kind == KPA) return u * (180.0 / kPi);
    return u;
}
// d(natural) / d(u)
__host__ __device__ inline double dnat_du(int kind, double p)
{
    if (kind == KSCALE || kind == KN) return p;
    if (kind == KPA) return 180.0 / kPi;
    return 1.0;
}

// ---------------------------------------------------------------- FP64 scalars
// digamma for x > 0: upward recurrence to x >= 10, then the Stirling series.
__device__ inline double digamma(double x)
{
    double s = 0.0;
    while (x < 10.0) {
        s -= 1.0 / x;
        x += 1.0;
    }
    double r = 1.0 / (x * x);
    double t = r * (1.0 / 12 - r * (1.0 / 120 - r * (1.0 / 252 - r * (1.0 / 240 - r * (1.0 / 132 - r * (691.0 / 32760 - r / 12))))));
    return s + log(x) - 0.5 / x - t;
}

// P(a, x) (regularised lower incomplete gamma) and dP/da from one pass over
// the series P = sum_k T_k, T_k = e^-x x^(a+k) / Gamma(a+k+1) (convergent for
// every x > 0), dT_k/da = T_k (ln x - psi(a+k+1)); T and psi by recurrence.
__device__ inline void gammainc_and_da(double a, double x, double *P, double *dPda)
{
    double lx = log(x);
    double T = exp(a * lx - x - lgamma(a + 1.0));
    double psi = digamma(a + 1.0);
    double sP = 0.0, sD = 0.0;
    for (int k = 0; k < 400; ++k) {
        if (k > 0) {
            T *= x / (a + k);
            psi += 1.0 / (a + k);
        }
        sP += T;
        sD += T * (lx - psi);
        if (k > x && T < 1e-17 * sP) break;
    }
    *P = sP;
    if (dPda) *dPda = sD;
}

// nu_n of the Sersic law: the root of P(2n, b) = 1/2 (the half-light
// condition), Newton with a bisection bracket; db/dn by implicit
// differentiation, -2 (dP/da) / (dP/dx).
__device__ inline double sersic_b(double n, double *dbdn)
{
    double a = 2.0 * n, lo = 0.0, hi = a + 20.0;
    double b = a - 1.0 / 3.0 + 4.0 / (405.0 * n);
    if (!(b > lo && b < hi)) b = 0.5 * a;
    double lga = lgamma(a);
    for (int it = 0; it < 100; ++it) {
        double P;
        gammainc_and_da(a, b, &P, nullptr);
        double f = P - 0.5;
        if (f > 0.0) hi = b; else lo = b;
        double fp = exp((a - 1.0) * log(b) - b - lga);
        double nb = b - f / fp;
        if (!(nb > lo && nb < hi)) nb = 0.5 * (lo + hi);
        double st = fabs(nb - b);
        b = nb;
        if (st < 1e-14 * b) break;
    }
    if (dbdn) {
        double P, dPa;
        gammainc_and_da(a, b, &P, &dPa);
        double dPx = exp((a - 1.0) * log(b) - b - lga);
        *dbdn = -2.0 * dPa / dPx;
    }
    return b;
}

// ---------------------------------------------------------------- components
// Every radial component carries its centre split into FP32 hi + lo parts so
// that offsets from the centre are exact to FP32 rounding of the offset itself,
// its orientation and its oversampling window (rows wi0..wi1, cols wj0..wj1).
struct Geo {
    float x0h, x0l, y0h, y0l, c, s, iq, iq2;
    int wi0, wi1, wj0, wj1;
};

__device__ inline void geo_prep(double x0, double y0, double q, double th, int H, int W, int osf, int osw, Geo &g)
{
    g.x0h = (float)x0;
    g.x0l = (float)(x0 - (double)g.x0h);
    g.y0h = (float)y0;
    g.y0l = (float)(y0 - (double)g.y0h);
    g.c = (float)cos(th);
    g.s = (float)sin(th);
    g.iq = (float)(1.0 / q);
    g.iq2 = (float)(1.0 / (q * q));
    // oversampled window: 'osw' x 'osw' pixels around the pixel holding the
    // centre, jc = floor(x0), ic = floor(H - y0), clipped to the cutout
    g.wi0 = 1; g.wi1 = 0; g.wj0 = 1; g.wj1 = 0;
    double jcd = floor(x0), icd = floor((double)H - y0);
    if (osf > 1 && osw > 0 && fabs(jcd) < 1e9 && fabs(icd) < 1e9) {
        int jc = (int)jcd, ic = (int)icd, hw = osw / 2;
        g.wi0 = max(ic - hw, 0); g.wi1 = min(ic + hw, H - 1);
        g.wj0 = max(jc - hw, 0); g.wj1 = min(jc + hw, W - 1);
    }
}

// offset of the point (x, y) = (xb + xs, yb - ys) from the centre, where xb, yb
// are integers (pixel corner) and xs, ys in (0, 1) the sub-pixel position
__device__ inline void offsets(const Geo &g, float xb, float xs, float yb, float ys, float &dx, float &dy)
{
    dx = ((xb - g.x0h) + xs) - g.x0l;
    dy = ((yb - g.y0h) - ys) - g.y0l;
}

struct RadialPt {
    float X, Y, r2, gmask;
};
__device__ inline RadialPt radial(const Geo &g, float dx, float dy)
{
    RadialPt p;
    p.X = g.c * dx + g.s * dy;
    p.Y = -g.s * dx + g.c * dy;
    p.r2 = p.X * p.X + p.Y * p.Y * g.iq2;
    p.gmask = 1.0f;
    if (p.r2 < 1e-12f) {        // cusp floor r^2 >= 1e-12 px^2: geometry derivatives vanish
        p.r2 = 1e-12f;
        p.gmask = 0.0f;
    }
    return p;
}

// Given I and dlnI/dr^2, the derivatives through r^2 with respect to the
// centre, the axis ratio (plus the direct -1/q of flux-normalised profiles)
// and the angle.
__device__ inline void geometry_derivs(const Geo &g, const RadialPt &p, float I, float dl, float dq_direct,
                                       float &dx0, float &dy0, float &dq, float &dth)
{
    float gd = I * dl * p.gmask;
    float Yq = p.Y * g.iq2;
    dx0 = gd * (-2.0f * p.X * g.c + 2.0f * Yq * g.s);
    dy0 = gd * (-2.0f * p.X * g.s - 2.0f * Yq * g.c);
    dq = gd * (-2.0f * p.Y * Yq * g.iq) + I * dq_direct;
    dth = gd * (2.0f * p.X * p.Y * (1.0f - g.iq2));
}

__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Sersic (Sec. 4.1): I = I_e exp(-b [(r/r_e)^(1/n) - 1]),
// I_e = F b^(2n) / (2 pi q r_e^2 n Gamma(2n) e^b).
// Values: I, then dI/d{x0, y0, mag, ln r_e, ln n, q, theta}.
struct SersicK {
    Geo g;
    float lnIe2, b, b2, inv2n, l2re2, bn, cn, nbp, bl2n;
    static constexpr int NV = 8;
};

__device__ inline void sersic_prep(const double *u, double m0, int H, int W, int osf, int osw, SersicK &k)
{
    double x0 = u[0], y0 = u[1], m = u[2], lnre = u[3], lnn = u[4], q = u[5], th = u[6];
    double n = exp(lnn);
    double bp;
    double b = sersic_b(n, &bp);
    double psi = digamma(2.0 * n);
    double lnIe = -0.4 * kLn10 * (m - m0) + 2.0 * n * log(b) - log(2.0 * kPi * q * n) - 2.0 * lnre
                  - lgamma(2.0 * n) - b;
    geo_prep(x0, y0, q, th, H, W, osf, osw, k.g);
    k.lnIe2 = (float)(lnIe * kLog2e);
    k.b = (float)b;
    k.b2 = (float)(b * kLog2e);
    k.inv2n = (float)(0.5 / n);
    k.l2re2 = (float)(2.0 * lnre * kLog2e);
    k.bn = (float)(b / n);
    // d ln I / d ln n = cn - n b' z + b z ln(r^2/re^2) / (2n)
    k.cn = (float)(n * (2.0 * log(b) + 2.0 * n * bp / b - 2.0 * psi) - 1.0);
    k.nbp = (float)(n * bp);
    k.bl2n = (float)(b * kLn2 / (2.0 * n));
}

__device__ inline void sersic_pt(const SersicK &k, float dx, float dy, float *v)
{
    RadialPt p = radial(k.g, dx, dy);
    float L2 = __log2f(p.r2) - k.l2re2;               // log2(r^2 / r_e^2)
    float z = exp2f(L2 * k.inv2n);                     // (r / r_e)^(1/n)
    float I = exp2f(k.lnIe2 - k.b2 * (z - 1.0f));
    float dl = -k.b * z * k.inv2n * frcp(p.r2);       // d ln I / d r^2
    float dx0, dy0, dq, dth;
    geometry_derivs(k.g, p, I, dl, -k.g.iq, dx0, dy0, dq, dth);
    v[0] = I;
    v[1] = dx0;
    v[2] = dy0;
    v[3] = kDMag * I;
    v[4] = I * (-2.0f + k.bn * z);
    v[5] = I * (k.cn - k.nbp * z + k.bl2n * z * L2);
    v[6] = dq;
    v[7] = dth;
}

// Exponential disk (Sec. 4.2.1): I = I0 exp(-r / r_s), I0 = F / (2 pi q r_s^2).
// Values: I, then dI/d{x0, y0, mag, ln r_s, q, theta}.
struct ExpDiskK {
    Geo g;
    float lnI02, irs, irs2;
    static constexpr int NV = 7;
};

__device__ inline void expdisk_prep(const double *u, double m0, int H, int W, int osf, int osw, ExpDiskK &k)
{
    double x0 = u[0], y0 = u[1], m = u[2], lnrs = u[3], q = u[4], th = u[5];
    double lnI0 = -0.4 * kLn10 * (m - m0) - log(2.0 * kPi * q) - 2.0 * lnrs;
    geo_prep(x0, y0, q, th, H, W, osf, osw, k.g);
    k.lnI02 = (float)(lnI0 * kLog2e);
    k.irs = (float)exp(-lnrs);
    k.irs2 = (float)(exp(-lnrs) * kLog2e);
}

__device__ inline void expdisk_pt(const ExpDiskK &k, float dx, float dy, float *v)
{
    RadialPt p = radial(k.g, dx, dy);
    float r = __builtin_amdgcn_sqrtf(p.r2);
    float I = exp2f(k.lnI02 - r * k.irs2);
    float dl = -0.5f * k.irs * frcp(r);               // d ln I / d r^2
    float dx0, dy0, dq, dth;
    geometry_derivs(k.g, p, I, dl, -k.g.iq, dx0, dy0, dq, dth);
    v[0] = I;
    v[1] = dx0;
    v[2] = dy0;
    v[3] = kDMag * I;
    v[4] = I * (-2.0f + r * k.irs);
    v[5] = dq;
    v[6] = dth;
}

// ---------------------------------------------------------------- families
// A family fixes, at compile time, the components of a model, the layout of
// the internal LM vector u and the image planes: plane 0 is the summed
// convolved light, plane 1 + k the derivative with respect to u_k (sky, the
// last entry of u, has the constant derivative 1 and no plane).

// Single Sersic + sky. u = x0 y0 mag ln r_e ln n q theta sky.
struct FamSersic {
    static constexpr int P = 8, NPL = 8, NCOMP = 1, SKY = 7;
    static constexpr int NWV = SersicK::NV;           // window values per pixel
    __host__ __device__ static constexpr int kind(int k)
    {
        return k == 0 ? KX0 : k == 1 ? KY0 : k == 2 ? KMAG : k == 3 ? KSCALE : k == 4 ? KN
             : k == 5 ? KQ : k == 6 ? KPA : KSKY;
    }
    struct Prep {
        SersicK s;
        float sky;
    };
    __device__ static void prep(const double *u, double m0, int H, int W, int osf, int osw, Prep &p)
    {
        sersic_prep(u, m0, H, W, osf, osw, p.s);
        p.sky = (float)u[7];
    }
    __device__ static const Geo &geo(const Prep &p, int) { return p.s.g; }
    __device__ static void comp_pt(const Prep &p, int, float dx, float dy, float *v) { sersic_pt(p.s, dx, dy, v); }
    // add component c's values v into the plane vector
    __device__ static void scatter(int, const float *v, float *pl)
    {
#pragma unroll
        for (int i = 0; i < 8; ++i) pl[i] += v[i];
    }
    // start vector from image moments: centre, magnitude, radius, axis ratio,
    // PA (deg), border sky; n = 2 for a lone Sersic
    __device__ static void default_guess(double xc, double yc, double mg, double r0, double q0, double pa0,
                                         double sky0, double, double *nat)
    {
        nat[0] = xc; nat[1] = yc; nat[2] = mg; nat[3] = r0; nat[4] = 2.0; nat[5] = q0; nat[6] = pa0; nat[7] = sky0;
    }
    // canonical form: (q index, theta index, scale indices)
    static constexpr int NCAN = 1;
    __host__ __device__ static void canon(int c, int &iq, int &ith, int &is0, int &is1)
    {
        iq = 5; ith = 6; is0 = 3; is1 = -1;
    }
};

// Sersic bulge + exponential disk with a shared centre + sky.
// u = x0 y0 | mag_b ln r_e ln n q_b theta_b | mag_d ln r_s q_d theta_d | sky.
struct FamBulgeDisk {
    static constexpr int P = 12, NPL = 12, NCOMP = 2, SKY = 11;
    static constexpr int NWV = SersicK::NV;           // the larger of the two
    __host__ __device__ static constexpr int kind(int k)
    {
        return k == 0 ? KX0 : k == 1 ? KY0 : k == 2 ? KMAG : k == 3 ? KSCALE : k == 4 ? KN
             : k == 5 ? KQ : k == 6 ? KPA : k == 7 ? KMAG : k == 8 ? KSCALE : k == 9 ? KQ
             : k == 10 ? KPA : KSKY;
    }
    struct Prep {
        SersicK s;
        ExpDiskK e;
        float sky;
    };
    __device__ static void prep(const double *u, double m0, int H, int W, int osf, int osw, Prep &p)
    {
        sersic_prep(u, m0, H, W, osf, osw, p.s);
        double ue[6] = {u[0], u[1], u[7], u[8], u[9], u[10]};
        expdisk_prep(ue, m0, H, W, osf, osw, p.e);
        p.sky = (float)u[11];
    }
    __device__ static const Geo &geo(const Prep &p, int c) { return c == 0 ? p.s.g : p.e.g; }
    __device__ static void comp_pt(const Prep &p, int c, float dx, float dy, float *v)
    {
        if (c == 0) sersic_pt(p.s, dx, dy, v);
        else expdisk_pt(p.e, dx, dy, v);
    }
    __device__ static void scatter(int c, const float *v, float *pl)
    {
        if (c == 0) {
#pragma unroll
            for (int i = 0; i < 8; ++i) pl[i] += v[i];
        } else {
            pl[0] += v[0];
            pl[1] += v[1];
            pl[2] += v[2];
#pragma unroll
            for (int i = 3; i < 7; ++i) pl[5 + i] += v[i];   // planes 8..11 = u 7..10
        }
    }
    // the flux is split evenly; bulge n = 4, r_e = r0 / 2; disk r_s = r0 / b_1
    __device__ static void default_guess(double xc, double yc, double mg, double r0, double q0, double pa0,
                                         double sky0, double, double *nat)
    {
        double ms = mg + 2.5 * log10(2.0);
        nat[0] = xc; nat[1] = yc;
        nat[2] = ms; nat[3] = 0.5 * r0; nat[4] = 4.0; nat[5] = q0; nat[6] = pa0;
        nat[7] = ms; nat[8] = r0 / 1.678347; nat[9] = q0; nat[10] = pa0;
        nat[11] = sky0;
    }
    static constexpr int NCAN = 2;
    __host__ __device__ static void canon(int c, int &iq, int &ith, int &is0, int &is1)
    {
        if (c == 0) { iq = 5; ith = 6; is0 = 3; is1 = -1; }
        else { iq = 9; ith = 10; is0 = 8; is1 = -1; }
    }
};

}  // namespace gm
