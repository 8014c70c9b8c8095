// gm_device.h -- device-side numerics of libgmfit: FP64 special functions for
// the per-galaxy scalar prologue, profile values and derivatives at one point,
// and the model families the kernels are compiled for.
//
// Precision: the light itself (the model plane) is evaluated and carried in
// FP64, so that chi^2 differences between nearby parameter vectors are exact
// to far below the step sizes the LM compares; the derivative planes are FP32.
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

// Butterfly sum over the 64 lanes of a wave; every lane gets the total, and
// the order of additions is fixed.
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// P(a, x) (regularised lower incomplete gamma) and dP/da, one wave: lane l
// sums the terms k = l, l + 64, l + 128 of the series P = sum_k T_k,
// T_k = e^-x x^(a+k) / Gamma(a+k+1), dT_k/da = T_k (ln x - psi(a+k+1)).
// 192 terms cover x <= a + 20 for a <= 20 to double precision.
__device__ inline void gammainc_wave(double a, double x, int lane, bool want_da, double *P, double *dPda)
{
    double lx = log(x), sp = 0.0, sd = 0.0;
#pragma unroll 1
    for (int m = 0; m < 3; ++m) {
        double k = (double)(lane + 64 * m);
        double T = exp((a + k) * lx - x - lgamma(a + k + 1.0));
        sp += T;
        if (want_da) sd += T * (lx - digamma(a + k + 1.0));
    }
    *P = wave_sum(sp);
    if (want_da) *dPda = wave_sum(sd);
}

// nu_n of the Sersic law (the b_n of Sec. 4.1): the root of P(2n, b) = 1/2,
// the half-light condition; Newton from the asymptotic expansion of
// Ciotti & Bertin (1999), safeguarded by a bisection bracket; db/dn by
// implicit differentiation, -2 (dP/da) / (dP/dx).  All lanes of one wave.
__device__ inline double sersic_b_wave(double n, int lane, double *dbdn)
{
    double a = 2.0 * n, lo = 0.0, hi = a + 20.0;
    double in = 1.0 / n;
    double b = a - 1.0 / 3.0 + in * (4.0 / 405.0 + in * (46.0 / 25515.0 + in * (131.0 / 1148175.0)));
    if (!(b > lo && b < hi)) b = 0.5 * a;
    double lga = lgamma(a);
#pragma unroll 1
    for (int it = 0; it < 60; ++it) {
        double P;
        gammainc_wave(a, b, lane, false, &P, nullptr);
        double f = P - 0.5;
        if (f > 0.0) hi = b; else lo = b;
        double fp = exp((a - 1.0) * log(b) - b - lga);
        double nb = b - f / fp;
        if (!(nb > lo && nb < hi)) nb = 0.5 * (lo + hi);
        double st = fabs(nb - b);
        b = nb;
        if (st < 1e-14 * b) break;
    }
    double P, dPa;
    gammainc_wave(a, b, lane, true, &P, &dPa);
    *dbdn = -2.0 * dPa / exp((a - 1.0) * log(b) - b - lga);
    return b;
}

// ---------------------------------------------------------------- components
// Orientation and oversampling window (rows wi0..wi1, cols wj0..wj1) of a
// radial component.
struct Geo {
    double x0, y0, c, s, iq2;
    float cf, sf, iqf, iq2f;
    int wi0, wi1, wj0, wj1;
};

__device__ inline void geo_prep(double x0, double y0, double q, double th, int H, int W, int osf, int osw, Geo &g)
{
    g.x0 = x0;
    g.y0 = y0;
    g.c = cos(th);
    g.s = sin(th);
    g.iq2 = 1.0 / (q * q);
    g.cf = (float)g.c;
    g.sf = (float)g.s;
    g.iqf = (float)(1.0 / q);
    g.iq2f = (float)g.iq2;
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

// A point in the component frame.  F64: rotated coordinates and r^2 in FP64
// (for the FP64 light), else FP32 from the FP64 offsets.
template <bool F64>
struct Pt {
    double X, Y, r2;
    float Xf, Yf, r2f, gmask;
};

template <bool F64>
__device__ inline Pt<F64> frame(const Geo &g, double dx, double dy)
{
    Pt<F64> p;
    if constexpr (F64) {
        p.X = g.c * dx + g.s * dy;
        p.Y = -g.s * dx + g.c * dy;
        p.r2 = p.X * p.X + p.Y * p.Y * g.iq2;
        p.gmask = 1.0f;
        if (p.r2 < 1e-12) {       // cusp floor r^2 >= 1e-12 px^2: geometry derivatives vanish
            p.r2 = 1e-12;
            p.gmask = 0.0f;
        }
        p.Xf = (float)p.X;
        p.Yf = (float)p.Y;
        p.r2f = (float)p.r2;
    } else {
        float dxf = (float)dx, dyf = (float)dy;
        p.Xf = g.cf * dxf + g.sf * dyf;
        p.Yf = -g.sf * dxf + g.cf * dyf;
        p.r2f = p.Xf * p.Xf + p.Yf * p.Yf * g.iq2f;
        p.gmask = 1.0f;
        if (p.r2f < 1e-12f) {
            p.r2f = 1e-12f;
            p.gmask = 0.0f;
        }
    }
    return p;
}

// Given I and d ln I / d r^2, the derivatives through r^2 with respect to the
// centre, the axis ratio (plus the direct -1/q of flux-normalised profiles)
// and the angle.
template <bool F64>
__device__ inline void geometry_derivs(const Geo &g, const Pt<F64> &p, float I, float dl, float dq_direct, float *d)
{
    float gd = I * dl * p.gmask;
    float Yq = p.Yf * g.iq2f;
    d[0] = gd * (-2.0f * p.Xf * g.cf + 2.0f * Yq * g.sf);
    d[1] = gd * (-2.0f * p.Xf * g.sf - 2.0f * Yq * g.cf);
    d[2] = gd * (-2.0f * p.Yf * Yq * g.iqf) + I * dq_direct;
    d[3] = gd * (2.0f * p.Xf * p.Yf * (1.0f - g.iq2f));
}

__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Sersic (Sec. 4.1): I = I_e exp(-b [(r/r_e)^(1/n) - 1]),
// I_e = F b^(2n) / (2 pi q r_e^2 n Gamma(2n) e^b).
// Derivatives (FP32): dI/d{x0, y0, mag, ln r_e, ln n, q, theta}.
struct SersicK {
    Geo g;
    double lnIe, b, inv2n, lnre2;
    float lnIe2f, bf, b2f, inv2nf, l2re2f, bnf, cnf, nbpf, bl2nf;
    static constexpr int ND = 7;
};

// All lanes of wave 0 call this (the b_n series is spread over the lanes).
__device__ inline void sersic_prep(const double *u, double m0, int H, int W, int osf, int osw, int lane, SersicK &k)
{
    double x0 = u[0], y0 = u[1], m = u[2], lnre = u[3], lnn = u[4], q = u[5], th = u[6];
    double n = exp(lnn);
    double bp;
    double b = sersic_b_wave(n, lane, &bp);
    double psi = digamma(2.0 * n);
    double lnIe = -0.4 * kLn10 * (m - m0) + 2.0 * n * log(b) - log(2.0 * kPi * q * n) - 2.0 * lnre
                  - lgamma(2.0 * n) - b;
    geo_prep(x0, y0, q, th, H, W, osf, osw, k.g);
    k.lnIe = lnIe;
    k.b = b;
    k.inv2n = 0.5 / n;
    k.lnre2 = 2.0 * lnre;
    k.lnIe2f = (float)(lnIe * kLog2e);
    k.bf = (float)b;
    k.b2f = (float)(b * kLog2e);
    k.inv2nf = (float)(0.5 / n);
    k.l2re2f = (float)(2.0 * lnre * kLog2e);
    k.bnf = (float)(b / n);
    // d ln I / d ln n = cn - n b' z + b z ln(r^2/re^2) / (2n)
    k.cnf = (float)(n * (2.0 * log(b) + 2.0 * n * bp / b - 2.0 * psi) - 1.0);
    k.nbpf = (float)(n * bp);
    k.bl2nf = (float)(b * kLn2 / (2.0 * n));
}

template <bool F64>
__device__ inline void sersic_pt(const SersicK &k, double dx, double dy, double &I64, float *d)
{
    Pt<F64> p = frame<F64>(k.g, dx, dy);
    float I, z, L2;
    if constexpr (F64) {
        double L = log(p.r2) - k.lnre2;                  // ln(r^2 / r_e^2)
        double zd = exp(L * k.inv2n);                    // (r / r_e)^(1/n)
        I64 = exp(k.lnIe - k.b * (zd - 1.0));
        I = (float)I64;
        z = (float)zd;
        L2 = (float)(L * kLog2e);
    } else {
        L2 = __log2f(p.r2f) - k.l2re2f;
        z = exp2f(L2 * k.inv2nf);
        I = exp2f(k.lnIe2f - k.b2f * (z - 1.0f));
        I64 = I;
    }
    float dl = -k.bf * z * k.inv2nf * frcp(p.r2f);     // d ln I / d r^2
    float gd[4];
    geometry_derivs<F64>(k.g, p, I, dl, -k.g.iqf, gd);
    d[0] = gd[0];
    d[1] = gd[1];
    d[2] = kDMag * I;
    d[3] = I * (-2.0f + k.bnf * z);
    d[4] = I * (k.cnf - k.nbpf * z + k.bl2nf * z * L2);
    d[5] = gd[2];
    d[6] = gd[3];
}

// Exponential disk (Sec. 4.2.1): I = I0 exp(-r / r_s), I0 = F / (2 pi q r_s^2).
// Derivatives: dI/d{x0, y0, mag, ln r_s, q, theta}.
struct ExpDiskK {
    Geo g;
    double lnI0, irs;
    float lnI02f, irsf, irs2f;
    static constexpr int ND = 6;
};

__device__ inline void expdisk_prep(const double *u, double m0, int H, int W, int osf, int osw, ExpDiskK &k)
{
    double x0 = u[0], y0 = u[1], m = u[2], lnrs = u[3], q = u[4], th = u[5];
    double lnI0 = -0.4 * kLn10 * (m - m0) - log(2.0 * kPi * q) - 2.0 * lnrs;
    geo_prep(x0, y0, q, th, H, W, osf, osw, k.g);
    k.lnI0 = lnI0;
    k.irs = exp(-lnrs);
    k.lnI02f = (float)(lnI0 * kLog2e);
    k.irsf = (float)k.irs;
    k.irs2f = (float)(k.irs * kLog2e);
}

template <bool F64>
__device__ inline void expdisk_pt(const ExpDiskK &k, double dx, double dy, double &I64, float *d)
{
    Pt<F64> p = frame<F64>(k.g, dx, dy);
    float I, r;
    if constexpr (F64) {
        double rd = sqrt(p.r2);
        I64 = exp(k.lnI0 - rd * k.irs);
        I = (float)I64;
        r = (float)rd;
    } else {
        r = __builtin_amdgcn_sqrtf(p.r2f);
        I = exp2f(k.lnI02f - r * k.irs2f);
        I64 = I;
    }
    float dl = -0.5f * k.irsf * frcp(r);                // d ln I / d r^2
    float gd[4];
    geometry_derivs<F64>(k.g, p, I, dl, -k.g.iqf, gd);
    d[0] = gd[0];
    d[1] = gd[1];
    d[2] = kDMag * I;
    d[3] = I * (-2.0f + r * k.irsf);
    d[4] = gd[2];
    d[5] = gd[3];
}

// ---------------------------------------------------------------- families
// A family fixes, at compile time, the components of a model, the layout of
// the internal LM vector u and the image planes: plane 0 is the summed
// convolved light (FP64), plane 1 + k the derivative with respect to u_k
// (FP32; sky, the last entry of u, has the constant derivative 1 and no plane).

// Single Sersic + sky. u = x0 y0 mag ln r_e ln n q theta sky.
struct FamSersic {
    static constexpr int P = 8, NPL = 8, NCOMP = 1, SKY = 7;
    static constexpr int ND = SersicK::ND;             // derivative values per window pixel
    __host__ __device__ static constexpr int kind(int k)
    {
        return k == 0 ? KX0 : k == 1 ? KY0 : k == 2 ? KMAG : k == 3 ? KSCALE : k == 4 ? KN
             : k == 5 ? KQ : k == 6 ? KPA : KSKY;
    }
    struct Prep {
        SersicK s;
        double sky;
    };
    __device__ static void prep(const double *u, double m0, int H, int W, int osf, int osw, int lane, Prep &p)
    {
        sersic_prep(u, m0, H, W, osf, osw, lane, p.s);
        p.sky = u[7];
    }
    __device__ static const Geo &geo(const Prep &p, int) { return p.s.g; }
    template <bool F64>
    __device__ static void comp_pt(const Prep &p, int, double dx, double dy, double &I, float *d)
    {
        sersic_pt<F64>(p.s, dx, dy, I, d);
    }
    // add component c's derivatives into the derivative planes (index = plane - 1)
    __device__ static void scatter(int, const float *d, float *dp)
    {
#pragma unroll
        for (int i = 0; i < 7; ++i) dp[i] += d[i];
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
    __host__ __device__ static void canon(int, int &iq, int &ith, int &is0, int &is1)
    {
        iq = 5; ith = 6; is0 = 3; is1 = -1;
    }
};

// Sersic bulge + exponential disk with a shared centre + sky.
// u = x0 y0 | mag_b ln r_e ln n q_b theta_b | mag_d ln r_s q_d theta_d | sky.
struct FamBulgeDisk {
    static constexpr int P = 12, NPL = 12, NCOMP = 2, SKY = 11;
    static constexpr int ND = SersicK::ND;             // the larger of the two
    __host__ __device__ static constexpr int kind(int k)
    {
        return k == 0 ? KX0 : k == 1 ? KY0 : k == 2 ? KMAG : k == 3 ? KSCALE : k == 4 ? KN
             : k == 5 ? KQ : k == 6 ? KPA : k == 7 ? KMAG : k == 8 ? KSCALE : k == 9 ? KQ
             : k == 10 ? KPA : KSKY;
    }
    struct Prep {
        SersicK s;
        ExpDiskK e;
        double sky;
    };
    __device__ static void prep(const double *u, double m0, int H, int W, int osf, int osw, int lane, Prep &p)
    {
        sersic_prep(u, m0, H, W, osf, osw, lane, p.s);
        double ue[6] = {u[0], u[1], u[7], u[8], u[9], u[10]};
        expdisk_prep(ue, m0, H, W, osf, osw, p.e);
        p.sky = u[11];
    }
    __device__ static const Geo &geo(const Prep &p, int c) { return c == 0 ? p.s.g : p.e.g; }
    template <bool F64>
    __device__ static void comp_pt(const Prep &p, int c, double dx, double dy, double &I, float *d)
    {
        if (c == 0) {
            sersic_pt<F64>(p.s, dx, dy, I, d);
        } else {
            expdisk_pt<F64>(p.e, dx, dy, I, d);
            d[6] = 0.0f;
        }
    }
    __device__ static void scatter(int c, const float *d, float *dp)
    {
        if (c == 0) {
#pragma unroll
            for (int i = 0; i < 7; ++i) dp[i] += d[i];
        } else {
            dp[0] += d[0];
            dp[1] += d[1];
#pragma unroll
            for (int i = 2; i < 6; ++i) dp[5 + i] += d[i];   // planes 8..11 = u 7..10
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
