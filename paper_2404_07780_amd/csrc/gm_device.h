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
// Ferrer a and King alpha (positive exponents) go through their log, Ferrer b
// and the boxiness as they are.
enum Kind : int { KX0 = 1, KY0, KMAG, KAMP, KSCALE, KN, KQ, KPA, KSKY, KSKYG, KBOX, KFA, KFB, KKAL };

__host__ __device__ inline bool log_kind(int kind) { return kind == KSCALE || kind == KN || kind == KFA || kind == KKAL; }

__host__ __device__ inline double nat_to_u(int kind, double p)
{
    if (log_kind(kind)) return log(p);
    if (kind == KPA) return p * (kPi / 180.0);
    return p;
}
__host__ __device__ inline double u_to_nat(int kind, double u)
{
    if (log_kind(kind)) return exp(u);
    if (kind == KPA) return u * (180.0 / kPi);
    return u;
}
// d(natural) / d(u)
__host__ __device__ inline double dnat_du(int kind, double p)
{
    if (log_kind(kind)) return p;
    if (kind == KPA) return 180.0 / kPi;
    return 1.0;
}

// ---------------------------------------------------------------- FP64 point functions
// Base-2 exponential and logarithm of the FP64 light at every region and
// window point (the library's exp and log are general-purpose and several
// times longer).  Both are within about 2 ulp of the exact values.
//
// 2^x: x = k + f with k = rint(x), |f| <= 1/2, 2^f = e^y with y = f ln 2,
// |y| <= 0.347, by its Taylor series to y^12 (remainder below 1e-17), scaled
// by 2^k (k clamped: 2^x is 0 or infinite there; a NaN x gives NaN).
__host__ __device__ inline double exp2_pt(double x)
{
    const double k = rint(x);
    const double y = (x - k) * kLn2;
    double p = 1.0 / 479001600.0;
    p = fma(p, y, 1.0 / 39916800.0);
    p = fma(p, y, 1.0 / 3628800.0);
    p = fma(p, y, 1.0 / 362880.0);
    p = fma(p, y, 1.0 / 40320.0);
    p = fma(p, y, 1.0 / 5040.0);
    p = fma(p, y, 1.0 / 720.0);
    p = fma(p, y, 1.0 / 120.0);
    p = fma(p, y, 1.0 / 24.0);
    p = fma(p, y, 1.0 / 6.0);
    p = fma(p, y, 0.5);
    p = fma(p, y, 1.0);
    p = fma(p, y, 1.0);
    return ldexp(p, (int)fmin(fmax(k, -2200.0), 2200.0));
}

// log2 x for finite x > 0: x = m 2^e with m in [1/sqrt 2, sqrt 2), and
// ln m = 2 atanh s = 2 (s + s^3/3 + s^5/5 + ...), s = (m - 1)/(m + 1),
// |s| <= 3 - 2 sqrt 2, summed to s^23 (remainder below 1e-18).
__host__ __device__ inline double log2_pt(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, z, 1.0 / 21.0);
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    p = fma(p, z, 1.0);
    return (double)e + s * (p * (2.0 * kLog2e));
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

// Cross-lane moves of an FP64 value: a DPP row move (CTRL a compile-time
// DPP control; lanes whose source falls outside the 16-lane row read 0) and
// the value of one lane (wave-uniform lane index).  The whole wave must be
// active.
template <int CTRL>
__device__ inline double dpp_move(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ inline double lane_value(double v, int lane)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)lo);
}

// Sum over the 64 lanes of a wave; every lane gets the total.  Within each
// 16-lane row a shift-and-add ladder (row_shr 1, 2, 4, 8) leaves the row sum
// in the row's last lane; the four row sums are then added in row order.
// The order of additions is fixed, so results are reproducible.
__device__ inline double wave_sum(double v)
{
    v += dpp_move<0x111>(v);
    v += dpp_move<0x112>(v);
    v += dpp_move<0x114>(v);
    v += dpp_move<0x118>(v);
    return ((lane_value(v, 15) + lane_value(v, 31)) + lane_value(v, 47)) + lane_value(v, 63);
}

// Inclusive prefix sum over the 64 lanes (lane l gets lanes 0..l), in a
// fixed order: the shift-and-add ladder of wave_sum within each 16-lane row,
// then the totals of the rows before.
__device__ inline double wave_scan(double v, int lane)
{
    v += dpp_move<0x111>(v);
    v += dpp_move<0x112>(v);
    v += dpp_move<0x114>(v);
    v += dpp_move<0x118>(v);
    const double t0 = lane_value(v, 15), t1 = lane_value(v, 31), t2 = lane_value(v, 47);
    const int row = lane >> 4;
    const double off = row == 0 ? 0.0 : row == 1 ? t0 : row == 2 ? t0 + t1 : (t0 + t1) + t2;
    return v + off;
}

// P(a, x) (regularised lower incomplete gamma) and dP/da, one wave: lane l
// sums the terms k = l, l + 64, l + 128 of the series P = sum_k T_k,
// T_k = e^-x x^(a+k) / Gamma(a+k+1), dT_k/da = T_k (ln x - psi(a+k+1)).
// ln Gamma(a+k+1) = ln Gamma(a+1) + sum_{j=1..k} ln(a+j) and
// psi(a+k+1) = psi(a+1) + sum_{j=1..k} 1/(a+j) are prefix sums over the
// lanes (lga1 = ln Gamma(a+1), psi1 = psi(a+1)).  192 terms cover
// x <= a + 20 for a <= 20 to double precision; a block of 64 terms is
// skipped once the last term of the previous block is below 1e-17 of the
// sum and the ratio of successive terms, x / (a + k), is below 1/2 (the rest
// of the series is then below twice that last term).
__device__ inline void gammainc_wave(double a, double x, double lga1, double psi1, int lane, bool want_da, double *P,
                                     double *dPda)
{
    double lx = log(x), sp = 0.0, sd = 0.0, clg = lga1, cps = psi1;
#pragma unroll 1
    for (int m = 0; m < 3; ++m) {
        const double k = (double)(lane + 64 * m);
        const double lg = wave_scan(k >= 1.0 ? log(a + k) : 0.0, lane);
        const double T = exp((a + k) * lx - x - (clg + lg));
        sp += T;
        clg += lane_value(lg, 63);
        if (want_da) {
            const double ps = wave_scan(k >= 1.0 ? 1.0 / (a + k) : 0.0, lane);
            sd += T * (lx - (cps + ps));
            cps += lane_value(ps, 63);
        }
        if (m < 2 && x < 0.5 * (a + 64.0 * (m + 1)) && lane_value(T, 63) < 1e-17 * wave_sum(sp)) break;
    }
    *P = wave_sum(sp);
    if (want_da) *dPda = wave_sum(sd);
}

// nu_n of the Sersic law (the b_n of Sec. 4.1): the root of P(2n, b) = 1/2,
// the half-light condition; Newton from the asymptotic expansion of
// Ciotti & Bertin (1999), safeguarded by a bisection bracket, stopped when
// the error after a Newton step, about |f''/(2 f')| step^2 with
// f''/f' = (a - 1)/b - 1, is below 1e-16 b (or a step is below 1e-14 b);
// db/dn by implicit differentiation, -2 (dP/da) / (dP/dx).  All lanes of
// one wave.  Also returns ln Gamma(2n) and psi(2n) (= psi(2n + 1) - 1/(2n)),
// which the solve computes on the way.
__device__ inline double sersic_b_wave(double n, int lane, double *dbdn, double *lg2n, double *psi2n)
{
    double a = 2.0 * n, lo = 0.0, hi = a + 20.0;
    double in = 1.0 / n;
    double b = a - 1.0 / 3.0 + in * (4.0 / 405.0 + in * (46.0 / 25515.0 + in * (131.0 / 1148175.0)));
    if (!(b > lo && b < hi)) b = 0.5 * a;
    const double lga = lgamma(a), lga1 = lga + log(a);
#pragma unroll 1
    for (int it = 0; it < 60; ++it) {
        double P;
        gammainc_wave(a, b, lga1, 0.0, lane, false, &P, nullptr);
        double f = P - 0.5;
        if (f > 0.0) hi = b; else lo = b;
        double fp = exp((a - 1.0) * log(b) - b - lga);
        double nb = b - f / fp;
        const bool newton = nb > lo && nb < hi;
        if (!newton) nb = 0.5 * (lo + hi);
        double st = fabs(nb - b);
        const double pred = 0.5 * fabs((a - 1.0) / b - 1.0) * st * st;
        b = nb;
        if (st < 1e-14 * b || (newton && pred < 1e-16 * b)) break;
    }
    double P, dPa;
    const double psi1 = digamma(a + 1.0);
    gammainc_wave(a, b, lga1, psi1, lane, true, &P, &dPa);
    *dbdn = -2.0 * dPa / exp((a - 1.0) * log(b) - b - lga);
    *lg2n = lga;
    *psi2n = psi1 - 1.0 / a;
    return b;
}

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 32 x 32 -> 64-bit multiplications with a Weyl-sequence key schedule.
struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Poisson(1) deviate by inversion of a uniform 32-bit word: the number of
// thresholds T_k <= x, T_k = floor(2^32 F(k)) for k = 0..11 with the CDF
// F(k) = e^-1 sum_{j<=k} 1/j! summed in that order in FP64 (12 for the
// remaining mass, below 1e-9).
struct Poisson1Table {
    uint32_t t[12];
};
__host__ __device__ constexpr Poisson1Table poisson1_table()
{
    Poisson1Table pt{};
    double term = 0.36787944117144233;      // e^-1, correctly rounded
    double cdf = term;
    pt.t[0] = (uint32_t)(cdf * 4294967296.0);
    for (int k = 1; k < 12; ++k) {
        term = term / (double)k;
        cdf = cdf + term;
        pt.t[k] = (uint32_t)(cdf * 4294967296.0);
    }
    return pt;
}
__host__ __device__ inline int poisson1(uint32_t x)
{
    constexpr Poisson1Table T = poisson1_table();
    int k = 0;
#pragma unroll
    for (int j = 0; j < 12; ++j) k += (x >= T.t[j]) ? 1 : 0;
    return k;
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

// ---------------------------------------------------------------- components
// Every component type provides: its LM slots (NS, kind(s)), the slots of
// its axis ratio, angle and scales (canonical form), an FP64 prologue
// prep(us, cst, ...) from its slot values us (u-space) and shape constants cst,
// a point evaluation pt<F64>(k, dx, dy, I, d) of the light I (FP64 if F64)
// and its FP32 derivatives d[s] = dI/du_s, and the moment-based start values.

// Sersic (Sec. 4.1): I = I_e exp(-b [(r/r_e)^(1/n) - 1]),
// I_e = F b^(2n) / (2 pi q r_e^2 n Gamma(2n) e^b).  Slots x0 y0 mag ln r_e ln n q theta.
struct Sersic {
    struct K {
        Geo g;
        double lnIe, b, inv2n, lnre2, lnIe2, b2, l2re2;
        float bf, inv2nf, l2re2f, lnIe2f, b2f, bnf, cnf, nbpf, bl2nf;
    };
    static constexpr int NS = 7, IQ = 5, ITH = 6, IS0 = 3, IS1 = -1;
    __host__ __device__ static constexpr int kind(int s)
    {
        return s == 0 ? KX0 : s == 1 ? KY0 : s == 2 ? KMAG : s == 3 ? KSCALE : s == 4 ? KN : s == 5 ? KQ : KPA;
    }
    // all lanes of wave 0 call this (the b_n series is spread over the lanes)
    __device__ static void prep(const double *u, const double *, double m0, int H, int W, int osf, int osw, int lane,
                                K &k)
    {
        double x0 = u[0], y0 = u[1], m = u[2], lnre = u[3], lnn = u[4], q = u[5], th = u[6];
        double n = exp(lnn);
        double bp, lg2n, psi;
        double b = sersic_b_wave(n, lane, &bp, &lg2n, &psi);
        double lnIe = -0.4 * kLn10 * (m - m0) + 2.0 * n * log(b) - log(2.0 * kPi * q * n) - 2.0 * lnre - lg2n - b;
        geo_prep(x0, y0, q, th, H, W, osf, osw, k.g);
        k.lnIe = lnIe;
        k.b = b;
        k.inv2n = 0.5 / n;
        k.lnre2 = 2.0 * lnre;
        k.lnIe2 = lnIe * kLog2e;
        k.b2 = b * kLog2e;
        k.l2re2 = 2.0 * lnre * kLog2e;
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
    __device__ static void pt(const K &k, double dx, double dy, double &I64, float *d)
    {
        Pt<F64> p = frame<F64>(k.g, dx, dy);
        float I, z, L2;
        if constexpr (F64) {
            const double L2d = log2_pt(p.r2) - k.l2re2;      // log2(r^2 / r_e^2)
            const double zd = exp2_pt(L2d * k.inv2n);        // (r / r_e)^(1/n)
            I64 = exp2_pt(k.lnIe2 - k.b2 * (zd - 1.0));
            I = (float)I64;
            z = (float)zd;
            L2 = (float)L2d;
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
    // natural start values: r_e = r0 (r0 / 2 next to another component), n = 2 (4)
    __device__ static void guess(double xc, double yc, double m, double r0, double q0, double pa0, double, int nrad,
                                 double *v)
    {
        v[0] = xc; v[1] = yc; v[2] = m; v[3] = nrad > 1 ? 0.5 * r0 : r0; v[4] = nrad > 1 ? 4.0 : 2.0;
        v[5] = q0; v[6] = pa0;
    }
};

// Boxy Sersic (Sec. 4.1, eqs. (r) and (rbox)): the Sersic law of the
// generalised radius r = (|X|^c + |Y/q|^c)^(1/c), c = B + 2, in the frame
// rotated by the position angle, and I_e multiplied by
// r_box = pi c / (2 beta(1/c, 1/c)).  Slots x0 y0 mag ln r_e ln n q theta B.
// With G = d ln I / d ln r = -b z / n (z = (r / r_e)^(1/n)):
//   d ln r / dX = A / (S X), d ln r / dY = Bq / (S Y), A = |X|^c,
//   Bq = |Y/q|^c, S = A + Bq (0 on an axis: c > 1);
//   d ln r / dq = -Bq / (q S);
//   d ln r / dc = -ln S / c^2 + (A ln|X| + Bq ln|Y/q|) / (c S);
//   d ln r_box / dc = 1/c + 2 (psi(1/c) - psi(2/c)) / c^2.
struct SersicBox {
    struct K : Sersic::K {
        double c, ic, iq;
        float cf, icf, dlrboxf;
    };
    static constexpr int NS = 8, IQ = 5, ITH = 6, IS0 = 3, IS1 = -1;
    __host__ __device__ static constexpr int kind(int s) { return s == 7 ? KBOX : Sersic::kind(s); }
    __device__ static void prep(const double *u, const double *cst, double m0, int H, int W, int osf, int osw,
                                int lane, K &k)
    {
        Sersic::prep(u, cst, m0, H, W, osf, osw, lane, k);
        const double c = u[7] + 2.0, ic = 1.0 / c;
        const double lnrbox = log(0.5 * kPi * c) - (2.0 * lgamma(ic) - lgamma(2.0 * ic));
        k.lnIe += lnrbox;
        k.lnIe2f = (float)(k.lnIe * kLog2e);
        k.c = c;
        k.ic = ic;
        k.iq = 1.0 / u[5];
        k.cf = (float)c;
        k.icf = (float)ic;
        k.dlrboxf = (float)(ic + 2.0 * (digamma(ic) - digamma(2.0 * ic)) * ic * ic);
    }
    template <bool F64>
    __device__ static void pt(const K &k, double dx, double dy, double &I64, float *d)
    {
        const Geo &g = k.g;
        float I, z, L2, Xf, Yf, lx, ly, lq, lc, gmask = 1.0f;
        if constexpr (F64) {
            const double X = g.c * dx + g.s * dy, Y = -g.s * dx + g.c * dy;
            const double ax = fabs(X), ay = fabs(Y) * k.iq;
            const double la = log(ax), lb = log(ay);
            const double A = exp(k.c * la), Bq = exp(k.c * lb), S = A + Bq;
            const double lS = log(S);
            double L = 2.0 * lS * k.ic - k.lnre2;              // ln(r^2 / r_e^2)
            const double fl = -27.631021115928547 - k.lnre2;   // r^2 >= 1e-12 px^2
            if (!(L >= fl)) {
                L = fl;
                gmask = 0.0f;
            }
            const double zd = exp(L * k.inv2n);
            I64 = exp(k.lnIe - k.b * (zd - 1.0));
            I = (float)I64;
            z = (float)zd;
            L2 = (float)(L * kLog2e);
            Xf = (float)X;
            Yf = (float)Y;
            lx = X != 0.0 ? (float)(A / (S * X)) : 0.0f;
            ly = Y != 0.0 ? (float)(Bq / (S * Y)) : 0.0f;
            lq = (float)(-Bq * k.iq / S);
            lc = (float)(-lS * k.ic * k.ic + ((ax > 0.0 ? A * la : 0.0) + (ay > 0.0 ? Bq * lb : 0.0)) * k.ic / S);
        } else {
            const float dxf = (float)dx, dyf = (float)dy;
            Xf = g.cf * dxf + g.sf * dyf;
            Yf = -g.sf * dxf + g.cf * dyf;
            const float ax = fabsf(Xf), ay = fabsf(Yf) * g.iqf;
            const float la2 = __log2f(ax), lb2 = __log2f(ay);
            const float A = exp2f(k.cf * la2), Bq = exp2f(k.cf * lb2), S = A + Bq;
            const float lS2 = __log2f(S);
            L2 = 2.0f * lS2 * k.icf - k.l2re2f;                 // log2(r^2 / r_e^2)
            const float fl = -39.863137f - k.l2re2f;
            if (!(L2 >= fl)) {
                L2 = fl;
                gmask = 0.0f;
            }
            z = exp2f(L2 * k.inv2nf);
            I = exp2f(k.lnIe2f - k.b2f * (z - 1.0f));
            I64 = I;
            lx = Xf != 0.0f ? A / (S * Xf) : 0.0f;
            ly = Yf != 0.0f ? Bq / (S * Yf) : 0.0f;
            lq = -Bq * g.iqf / S;
            lc = (float)kLn2 * (-lS2 * k.icf * k.icf + ((ax > 0.0f ? A * la2 : 0.0f) + (ay > 0.0f ? Bq * lb2 : 0.0f)) * k.icf / S);
        }
        const float gd = I * (-2.0f * k.bf * z * k.inv2nf) * gmask;     // I d ln I / d ln r
        d[0] = gd * (-g.cf * lx + g.sf * ly);
        d[1] = gd * (-g.sf * lx - g.cf * ly);
        d[2] = kDMag * I;
        d[3] = I * (-2.0f + k.bnf * z);
        d[4] = I * (k.cnf - k.nbpf * z + k.bl2nf * z * L2);
        d[5] = gd * lq - I * g.iqf;
        d[6] = gd * (Yf * lx - Xf * ly);
        d[7] = I * k.dlrboxf + gd * lc;
    }
    __device__ static void guess(double xc, double yc, double m, double r0, double q0, double pa0, double pk,
                                 int nrad, double *v)
    {
        Sersic::guess(xc, yc, m, r0, q0, pa0, pk, nrad, v);
        v[7] = 0.0;
    }
};

// Exponential disk (Sec. 4.2.1): I = I0 exp(-r / r_s), I0 = F / (2 pi q r_s^2).
// Slots x0 y0 mag ln r_s q theta.
struct ExpDisk {
    struct K {
        Geo g;
        double lnI0, irs;
        float lnI02f, irsf, irs2f;
    };
    static constexpr int NS = 6, IQ = 4, ITH = 5, IS0 = 3, IS1 = -1;
    __host__ __device__ static constexpr int kind(int s)
    {
        return s == 0 ? KX0 : s == 1 ? KY0 : s == 2 ? KMAG : s == 3 ? KSCALE : s == 4 ? KQ : KPA;
    }
    __device__ static void prep(const double *u, const double *, double m0, int H, int W, int osf, int osw, int,
                                K &k)
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
    __device__ static void pt(const K &k, double dx, double dy, double &I64, float *d)
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
    __device__ static void guess(double xc, double yc, double m, double r0, double q0, double pa0, double, int,
                                 double *v)
    {
        v[0] = xc; v[1] = yc; v[2] = m; v[3] = r0 / 1.678347; v[4] = q0; v[5] = pa0;
    }
};

// Modified Ferrer (Sec. 4.2.2): I = I0 [1 - (r/r_out)^(2-b)]^a inside r_out, 0
// beyond; I0 = F / (pi q r_out^2 a beta(a, 1 + 2/(2-b))).  Shape constants
// cst = {a, b}.  Slots x0 y0 mag ln r_out q theta.
struct Ferrer {
    struct K {
        Geo g;
        double lnI0, a, e2, lnro2;          // e2 = (2 - b) / 2
        float af, ef, iro2f;
    };
    static constexpr int NS = 6, IQ = 4, ITH = 5, IS0 = 3, IS1 = -1;
    __host__ __device__ static constexpr int kind(int s) { return ExpDisk::kind(s); }
    __device__ static void prep(const double *u, const double *cst, double m0, int H, int W, int osf, int osw, int,
                                K &k)
    {
        double x0 = u[0], y0 = u[1], m = u[2], lnro = u[3], q = u[4], th = u[5];
        double a = cst[0], bb = cst[1], c2 = 1.0 + 2.0 / (2.0 - bb);
        double lbeta = lgamma(a) + lgamma(c2) - lgamma(a + c2);
        geo_prep(x0, y0, q, th, H, W, osf, osw, k.g);
        k.lnI0 = -0.4 * kLn10 * (m - m0) - log(kPi * q * a) - 2.0 * lnro - lbeta;
        k.a = a;
        k.e2 = 0.5 * (2.0 - bb);
        k.lnro2 = 2.0 * lnro;
        k.af = (float)a;
        k.ef = (float)(2.0 - bb);
        k.iro2f = (float)exp(-2.0 * lnro);
    }
    template <bool F64>
    __device__ static void pt(const K &k, double dx, double dy, double &I64, float *d)
    {
        Pt<F64> p = frame<F64>(k.g, dx, dy);
        float I, u, omu;
        if constexpr (F64) {
            double lnu = k.e2 * (log(p.r2) - k.lnro2);     // ln (r/r_out)^(2-b)
            if (lnu >= 0.0) {
                I64 = 0.0;
                for (int s = 0; s < NS; ++s) d[s] = 0.0f;
                return;
            }
            double omud = -expm1(lnu);
            I64 = exp(k.lnI0 + k.a * log(omud));
            I = (float)I64;
            u = (float)exp(lnu);
            omu = (float)omud;
        } else {
            float lnu = 0.5f * k.ef * __logf(p.r2f * k.iro2f);
            if (lnu >= 0.0f) {
                I64 = 0.0;
                for (int s = 0; s < NS; ++s) d[s] = 0.0f;
                return;
            }
            omu = -expm1f(lnu);
            u = 1.0f - omu;
            I = __expf((float)k.lnI0 + k.af * __logf(omu));
            I64 = I;
        }
        float dl = -k.af * k.ef * u * frcp(2.0f * p.r2f * omu);   // d ln I / d r^2
        float gd[4];
        geometry_derivs<F64>(k.g, p, I, dl, -k.g.iqf, gd);
        d[0] = gd[0];
        d[1] = gd[1];
        d[2] = kDMag * I;
        d[3] = I * (-2.0f + k.af * k.ef * u * frcp(omu));
        d[4] = gd[2];
        d[5] = gd[3];
    }
    __device__ static void guess(double xc, double yc, double m, double r0, double q0, double pa0, double, int,
                                 double *v)
    {
        v[0] = xc; v[1] = yc; v[2] = m; v[3] = r0; v[4] = q0; v[5] = pa0;
    }
};

// Empirical King (Sec. 4.2.3, eq. (BE_S) with the terms of the second bracket
// in the order that gives I(0) = I0 and I(r_t) = 0):
// I = I0 [(S - A) / (1 - A)]^alpha, S = (1 + r^2/r_c^2)^(-1/alpha),
// A = (1 + r_t^2/r_c^2)^(-1/alpha); 0 beyond r_t.  cst = {alpha}.
// Slots x0 y0 I0 ln r_c ln r_t q theta.
struct King {
    struct K {
        Geo g;
        double I0, al, ial, irc2, A, rt2;
        float I0f, alf, ialf, irc2f, Af, dA_rcf, rt2f;
    };
    static constexpr int NS = 7, IQ = 5, ITH = 6, IS0 = 3, IS1 = 4;
    __host__ __device__ static constexpr int kind(int s)
    {
        return s == 0 ? KX0 : s == 1 ? KY0 : s == 2 ? KAMP : s == 3 ? KSCALE : s == 4 ? KSCALE : s == 5 ? KQ : KPA;
    }
    __device__ static void prep(const double *u, const double *cst, double, int H, int W, int osf, int osw, int,
                                K &k)
    {
        double x0 = u[0], y0 = u[1], I0 = u[2], lnrc = u[3], lnrt = u[4], q = u[5], th = u[6];
        double al = cst[0];
        double rc = exp(lnrc), rt = exp(lnrt);
        double T = 1.0 + (rt / rc) * (rt / rc);
        geo_prep(x0, y0, q, th, H, W, osf, osw, k.g);
        k.I0 = I0;
        k.al = al;
        k.ial = 1.0 / al;
        k.irc2 = 1.0 / (rc * rc);
        k.A = pow(T, -1.0 / al);
        k.rt2 = rt * rt;
        k.I0f = (float)I0;
        k.alf = (float)al;
        k.ialf = (float)(1.0 / al);
        k.irc2f = (float)k.irc2;
        k.Af = (float)k.A;
        k.dA_rcf = (float)(2.0 * k.A * (T - 1.0) / (al * T));     // dA / d ln r_c
        k.rt2f = (float)k.rt2;
    }
    template <bool F64>
    __device__ static void pt(const K &k, double dx, double dy, double &I64, float *d)
    {
        Pt<F64> p = frame<F64>(k.g, dx, dy);
        float shape, s, S, D;
        if constexpr (F64) {
            if (p.r2 >= k.rt2) {
                I64 = 0.0;
                for (int q = 0; q < NS; ++q) d[q] = 0.0f;
                return;
            }
            double sd = 1.0 + p.r2 * k.irc2;
            double Sd = exp(-k.ial * log(sd));
            double Dd = Sd - k.A;
            double shd = exp(k.al * log(Dd / (1.0 - k.A)));
            I64 = k.I0 * shd;
            shape = (float)shd;
            s = (float)sd;
            S = (float)Sd;
            D = (float)Dd;
        } else {
            if (p.r2f >= k.rt2f) {
                I64 = 0.0;
                for (int q = 0; q < NS; ++q) d[q] = 0.0f;
                return;
            }
            s = 1.0f + p.r2f * k.irc2f;
            S = __expf(-k.ialf * __logf(s));
            D = S - k.Af;
            shape = __expf(k.alf * __logf(D / (1.0f - k.Af)));
            I64 = k.I0f * shape;
        }
        float I = k.I0f * shape;
        float iD = frcp(D), iomA = frcp(1.0f - k.Af);
        float dl = -S * k.irc2f * frcp(s) * iD;              // d ln I / d r^2
        float gd[4];
        geometry_derivs<F64>(k.g, p, I, dl, 0.0f, gd);
        float dS_rc = 2.0f * S * (s - 1.0f) * k.ialf * frcp(s);
        d[0] = gd[0];
        d[1] = gd[1];
        d[2] = shape;
        d[3] = I * k.alf * (k.dA_rcf * iomA + (dS_rc - k.dA_rcf) * iD);
        d[4] = I * k.alf * (-k.dA_rcf * iomA + k.dA_rcf * iD);
        d[5] = gd[2];
        d[6] = gd[3];
    }
    __device__ static void guess(double xc, double yc, double, double r0, double q0, double pa0, double pk, int,
                                 double *v)
    {
        v[0] = xc; v[1] = yc; v[2] = pk; v[3] = 0.5 * r0; v[4] = 4.0 * r0; v[5] = q0; v[6] = pa0;
    }
};

// Ferrer with free shape exponents (Sec. 4.2.2): slots x0 y0 mag ln r_out q
// theta ln a b.  With u = (r / r_out)^(2-b) and c2 = 1 + 2 / (2 - b):
//   d ln I / d a = ln(1 - u) - 1/a - (psi(a) - psi(a + c2)),
//   d ln I / d b = a (u / (1 - u)) ln(r / r_out) - 2 (psi(c2) - psi(a + c2)) / (2 - b)^2,
// the psi terms from I0 = F / (pi q r_out^2 a beta(a, c2)).
struct FerrerFree {
    struct K : Ferrer::K {
        float dlaf, dlbf;
    };
    static constexpr int NS = 8, IQ = 4, ITH = 5, IS0 = 3, IS1 = -1;
    __host__ __device__ static constexpr int kind(int s) { return s == 6 ? KFA : s == 7 ? KFB : Ferrer::kind(s); }
    __device__ static void prep(const double *u, const double *, double m0, int H, int W, int osf, int osw, int lane,
                                K &k)
    {
        const double a = exp(u[6]), bb = u[7], c2 = 1.0 + 2.0 / (2.0 - bb);
        const double shape[2] = {a, bb};
        Ferrer::prep(u, shape, m0, H, W, osf, osw, lane, k);
        k.dlaf = (float)(-1.0 / a - (digamma(a) - digamma(a + c2)));
        k.dlbf = (float)(-2.0 * (digamma(c2) - digamma(a + c2)) / ((2.0 - bb) * (2.0 - bb)));
    }
    template <bool F64>
    __device__ static void pt(const K &k, double dx, double dy, double &I64, float *d)
    {
        Pt<F64> p = frame<F64>(k.g, dx, dy);
        float I, u, omu, lnuf, lomu;
        if constexpr (F64) {
            double lnu = k.e2 * (log(p.r2) - k.lnro2);     // ln (r/r_out)^(2-b)
            if (lnu >= 0.0) {
                I64 = 0.0;
                for (int s = 0; s < NS; ++s) d[s] = 0.0f;
                return;
            }
            double omud = -expm1(lnu), lo = log(omud);
            I64 = exp(k.lnI0 + k.a * lo);
            I = (float)I64;
            u = (float)exp(lnu);
            omu = (float)omud;
            lnuf = (float)lnu;
            lomu = (float)lo;
        } else {
            lnuf = 0.5f * k.ef * __logf(p.r2f * k.iro2f);
            if (lnuf >= 0.0f) {
                I64 = 0.0;
                for (int s = 0; s < NS; ++s) d[s] = 0.0f;
                return;
            }
            omu = -expm1f(lnuf);
            u = 1.0f - omu;
            lomu = __logf(omu);
            I = __expf((float)k.lnI0 + k.af * lomu);
            I64 = I;
        }
        const float iomu = frcp(omu);
        float dl = -k.af * k.ef * u * frcp(2.0f * p.r2f * omu);   // d ln I / d r^2
        float gd[4];
        geometry_derivs<F64>(k.g, p, I, dl, -k.g.iqf, gd);
        d[0] = gd[0];
        d[1] = gd[1];
        d[2] = kDMag * I;
        d[3] = I * (-2.0f + k.af * k.ef * u * iomu);
        d[4] = gd[2];
        d[5] = gd[3];
        d[6] = I * k.af * (lomu + k.dlaf);
        d[7] = I * (k.af * u * iomu * lnuf * frcp(k.ef) + k.dlbf);
    }
    __device__ static void guess(double xc, double yc, double m, double r0, double q0, double pa0, double pk, int nrad,
                                 double *v)
    {
        Ferrer::guess(xc, yc, m, r0, q0, pa0, pk, nrad, v);
        v[6] = 0.5;     // the values printed in Appendix C
        v[7] = 1.9;
    }
};

// King with a free alpha (Sec. 4.2.3): slots x0 y0 I0 ln r_c ln r_t q theta
// ln alpha.  With ln(I / I0) = alpha [ln(S - A) - ln(1 - A)], S = s^(-1/alpha),
// A = T^(-1/alpha), T = 1 + r_t^2 / r_c^2:
//   d I / d ln alpha = I (alpha ln((S - A)/(1 - A)) + (S ln s - A ln T)/(S - A) + A ln T/(1 - A)).
struct KingFree {
    struct K : King::K {
        float lnTf;
    };
    static constexpr int NS = 8, IQ = 5, ITH = 6, IS0 = 3, IS1 = 4;
    __host__ __device__ static constexpr int kind(int s) { return s == 7 ? KKAL : King::kind(s); }
    __device__ static void prep(const double *u, const double *, double m0, int H, int W, int osf, int osw, int lane,
                                K &k)
    {
        const double al[1] = {exp(u[7])};
        King::prep(u, al, m0, H, W, osf, osw, lane, k);
        k.lnTf = (float)log(1.0 + exp(2.0 * (u[4] - u[3])));
    }
    template <bool F64>
    __device__ static void pt(const K &k, double dx, double dy, double &I64, float *d)
    {
        Pt<F64> p = frame<F64>(k.g, dx, dy);
        float shape, s, S, D, lns, lDA;
        if constexpr (F64) {
            if (p.r2 >= k.rt2) {
                I64 = 0.0;
                for (int q = 0; q < NS; ++q) d[q] = 0.0f;
                return;
            }
            double sd = 1.0 + p.r2 * k.irc2, ls = log(sd);
            double Sd = exp(-k.ial * ls);
            double Dd = Sd - k.A;
            double lr = log(Dd / (1.0 - k.A));
            double shd = exp(k.al * lr);
            I64 = k.I0 * shd;
            shape = (float)shd;
            s = (float)sd;
            S = (float)Sd;
            D = (float)Dd;
            lns = (float)ls;
            lDA = (float)lr;
        } else {
            if (p.r2f >= k.rt2f) {
                I64 = 0.0;
                for (int q = 0; q < NS; ++q) d[q] = 0.0f;
                return;
            }
            s = 1.0f + p.r2f * k.irc2f;
            lns = __logf(s);
            S = __expf(-k.ialf * lns);
            D = S - k.Af;
            lDA = __logf(D / (1.0f - k.Af));
            shape = __expf(k.alf * lDA);
            I64 = k.I0f * shape;
        }
        float I = k.I0f * shape;
        float iD = frcp(D), iomA = frcp(1.0f - k.Af);
        float dl = -S * k.irc2f * frcp(s) * iD;              // d ln I / d r^2
        float gd[4];
        geometry_derivs<F64>(k.g, p, I, dl, 0.0f, gd);
        float dS_rc = 2.0f * S * (s - 1.0f) * k.ialf * frcp(s);
        d[0] = gd[0];
        d[1] = gd[1];
        d[2] = shape;
        d[3] = I * k.alf * (k.dA_rcf * iomA + (dS_rc - k.dA_rcf) * iD);
        d[4] = I * k.alf * (-k.dA_rcf * iomA + k.dA_rcf * iD);
        d[5] = gd[2];
        d[6] = gd[3];
        d[7] = I * (k.alf * lDA + (S * lns - k.Af * k.lnTf) * iD + k.Af * k.lnTf * iomA);
    }
    __device__ static void guess(double xc, double yc, double m, double r0, double q0, double pa0, double pk, int nrad,
                                 double *v)
    {
        King::guess(xc, yc, m, r0, q0, pa0, pk, nrad, v);
        v[7] = 2.0;
    }
};

// Gaussian (Sec. 4.2.4): I = I0 exp(-r^2 / (2 sigma^2)), FWHM = 2 sqrt(2 ln 2) sigma.
// Slots x0 y0 I0 ln fwhm q theta.
struct Gaussian {
    struct K {
        Geo g;
        double I0, i2s2;
        float I0f, i2s2f;
    };
    static constexpr int NS = 6, IQ = 4, ITH = 5, IS0 = 3, IS1 = -1;
    __host__ __device__ static constexpr int kind(int s)
    {
        return s == 0 ? KX0 : s == 1 ? KY0 : s == 2 ? KAMP : s == 3 ? KSCALE : s == 4 ? KQ : KPA;
    }
    __device__ static void prep(const double *u, const double *, double, int H, int W, int osf, int osw, int, K &k)
    {
        double sg = exp(u[3]) / (2.0 * sqrt(2.0 * kLn2));
        geo_prep(u[0], u[1], u[4], u[5], H, W, osf, osw, k.g);
        k.I0 = u[2];
        k.i2s2 = 0.5 / (sg * sg);
        k.I0f = (float)u[2];
        k.i2s2f = (float)k.i2s2;
    }
    template <bool F64>
    __device__ static void pt(const K &k, double dx, double dy, double &I64, float *d)
    {
        Pt<F64> p = frame<F64>(k.g, dx, dy);
        float shape;
        if constexpr (F64) {
            double shd = exp(-p.r2 * k.i2s2);
            I64 = k.I0 * shd;
            shape = (float)shd;
        } else {
            shape = __expf(-p.r2f * k.i2s2f);
            I64 = k.I0f * shape;
        }
        float I = k.I0f * shape;
        float gd[4];
        geometry_derivs<F64>(k.g, p, I, -k.i2s2f, 0.0f, gd);
        d[0] = gd[0];
        d[1] = gd[1];
        d[2] = shape;
        d[3] = I * 2.0f * p.r2f * k.i2s2f;
        d[4] = gd[2];
        d[5] = gd[3];
    }
    __device__ static void guess(double xc, double yc, double, double r0, double q0, double pa0, double pk, int,
                                 double *v)
    {
        v[0] = xc; v[1] = yc; v[2] = pk; v[3] = r0; v[4] = q0; v[5] = pa0;
    }
};

// Moffat (Sec. 4.2.5): I = I0 [1 + (r/r_d)^2]^(-beta),
// r_d = FWHM / (2 sqrt(2^(1/beta) - 1)), I0 = (beta - 1) F / (pi q r_d^2).
// cst = {beta}.  Slots x0 y0 mag ln fwhm q theta.
struct Moffat {
    struct K {
        Geo g;
        double lnI0, be, ird2;
        float bef, ird2f, rd2f;
    };
    static constexpr int NS = 6, IQ = 4, ITH = 5, IS0 = 3, IS1 = -1;
    __host__ __device__ static constexpr int kind(int s) { return ExpDisk::kind(s); }
    __device__ static void prep(const double *u, const double *cst, double m0, int H, int W, int osf, int osw, int,
                                K &k)
    {
        double be = cst[0];
        double rd = exp(u[3]) / (2.0 * sqrt(pow(2.0, 1.0 / be) - 1.0));
        geo_prep(u[0], u[1], u[4], u[5], H, W, osf, osw, k.g);
        k.lnI0 = -0.4 * kLn10 * (u[2] - m0) + log(be - 1.0) - log(kPi * u[4] * rd * rd);
        k.be = be;
        k.ird2 = 1.0 / (rd * rd);
        k.bef = (float)be;
        k.ird2f = (float)k.ird2;
        k.rd2f = (float)(rd * rd);
    }
    template <bool F64>
    __device__ static void pt(const K &k, double dx, double dy, double &I64, float *d)
    {
        Pt<F64> p = frame<F64>(k.g, dx, dy);
        float I;
        if constexpr (F64) {
            I64 = exp(k.lnI0 - k.be * log1p(p.r2 * k.ird2));
            I = (float)I64;
        } else {
            I = __expf((float)k.lnI0 - k.bef * __logf(1.0f + p.r2f * k.ird2f));
            I64 = I;
        }
        float idn = frcp(k.rd2f + p.r2f);
        float gd[4];
        geometry_derivs<F64>(k.g, p, I, -k.bef * idn, -k.g.iqf, gd);
        d[0] = gd[0];
        d[1] = gd[1];
        d[2] = kDMag * I;
        d[3] = I * (-2.0f + 2.0f * k.bef * p.r2f * idn);
        d[4] = gd[2];
        d[5] = gd[3];
    }
    __device__ static void guess(double xc, double yc, double m, double r0, double q0, double pa0, double, int,
                                 double *v)
    {
        v[0] = xc; v[1] = yc; v[2] = m; v[3] = r0; v[4] = q0; v[5] = pa0;
    }
};

// ---------------------------------------------------------------- families
// A family fixes, at compile time, the components of a model, the layout of
// the internal LM vector u and the image planes: plane 0 is the summed light
// of the components (FP64), plane plane(k) the derivative with respect to u_k
// (FP32).  Two variables have no plane: sky (derivative 1) and DER, the
// magnitude whose derivative follows from the light by linearity -- the light
// of a component is proportional to 10^(-0.4 m), so d M / d m = -0.4 ln 10
// times the component's convolved light.  Only one-component families use it:
// for a pair the second magnitude's derivative would be the total light minus
// the first component's FP32 plane, which amplifies that plane's rounding by
// the flux ratio of the components.  DER = -1 also when the flux parameter is
// an amplitude (dividing by it would fail at zero).

// One component + sky: u = the component's slots, then sky.
// One radial component and a flat sky, or (TILT) the tilted-plane sky of
// Appendix D, eq. (new_sky_I): sky + kx (x - W/2) + ky (y - H/2), whose two
// gradient variables follow the sky in the LM vector.
template <class C, bool TILT = false>
struct FamSingle {
    static constexpr int P = C::NS + (TILT ? 3 : 1), NCOMP = 1, NRAD = 1, SKY = C::NS, ND = C::NS;
    static constexpr int DER = C::kind(2) == KMAG ? 2 : -1;
    static constexpr int NPL = 1 + C::NS - (DER >= 0 ? 1 : 0);
    __host__ __device__ static constexpr int kind(int k)
    {
        return k < C::NS ? C::kind(k) : k == SKY ? KSKY : KSKYG;
    }
    __host__ __device__ static constexpr int plane(int k)
    {
        return (k >= SKY || k == DER) ? -1 : (DER >= 0 && k > DER) ? k : k + 1;
    }
    // the sky's columns of the Jacobian are analytic: 1, x - W/2, y - H/2
    __host__ __device__ static constexpr bool analytic(int k) { return k >= SKY; }
    __device__ static float analytic_value(int k, float dx, float dy)
    {
        return k == SKY ? 1.0f : k == SKY + 1 ? dx : dy;
    }
    // d M / d u_DER at a pixel from the convolved light acc0 and planes acc
    __device__ static float derived(double acc0, const float *) { return kDMag * (float)acc0; }
    struct Prep {
        typename C::K k0;
        double sky, gx, gy;
    };
    __device__ static void prep(const double *u, const double *cst, double m0, int H, int W, int osf, int osw,
                                int lane, Prep &p)
    {
        C::prep(u, cst, m0, H, W, osf, osw, lane, p.k0);
        p.sky = u[SKY];
        p.gx = TILT ? u[SKY + 1] : 0.0;
        p.gy = TILT ? u[SKY + 2] : 0.0;
    }
    // the unconvolved sky at a pixel at (dx, dy) from the cutout's centre
    __device__ static double sky_at(const Prep &p, double dx, double dy)
    {
        if constexpr (TILT) return p.sky + p.gx * dx + p.gy * dy;
        else return p.sky;
    }
    __device__ static const Geo &geo(const Prep &p, int) { return p.k0.g; }
    template <bool F64>
    __device__ static void comp_pt(const Prep &p, int, double dx, double dy, double &I, float *d)
    {
        C::template pt<F64>(p.k0, dx, dy, I, d);
    }
    // component derivatives into the derivative planes (index = plane - 1)
    __device__ static void scatter(int, const float *d, float *dp)
    {
#pragma unroll
        for (int i = 0; i < C::NS; ++i)
            if (plane(i) > 0) dp[plane(i) - 1] += d[i];
    }
    __device__ static void default_guess(double xc, double yc, double m, double r0, double q0, double pa0,
                                         double sky0, double pk, double *nat)
    {
        C::guess(xc, yc, m, r0, q0, pa0, pk, NRAD, nat);
        nat[SKY] = sky0;
        if (TILT) nat[SKY + 1] = nat[SKY + 2] = 0.0;
    }
    static constexpr int NCAN = 1;
    __host__ __device__ static void canon(int, int &iq, int &ith, int &is0, int &is1)
    {
        iq = C::IQ; ith = C::ITH; is0 = C::IS0; is1 = C::IS1;
    }
};

// Two components with a shared centre + sky:
// u = x0 y0 | C1 slots 2.. | C2 slots 2.. | sky.  cst: C1's constants at
// cst[0..1], C2's at cst[2..3].
template <class C1, class C2>
struct FamPair {
    static constexpr int O2 = C1::NS - 2;                  // C2 slot s >= 2 sits at u[O2 + s]
    static constexpr int P = C1::NS + C2::NS - 2 + 1, NCOMP = 2, NRAD = 2, SKY = P - 1;
    static constexpr int ND = C1::NS > C2::NS ? C1::NS : C2::NS;
    static constexpr int DER = -1, NPL = P;
    __host__ __device__ static constexpr int plane(int k) { return k == SKY ? -1 : k + 1; }
    __host__ __device__ static constexpr bool analytic(int k) { return k == SKY; }
    __device__ static float analytic_value(int, float, float) { return 1.0f; }
    __device__ static float derived(double, const float *) { return 0.0f; }
    __host__ __device__ static constexpr int kind(int k)
    {
        return k < C1::NS ? C1::kind(k) : k < SKY ? C2::kind(k - O2) : KSKY;
    }
    struct Prep {
        typename C1::K k0;
        typename C2::K k1;
        double sky;
    };
    __device__ static void prep(const double *u, const double *cst, double m0, int H, int W, int osf, int osw,
                                int lane, Prep &p)
    {
        C1::prep(u, cst, m0, H, W, osf, osw, lane, p.k0);
        double u2[C2::NS];
        u2[0] = u[0];
        u2[1] = u[1];
        for (int s = 2; s < C2::NS; ++s) u2[s] = u[O2 + s];
        C2::prep(u2, cst + 2, m0, H, W, osf, osw, lane, p.k1);
        p.sky = u[SKY];
    }
    __device__ static double sky_at(const Prep &p, double, double) { return p.sky; }
    __device__ static const Geo &geo(const Prep &p, int c) { return c == 0 ? p.k0.g : p.k1.g; }
    template <bool F64>
    __device__ static void comp_pt(const Prep &p, int c, double dx, double dy, double &I, float *d)
    {
        if (c == 0) C1::template pt<F64>(p.k0, dx, dy, I, d);
        else C2::template pt<F64>(p.k1, dx, dy, I, d);
    }
    __device__ static void scatter(int c, const float *d, float *dp)
    {
        if (c == 0) {
#pragma unroll
            for (int i = 0; i < C1::NS; ++i) dp[plane(i) - 1] += d[i];
        } else {
            dp[plane(0) - 1] += d[0];
            dp[plane(1) - 1] += d[1];
#pragma unroll
            for (int i = 2; i < C2::NS; ++i)
                if (plane(O2 + i) > 0) dp[plane(O2 + i) - 1] += d[i];
        }
    }
    __device__ static void default_guess(double xc, double yc, double m, double r0, double q0, double pa0,
                                         double sky0, double pk, double *nat)
    {
        double v2[C2::NS];
        C1::guess(xc, yc, m, r0, q0, pa0, pk, NRAD, nat);
        C2::guess(xc, yc, m, r0, q0, pa0, pk, NRAD, v2);
        for (int s = 2; s < C2::NS; ++s) nat[O2 + s] = v2[s];
        nat[SKY] = sky0;
    }
    static constexpr int NCAN = 2;
    __host__ __device__ static void canon(int c, int &iq, int &ith, int &is0, int &is1)
    {
        if (c == 0) {
            iq = C1::IQ; ith = C1::ITH; is0 = C1::IS0; is1 = C1::IS1;
        } else {
            iq = O2 + C2::IQ; ith = O2 + C2::ITH;
            is0 = C2::IS0 >= 2 ? O2 + C2::IS0 : -1;
            is1 = C2::IS1 >= 2 ? O2 + C2::IS1 : -1;
        }
    }
};

using FamSersic = FamSingle<Sersic>;
using FamSersicTilt = FamSingle<Sersic, true>;
using FamSersicBox = FamSingle<SersicBox>;
using FamFerrerFree = FamSingle<FerrerFree>;
using FamKingFree = FamSingle<KingFree>;
using FamBulgeDisk = FamPair<Sersic, ExpDisk>;
using FamSersicBar = FamPair<Sersic, Ferrer>;

}  // namespace gm
