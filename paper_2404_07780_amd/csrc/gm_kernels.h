// gm_kernels.h -- gfx950 kernels of libgmfit.
//
// Work decomposition.  A galaxy's cutout is processed in 32 x 32 output tiles
// by one 256-thread workgroup.  For a tile, the light (FP64) and its FP32
// derivatives with respect to every LM variable are evaluated on the tile's
// (32 + K - 1)^2 input region straight into LDS, one plane per quantity; the
// oversampled central window is evaluated once per model evaluation into a
// small LDS table.  Each thread then convolves a 1 x 4 strip of outputs of
// every plane with the PSF (true convolution, zero padding), streaming one
// row segment from LDS per PSF row and reading the PSF through the scalar
// cache; the results stay in registers.  When the planes of a model do not fit
// LDS together (or fit only one workgroup per CU) they are processed in NG
// groups, re-evaluating the profile per group (only the first group needs the
// FP64 light).  The fitting kernel turns the convolved planes into residuals
// and FP64 normal-equation sums without writing any image to memory.
//
// gm_fit_batch runs one persistent kernel: each workgroup pulls galaxies, in
// descending-cost order, from an atomic queue and runs the whole
// Levenberg-Marquardt iteration for a galaxy; thread 0 does the FP64 damped
// Cholesky solve and accept/reject between evaluations.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "gmfit.h"
#include "gm_device.h"

namespace gm {

constexpr int TILE = 32;
constexpr int NT = 256;
constexpr int NWAVE = NT / 64;
constexpr int MAXP = 16;
constexpr int MAXWIN = 25;      // oversampled window of at most 5 x 5 pixels
constexpr int MAXOSF = 16;      // sub-samples per pixel side

struct Meta {
    int32_t h, w, k, pad;
    int64_t img_off, psf_off;
};

// Model description passed by value: internal LM index -> column of the
// caller's parameter vector (-1: fixed at fixedv, natural units).
struct ModelArgs {
    int p;
    int col[MAXP];
    double fixedv[MAXP];
    double cst[4];          // shape constants: component 0 at [0..1], component 1 at [2..3]
    double m0;
    int osf, osw;
    int nflux;              // components whose magnitude/amplitude is fitted (start-vector flux split)
};

struct BatchArgs {
    const Meta *meta;
    const float *data, *sigma, *psf;
    const uint8_t *omega;
};

__device__ inline int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Input-region geometry of a tile for PSF side K (row pitch IWP in elements).
__host__ __device__ constexpr int region_h(int K) { return TILE + K - 1; }
// Row pitch: the 32 outputs' 16-byte-aligned input segments need
// 28 + 4 ceil((K + 3) / 4) floats.
__host__ __device__ constexpr int region_wp(int K) { return 28 + 4 * ((K + 3 + 3) / 4); }

// FP64 light plane rows: with a pitch of 48 doubles (PSF side 15) the 16-byte
// reads of two adjacent rows (one 16-lane group) fall on the same LDS banks;
// odd rows stored 2 doubles (16 bytes) further on read conflict-free
// (measured with the bank-conflict counter).  The pitch has the 2 spare
// doubles this needs.
template <int KT>
__host__ __device__ constexpr bool shift64()
{
    return KT > 0 && region_wp(KT) == 48 && region_h(KT) + 2 <= 48;
}

// Output strip of thread tid in a tile: row r, columns 4 cg .. 4 cg + 3.  Wave
// w covers rows 8w .. 8w + 7, 8 lanes per row.  When the row pitch is 8
// (mod 16) floats (PSF sides 7, 9, 23, 25, ...), adjacent rows' 16-byte
// segment reads overlap on three quarters of the LDS banks; the two 8-lane
// halves of each 16-lane group then take rows 4 apart (4 x pitch = 32 mod 64),
// which measured 6% faster fits at K = 25.  Other pitches keep rows in order
// (the paired mapping measured 1% slower at K = 15).
__host__ __device__ inline int strip_gap(int IWP) { return (IWP % 16 == 8) ? 4 : 0; }
__device__ inline void strip_of(int tid, int K, int &r, int &cg)
{
    const int lane = tid & 63, w = tid >> 6, gi = lane >> 4, h = (lane >> 3) & 1;
    cg = lane & 7;
    int rb;
    if (strip_gap(region_wp(K)) == 4) rb = gi + 4 * h;
    else rb = lane >> 3;
    r = 8 * w + rb;
}

// Plane groups: plane 0 (FP64) counts two units, the others one; groups are
// contiguous and balanced in units.
__host__ __device__ constexpr int group_bound(int npl, int ng, int g)
{
    if (g <= 0) return 0;
    if (g >= ng) return npl;
    int target = ((npl + 1) * g + ng - 1) / ng, acc = 0;
    for (int q = 0; q < npl; ++q) {
        acc += (q == 0 ? 2 : 1);
        if (acc >= target) return q + 1;
    }
    return npl;
}
__host__ __device__ constexpr int group_units(int npl, int ng, int g)
{
    int lo = group_bound(npl, ng, g), hi = group_bound(npl, ng, g + 1);
    return hi - lo + (lo == 0 ? 1 : 0);
}
__host__ __device__ constexpr int max_group_units(int npl, int ng)
{
    int m = 0;
    for (int g = 0; g < ng; ++g) m = group_units(npl, ng, g) > m ? group_units(npl, ng, g) : m;
    return m;
}

template <class F, int NG>
__host__ __device__ inline size_t planes_bytes(int K)
{
    return (size_t)max_group_units(F::NPL, NG) * region_h(K) * region_wp(K) * sizeof(float);
}

// ---------------------------------------------------------------- per-evaluation state in LDS
// Tiles a thread sums its FP32 partial products of g and J^T W J over before
// they are added, per wave, to FP64 running sums (EvalShared::nacc): a thread
// then never sums more than 4 x 16 = 64 pixels in FP32, whatever the cutout's
// size.  Cutouts of up to 16 tiles (128 x 128) never flush.
constexpr int FLUSH_TILES = 16;

template <class F>
struct EvalShared {
    typename F::Prep prep;
    double win0[F::NCOMP][MAXWIN];
    float win[F::NCOMP][MAXWIN][F::ND];
    double nacc[NWAVE][F::P + F::P * (F::P + 1) / 2];     // per-wave FP64 sums of the flushed partials
};

// scratch needed by the window tables (in the plane buffer)
template <class F>
__host__ __device__ constexpr size_t window_scratch_bytes()
{
    return (size_t)MAXWIN * MAXOSF * (sizeof(double) + F::ND * sizeof(float));
}

// Dynamic LDS of the evaluating kernels: the plane buffer (which also hosts
// the window partial sums, the wave partial sums of the normal equations and
// the thread-0 solver temporaries), then a copy of the galaxy's PSF with rows
// padded to psf_pitch floats (16-byte aligned rows).
__host__ __device__ inline int psf_pitch(int K) { return (K + 3) & ~3; }
template <class F, int NG>
__host__ __device__ inline size_t lds_main_bytes(int K)
{
    size_t m = planes_bytes<F, NG>(K);
    const size_t sums = (size_t)NWAVE * (1 + F::P + F::P * (F::P + 1) / 2) * 8, solve = (size_t)3 * F::P * F::P * 8;
    m = m > sums ? m : sums;
    m = m > solve ? m : solve;
    m = m > window_scratch_bytes<F>() ? m : window_scratch_bytes<F>();
    return (m + 15) & ~(size_t)15;
}
template <class F, int NG>
__host__ __device__ inline size_t lds_total_bytes(int K)
{
    return lds_main_bytes<F, NG>(K) + (size_t)K * psf_pitch(K) * sizeof(float);
}

// Copy the PSF (K x K, global) into its LDS rows; the caller's next barrier
// publishes it.
template <class F, int NG>
__device__ inline const float *stage_psf(float *planes, const float *psf, int K)
{
    float *d = planes + lds_main_bytes<F, NG>(K) / sizeof(float);
    const int kp = psf_pitch(K);
    for (int i = threadIdx.x; i < K * K; i += NT) {
        const int u = i / K;
        d[u * kp + (i - u * K)] = psf[i];
    }
    return d;
}

// Scalar prologue (wave 0) + oversampled window tables (all threads).
// u: LDS (FP64, internal).  scratch: the idle plane buffer.
template <class F>
__device__ void eval_prologue(const double *u, const ModelArgs &ma, int H, int W, EvalShared<F> &sh, float *scratch)
{
    const int tid = threadIdx.x;
    if (tid < 64) {
        typename F::Prep lp;
        F::prep(u, ma.cst, ma.m0, H, W, ma.osf, ma.osw, tid, lp);
        if (tid == 0) sh.prep = lp;
    }
    __syncthreads();
    const int f = ma.osf;
    const double invf = 1.0 / (double)f;
    double *sd = reinterpret_cast<double *>(scratch);
    float *sf = scratch + 2 * MAXWIN * MAXOSF;
#pragma unroll 1
    for (int c = 0; c < F::NCOMP; ++c) {
        const Geo &g = F::geo(sh.prep, c);
        const int ww = g.wj1 - g.wj0 + 1, wh = g.wi1 - g.wi0 + 1;
        if (ww <= 0 || wh <= 0) continue;
        const int nwin = ww * wh, items = nwin * f;
        // each item: one sub-row (t) of one window pixel, summed over s
        for (int it = tid; it < items; it += NT) {
            int pix = it / f, t = it - pix * f;
            int i = g.wi0 + pix / ww, j = g.wj0 + pix % ww;
            double aI = 0.0;
            float ad[F::ND];
#pragma unroll
            for (int q = 0; q < F::ND; ++q) ad[q] = 0.0f;
            const double dy = ((double)(H - i) - ((double)t + 0.5) * invf) - g.y0;
            for (int s = 0; s < f; ++s) {
                const double dx = ((double)j + ((double)s + 0.5) * invf) - g.x0;
                double I;
                float d[F::ND] = {};
                F::template comp_pt<true>(sh.prep, c, dx, dy, I, d);
                aI += I;
#pragma unroll
                for (int q = 0; q < F::ND; ++q) ad[q] += d[q];
            }
            sd[it] = aI;
#pragma unroll
            for (int q = 0; q < F::ND; ++q) sf[it * F::ND + q] = ad[q];
        }
        __syncthreads();
        const double norm = 1.0 / (double)(f * f);
        for (int pix = tid; pix < nwin; pix += NT) {
            double s0 = 0.0;
            for (int t = 0; t < f; ++t) s0 += sd[pix * f + t];
            sh.win0[c][pix] = s0 * norm;
#pragma unroll
            for (int q = 0; q < F::ND; ++q) {
                float s = 0.0f;
                for (int t = 0; t < f; ++t) s += sf[(pix * f + t) * F::ND + q];
                sh.win[c][pix][q] = s * (float)norm;
            }
        }
        __syncthreads();
    }
}

// Light (FP64 if F64) and derivative planes (dp[q - 1] for plane q) of the
// convolved components at pixel (i, j).
template <class F, bool F64>
__device__ inline void planes_at(const EvalShared<F> &sh, int i, int j, int H, double &v0, float *dp)
{
    v0 = 0.0;
#pragma unroll
    for (int q = 0; q < F::NPL - 1; ++q) dp[q] = 0.0f;
#pragma unroll
    for (int c = 0; c < F::NCOMP; ++c) {
        const Geo &g = F::geo(sh.prep, c);
        double I;
        float d[F::ND] = {};
        if (i >= g.wi0 && i <= g.wi1 && j >= g.wj0 && j <= g.wj1) {
            const int pix = (i - g.wi0) * (g.wj1 - g.wj0 + 1) + (j - g.wj0);
            I = sh.win0[c][pix];
#pragma unroll
            for (int q = 0; q < F::ND; ++q) d[q] = sh.win[c][pix][q];
        } else {
            const double dx = ((double)j + 0.5) - g.x0;
            const double dy = ((double)(H - i) - 0.5) - g.y0;
            F::template comp_pt<F64>(sh.prep, c, dx, dy, I, d);
        }
        v0 += I;
        F::scatter(c, d, dp);
    }
}

// Fill the LDS planes LO..HI-1 of the input region of the tile at (ti0, tj0).
// Layout: if LO == 0 the FP64 light plane comes first (two float units),
// then the FP32 planes in order.  Region points outside the image are the
// convolution's zero padding; the points inside form a rectangle whose
// profile values are spread linearly over all threads of the workgroup.
template <class F, int LO, int HI, bool SH = false>
__device__ void fill_region(const EvalShared<F> &sh, float *buf, int H, int W, int K, int ti0, int tj0)
{
    const int IH = region_h(K), IWP = region_wp(K), IW = TILE + K - 1, c = (K - 1) / 2;
    const int plane_sz = IH * IWP;
    double *b0 = reinterpret_cast<double *>(buf);
    float *bf = (LO == 0) ? buf + 2 * plane_sz : buf;
    constexpr int QLO = LO == 0 ? 1 : LO;
    // region rows r0..r1-1 and columns c0..c1-1 lie inside the image
    const int r0 = max(0, c - ti0), r1 = min(IH, H + c - ti0);
    const int c0 = max(0, c - tj0), c1 = min(IW, W + c - tj0);
    // region point (ri, ci); SH: odd rows of the FP64 plane 2 further on
    auto store = [&](int ri, int ci, double v0, const float *dp) {
        const int idx = ri * IWP + ci;
        if constexpr (LO == 0) b0[SH ? idx + 2 * (ri & 1) : idx] = v0;
#pragma unroll
        for (int q = QLO; q < HI; ++q) bf[(q - QLO) * plane_sz + idx] = dp[q - 1];
    };
    const bool edge = r0 > 0 || r1 < IH || c0 > 0 || c1 < IW;
    if (edge) {
        float z[F::NPL - 1];
#pragma unroll
        for (int q = 0; q < F::NPL - 1; ++q) z[q] = 0.0f;
        for (int t = threadIdx.x; t < IH * IW; t += NT) {
            const int ri = t / IW, ci = t - ri * IW;
            if (ri < r0 || ri >= r1 || ci < c0 || ci >= c1) store(ri, ci, 0.0, z);
        }
    }
    const int nc = c1 - c0, npts = (r1 - r0) * nc;
    // row of a linear index by a float product: (t + 0.5) / nc is below the
    // row count (< 2^8) and at least 1/(2 nc) > 2^-9 away from an integer,
    // while the float rounding moves it by less than 2^-14
    const float rnc = 1.0f / (float)nc;
    for (int t = threadIdx.x; t < npts; t += NT) {
        const int rr = (int)(((float)t + 0.5f) * rnc), ri = r0 + rr, ci = c0 + (t - rr * nc);
        double v0;
        float dp[F::NPL - 1];
        planes_at<F, LO == 0>(sh, ti0 - c + ri, tj0 - c + ci, H, v0, dp);
        store(ri, ci, v0, dp);
    }
}

// The PSF is read through the constant address space with a wave-uniform
// offset: such loads are scalar (s_load through the scalar cache) and the taps
// reach the FMAs as SGPR operands.
typedef __attribute__((address_space(4))) const float cfloat;

__device__ inline int64_t uniform64(int64_t x)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One PSF row (KT taps) against a row segment: acc[t] += sum_v p[v] seg[t + KT-1-v].
template <int KT, typename T, typename PR>
__device__ inline void row_fma(const T *seg, PR pr, T &a0, T &a1, T &a2, T &a3)
{
#pragma unroll
    for (int v = 0; v < KT; ++v) {
        const T pv = (T)pr[v];
        a0 = fma(pv, seg[KT - 1 - v], a0);
        a1 = fma(pv, seg[KT - v], a1);
        a2 = fma(pv, seg[KT + 1 - v], a2);
        a3 = fma(pv, seg[KT + 2 - v], a3);
    }
}

// Load the (KT + 3)-element row segment at p (16-byte aligned) into seg.
template <int KT, typename T>
__device__ inline void load_seg(const T *p, T *seg)
{
    constexpr int PER = 16 / sizeof(T);
    constexpr int NV = (KT + 3 + PER - 1) / PER;
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    const V *rp = reinterpret_cast<const V *>(p);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        V t = rp[q];
        if constexpr (sizeof(T) == 4) {
            seg[4 * q] = t.x; seg[4 * q + 1] = t.y; seg[4 * q + 2] = t.z; seg[4 * q + 3] = t.w;
        } else {
            seg[2 * q] = t.x; seg[2 * q + 1] = t.y;
        }
    }
}

// Taps v0 .. v1-1 of one PSF row against the segment elements e0 .. (e0 a
// multiple of the 16-byte vector width): acc[t] += sum_v p[v] seg[KT-1-v+t].
template <int KT, int V0, int V1, int E0, typename T, typename PR>
__device__ inline void row_part(const T *rp, PR pr, T &a0, T &a1, T &a2, T &a3)
{
    constexpr int PER = 16 / sizeof(T);
    constexpr int N = ((KT + 2 - V0) - E0 + 1 + PER - 1) / PER * PER;
    T seg[N];
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    const V *vp = reinterpret_cast<const V *>(rp + E0);
#pragma unroll
    for (int q = 0; q < N / PER; ++q) {
        V t = vp[q];
        if constexpr (sizeof(T) == 4) {
            seg[4 * q] = t.x; seg[4 * q + 1] = t.y; seg[4 * q + 2] = t.z; seg[4 * q + 3] = t.w;
        } else {
            seg[2 * q] = t.x; seg[2 * q + 1] = t.y;
        }
    }
#pragma unroll
    for (int v = V0; v < V1; ++v) {
        const T pv = (T)pr[v];
        a0 = fma(pv, seg[KT - 1 - v - E0], a0);
        a1 = fma(pv, seg[KT - v - E0], a1);
        a2 = fma(pv, seg[KT + 1 - v - E0], a2);
        a3 = fma(pv, seg[KT + 2 - v - E0], a3);
    }
}

// Convolve one plane (elements of type T, row pitch IWP) for a 1 x 4 output
// strip with a compile-time PSF side (the Adam fit's planes).  Up to side 15,
// FP32 planes load the segment of the next PSF row while the current one is
// used and the FP64 plane, whose segment is twice as large, loads one row at
// a time.  Wider
// PSFs take each row in two halves of taps, each with only the part of the
// segment it reads, so that the kernel fits two workgroups' registers.
template <int KT, typename T>
__device__ inline void conv_plane(const T *base, int r, int IWP, const cfloat *psf, T (&out)[4])
{
    constexpr int PER = 16 / sizeof(T);
    constexpr int SEG = ((KT + 3 + PER - 1) / PER) * PER;
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    if constexpr (KT > 15) {
        // taps v < VS read elements from ES on, taps v >= VS elements from 0
        constexpr int ES = 4 * ((KT - 1) / 8), VS = KT - ES;
#pragma unroll 1
        for (int u = 0; u < KT; ++u) {
            const T *rp = base + (r + KT - 1 - u) * IWP;
            row_part<KT, 0, VS, ES>(rp, psf + u * KT, a0, a1, a2, a3);
            row_part<KT, VS, KT, 0>(rp, psf + u * KT, a0, a1, a2, a3);
        }
    } else if constexpr (sizeof(T) == 4) {
        T sa[SEG], sb[SEG];
        load_seg<KT>(base + (r + KT - 1) * IWP, sa);
#pragma unroll 1
        for (int u = 0; u + 1 < KT; u += 2) {
            load_seg<KT>(base + (r + KT - 2 - u) * IWP, sb);
            row_fma<KT>(sa, psf + u * KT, a0, a1, a2, a3);
            if (u + 2 < KT) load_seg<KT>(base + (r + KT - 3 - u) * IWP, sa);
            row_fma<KT>(sb, psf + (u + 1) * KT, a0, a1, a2, a3);
        }
        if (KT & 1) row_fma<KT>(sa, psf + (KT - 1) * KT, a0, a1, a2, a3);
    } else {
        T sa[SEG];
#pragma unroll 1
        for (int u = 0; u < KT; ++u) {
            load_seg<KT>(base + (r + KT - 1 - u) * IWP, sa);
            row_fma<KT>(sa, psf + u * KT, a0, a1, a2, a3);
        }
    }
    out[0] = a0; out[1] = a1; out[2] = a2; out[3] = a3;
}

// Any PSF side (slow path): taps read one by one from LDS.
template <typename T>
__device__ inline void conv_plane_any(const T *base, int r, int K, int IWP, const cfloat *psf, T (&out)[4])
{
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int u = 0; u < K; ++u) {
        const T *rp = base + (r + K - 1 - u) * IWP;
        const cfloat *pr = psf + u * K;
        for (int v = 0; v < K; ++v) {
            const T pv = (T)pr[v];
            const T *sp = rp + K - 1 - v;
            a0 = fma(pv, sp[0], a0);
            a1 = fma(pv, sp[1], a1);
            a2 = fma(pv, sp[2], a2);
            a3 = fma(pv, sp[3], a3);
        }
    }
    out[0] = a0; out[1] = a1; out[2] = a2; out[3] = a3;
}

// The taps of PSF row u from its LDS copy (rows of KP = psf_pitch floats).
template <int KP>
__device__ inline void load_taps(const float *psl, int u, float (&tp)[KP])
{
    const float4 *tv = reinterpret_cast<const float4 *>(psl + u * KP);
#pragma unroll
    for (int q = 0; q < KP / 4; ++q) {
        const float4 t = tv[q];
        tp[4 * q] = t.x; tp[4 * q + 1] = t.y; tp[4 * q + 2] = t.z; tp[4 * q + 3] = t.w;
    }
}

// PSF sides above 15: the planes of a group row by row of the PSF, every
// plane of the group under one row's taps.  A row's taps are scalar loads,
// which complete out of order with the LDS reads of the segments: with them
// loaded once per PSF row, no scalar load is outstanding while the planes of
// the row run, so the segment reads of the next plane overlap the products of
// the current one.  Each accumulator sees the products in the order of the
// plane-by-plane loop (rows, then taps).
template <class F, int KT, int LO, int HI>
__device__ inline void conv_group_wide(const float *__restrict__ buf, const cfloat *psf, int r, int cg,
                                       double (&acc0)[4], float (&acc)[F::NPL][4])
{
    constexpr int IH = TILE + KT - 1, IWP = (28 + 4 * ((KT + 3 + 3) / 4));
    constexpr int plane_sz = IH * IWP;
    constexpr int QLO = LO == 0 ? 1 : LO;
    const float *bf = ((LO == 0) ? buf + 2 * plane_sz : buf) + 4 * cg;
    const double *b64 = reinterpret_cast<const double *>(buf) + 4 * cg;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
    float a[HI - QLO][4];
#pragma unroll
    for (int pl = 0; pl < HI - QLO; ++pl) a[pl][0] = a[pl][1] = a[pl][2] = a[pl][3] = 0.0f;
#pragma unroll 1
    for (int u = 0; u < KT; ++u) {
        const int ro = (r + KT - 1 - u) * IWP;
        const cfloat *pr = psf + u * KT;
        // wide PSFs: each row in two halves of taps, each with only the part
        // of the segment it reads (taps v < VS read elements from ES on)
        constexpr int ES = 4 * ((KT - 1) / 8), VS = KT - ES;
        if constexpr (LO == 0) {
            row_part<KT, 0, VS, ES>(b64 + ro, pr, d0, d1, d2, d3);
            row_part<KT, VS, KT, 0>(b64 + ro, pr, d0, d1, d2, d3);
        }
#pragma unroll
        for (int pl = 0; pl < HI - QLO; ++pl) {
            row_part<KT, 0, VS, ES>(bf + pl * plane_sz + ro, pr, a[pl][0], a[pl][1], a[pl][2], a[pl][3]);
            row_part<KT, VS, KT, 0>(bf + pl * plane_sz + ro, pr, a[pl][0], a[pl][1], a[pl][2], a[pl][3]);
        }
    }
    if constexpr (LO == 0) {
        acc0[0] = d0; acc0[1] = d1; acc0[2] = d2; acc0[3] = d3;
    }
#pragma unroll
    for (int pl = QLO; pl < HI; ++pl)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[pl][t] = a[pl - QLO][t];
}

// PSF sides up to 15.  Every load of the loops is an LDS read (the taps
// from the PSF's LDS copy, the segments from the planes), and LDS reads
// complete in order, so a wait covers exactly the reads a product needs and
// the reads issued after them stay in flight.  The FP64 plane runs first, on
// its own, with the segment and taps of the next PSF row loaded while the
// current row is used; then the FP32 planes, row by row of the PSF with every
// plane under the row's taps, each plane's segment loaded while the previous
// plane's products run.  Each accumulator sees the products in the same order
// (rows, then taps).
template <class F, int KT, int LO, int HI>
__device__ inline void conv_group_rows(const float *__restrict__ buf, const float *__restrict__ psl, int r, int cg,
                                       double (&acc0)[4], float (&acc)[F::NPL][4])
{
    constexpr int KP = (KT + 3) & ~3;
    constexpr int IH = TILE + KT - 1, IWP = (28 + 4 * ((KT + 3 + 3) / 4));
    constexpr int plane_sz = IH * IWP;
    constexpr int QLO = LO == 0 ? 1 : LO, NP = HI - QLO;
    constexpr int SEG32 = ((KT + 3 + 3) / 4) * 4, SEG64 = ((KT + 3 + 1) / 2) * 2;
    const float *bf = ((LO == 0) ? buf + 2 * plane_sz : buf) + 4 * cg;
    const float *rowp = bf + (r + KT - 1) * IWP;          // row of PSF row 0; PSF row u is -u * IWP
    if constexpr (LO == 0) {
        // rows of even u start at pe - u IWP, of odd u at po - (u - 1) IWP (the
        // row parity, and so the shift64 offset, alternates with u)
        const int rr0 = r + KT - 1;
        const double *b64 = reinterpret_cast<const double *>(buf) + 4 * cg;
        const double *pe = b64 + rr0 * IWP + (shift64<KT>() ? 2 * (rr0 & 1) : 0);
        const double *po = b64 + (rr0 - 1) * IWP + (shift64<KT>() ? 2 * ((rr0 - 1) & 1) : 0);
        double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
        double sa[SEG64], sb[SEG64];
        float ta[KP], tb[KP];
        load_taps<KP>(psl, 0, ta);
        load_seg<KT>(pe, sa);
#pragma unroll 1
        for (int u = 0; u + 1 < KT; u += 2) {
            load_taps<KP>(psl, u + 1, tb);
            load_seg<KT>(po - u * IWP, sb);
            row_fma<KT>(sa, ta, d0, d1, d2, d3);
            if (u + 2 < KT) {
                load_taps<KP>(psl, u + 2, ta);
                load_seg<KT>(pe - (u + 2) * IWP, sa);
            }
            row_fma<KT>(sb, tb, d0, d1, d2, d3);
        }
        if (KT & 1) row_fma<KT>(sa, ta, d0, d1, d2, d3);
        acc0[0] = d0; acc0[1] = d1; acc0[2] = d2; acc0[3] = d3;
    }
    float a[NP > 0 ? NP : 1][4];
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) a[pl][0] = a[pl][1] = a[pl][2] = a[pl][3] = 0.0f;
    if constexpr (NP > 0) {
#pragma unroll 1
        for (int u = 0; u < KT; ++u) {
            float tp[KP];
            load_taps<KP>(psl, u, tp);
            const float *ro = rowp - u * IWP;
            float sg[2][SEG32];
            load_seg<KT>(ro, sg[0]);
            constexpr int NRD = (KT + 3 + 3) / 4;      // 16-byte reads per segment
            __builtin_amdgcn_sched_group_barrier(0x100, KP / 4 + NRD, 0);
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) {
                if (pl + 1 < NP) {
                    load_seg<KT>(ro + (pl + 1) * plane_sz, sg[(pl + 1) & 1]);
                    __builtin_amdgcn_sched_group_barrier(0x100, NRD, 0);
                }
                row_fma<KT>(sg[pl & 1], tp, a[pl][0], a[pl][1], a[pl][2], a[pl][3]);
                __builtin_amdgcn_sched_group_barrier(0x002, 4 * KT, 0);
            }
        }
    }
#pragma unroll
    for (int pl = QLO; pl < HI; ++pl)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[pl][t] = a[pl - QLO][t];
}

// Convolve planes LO..HI-1 for this thread's 1 x 4 output strip (tile row r,
// columns 4 cg .. 4 cg + 3): plane 0 in FP64, the derivative planes in FP32.
// KT > 0: compile-time PSF side; 0: any K.
template <class F, int KT, int LO, int HI>
__device__ inline void conv_group(const float *__restrict__ buf, int K, const cfloat *psf, const float *psl, int r,
                                  int cg, double (&acc0)[4], float (&acc)[F::NPL][4])
{
    if constexpr (KT > 15) {
        conv_group_wide<F, KT, LO, HI>(buf, psf, r, cg, acc0, acc);
    } else if constexpr (KT > 0) {
        conv_group_rows<F, KT, LO, HI>(buf, psl, r, cg, acc0, acc);
    } else {
        const int IH = region_h(K), IWP = region_wp(K);
        const int plane_sz = IH * IWP;
        constexpr int QLO = LO == 0 ? 1 : LO;
        const float *bf = (LO == 0) ? buf + 2 * plane_sz : buf;
        if constexpr (LO == 0)
            conv_plane_any<double>(reinterpret_cast<const double *>(buf) + 4 * cg, r, K, IWP, psf, acc0);
#pragma unroll
        for (int pl = QLO; pl < HI; ++pl) conv_plane_any<float>(bf + (pl - QLO) * plane_sz + 4 * cg, r, K, IWP, psf, acc[pl]);
    }
}

// All groups of one tile: fill, convolve, leave the buffer idle.
template <class F, int KT, int NG, int G = 0>
__device__ inline void tile_planes(const EvalShared<F> &sh, float *buf, int H, int W, int K, int ti0, int tj0,
                                   const cfloat *psf, const float *psl, int r, int cg, double (&acc0)[4],
                                   float (&acc)[F::NPL][4])
{
    if constexpr (G < NG) {
        constexpr int LO = group_bound(F::NPL, NG, G), HI = group_bound(F::NPL, NG, G + 1);
        fill_region<F, LO, HI, shift64<KT>()>(sh, buf, H, W, K, ti0, tj0);
        __syncthreads();
        conv_group<F, KT, LO, HI>(buf, K, psf, psl, r, cg, acc0, acc);
        __syncthreads();
        tile_planes<F, KT, NG, G + 1>(sh, buf, H, W, K, ti0, tj0, psf, psl, r, cg, acc0, acc);
    }
}

// d M / d u_k at output column t of this thread's strip.
// (dx, dy): the pixel's offset from the cutout's centre (analytic sky columns).
template <class F>
__device__ inline float jac_at(int k, int t, const double (&acc0)[4], const float (&acc)[F::NPL][4], float dx,
                               float dy)
{
    if (F::analytic(k)) return F::analytic_value(k, dx, dy);
    if (k == F::DER) {
        float col[F::NPL];
#pragma unroll
        for (int q = 0; q < F::NPL; ++q) col[q] = acc[q][t];
        return F::derived(acc0[t], col);
    }
    return acc[F::plane(k)][t];
}

__device__ inline float pixel_weight(const BatchArgs &ba, int64_t idx, float &d)
{
    d = ba.data[idx];
    float s = ba.sigma[idx];
    bool ok = (ba.omega == nullptr || ba.omega[idx] != 0) && s > 0.0f && isfinite(s) && isfinite(d);
    return ok ? 1.0f / (s * s) : 0.0f;
}

// pixel_weight of the four pixels j0 .. j0 + 3 of the row starting at rowoff,
// read together (columns past W - 1 read pixel W - 1; the caller skips them):
// one wait for the strip instead of one per pixel.
__device__ inline void strip_weights(const BatchArgs &ba, int64_t rowoff, int j0, int W, float (&d)[4],
                                     float (&w)[4])
{
    float s[4];
    int m[4] = {1, 1, 1, 1};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t idx = rowoff + min(j0 + t, W - 1);
        d[t] = ba.data[idx];
        s[t] = ba.sigma[idx];
    }
    if (ba.omega) {
#pragma unroll
        for (int t = 0; t < 4; ++t) m[t] = ba.omega[rowoff + min(j0 + t, W - 1)];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bool ok = m[t] != 0 && s[t] > 0.0f && isfinite(s[t]) && isfinite(d[t]);
        w[t] = ok ? 1.0f / (s[t] * s[t]) : 0.0f;
    }
}

// A bootstrap replica (r >= 0) of galaxy g: every pixel weight is multiplied
// by a Poisson(1) deviate drawn from Philox4x32-10 keyed by (k0, k1), counter
// {pixel / 4, g, r, 1}, word pixel mod 4 (pixel: row-major index in the
// cutout).  r < 0: the plain weights.
struct BootArgs {
    uint32_t k0, k1;
    int g, r;
};

// Poisson(1) multipliers of the four consecutive pixels pix0 .. pix0 + 3.
__device__ inline void boot_weights(const BootArgs &bt, int64_t pix0, float (&m)[4])
{
    const uint32_t q0 = (uint32_t)(pix0 >> 2), off = (uint32_t)(pix0 & 3);
    const U4 a = philox4x32_10(U4{q0, (uint32_t)bt.g, (uint32_t)bt.r, 1u}, bt.k0, bt.k1);
    U4 b = a;
    if (off != 0) b = philox4x32_10(U4{q0 + 1u, (uint32_t)bt.g, (uint32_t)bt.r, 1u}, bt.k0, bt.k1);
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) m[t] = (float)poisson1(w[off + t]);
}

// One model evaluation at u (LDS): chi^2, g = J^T W r and A = J^T W J
// (internal LM variables), written to out_chi2/out_g/out_A (LDS, A full
// P x P).  All threads of the workgroup call it.
//
// A team of tsize workgroups shares one evaluation: the workgroup of rank
// trank takes the tiles whose row-major index is trank modulo tsize, and its
// outputs are the partial sums over those tiles (tsize = 1: the whole image).
template <class F, int KT, int NG>
__device__ void evaluate(const double *u, const ModelArgs &ma, const BatchArgs &ba, const Meta &me, EvalShared<F> &sh,
                         float *planes, double *out_chi2, double *out_g, double *out_A,
                         const BootArgs &bt = BootArgs{0u, 0u, 0, -1}, int trank = 0, int tsize = 1)
{
    constexpr int P = F::P;
    constexpr int NR = 1 + P + P * (P + 1) / 2;
    const int H = me.h, W = me.w, K = me.k;
    const int tid = threadIdx.x;
    const float *psl = stage_psf<F, NG>(planes, ba.psf + uniform64(me.psf_off), K);
    eval_prologue<F>(u, ma, H, W, sh, planes);
    const cfloat *psf = (const cfloat *)(ba.psf + uniform64(me.psf_off));
    // Per-thread partial sums: chi^2 in FP64 (it decides accept/reject), g and
    // A in FP32 over at most FLUSH_TILES tiles (64 pixels), then FP64.
    double c2 = 0.0;
    float red[NR - 1];
#pragma unroll
    for (int q = 0; q < NR - 1; ++q) red[q] = 0.0f;
    int r, cg;
    strip_of(tid, K, r, cg);
    const int nty = (H + TILE - 1) / TILE, ntx = (W + TILE - 1) / TILE;
    const int lane = tid & 63, wave = tid >> 6;
    const int ntiles = nty * ntx;
    const int mine = (ntiles - trank + tsize - 1) / tsize;        // tiles of this workgroup
    const bool flushes = mine > FLUSH_TILES;                      // uniform over the workgroup
    if (flushes && lane == 0)
        for (int q = 0; q < NR - 1; ++q) sh.nacc[wave][q] = 0.0;
    int since_flush = 0;
    for (int ti = trank; ti < ntiles; ti += tsize) {
        {
            const int ty = ti / ntx, tx = ti - ty * ntx;
            if (since_flush == FLUSH_TILES) {
                // the FP32 partials of the last FLUSH_TILES tiles into the wave's FP64 sums
#pragma unroll
                for (int q = 0; q < NR - 1; ++q) {
                    const double v = wave_sum((double)red[q]);
                    if (lane == 0) sh.nacc[wave][q] += v;
                    red[q] = 0.0f;
                }
                since_flush = 0;
            }
            ++since_flush;
            const int ti0 = ty * TILE, tj0 = tx * TILE;
            double acc0[4];
            float acc[F::NPL][4];
            tile_planes<F, KT, NG>(sh, planes, H, W, K, ti0, tj0, psf, psl, r, cg, acc0, acc);
            const int i = ti0 + r;
            if (i < H) {
                float bw[4] = {1.0f, 1.0f, 1.0f, 1.0f};
                if (bt.r >= 0) boot_weights(bt, (int64_t)i * W + tj0 + 4 * cg, bw);
                float dv[4], wv[4];
                strip_weights(ba, me.img_off + (int64_t)i * W, tj0 + 4 * cg, W, dv, wv);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int j = tj0 + 4 * cg + t;
                    if (j >= W) continue;
                    const float d = dv[t];
                    const float wgt = wv[t] * bw[t];
                    if (wgt == 0.0f) continue;
                    const double pdx = ((double)j + 0.5) - 0.5 * W, pdy = 0.5 * H - ((double)i + 0.5);
                    const double res = (double)d - (acc0[t] + F::sky_at(sh.prep, pdx, pdy));
                    c2 = fma((double)wgt * res, res, c2);
                    const float wr = wgt * (float)res;
                    const float fdx = (float)pdx, fdy = (float)pdy;
#pragma unroll
                    for (int k = 0; k < P; ++k) {
                        const float Jk = jac_at<F>(k, t, acc0, acc, fdx, fdy);
                        red[k] = fmaf(wr, Jk, red[k]);
                        const float wj = wgt * Jk;
#pragma unroll
                        for (int l = 0; l <= k; ++l) {
                            const float Jl = jac_at<F>(l, t, acc0, acc, fdx, fdy);
                            red[P + k * (k + 1) / 2 + l] = fmaf(wj, Jl, red[P + k * (k + 1) / 2 + l]);
                        }
                    }
                }
            }
        }
    }
    // fixed-order reduction in FP64: within each wave, then the waves in order
    // (the plane buffer is idle after the last tile's barrier: reuse it)
    double *sred = reinterpret_cast<double *>(planes);
    {
        double v = wave_sum(c2);
        if (lane == 0) sred[wave * NR] = v;
    }
#pragma unroll
    for (int q = 1; q < NR; ++q) {
        double v = wave_sum((double)red[q - 1]);
        if (lane == 0) sred[wave * NR + q] = flushes ? sh.nacc[wave][q - 1] + v : v;
    }
    __syncthreads();
    for (int q = tid; q < NR; q += NT) {
        double s = sred[q];
        for (int wv = 1; wv < NWAVE; ++wv) s += sred[wv * NR + q];
        if (q == 0) {
            *out_chi2 = s;
        } else if (q <= P) {
            out_g[q - 1] = s;
        } else {
            int e = q - 1 - P, k = 0;
            while ((k + 1) * (k + 2) / 2 <= e) ++k;
            int l = e - k * (k + 1) / 2;
            out_A[k * P + l] = s;
            out_A[l * P + k] = s;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- small FP64 algebra (one thread)
// Cholesky L L^T = M of a P x P matrix; returns false if not positive definite.
template <int P>
__device__ bool chol(const double *M, double *L)
{
    for (int i = 0; i < P * P; ++i) L[i] = 0.0;
    for (int j = 0; j < P; ++j) {
        double d = M[j * P + j];
        for (int k = 0; k < j; ++k) d -= L[j * P + k] * L[j * P + k];
        if (!(d > 0.0) || !isfinite(d)) return false;
        double lj = sqrt(d);
        L[j * P + j] = lj;
        for (int i = j + 1; i < P; ++i) {
            double s = M[i * P + j];
            for (int k = 0; k < j; ++k) s -= L[i * P + k] * L[j * P + k];
            L[i * P + j] = s / lj;
        }
    }
    return true;
}

template <int P>
__device__ void chol_solve(const double *L, const double *b, double *x)
{
    double y[P];
    for (int i = 0; i < P; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * P + k] * y[k];
        y[i] = s / L[i * P + i];
    }
    for (int i = P - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < P; ++k) s -= L[k * P + i] * x[k];
        x[i] = s / L[i * P + i];
    }
}

template <int P>
__device__ void chol_inverse(const double *L, double *inv)
{
    for (int j = 0; j < P; ++j) {
        double e[P], col[P];
        for (int i = 0; i < P; ++i) e[i] = (i == j) ? 1.0 : 0.0;
        chol_solve<P>(L, e, col);
        for (int i = 0; i < P; ++i) inv[i * P + j] = col[i];
    }
}

// Fixed parameters: their rows and columns of A are replaced by the identity
// and their gradient by 0, so that they never move.
template <int P>
__device__ void project_fixed(const int *freev, double *A, double *g)
{
    for (int k = 0; k < P; ++k) {
        if (freev[k]) continue;
        for (int l = 0; l < P; ++l) {
            A[k * P + l] = 0.0;
            A[l * P + k] = 0.0;
        }
        A[k * P + k] = 1.0;
        g[k] = 0.0;
    }
}

// Bounds of the LM variables (natural units: centres inside the cutout,
// scales in [0.1, 2 max(H, W)] px, Sersic n in [0.2, 10], q in [0.05, 20]).

// Canonical form of every component: q > 1 -> (1/q, scale * q, theta + pi/2),
// then theta wrapped into [0, pi).  u in internal layout; natural output.
template <class F>
__device__ void canonical_nat(const double *u, const int *freev, double *nat)
{
    for (int k = 0; k < F::P; ++k) nat[k] = u_to_nat(F::kind(k), u[k]);
    for (int c = 0; c < F::NCAN; ++c) {
        int iq, ith, is0, is1;
        F::canon(c, iq, ith, is0, is1);
        if (freev[iq] && freev[ith] && nat[iq] > 1.0) {
            double qo = nat[iq];
            nat[iq] = 1.0 / qo;
            if (is0 >= 0) nat[is0] *= qo;
            if (is1 >= 0) nat[is1] *= qo;
            nat[ith] += 90.0;
        }
        if (freev[ith]) {
            double pa = fmod(nat[ith], 180.0);
            if (pa < 0.0) pa += 180.0;
            if (pa >= 180.0) pa -= 180.0;
            nat[ith] = pa;
        }
    }
}

// Covariance errors of a fit, sqrt(diag (J^T W J)^-1) (Sec. 5.2), from the
// normal matrix of the last accepted evaluation (J^T W J at u), in natural
// units of the canonical form written by canonical_nat.  Where that form
// flips a component (q -> 1/q, each scale s -> s q, theta -> theta + pi/2),
// the model image is unchanged, so the Jacobian in the canonical variables is
// J Phi^-1 with Phi the Jacobian of the flip in the LM variables (ln s' =
// ln s + ln q, q' = 1/q) and the covariance becomes Phi (J^T W J)^-1 Phi^T:
// the errors gm_param_errors computes at the canonical parameters, without
// another evaluation.  Fixed slots have identity rows (as in the error
// kernel); a matrix that is not positive definite gives NaN.  One thread,
// every array in LDS and every loop rolled, so that it adds no registers to
// the fit's loops; scratch: 3 P^2 + 2 P doubles.  A is overwritten.
template <class F>
__device__ void fit_errors(double *A, double *g, const double *u, const int *freev, const ModelArgs &ma, double *err,
                           double *scratch)
{
    constexpr int P = F::P;
    double *L = scratch, *inv = L + P * P, *phi = inv + P * P, *nat = phi + P * P, *y = nat + P;
    project_fixed<P>(freev, A, g);
    // Cholesky A = L L^T
    bool ok = true;
#pragma unroll 1
    for (int j = 0; j < P && ok; ++j) {
        double d = A[j * P + j];
#pragma unroll 1
        for (int k = 0; k < j; ++k) d -= L[j * P + k] * L[j * P + k];
        if (!(d > 0.0) || !isfinite(d)) {
            ok = false;
            break;
        }
        const double lj = sqrt(d);
        L[j * P + j] = lj;
#pragma unroll 1
        for (int i = j + 1; i < P; ++i) {
            double t = A[i * P + j];
#pragma unroll 1
            for (int k = 0; k < j; ++k) t -= L[i * P + k] * L[j * P + k];
            L[i * P + j] = t / lj;
        }
    }
    if (!ok) {
#pragma unroll 1
        for (int k = 0; k < P; ++k)
            if (ma.col[k] >= 0) err[ma.col[k]] = NAN;
        return;
    }
    // inverse, column by column: L y = e_j, then L^T x = y
#pragma unroll 1
    for (int j = 0; j < P; ++j) {
#pragma unroll 1
        for (int i = 0; i < P; ++i) {
            double t = (i == j) ? 1.0 : 0.0;
#pragma unroll 1
            for (int k = 0; k < i; ++k) t -= L[i * P + k] * y[k];
            y[i] = t / L[i * P + i];
        }
#pragma unroll 1
        for (int i = P - 1; i >= 0; --i) {
            double t = y[i];
#pragma unroll 1
            for (int k = i + 1; k < P; ++k) t -= L[k * P + i] * inv[k * P + j];
            inv[i * P + j] = t / L[i * P + i];
        }
    }
    // Phi: identity, with the flip's rows for components canonical_nat flips
#pragma unroll 1
    for (int k = 0; k < P * P; ++k) phi[k] = (k % (P + 1) == 0) ? 1.0 : 0.0;
#pragma unroll 1
    for (int c = 0; c < F::NCAN; ++c) {
        int iq, ith, is0, is1;
        F::canon(c, iq, ith, is0, is1);
        const double q = u[iq];
        if (freev[iq] && freev[ith] && q > 1.0) {
            phi[iq * P + iq] = -1.0 / (q * q);
            if (is0 >= 0) phi[is0 * P + iq] = 1.0 / q;
            if (is1 >= 0) phi[is1 * P + iq] = 1.0 / q;
        }
    }
    canonical_nat<F>(u, freev, nat);
    // diag(Phi inv Phi^T)
#pragma unroll 1
    for (int a = 0; a < P; ++a) {
        if (ma.col[a] < 0) continue;
        double v = 0.0;
#pragma unroll 1
        for (int k = 0; k < P; ++k) {
            if (phi[a * P + k] == 0.0) continue;
            double t = 0.0;
#pragma unroll 1
            for (int l = 0; l < P; ++l) t += inv[k * P + l] * phi[a * P + l];
            v += phi[a * P + k] * t;
        }
        err[ma.col[a]] = sqrt(v) * fabs(dnat_du(F::kind(a), nat[a]));
    }
}

// ---------------------------------------------------------------- LM kernel
template <class F>
struct LMShared {
    double u[F::P], ut[F::P], g[F::P], gt[F::P], A[F::P * F::P], At[F::P * F::P];
    double Dg[F::P], sig[F::P], delta[F::P];
    double chi2, chi2t, lambda;
    int freev[F::P];
    int t, status, fresh, apd, action, max_iter;
    int gal;
    int tok;                  // team: the last wait ended in time
};

struct FitArgs {
    const int *order;
    const int *active;        // nullable: galaxies with active[g] == 0 are skipped
    int n_gal;
    int *queue;
    double *params, *chi2;
    int *niter, *status;
    double *err;              // nullable: covariance errors at the fit [n_gal][p]
    int max_iter;
    double lambda0, tol;
    // Refit (nullable refit_start): a galaxy whose fit from params ends other
    // than CONVERGED within first_max_iter trials, or whose valid[g] is 0 (its
    // params are not a usable start), is fitted again, at once and by the same
    // workgroup, from refit_start[g] with max_iter trials; niter counts the
    // trials of both fits and refit_code[g] (nullable) is 0 (first fit), 1
    // (unusable start) or 2 (refitted).
    const double *refit_start;
    const int *valid;
    int *refit_code;
    int first_max_iter;
    // Bootstrap (n_boot > 0): fit index i is replica i % n_boot of galaxy
    // i / n_boot (BootArgs, key (boot_k0, boot_k1)); n_gal counts fit indices.
    int n_boot;
    uint32_t boot_k0, boot_k1;
    // Teams (nullable items): queue entry i is items[i] instead of order[i];
    // n_gal then counts the entries.  A fit with team size G > 1 is served by
    // G workgroups through its TeamCtl (ctl[team]) and its G partial-sum
    // slots (part + team * part_stride + rank * NR); spin_limit bounds every
    // wait of a team member, in wall-clock ticks.
    const struct TeamItem *items;
    struct TeamCtl *ctl;
    double *part;
    int64_t part_stride;
    int64_t spin_limit;
};

enum { ACT_EVAL = 0, ACT_RETRY = 1, ACT_DONE = 2 };

// ---------------------------------------------------------------- teams of workgroups
// A fit served by G workgroups: the leader (rank 0) runs the LM, and each
// evaluation is shared by the team -- the leader publishes the point (its
// LM variables and the command ACT_EVAL, epoch by epoch), every member
// evaluates its tiles and delivers its partial sums (chi^2, g, the lower
// triangle of A in FP64), the leader adds the G partials in rank order (a
// fixed order: results do not depend on timing) and takes the LM step.  The
// leader ends the team with ACT_DONE.  All G workgroups hold their queue
// entries at once (consecutive entries of the persistent grid, which is never
// smaller than a team), so every wait ends; each wait is nonetheless bounded
// by spin_limit, after which the fit ends with GM_ST_TEAM_TIMEOUT.
struct TeamItem {
    int32_t fit, rank, size, team;
};

struct TeamCtl {
    int cmd;                  // commands published so far (the epoch of the last one + 1)
    int action;               // the last command: ACT_EVAL or ACT_DONE
    int arrive;               // partial sums delivered so far, over all epochs
    int pad;
    double u[MAXP];           // the point of the last ACT_EVAL
};

__device__ inline int team_load(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0: wait until *p >= target (acquire) or the limit passes; true if reached.
__device__ inline bool team_wait(const int *p, int target, int64_t limit)
{
    const int64_t t0 = wall_clock64();
    while (team_load(p) < target) {
        if (wall_clock64() - t0 > limit) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Entry q of the NR = 1 + P + P (P + 1) / 2 sums of an evaluation: chi^2, g,
// then A's lower triangle row by row.
template <int P>
__device__ inline double sum_entry(int q, double chi2, const double *g, const double *A)
{
    if (q == 0) return chi2;
    if (q <= P) return g[q - 1];
    int e = q - 1 - P, k = 0;
    while ((k + 1) * (k + 2) / 2 <= e) ++k;
    return A[k * P + (e - k * (k + 1) / 2)];
}

template <int P>
__device__ inline void set_entry(int q, double v, double *chi2, double *g, double *A)
{
    if (q == 0) {
        *chi2 = v;
    } else if (q <= P) {
        g[q - 1] = v;
    } else {
        int e = q - 1 - P, k = 0;
        while ((k + 1) * (k + 2) / 2 <= e) ++k;
        const int l = e - k * (k + 1) / 2;
        A[k * P + l] = v;
        A[l * P + k] = v;
    }
}

// All threads: this workgroup's partial sums (LDS) into its slot, made visible
// at device scope before thread 0 counts the delivery.
template <int P>
__device__ inline void team_deliver(TeamCtl *ctl, double *slot, double chi2, const double *g, const double *A)
{
    constexpr int NR = 1 + P + P * (P + 1) / 2;
    for (int q = threadIdx.x; q < NR; q += NT) slot[q] = sum_entry<P>(q, chi2, g, A);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&ctl->arrive, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- wave-parallel LM step
// One wave runs the LM bookkeeping between evaluations.  Lane r < P holds row
// r of the P x P normal matrix; the Cholesky factorisation is row-parallel
// (the pivot row is broadcast with readlane at every step), and the
// triangular solves and the diagonal of the inverse are computed by every
// lane from broadcast values.  Sums run in the same order as the textbook
// one-thread algorithm.

// L (lane r: row r) of M (lane r: row r); false if M is not positive definite.
template <int P>
__device__ inline bool chol_rows(const double (&m)[P], double (&l)[P], int lane)
{
#pragma unroll
    for (int k = 0; k < P; ++k) l[k] = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double lj[P > 1 ? P - 1 : 1];
#pragma unroll
        for (int k = 0; k < j; ++k) lj[k] = lane_value(l[k], j);
        double d = lane_value(m[j], j);
#pragma unroll
        for (int k = 0; k < j; ++k) d -= lj[k] * lj[k];
        if (!(d > 0.0) || !isfinite(d)) return false;
        const double ljj = sqrt(d);
        double sr = m[j];
#pragma unroll
        for (int k = 0; k < j; ++k) sr -= l[k] * lj[k];
        l[j] = lane > j ? sr / ljj : (lane == j ? ljj : 0.0);
    }
    return true;
}

// x = (L L^T)^-1 b, with b and the result as wave-uniform arrays.
template <int P>
__device__ inline void chol_solve_rows(const double (&l)[P], const double (&b)[P], double (&x)[P])
{
    double y[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        double t = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) t -= lane_value(l[k], i) * y[k];
        y[i] = t / lane_value(l[i], i);
    }
#pragma unroll
    for (int i = P - 1; i >= 0; --i) {
        double t = y[i];
#pragma unroll
        for (int k = i + 1; k < P; ++k) t -= lane_value(l[i], k) * x[k];
        x[i] = t / lane_value(l[i], i);
    }
}

// diag((L L^T)^-1)_c = sum_i (L^-1)_ic^2, as a wave-uniform array.
template <int P>
__device__ inline void chol_inv_diag_rows(const double (&l)[P], double (&dg)[P])
{
#pragma unroll
    for (int c = 0; c < P; ++c) {
        double z[P];
        double acc = 0.0;
#pragma unroll
        for (int i = c; i < P; ++i) {
            double t = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int k = c; k < i; ++k) t -= lane_value(l[k], i) * z[k];
            z[i] = t / lane_value(l[i], i);
            acc += z[i] * z[i];
        }
        dg[c] = acc;
    }
}

// v limited to [lo, hi] by comparisons: a NaN stays NaN (fmin/fmax would
// replace it by a bound), so a non-finite start or step gives a non-finite
// chi^2 and is never taken for a point inside the bounds.
__device__ inline double clamp_to(double v, double lo, double hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

// Bounds of the LM variables (internal units: ln of scales, n and a, radians).
template <class F>
__device__ inline double clamp_var(int k, double v, int H, int W)
{
    const double big = 2.0 * (H > W ? H : W);
    switch (F::kind(k)) {
    case KX0: return clamp_to(v, 0.0, (double)W);
    case KY0: return clamp_to(v, 0.0, (double)H);
    case KSCALE: return clamp_to(v, log(0.1), log(big));
    case KN: return clamp_to(v, log(0.2), log(10.0));
    case KQ: return clamp_to(v, 0.05, 20.0);
    case KBOX: return clamp_to(v, -0.9, 2.0);
    case KFA: return clamp_to(v, log(0.1), log(10.0));
    case KFB: return clamp_to(v, -1.0, 1.95);
    case KKAL: return clamp_to(v, log(0.5), log(10.0));
    default: return v;
    }
}

template <class F>
__device__ void clamp_u(double *u, int H, int W)
{
    for (int k = 0; k < F::P; ++k) u[k] = clamp_var<F>(k, u[k], H, W);
}

// Wave 0, all lanes: absorb the evaluation just made (the start point, or a
// trial: accept if chi^2 decreased, else raise the damping), then choose the
// next trial point or finish.
//   Start: A, g from the evaluation, fixed rows/columns replaced by the
//     identity and their gradient by 0; lambda = lambda0.
//   Stop test at every newly accepted state: the undamped Gauss-Newton step
//     A^-1 g in units of sigma_k = sqrt([A^-1]_kk) below tol -> CONVERGED
//     (while A is not positive definite: the damped step against
//     1/sqrt(D_kk)).
//   Trial: (A + lambda D) delta = g with D = diag(max(A_kk, 1e-12 max A_kk))
//     of the current accepted A; a failed factorisation raises lambda by 10
//     and counts the trial; lambda > 1e9 -> STALLED; max_iter trials ->
//     MAXITER.
template <class F>
__device__ void lm_step_wave(LMShared<F> &s, const FitArgs &fa, int H, int W)
{
    constexpr int P = F::P;
    const int lane = threadIdx.x & 63;
    const bool row = lane < P;
    const int r = row ? lane : 0;
    bool fv[P];
#pragma unroll
    for (int k = 0; k < P; ++k) fv[k] = s.freev[k] != 0;
    bool fr = false;
#pragma unroll
    for (int k = 0; k < P; ++k)
        if (k == r) fr = fv[k];
    int t = s.t, action = s.action, status = s.status, fresh = s.fresh, apd = s.apd;
    double lambda = s.lambda, chi2 = s.chi2;
    double a[P];
    double gr, ur = s.u[r], dgr = s.Dg[r], sgr = s.sig[r];
    bool newA = false, accepted = false;
    if (t < 0 || action == ACT_EVAL) {
        const double chi2t = s.chi2t;
        const bool take = t < 0 || (isfinite(chi2t) && chi2t < chi2);
        if (take) {
#pragma unroll
            for (int k = 0; k < P; ++k) a[k] = (fr && fv[k]) ? s.At[r * P + k] : (r == k ? 1.0 : 0.0);
            gr = fr ? s.gt[r] : 0.0;
            newA = true;
            chi2 = chi2t;
            if (t < 0) {
                t = 0;
                if (!isfinite(chi2)) {
                    status = GM_ST_NONFINITE;
                    action = ACT_DONE;
                }
            } else {
                accepted = true;
                ur = s.ut[r];
                lambda = fmax(lambda / 10.0, 1e-9);
                fresh = 1;
            }
        } else {
            lambda *= 10.0;
            if (lambda > 1e9) {
                status = GM_ST_STALLED;
                action = ACT_DONE;
            }
        }
    }
    if (!newA) {
#pragma unroll
        for (int k = 0; k < P; ++k) a[k] = s.A[r * P + k];
        gr = s.g[r];
    }
    double utr = ur;
    bool proposed = false;
    if (action != ACT_DONE) {
        if (t >= s.max_iter) {
            status = GM_ST_MAXITER;
            action = ACT_DONE;
        } else {
            t += 1;
            double gv[P];
#pragma unroll
            for (int k = 0; k < P; ++k) gv[k] = lane_value(gr, k);
            bool stop = false;
            if (fresh) {
                double drr = 0.0;
#pragma unroll
                for (int k = 0; k < P; ++k)
                    if (k == r) drr = a[k];
                double amax = 0.0;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    const double dk = lane_value(drr, k);
                    if (fv[k] && dk > amax) amax = dk;
                }
                dgr = fr ? (drr > 1e-12 * amax ? drr : 1e-12 * amax) : 1.0;
                double l[P];
                apd = chol_rows<P>(a, l, lane) ? 1 : 0;
                if (apd) {
                    double idg[P], dv[P];
                    chol_inv_diag_rows<P>(l, idg);
                    chol_solve_rows<P>(l, gv, dv);
                    double smax = 0.0;
#pragma unroll
                    for (int k = 0; k < P; ++k) {
                        const double sk = sqrt(idg[k]);
                        if (k == r) sgr = sk;
                        const double q = fabs(dv[k]) / sk;
                        if (!(q <= smax)) smax = q;
                    }
                    if (smax < fa.tol) {
                        t -= 1;
                        status = GM_ST_CONVERGED;
                        action = ACT_DONE;
                        stop = true;
                    }
                } else {
                    sgr = 1.0 / sqrt(dgr);
                }
                fresh = 0;
            }
            if (!stop) {
                double m[P], l[P];
#pragma unroll
                for (int k = 0; k < P; ++k) m[k] = a[k] + (k == r ? lambda * dgr : 0.0);
                if (!chol_rows<P>(m, l, lane)) {
                    lambda *= 10.0;
                    if (lambda > 1e9) {
                        status = GM_ST_STALLED;
                        action = ACT_DONE;
                    } else {
                        action = ACT_RETRY;
                    }
                } else {
                    double dv[P];
                    chol_solve_rows<P>(l, gv, dv);
                    bool conv = false;
                    if (!apd) {
                        double smax = 0.0;
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            const double q = fabs(dv[k]) / lane_value(sgr, k);
                            if (!(q <= smax)) smax = q;
                        }
                        conv = smax < fa.tol;
                    }
                    if (conv) {
                        t -= 1;
                        status = GM_ST_CONVERGED;
                        action = ACT_DONE;
                    } else {
                        double dr = 0.0;
#pragma unroll
                        for (int k = 0; k < P; ++k)
                            if (k == r) dr = dv[k];
                        utr = clamp_var<F>(r, ur + (fr ? dr : 0.0), H, W);
                        proposed = true;
                        action = ACT_EVAL;
                    }
                }
            }
        }
    }
    if (row) {
        if (newA) {
#pragma unroll
            for (int k = 0; k < P; ++k) s.A[r * P + k] = a[k];
            s.g[r] = gr;
        }
        if (accepted) s.u[r] = ur;
        if (proposed) s.ut[r] = utr;
        s.Dg[r] = dgr;
        s.sig[r] = sgr;
    }
    if (lane == 0) {
        s.t = t;
        s.action = action;
        s.status = status;
        s.fresh = fresh;
        s.apd = apd;
        s.lambda = lambda;
        s.chi2 = chi2;
    }
}

template <class F>
__device__ void load_u(LMShared<F> &s, const ModelArgs &ma, const double *params)
{
    for (int k = 0; k < F::P; ++k) {
        int c = ma.col[k];
        double nat = c >= 0 ? params[c] : ma.fixedv[k];
        s.u[k] = nat_to_u(F::kind(k), nat);
        s.freev[k] = c >= 0;
    }
}

// Workgroups per CU that the fit kernel's register allocation targets.  Two
// (at most 256 VGPRs per lane) let one workgroup's profile evaluation,
// prologue and LM step overlap the other's convolution, where the plane
// buffers of two fit in LDS.  The one-component families fit them without
// spills inside loops (measured 1.38x faster Sersic fits at 64 x 64, PSF
// side 15); the two-component models need more registers than that for
// their accumulators and keep one (as does the error kernel, which would
// spill inside its loops).  Where a workgroup's LDS (plane buffer, PSF
// copies, static state) leaves room for one per CU only, the target is one
// too: the second workgroup's registers could never be used, and the 256
// VGPR cap made the wide-PSF kernels spill.
template <class F, int KT, int NG>
__host__ __device__ constexpr int min_wg()
{
    if (F::NCOMP != 1) return 1;
    if (KT == 0) return 2;
    const size_t planes = (size_t)max_group_units(F::NPL, NG) * region_h(KT) * region_wp(KT) * sizeof(float);
    const size_t psf = (size_t)KT * ((KT + 3) & ~3) * (sizeof(float) + sizeof(double));
    const size_t per_wg = planes + psf + sizeof(EvalShared<F>) + sizeof(LMShared<F>) + 1024;
    return 2 * per_wg <= (size_t)160 * 1024 ? 2 : 1;
}

// Team steps around the one evaluation site of lm_fit_kernel.
// Leader: publish the point s.ut of the epoch-th shared evaluation.
template <class F>
__device__ inline void team_publish(const LMShared<F> &s, TeamCtl *ctl, int epoch)
{
    const int tid = threadIdx.x;
    if (tid < F::P) ctl->u[tid] = s.ut[tid];
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        ctl->action = ACT_EVAL;
        __hip_atomic_store(&ctl->cmd, epoch + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Member: wait for the leader's command of the epoch-th evaluation; s.action
// and (for ACT_EVAL) s.ut take it.  A wait past the spin limit reads as ACT_DONE.
template <class F>
__device__ inline void team_command(LMShared<F> &s, const TeamCtl *ctl, int epoch, int64_t limit)
{
    if (threadIdx.x == 0) {
        // the command's fields are read atomically (never through a cache of
        // uniform loads), after the acquire of cmd
        const bool got = team_wait(&ctl->cmd, epoch + 1, limit);
        const int act = got ? __hip_atomic_load(&ctl->action, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : ACT_DONE;
        s.action = act;
        if (act == ACT_EVAL)
            for (int k = 0; k < F::P; ++k)
                s.ut[k] = __hip_atomic_load(&ctl->u[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// Leader, after its own delivery: wait for the team's tsize deliveries of the
// epoch-th evaluation and add the partial sums in rank order into s.chi2t,
// s.gt, s.At.  False if they did not arrive within the limit.
template <class F>
__device__ inline bool team_collect(LMShared<F> &s, TeamCtl *ctl, const double *slots, int tsize, int epoch,
                                    int64_t limit)
{
    constexpr int P = F::P, NR = 1 + P + P * (P + 1) / 2;
    const int tid = threadIdx.x;
    if (tid == 0) s.tok = team_wait(&ctl->arrive, tsize * (epoch + 1), limit) ? 1 : 0;
    __syncthreads();
    const bool ok = uniform(s.tok) != 0;
    if (ok) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (int q = tid; q < NR; q += NT) {
            double v = slots[q];
            for (int r = 1; r < tsize; ++r) v += slots[(int64_t)r * NR + q];
            set_entry<P>(q, v, &s.chi2t, s.gt, s.At);
        }
    }
    __syncthreads();
    return ok;
}

// Persistent LM fits: each workgroup takes queue entries (a fit, or one rank
// of a team sharing a fit) until the queue is empty.  One workgroup, or the
// leader of a team, runs the LM of its fit (a fit from params, then possibly
// the refit from refit_start); members follow the leader's commands.  The
// model is evaluated at a single site for all three roles.
template <class F, int KT, int NG>
__global__ __launch_bounds__(NT, (min_wg<F, KT, NG>())) void lm_fit_kernel(ModelArgs ma, BatchArgs ba, FitArgs fa)
{
    extern __shared__ float4 dyn_lds[];
    float *planes = reinterpret_cast<float *>(dyn_lds);
    __shared__ EvalShared<F> esh;
    __shared__ LMShared<F> s;
    constexpr int NR = 1 + F::P + F::P * (F::P + 1) / 2;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s.gal = atomicAdd(fa.queue, 1);
        __syncthreads();
        const int qi = uniform(s.gal);
        if (qi >= fa.n_gal) break;
        int g, trank = 0, tsize = 1, team = 0;
        if (fa.items) {
            const TeamItem it = fa.items[qi];
            g = uniform(it.fit);
            trank = uniform(it.rank);
            tsize = uniform(it.size);
            team = uniform(it.team);
        } else {
            g = uniform(fa.order[qi]);
        }
        if (fa.active && uniform(fa.active[g]) == 0) {
            __syncthreads();      // s.gal is rewritten by thread 0 next
            continue;
        }
        const int src = fa.n_boot > 0 ? g / fa.n_boot : g;
        const BootArgs bt{fa.boot_k0, fa.boot_k1, src, fa.n_boot > 0 ? g - src * fa.n_boot : -1};
        const Meta me = ba.meta[src];
        const bool member = trank > 0;
        TeamCtl *ctl = tsize > 1 ? fa.ctl + team : nullptr;
        double *slots = tsize > 1 ? fa.part + (int64_t)team * fa.part_stride : nullptr;
        // phase 0: the fit from params; phase 1: the refit from refit_start
        const bool refit = fa.refit_start != nullptr;
        const int first = (!member && refit && fa.valid && uniform(fa.valid[g]) == 0) ? 1 : 0;
        int t0 = 0, phase = first, epoch = 0;
        bool phase_start = !member;
        for (;;) {
            if (phase_start) {
                if (tid == 0) {
                    load_u<F>(s, ma, (phase ? fa.refit_start : fa.params) + (int64_t)g * ma.p);
                    clamp_u<F>(s.u, me.h, me.w);
                    for (int k = 0; k < F::P; ++k) s.ut[k] = s.u[k];
                    s.t = -1;             // -1: the next evaluation is the start point
                    s.status = GM_ST_MAXITER;
                    s.max_iter = (refit && phase == 0) ? fa.first_max_iter : fa.max_iter;
                    s.lambda = fa.lambda0;
                    s.fresh = 1;
                    s.apd = 0;
                    s.chi2 = 0.0;
                    s.action = ACT_EVAL;
                    for (int k = 0; k < F::P; ++k) {
                        s.Dg[k] = 1.0;
                        s.sig[k] = 1.0;
                    }
                }
                __syncthreads();
                phase_start = false;
            }
            if (member) team_command<F>(s, ctl, epoch, fa.spin_limit);
            const int act = uniform(s.action);
            if (act == ACT_DONE) {
                if (member) break;
                if (uniform(s.status) == GM_ST_TEAM_TIMEOUT || phase == 1) break;
                if (!refit || uniform(s.status) == GM_ST_CONVERGED) {
                    t0 = -1;          // no refit
                    break;
                }
                t0 = uniform(s.t);
                __syncthreads();      // every thread has read s before thread 0 reloads it
                phase = 1;
                phase_start = true;
                continue;
            }
            if (act == ACT_EVAL) {
                if (tsize > 1 && !member) team_publish<F>(s, ctl, epoch);
                // the evaluation site: the whole image, or this rank's tiles of it
                evaluate<F, KT, NG>(s.ut, ma, ba, me, esh, planes, &s.chi2t, s.gt, s.At, bt, trank, tsize);
                if (tsize > 1) {
                    team_deliver<F::P>(ctl, slots + (int64_t)trank * NR, s.chi2t, s.gt, s.At);
                    if (!member && !team_collect<F>(s, ctl, slots, tsize, epoch, fa.spin_limit)) {
                        if (tid == 0) {
                            s.status = GM_ST_TEAM_TIMEOUT;
                            s.action = ACT_DONE;
                        }
                        __syncthreads();
                        continue;
                    }
                    ++epoch;
                }
            }
            if (!member && tid < 64) lm_step_wave<F>(s, fa, me.h, me.w);
            __syncthreads();
        }
        if (member) {
            __syncthreads();          // s.gal is rewritten by thread 0 next
            continue;
        }
        if (tsize > 1 && tid == 0) {
            // end the team (epoch + 2 exceeds every epoch a member can be waiting for)
            ctl->action = ACT_DONE;
            __hip_atomic_store(&ctl->cmd, epoch + 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (uniform(s.status) == GM_ST_TEAM_TIMEOUT) t0 = -1;
        if (tid == 0) {
            double nat[F::P];
            canonical_nat<F>(s.u, s.freev, nat);
            double *out = fa.params + (int64_t)g * ma.p;
            for (int k = 0; k < F::P; ++k)
                if (ma.col[k] >= 0) out[ma.col[k]] = nat[k];
            fa.chi2[g] = s.chi2;
            fa.niter[g] = s.t + (t0 > 0 ? t0 : 0);
            fa.status[g] = s.status;
            if (fa.refit_code) fa.refit_code[g] = t0 < 0 ? 0 : (first ? 1 : 2);
            if (fa.err)
                fit_errors<F>(s.A, s.g, s.u, s.freev, ma, fa.err + (int64_t)g * ma.p,
                              reinterpret_cast<double *>(planes));
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- covariance errors
struct ErrArgs {
    const double *params;
    double *err, *cov;
    int n_gal;
};

template <class F, int KT, int NG>
__global__ __launch_bounds__(NT) void errors_kernel(ModelArgs ma, BatchArgs ba, ErrArgs ea)
{
    extern __shared__ float4 dyn_lds[];
    float *planes = reinterpret_cast<float *>(dyn_lds);
    __shared__ EvalShared<F> esh;
    __shared__ LMShared<F> s;
    constexpr int P = F::P;
    const int tid = threadIdx.x;
    for (int g = blockIdx.x; g < ea.n_gal; g += gridDim.x) {
        const Meta me = ba.meta[g];
        if (tid == 0) load_u<F>(s, ma, ea.params + (int64_t)g * ma.p);
        __syncthreads();
        evaluate<F, KT, NG>(s.u, ma, ba, me, esh, planes, &s.chi2, s.g, s.A);
        if (tid == 0) {
            // thread-0 temporaries in the idle plane buffer
            double *L = reinterpret_cast<double *>(planes);
            double *inv = L + P * P;
            project_fixed<P>(s.freev, s.A, s.g);
            const int p = ma.p;
            double *err = ea.err + (int64_t)g * p;
            double *cov = ea.cov ? ea.cov + (int64_t)g * p * p : nullptr;
            if (chol<P>(s.A, L)) {
                chol_inverse<P>(L, inv);
                for (int a = 0; a < P; ++a) {
                    if (ma.col[a] < 0) continue;
                    double na = u_to_nat(F::kind(a), s.u[a]);
                    double sa = dnat_du(F::kind(a), na);
                    err[ma.col[a]] = sqrt(inv[a * P + a]) * fabs(sa);
                    if (cov)
                        for (int b = 0; b < P; ++b) {
                            if (ma.col[b] < 0) continue;
                            double nb = u_to_nat(F::kind(b), s.u[b]);
                            cov[ma.col[a] * p + ma.col[b]] = sa * inv[a * P + b] * dnat_du(F::kind(b), nb);
                        }
                }
            } else {
                for (int a = 0; a < p; ++a) err[a] = NAN;
                if (cov)
                    for (int a = 0; a < p * p; ++a) cov[a] = NAN;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- model image / Jacobian
struct TileItem {
    int32_t gal, ty, tx, pad;
};

struct ImageArgs {
    const TileItem *tiles;
    int n_tiles;
    const double *params;
    float *out;          // model (mode 0) or Jacobian (mode 1)
    int mode;            // 2: adjoint, per-tile partials of J^T gin into part
    const float *gin;    // mode 2: weights of the pixels (image layout)
    double *part;        // mode 2: [n_tiles][P] partial sums (internal variable order)
};

template <class F, int KT, int NG>
__global__ __launch_bounds__(NT) void image_kernel(ModelArgs ma, BatchArgs ba, ImageArgs ia)
{
    extern __shared__ float4 dyn_lds[];
    float *planes = reinterpret_cast<float *>(dyn_lds);
    __shared__ EvalShared<F> esh;
    __shared__ double su[F::P];
    __shared__ double sdu[F::P];        // d u / d p (natural units)
    __shared__ int sfree[F::P];
    __shared__ double sv[NWAVE][F::P];
    constexpr int P = F::P;
    const int tid = threadIdx.x;
    for (int it = blockIdx.x; it < ia.n_tiles; it += gridDim.x) {
        const TileItem ti = ia.tiles[it];
        const int g = uniform(ti.gal);
        const Meta me = ba.meta[g];
        const int H = me.h, W = me.w, K = me.k;
        if (tid == 0) {
            const double *pp = ia.params + (int64_t)g * ma.p;
            for (int k = 0; k < P; ++k) {
                int c = ma.col[k];
                su[k] = nat_to_u(F::kind(k), c >= 0 ? pp[c] : ma.fixedv[k]);
                sdu[k] = 1.0 / dnat_du(F::kind(k), u_to_nat(F::kind(k), su[k]));
                sfree[k] = c >= 0;
            }
        }
        const float *psl = stage_psf<F, NG>(planes, ba.psf + uniform64(me.psf_off), K);
        __syncthreads();
        eval_prologue<F>(su, ma, H, W, esh, planes);
        const int ti0 = ti.ty * TILE, tj0 = ti.tx * TILE;
        int r, cg;
        strip_of(tid, K, r, cg);
        double acc0[4];
        float acc[F::NPL][4];
        tile_planes<F, KT, NG>(esh, planes, H, W, K, ti0, tj0, (const cfloat *)(ba.psf + uniform64(me.psf_off)), psl,
                               r, cg, acc0, acc);
        const int i = ti0 + r;
        double v[P];
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = 0.0;
        if (i < H) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int j = tj0 + 4 * cg + t;
                if (j >= W) continue;
                const int64_t pix = (int64_t)i * W + j;
                const double pdx = ((double)j + 0.5) - 0.5 * W, pdy = 0.5 * H - ((double)i + 0.5);
                const float fdx = (float)pdx, fdy = (float)pdy;
                if (ia.mode == 0) {
                    ia.out[me.img_off + pix] = (float)(acc0[t] + F::sky_at(esh.prep, pdx, pdy));
                } else if (ia.mode == 1) {
                    float *jo = ia.out + (int64_t)ma.p * me.img_off;
#pragma unroll
                    for (int k = 0; k < P; ++k) {
                        if (!sfree[k]) continue;
                        float jv = jac_at<F>(k, t, acc0, acc, fdx, fdy);
                        jo[(int64_t)ma.col[k] * H * W + pix] = jv * (float)sdu[k];
                    }
                } else {
                    const double gw = (double)ia.gin[me.img_off + pix];
#pragma unroll
                    for (int k = 0; k < P; ++k) v[k] += (double)jac_at<F>(k, t, acc0, acc, fdx, fdy) * gw;
                }
            }
        }
        if (ia.mode == 2) {
            // fixed-order reduction: wave butterflies, then the waves in order
            const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const double w = wave_sum(v[k]);
                if (lane == 0) sv[wave][k] = w;
            }
            __syncthreads();
            if (tid < P) {
                double sacc = sv[0][tid];
                for (int w = 1; w < NWAVE; ++w) sacc += sv[w][tid];
                ia.part[(int64_t)it * P + tid] = sacc * sdu[tid];
            }
        }
        __syncthreads();
    }
}

// Sum of the tile partials of each galaxy (tiles tstart[g] .. tstart[g+1]-1, in
// order) into its gradient row; fixed columns of the row are left at 0.
static __global__ void vjp_reduce_kernel(int n_gal, int P, ModelArgs ma, const int *tstart, const double *part,
                                  double *grad)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_gal) return;
    double *row = grad + (int64_t)g * ma.p;
    for (int c = 0; c < ma.p; ++c) row[c] = 0.0;
    for (int k = 0; k < P; ++k) {
        if (ma.col[k] < 0) continue;
        double s = 0.0;
        for (int t = tstart[g]; t < tstart[g + 1]; ++t) s += part[(int64_t)t * P + k];
        row[ma.col[k]] = s;
    }
}

// ---------------------------------------------------------------- default guess
struct GuessArgs {
    double *params, *moments;
    int n_gal;
};

__device__ inline double block_sum(double v, double *sred)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sred[wave] = v;
    __syncthreads();
    double s = sred[0];
    for (int w = 1; w < NWAVE; ++w) s += sred[w];
    return s;
}

// Image moments of one galaxy (all threads of the workgroup call this):
// sky0 = mean of the usable pixels in the 2-px frame; S = usable pixels with
// D - sky0 > 3 sigma; flux, flux-weighted centroid and central second moments
// over S; r0 = 1.1774 sqrt(lambda+), q0 = sqrt(lambda-/lambda+), theta0 =
// atan2(2 Mxy, Mxx - Myy) / 2, m_g = m0 - 2.5 log10 max(F0, 1e-3); fewer
// than 5 pixels in S: the cutout centre, r0 = 3, q0 = 1, theta0 = 0.
struct Moments {
    double sky0, f0, xc, yc, r0, q0, th0, mg, pk;
};

// Pixels per thread that a moments pass reads at once.
constexpr int kMomU = 4;

// This thread's pixels q0 + u NT (u < kMomU) of a cutout of npix pixels at
// off: data d, sigma s and ok = (pixel_weight != 0) (false past the cutout,
// whose reads take its last pixel), all reads issued before any value is
// used, the mask's in one uniform branch: one wait per batch.
__device__ inline void moment_pixels(const BatchArgs &ba, int64_t off, int q0, int npix, float (&d)[kMomU],
                                     float (&s)[kMomU], bool (&ok)[kMomU])
{
    int m[kMomU];
#pragma unroll
    for (int u = 0; u < kMomU; ++u) {
        const int64_t idx = off + min(q0 + u * NT, npix - 1);
        d[u] = ba.data[idx];
        s[u] = ba.sigma[idx];
        m[u] = 1;
    }
    if (ba.omega) {
#pragma unroll
        for (int u = 0; u < kMomU; ++u) m[u] = ba.omega[off + min(q0 + u * NT, npix - 1)];
    }
#pragma unroll
    for (int u = 0; u < kMomU; ++u) {
        const bool use = m[u] != 0 && s[u] > 0.0f && isfinite(s[u]) && isfinite(d[u]);
        ok[u] = q0 + u * NT < npix && (use ? 1.0f / (s[u] * s[u]) : 0.0f) != 0.0f;
    }
}

__device__ inline Moments image_moments(const BatchArgs &ba, const Meta &me, double m0, double *sred)
{
    const int tid = threadIdx.x;
    const int H = me.h, W = me.w;
    // row of pixel q by a float product: cutouts are at most 1024 x 1024, so (q + 0.5) / W is
    // below 1024 and at least 1 / (2 W) >= 2^-11 away from an integer, while the float
    // rounding of the product moves it by less than 2^-13
    const int npix = H * W;
    const float rW = 1.0f / (float)W;
    // each thread takes its pixels q = tid + k NT in increasing k, kMomU at a time
    double ss = 0.0, sc = 0.0;
    for (int q0 = tid; q0 < npix; q0 += kMomU * NT) {
        float d[kMomU], sg[kMomU];
        bool ok[kMomU];
        moment_pixels(ba, me.img_off, q0, npix, d, sg, ok);
#pragma unroll
        for (int u = 0; u < kMomU; ++u) {
            const int q = q0 + u * NT;
            const int i = (int)(((float)q + 0.5f) * rW), j = q - i * W;
            if (ok[u] && (i < 2 || i >= H - 2 || j < 2 || j >= W - 2)) {
                ss += d[u];
                sc += 1.0;
            }
        }
    }
    ss = block_sum(ss, sred);
    sc = block_sum(sc, sred);
    Moments mo;
    mo.sky0 = sc > 0.0 ? ss / sc : 0.0;
    double f0 = 0.0, fx = 0.0, fy = 0.0, cnt = 0.0, pk = 0.0;
    for (int q0 = tid; q0 < npix; q0 += kMomU * NT) {
        float d[kMomU], sg[kMomU];
        bool ok[kMomU];
        moment_pixels(ba, me.img_off, q0, npix, d, sg, ok);
#pragma unroll
        for (int u = 0; u < kMomU; ++u) {
            const double dp = (double)d[u] - mo.sky0;
            if (!ok[u] || !(dp > 3.0 * (double)sg[u])) continue;
            const int q = q0 + u * NT;
            const int i = (int)(((float)q + 0.5f) * rW), j = q - i * W;
            double x = j + 0.5, y = (double)H - i - 0.5;
            f0 += dp; fx += dp * x; fy += dp * y; cnt += 1.0;
            pk = fmax(pk, dp);
        }
    }
    f0 = block_sum(f0, sred);
    fx = block_sum(fx, sred);
    fy = block_sum(fy, sred);
    cnt = block_sum(cnt, sred);
    {   // block max of the peak
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) pk = fmax(pk, __shfl_xor(pk, o, 64));
        __syncthreads();
        if (lane == 0) sred[wave] = pk;
        __syncthreads();
        pk = sred[0];
        for (int w = 1; w < NWAVE; ++w) pk = fmax(pk, sred[w]);
    }
    mo.f0 = f0;
    mo.pk = pk > 0.0 ? pk : 1.0;
    mo.xc = 0.5 * W; mo.yc = 0.5 * H; mo.r0 = 3.0; mo.q0 = 1.0; mo.th0 = 0.0;
    const bool have = cnt >= 5.0 && f0 > 0.0;
    double mxx = 0.0, myy = 0.0, mxy = 0.0;
    if (have) {
        mo.xc = fx / f0;
        mo.yc = fy / f0;
        for (int q0 = tid; q0 < npix; q0 += kMomU * NT) {
            float d[kMomU], sg[kMomU];
            bool ok[kMomU];
            moment_pixels(ba, me.img_off, q0, npix, d, sg, ok);
#pragma unroll
            for (int u = 0; u < kMomU; ++u) {
                const double dp = (double)d[u] - mo.sky0;
                if (!ok[u] || !(dp > 3.0 * (double)sg[u])) continue;
                const int q = q0 + u * NT;
                const int i = (int)(((float)q + 0.5f) * rW), j = q - i * W;
                double dx = j + 0.5 - mo.xc, dy = (double)H - i - 0.5 - mo.yc;
                mxx += dp * dx * dx; myy += dp * dy * dy; mxy += dp * dx * dy;
            }
        }
    }
    mxx = block_sum(mxx, sred);
    myy = block_sum(myy, sred);
    mxy = block_sum(mxy, sred);
    if (have) {
        mxx /= f0; myy /= f0; mxy /= f0;
        double tr = 0.5 * (mxx + myy), dd = sqrt(0.25 * (mxx - myy) * (mxx - myy) + mxy * mxy);
        double lp = tr + dd, lm = fmax(tr - dd, 0.0);
        mo.q0 = lp > 0.0 ? sqrt(lm / lp) : 1.0;
        mo.q0 = fmin(fmax(mo.q0, 0.1), 1.0);
        mo.th0 = 0.5 * atan2(2.0 * mxy, mxx - myy);
        mo.r0 = 1.1774 * sqrt(fmax(lp, 0.0));
        mo.r0 = fmin(fmax(mo.r0, 1.0), 0.25 * W);
    }
    mo.mg = m0 - 2.5 * log10(fmax(f0, 1e-3));
    return mo;
}

// The default start of one galaxy from its image moments, written into its
// parameter row through the model's column map.
template <class F>
__device__ inline void moments_guess(const ModelArgs &ma, const Moments &mo, double *out)
{
    double pa0 = mo.th0 * 180.0 / kPi;
    if (pa0 < 0.0) pa0 += 180.0;
    double nat[F::P];
    const double ms = mo.mg + 2.5 * log10((double)(ma.nflux > 1 ? ma.nflux : 1));
    F::default_guess(mo.xc, mo.yc, ms, mo.r0, mo.q0, pa0, mo.sky0, mo.pk, nat);
    for (int k = 0; k < F::P; ++k)
        if (ma.col[k] >= 0) out[ma.col[k]] = nat[k];
}

template <class F>
__global__ __launch_bounds__(NT) void guess_kernel(ModelArgs ma, BatchArgs ba, GuessArgs ga)
{
    __shared__ double sred[NWAVE];
    const int tid = threadIdx.x;
    for (int g = blockIdx.x; g < ga.n_gal; g += gridDim.x) {
        const Meta me = ba.meta[g];
        const Moments mo = image_moments(ba, me, ma.m0, sred);
        if (tid == 0) {
            if (ga.moments) {
                double *m6 = ga.moments + (int64_t)g * 6;
                m6[0] = mo.xc - 0.5 * me.w; m6[1] = mo.yc - 0.5 * me.h; m6[2] = mo.mg;
                m6[3] = log(mo.r0); m6[4] = mo.q0; m6[5] = mo.th0;
            }
            moments_guess<F>(ma, mo, ga.params + (int64_t)g * ma.p);
        }
        __syncthreads();
    }
}

// The same start from moments a feature pass has already stored: mom8[g] =
// {sky0, F0, xc, yc, m_g, r0, q0, theta0} and the peak pk[g]; one thread per
// galaxy.
template <class F>
__global__ void guess_stored_kernel(ModelArgs ma, int n_gal, const double *mom8, const double *pk, double *params)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_gal) return;
    const double *o = mom8 + (int64_t)g * 8;
    Moments mo;
    mo.sky0 = o[0]; mo.f0 = o[1]; mo.xc = o[2]; mo.yc = o[3];
    mo.mg = o[4]; mo.r0 = o[5]; mo.q0 = o[6]; mo.th0 = o[7];
    mo.pk = pk[g];
    moments_guess<F>(ma, mo, params + (int64_t)g * ma.p);
}

static __global__ void fill_int_kernel(int *p, int v) { *p = v; }

static __global__ void fill_ints_kernel(int *p, int n, int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace gm
