// gm_mlp.hip -- the learned proposal of libgmfit.
//
// A small MLP maps a flux-normalised 32 x 32 image of a galaxy plus six image
// moments to the seven Sersic parameters an LM fit starts from; plain LM from
// the moment-based guess is both its fallback and the judge of its error.
// The paper motivates a learned start by the neural parameter estimators it
// reviews (Sec. 1) and by its own need to set initial parameters by hand
// (Sec. 7); the network, the features and the target encoding are this
// library's design (include/gmfit.h states them).
//
// Dense layers run as BF16 matrix-core GEMMs (v_mfma_f32_16x16x32_bf16) with
// FP32 accumulation and fused epilogues: bias + GELU (+ the FP32
// pre-activation kept for the backward pass), bias only, plain FP32 (weight
// gradients) and the GELU derivative of the backward pass.  One 256-thread
// workgroup computes a 64 x 64 output tile; each of its four waves owns a
// 32 x 32 quarter as 2 x 2 MFMA blocks; operands are staged through LDS in
// 32-deep K slices, both stored K-contiguous so that every lane fetches its
// eight BF16 operands with one 16-byte LDS read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "gm_launch.h"

using namespace gm;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// feature and target encoding (include/gmfit.h)
constexpr int kInDim = 1056, kNOut = 7, kCells = 32;
constexpr double kXScale = 32.0;
constexpr double kMagScale = 0.5, kLnReOff = 1.7, kLnReScale = 0.6, kLnNOff = 0.6, kLnNScale = 0.6;
constexpr double kEScale = 0.3, kECap = 0.9;

// ------------------------------------------------------------ BF16 -------
__device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                               // nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ inline float gelu_grad_f(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ------------------------------------------------------------ GEMM -------
constexpr int GT = 64;           // output tile side
constexpr int GK = 32;           // K slice
constexpr int LDK = GK + 8;      // LDS row pitch in BF16 elements (80 bytes)

enum { EPI_GELU = 0, EPI_BIAS = 1, EPI_F32 = 2, EPI_DGELU = 3 };

// C[m][n] = sum_k A(m, k) B(k, n).
//   A(m, k) = a[amap(m) * lda + k]  (AT = false)  or  a[amap(k) * lda + m]  (AT = true)
//   B(k, n) = b[n * ldb + k]        (BT = true)   or  b[bmap(k) * ldb + n]  (BT = false)
// amap / bmap: optional row gathers (null: identity).  The contiguous extent
// of each operand (K for a K-contiguous one, M or N otherwise) is a multiple
// of 8 and every row starts 16-byte aligned.
struct GemmArgs {
    int M, N, K;
    const uint16_t *a;
    int64_t lda;
    const int *amap;
    const uint16_t *b;
    int64_t ldb;
    const int *bmap;
    const float *bias;       // EPI_GELU, EPI_BIAS
    float *cf;               // FP32 output (EPI_GELU: pre-activation, nullable)
    int64_t ldcf;
    uint16_t *cb;            // BF16 output (EPI_GELU, EPI_DGELU)
    int64_t ldcb;
    const float *z;          // EPI_DGELU: pre-activation of the layer below
    int64_t ldz;
};

// Staging of one 64 x 32 (rows x K) operand slice into an LDS tile
// T[r][k] (pitch LDK), zero outside R x K, in three steps so that the global
// reads of the next slice can be issued before the matrix-core work on the
// current one: gather_piece (the row indices of an optional row map),
// read_piece (global -> registers), put (registers -> LDS).  A workgroup
// gathers for both operands before it reads either: the memory counter the
// reads wait on counts in order, so a gather issued after a data read would
// make that read a wait of its own.  Both are called with k0 < K (K: the end
// of the workgroup's K range) and R >= 1.
//
// K-contiguous operand X(r, k) = P[map(r) * ld + k]: each thread reads eight
// consecutive K values of one row (16 bytes) and stores them with one
// 16-byte LDS write.
struct KMajorPiece {
    u32x4 v;
    int64_t row;
};

__device__ inline void gather_kmajor(KMajorPiece &f, const int *map, int r0, int R, int, int)
{
    const int rr = r0 + (threadIdx.x >> 2);
    f.row = map ? (int64_t)map[min(rr, R - 1)] : (int64_t)rr;
}

__device__ inline void read_kmajor(KMajorPiece &f, const uint16_t *P, int64_t ld, int r0, int R, int k0, int K)
{
    const int t = threadIdx.x;
    const int rr = r0 + (t >> 2), k = k0 + (t & 3) * 8;
    f.v = u32x4{0u, 0u, 0u, 0u};
    if (rr < R && k < K) f.v = *reinterpret_cast<const u32x4 *>(P + f.row * ld + k);
}

__device__ inline void put_kmajor(uint16_t *T, const KMajorPiece &f)
{
    const int t = threadIdx.x;
    *reinterpret_cast<u32x4 *>(T + (t >> 2) * LDK + (t & 3) * 8) = f.v;
}

// R-contiguous operand X(r, k) = P[map(k) * ld + r]: each thread reads an
// adjacent pair of rows (4 bytes) in four consecutive K rows and writes the
// transposed values, four K values per row, as two 8-byte LDS stores (R is a
// multiple of 8, so a pair is either inside R or outside it).
struct RMajorPiece {
    uint32_t v[4];
    int64_t row[4];
};

__device__ inline void gather_rmajor(RMajorPiece &f, const int *map, int, int, int k0, int K)
{
    const int kq = 4 * (threadIdx.x >> 5);
    // one branch on the map for the four indices, each clamped to K - 1
    // rather than guarded (a guarded read ends in a wait)
#pragma unroll
    for (int e = 0; e < 4; ++e) f.row[e] = k0 + kq + e;
    if (map) {
#pragma unroll
        for (int e = 0; e < 4; ++e) f.row[e] = map[min(k0 + kq + e, K - 1)];
    }
}

__device__ inline void read_rmajor(RMajorPiece &f, const uint16_t *P, int64_t ld, int r0, int R, int k0, int K)
{
    const int t = threadIdx.x;
    const int rr = r0 + 2 * (t & 31), kq = 4 * (t >> 5);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        f.v[e] = 0u;
        if (k0 + kq + e < K && rr < R) f.v[e] = *reinterpret_cast<const uint32_t *>(P + f.row[e] * ld + rr);
    }
}

__device__ inline void put_rmajor(uint16_t *T, const RMajorPiece &f)
{
    const int t = threadIdx.x;
    const int rp = 2 * (t & 31), kq = 4 * (t >> 5);
    // row rp: the low halves of the four words; row rp + 1: the high halves
    const u32x2 lo = {(f.v[0] & 0xffffu) | (f.v[1] << 16), (f.v[2] & 0xffffu) | (f.v[3] << 16)};
    const u32x2 hi = {(f.v[0] >> 16) | (f.v[1] & 0xffff0000u), (f.v[2] >> 16) | (f.v[3] & 0xffff0000u)};
    *reinterpret_cast<u32x2 *>(T + rp * LDK + kq) = lo;
    *reinterpret_cast<u32x2 *>(T + (rp + 1) * LDK + kq) = hi;
}

template <bool RMAJOR>
struct PieceOf {
    typedef KMajorPiece type;
};
template <>
struct PieceOf<true> {
    typedef RMajorPiece type;
};

template <bool RMAJOR>
__device__ inline void gather_piece(typename PieceOf<RMAJOR>::type &f, const int *map, int r0, int R, int k0, int K)
{
    if constexpr (RMAJOR)
        gather_rmajor(f, map, r0, R, k0, K);
    else
        gather_kmajor(f, map, r0, R, k0, K);
}

template <bool RMAJOR>
__device__ inline void read_piece(typename PieceOf<RMAJOR>::type &f, const uint16_t *P, int64_t ld, int r0, int R,
                                  int k0, int K)
{
    if constexpr (RMAJOR)
        read_rmajor(f, P, ld, r0, R, k0, K);
    else
        read_kmajor(f, P, ld, r0, R, k0, K);
}

template <bool RMAJOR>
__device__ inline void put(uint16_t *T, const typename PieceOf<RMAJOR>::type &f)
{
    if constexpr (RMAJOR)
        put_rmajor(T, f);
    else
        put_kmajor(T, f);
}

// C = A B over the K range [kbeg, kend) of this workgroup's split (blockIdx.z
// of gridDim.z splits, each a whole number of K slices): the splits of an
// EPI_F32 product write their partial sums to cf + z * M * ldcf, which
// reduce_splits_kernel adds in split order.
template <bool AT, bool BT, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[GT * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[GT * LDK];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = 8 * (lane >> 4);
    const int nsl = (g.K + GK - 1) / GK, per = (nsl + gridDim.z - 1) / gridDim.z;
    const int kbeg = blockIdx.z * per * GK, kend = min(g.K, kbeg + per * GK);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    typename PieceOf<AT>::type fa;
    typename PieceOf<!BT>::type fb;
    const int *bmap = BT ? nullptr : g.bmap;
    if (kbeg < kend) {
        gather_piece<AT>(fa, g.amap, m0, g.M, kbeg, kend);
        gather_piece<!BT>(fb, bmap, n0, g.N, kbeg, kend);
        read_piece<AT>(fa, g.a, g.lda, m0, g.M, kbeg, kend);
        read_piece<!BT>(fb, g.b, g.ldb, n0, g.N, kbeg, kend);
    }
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        put<AT>(As, fa);
        put<!BT>(Bs, fb);
        __syncthreads();
        if (k0 + GK < kend) {       // the next slice's global reads overlap this slice's products
            gather_piece<AT>(fa, g.amap, m0, g.M, k0 + GK, kend);
            gather_piece<!BT>(fb, bmap, n0, g.N, k0 + GK, kend);
            read_piece<AT>(fa, g.a, g.lda, m0, g.M, k0 + GK, kend);
            read_piece<!BT>(fb, g.b, g.ldb, n0, g.N, k0 + GK, kend);
        }
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            af[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(&As[(wm + 16 * i + lr) * LDK + lk]));
#pragma unroll
        for (int j = 0; j < 2; ++j)
            bfr[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(&Bs[(wn + 16 * j + lr) * LDK + lk]));
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    float *cf = g.cf;
    if (EPI == EPI_F32) cf += (int64_t)blockIdx.z * g.M * g.ldcf;
    // lane holds C[4 (lane / 16) + r][lane % 16] of each 16 x 16 block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + lr;
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[i][j][r];
                if (EPI == EPI_GELU) {
                    const float zz = v + g.bias[n];
                    if (cf) cf[(int64_t)m * g.ldcf + n] = zz;
                    g.cb[(int64_t)m * g.ldcb + n] = f2bf(gelu_f(zz));
                } else if (EPI == EPI_BIAS) {
                    cf[(int64_t)m * g.ldcf + n] = v + g.bias[n];
                } else if (EPI == EPI_F32) {
                    cf[(int64_t)m * g.ldcf + n] = v;
                } else {
                    g.cb[(int64_t)m * g.ldcb + n] = f2bf(v * gelu_grad_f(g.z[(int64_t)m * g.ldz + n]));
                }
            }
}

// out[m][n] = sum over the splits z = 0 .. S-1, in that order, of
// part[z][m][n] (pitch N).
__global__ __launch_bounds__(256) void reduce_splits_kernel(int M, int N, int S, const float *part, float *out,
                                                            int64_t ldo)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * N) return;
    const int m = (int)(e / N), n = (int)(e - (int64_t)m * N);
    float s = 0.0f;
    for (int z = 0; z < S; ++z) s += part[(int64_t)z * M * N + e];
    out[(int64_t)m * ldo + n] = s;
}

// ------------------------------------------------ loss, grads, AdamW ----
// dO[m][j] = bf16(2 (out - t) / (n n_out)) for j < n_out, else 0; per-block
// FP64 partial sums of the squared error (fixed order).
__global__ __launch_bounds__(256) void mse_kernel(int n, int out_dim, int n_out, const float *out,
                                                  const float *tgt, const int *rows, uint16_t *dout, double *part)
{
    __shared__ double sred[NWAVE];
    const int rows_per_block = 256 / 16;
    const int m = blockIdx.x * rows_per_block + (threadIdx.x >> 4);
    const int j = threadIdx.x & 15;
    const float inv = 2.0f / ((float)n * (float)n_out);
    double e2 = 0.0;
    if (m < n) {
        const int64_t tr = rows ? (int64_t)rows[m] : (int64_t)m;
        for (int jj = j; jj < out_dim; jj += 16) {
            float d = 0.0f;
            if (jj < n_out) {
                d = out[(int64_t)m * out_dim + jj] - tgt[tr * out_dim + jj];
                e2 += (double)d * (double)d;
            }
            dout[(int64_t)m * out_dim + jj] = f2bf(d * inv);
        }
    }
    e2 = block_sum(e2, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = e2;
}

__global__ void loss_final_kernel(int nparts, const double *part, double scale, double *loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += part[i];
    *loss = s * scale;
}

// Column sums of a BF16 [M][N] matrix in two fixed-order passes: partial sums
// over row slices (blockIdx.y, wave), then their sum.
constexpr int kColSlices = 16;

__global__ __launch_bounds__(256) void colsum_part_kernel(int M, int N, const uint16_t *x, int64_t ldx, float *part)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + lane;
    const int nslice = kColSlices * NWAVE, slice = blockIdx.y * NWAVE + wave;
    const int per = (M + nslice - 1) / nslice;
    const int r0 = slice * per, r1 = min(M, r0 + per);
    if (n >= N) return;
    float s = 0.0f;
    for (int m = r0; m < r1; ++m) s += bf2f(x[(int64_t)m * ldx + n]);
    part[(int64_t)slice * N + n] = s;
}

__global__ void colsum_final_kernel(int N, const float *part, float *out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int i = 0; i < kColSlices * NWAVE; ++i) s += part[(int64_t)i * N + n];
    out[n] = s;
}

// Decoupled weight decay Adam (Loshchilov and Hutter), then the BF16 copy.
__global__ void adamw_kernel(int64_t count, float *p, uint16_t *pb, const float *grad, float *m, float *v, float lr,
                             float b1, float b2, float eps, float wd, float bc1, float bc2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = grad[i];
        float pi = p[i] * (1.0f - lr * wd);
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        pi -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
        m[i] = mi;
        v[i] = vi;
        p[i] = pi;
        pb[i] = f2bf(pi);
    }
}

__global__ void sync_bf16_kernel(int64_t count, const float *p, uint16_t *pb)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        pb[i] = f2bf(p[i]);
}

// ------------------------------------------------------- features -------
// mom8[g] = {sky0, F0, xc, yc, m_g, r0, q0, theta0}, pk[g] = the peak (both nullable)
__global__ __launch_bounds__(NT) void features_kernel(BatchArgs ba, double m0, int n_gal, uint16_t *x, int64_t ldx,
                                                      double *mom8, double *pk)
{
    __shared__ double sred[NWAVE];
    for (int g = blockIdx.x; g < n_gal; g += gridDim.x) {
        const Meta me = ba.meta[g];
        const Moments mo = image_moments(ba, me, m0, sred);
        const int H = me.h, W = me.w;
        const double f0 = fmax(mo.f0, 1.0);
        const double area = (double)H * W / (double)(kCells * kCells);
        uint16_t *xg = x + (int64_t)g * ldx;
        for (int c = threadIdx.x; c < kCells * kCells; c += NT) {
            const int a = c / kCells, b = c % kCells;
            const double rlo = a * (double)H / kCells, rhi = (a + 1) * (double)H / kCells;
            const double clo = b * (double)W / kCells, chi = (b + 1) * (double)W / kCells;
            const int i0 = (int)floor(rlo), i1 = min(H - 1, (int)ceil(rhi) - 1);
            const int j0 = (int)floor(clo), j1 = min(W - 1, (int)ceil(chi) - 1);
            double num = 0.0, den = 0.0;
            for (int i = i0; i <= i1; ++i) {
                const double orow = fmin(i + 1.0, rhi) - fmax((double)i, rlo);
                if (!(orow > 0.0)) continue;
                for (int j = j0; j <= j1; ++j) {
                    const double ocol = fmin(j + 1.0, chi) - fmax((double)j, clo);
                    if (!(ocol > 0.0)) continue;
                    float d;
                    if (pixel_weight(ba, me.img_off + (int64_t)i * W + j, d) == 0.0f) continue;
                    const double wgt = orow * ocol;
                    num += wgt * ((double)d - mo.sky0);
                    den += wgt;
                }
            }
            const double v = den > 0.0 ? num / den * area : 0.0;
            xg[c] = f2bf((float)(kXScale * v / f0));
        }
        const int t = threadIdx.x;
        if (t < kInDim - kCells * kCells && kCells * kCells + t < ldx) {
            const double e0 = (1.0 - mo.q0) / (1.0 + mo.q0);
            double f = 0.0;
            switch (t) {
            case 0: f = (mo.xc - 0.5 * W) / 2.0; break;
            case 1: f = (mo.yc - 0.5 * H) / 2.0; break;
            case 2: f = (mo.mg - 14.0) / 2.0; break;
            case 3: f = log(mo.r0) - 1.5; break;
            case 4: f = e0 * cos(2.0 * mo.th0); break;
            case 5: f = e0 * sin(2.0 * mo.th0); break;
            default: break;
            }
            xg[kCells * kCells + t] = f2bf((float)f);
        }
        if (t == 0 && mom8) {
            double *o = mom8 + (int64_t)g * 8;
            o[0] = mo.sky0; o[1] = mo.f0; o[2] = mo.xc; o[3] = mo.yc;
            o[4] = mo.mg; o[5] = mo.r0; o[6] = mo.q0; o[7] = mo.th0;
        }
        if (t == 0 && pk) pk[g] = mo.pk;
        __syncthreads();
    }
}

// ------------------------------------------------ targets / decoding ----
// Sersic slots in the family's internal order: x0 y0 mag re n q pa, sky at 7.
__global__ void targets_kernel(int n_gal, ModelArgs ma, const double *truth, const double *mom8, float *tgt,
                               int out_dim)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_gal) return;
    const double *tp = truth + (int64_t)g * ma.p;
    double v[7];
    for (int k = 0; k < 7; ++k) v[k] = ma.col[k] >= 0 ? tp[ma.col[k]] : ma.fixedv[k];
    double q = v[5], re = v[3], pa = v[6];
    if (q > 1.0) {                       // the same ellipse with q <= 1
        re *= q;
        q = 1.0 / q;
        pa += 90.0;
    }
    const double *mo = mom8 + (int64_t)g * 8;
    const double e = (1.0 - q) / (1.0 + q), th = pa * (kPi / 180.0);
    float *t = tgt + (int64_t)g * out_dim;
    t[0] = (float)(v[0] - mo[2]);
    t[1] = (float)(v[1] - mo[3]);
    t[2] = (float)((v[2] - mo[4]) / kMagScale);
    t[3] = (float)((log(re) - kLnReOff) / kLnReScale);
    t[4] = (float)((log(v[4]) - kLnNOff) / kLnNScale);
    t[5] = (float)(e * cos(2.0 * th) / kEScale);
    t[6] = (float)(e * sin(2.0 * th) / kEScale);
    for (int k = kNOut; k < out_dim; ++k) t[k] = 0.0f;
}

__global__ void decode_kernel(int n_gal, ModelArgs ma, const Meta *meta, const float *out, int out_dim,
                              const double *mom8, double *params, int *valid)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_gal) return;
    const float *o = out + (int64_t)g * out_dim;
    const double *mo = mom8 + (int64_t)g * 8;
    const int H = meta[g].h, W = meta[g].w;
    double v[8];
    v[0] = mo[2] + (double)o[0];
    v[1] = mo[3] + (double)o[1];
    v[2] = mo[4] + kMagScale * (double)o[2];
    v[3] = exp(kLnReOff + kLnReScale * (double)o[3]);
    v[4] = exp(kLnNOff + kLnNScale * (double)o[4]);
    const double e1 = kEScale * (double)o[5], e2 = kEScale * (double)o[6];
    const double e = fmin(hypot(e1, e2), kECap);
    v[5] = (1.0 - e) / (1.0 + e);
    double pa = 0.5 * atan2(e2, e1) * (180.0 / kPi);
    if (pa < 0.0) pa += 180.0;
    if (pa >= 180.0) pa -= 180.0;
    v[6] = pa;
    v[7] = mo[0];
    bool ok = true;
    for (int k = 0; k < 8; ++k) ok = ok && isfinite(v[k]);
    const double big = 2.0 * max(H, W);
    ok = ok && v[0] >= 0.0 && v[0] <= W && v[1] >= 0.0 && v[1] <= H && v[3] >= 0.1 && v[3] <= big && v[4] >= 0.2 &&
         v[4] <= 10.0;
    double *pp = params + (int64_t)g * ma.p;
    for (int k = 0; k < 8; ++k)
        if (ma.col[k] >= 0) pp[ma.col[k]] = v[k];
    valid[g] = ok ? 1 : 0;
}

// ------------------------------------------------ synthetic noise -------
// Box-Muller on two 32-bit words: u1 in (0, 1], u2 in [0, 1).
__device__ inline void box_muller(uint32_t a, uint32_t b, double &z0, double &z1)
{
    const double u1 = ((double)a + 1.0) * 2.3283064365386963e-10;
    const double u2 = (double)b * 2.3283064365386963e-10;
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincos(2.0 * kPi * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// D = F U + sky + sigma z with F = snr sigma / max(U) (the peak SNR of the
// noiseless galaxy), z standard normal from Philox keyed by the seed with
// counter {pixel quad, galaxy index (64 bit), 0}.  mag[g * stride] = m0 - 2.5 log10 F.
__global__ __launch_bounds__(NT) void synth_kernel(const Meta *meta, int n_gal, const float *unit, const double *snr,
                                                   const double *sky, float sigma, double m0, uint32_t k0,
                                                   uint32_t k1, int64_t first, float *data, float *sig, double *mag,
                                                   int mag_stride)
{
    __shared__ float smax[NWAVE];
    for (int g = blockIdx.x; g < n_gal; g += gridDim.x) {
        const Meta me = meta[g];
        const int64_t npix = (int64_t)me.h * me.w;
        const float *u = unit + me.img_off;
        float pk = -INFINITY;
        for (int64_t i = threadIdx.x; i < npix; i += NT) pk = fmaxf(pk, u[i]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) pk = fmaxf(pk, __shfl_xor(pk, o, 64));
        __syncthreads();
        if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = pk;
        __syncthreads();
        pk = smax[0];
        for (int w = 1; w < NWAVE; ++w) pk = fmaxf(pk, smax[w]);
        const double F = snr[g] * (double)sigma / (double)pk;
        const double sk = sky[g];
        if (threadIdx.x == 0 && mag) mag[(int64_t)g * mag_stride] = m0 - 2.5 * log10(F);
        const uint64_t gi = (uint64_t)(first + g);
        for (int64_t qd = threadIdx.x; qd < (npix + 3) / 4; qd += NT) {
            const U4 r = philox4x32_10(U4{(uint32_t)qd, (uint32_t)gi, (uint32_t)(gi >> 32), 0u}, k0, k1);
            double z[4];
            box_muller(r.x, r.y, z[0], z[1]);
            box_muller(r.z, r.w, z[2], z[3]);
            for (int e = 0; e < 4; ++e) {
                const int64_t i = 4 * qd + e;
                if (i >= npix) break;
                data[me.img_off + i] = (float)(F * (double)u[i] + sk + (double)sigma * z[e]);
                if (sig) sig[me.img_off + i] = sigma;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- host side -------
int ensure_ws(gm_ctx *c, size_t bytes)
{
    if (c->mlp_ws_bytes >= bytes) return GM_OK;
    if (c->mlp_ws) {
        if (hipDeviceSynchronize() != hipSuccess) return GM_EHIP;
        (void)hipFree(c->mlp_ws);
        c->mlp_ws = nullptr;
        c->mlp_ws_bytes = 0;
    }
    size_t nb = std::max(bytes, (size_t)1 << 22);
    if (hipMalloc(&c->mlp_ws, nb) != hipSuccess) return GM_ENOMEM;
    c->mlp_ws_bytes = nb;
    return GM_OK;
}

// bump allocator over the workspace (256-byte aligned pieces)
struct Carve {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        T *p = reinterpret_cast<T *>(base + off);
        off += (count * sizeof(T) + 255) & ~(size_t)255;
        return p;
    }
};

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

int n_layers(const gm_mlp *m) { return m->n_hidden + 1; }

int layer_in(const gm_mlp *m, int l) { return l == 0 ? m->in_dim : m->hidden; }
int layer_out(const gm_mlp *m, int l) { return l == n_layers(m) - 1 ? m->out_dim : m->hidden; }

// offsets of W_l and b_l in the flat parameter vector
int64_t w_off(const gm_mlp *m, int l)
{
    int64_t off = 0;
    for (int i = 0; i < l; ++i) off += (int64_t)layer_out(m, i) * layer_in(m, i) + layer_out(m, i);
    return off;
}
int64_t b_off(const gm_mlp *m, int l) { return w_off(m, l) + (int64_t)layer_out(m, l) * layer_in(m, l); }

int64_t count_params(const gm_mlp *m) { return w_off(m, n_layers(m)); }

int check_mlp(const gm_mlp *m, bool train)
{
    if (!m || m->in_dim < 8 || m->hidden < 8 || m->n_hidden < 1 || m->n_hidden > 16 || m->out_dim < 8 ||
        m->n_out < 1 || m->n_out > m->out_dim)
        return GM_EINVAL;
    if (m->in_dim % 8 || m->hidden % 8 || m->out_dim % 8) return GM_EINVAL;
    if (m->in_dim > 65536 || m->hidden > 65536 || m->out_dim > 65536) return GM_EINVAL;
    if (!m->params || !m->params_bf16 || !aligned16(m->params_bf16)) return GM_EINVAL;
    if (train && (!m->grad || !m->adam_m || !m->adam_v)) return GM_EINVAL;
    return GM_OK;
}

int launch_gemm_rc() { return hipGetLastError() == hipSuccess ? GM_OK : GM_EHIP; }

template <bool AT, bool BT, int EPI>
int gemm(const GemmArgs &g, hipStream_t st)
{
    if (g.M <= 0 || g.N <= 0) return GM_OK;
    dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT, 1);
    hipLaunchKernelGGL((gemm_kernel<AT, BT, EPI>), grid, dim3(256), 0, st, g);
    return launch_gemm_rc();
}

// K splits of a weight-gradient product (C = A^T B over a long K, the
// mini-batch): enough workgroups to fill the chip (the output has only
// (M / 64) (N / 64) tiles: 136 for the first layer, 64 for the hidden ones)
// while each split keeps at least 256 of K.
int dw_splits(int M, int N, int K)
{
    const int tiles = ((M + GT - 1) / GT) * ((N + GT - 1) / GT);
    int s = 1;
    while (s < 16 && tiles * s < 1024 && (K + 2 * s - 1) / (2 * s) >= 256) s *= 2;
    return s;
}

size_t dw_part_floats(int M, int N, int K)
{
    const int s = dw_splits(M, N, K);
    return s > 1 ? (size_t)s * M * N : 0;
}

// C (FP32, pitch ldcf) = A^T B with A(m, k) = a[k * lda + m] and B(k, n) =
// b[bmap(k) * ldb + n]: the weight gradients.  With more than one split the
// splits write partial sums to `part` (dw_part_floats(M, N, K) floats) and a
// second kernel adds them in split order, so the result does not depend on
// timing.
int gemm_dw(GemmArgs g, float *part, hipStream_t st)
{
    if (g.M <= 0 || g.N <= 0) return GM_OK;
    const int s = dw_splits(g.M, g.N, g.K);
    if (s == 1) return gemm<true, false, EPI_F32>(g, st);
    float *out = g.cf;
    const int64_t ldo = g.ldcf;
    g.cf = part;
    g.ldcf = g.N;
    dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT, s);
    hipLaunchKernelGGL((gemm_kernel<true, false, EPI_F32>), grid, dim3(256), 0, st, g);
    if (hipGetLastError() != hipSuccess) return GM_EHIP;
    const int64_t cnt = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(reduce_splits_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, g.M, g.N, s,
                       part, out, ldo);
    return launch_gemm_rc();
}

// Forward pass of n rows of x (BF16, row pitch ldx, optional row gather).
// Y[l] receives the BF16 output of hidden layer l and Z[l] (nullable) its
// FP32 pre-activation; out [n][out_dim] FP32.
int forward_pass(const gm_mlp *m, int n, const uint16_t *x, int64_t ldx, const int *rows, uint16_t *const *Y,
                 float *const *Z, float *out, hipStream_t st)
{
    const int L = n_layers(m);
    const uint16_t *wb = m->params_bf16;
    for (int l = 0; l < L; ++l) {
        GemmArgs g{};
        g.M = n;
        g.N = layer_out(m, l);
        g.K = layer_in(m, l);
        g.a = l == 0 ? x : Y[l - 1];
        g.lda = l == 0 ? ldx : m->hidden;
        g.amap = l == 0 ? rows : nullptr;
        g.b = wb + w_off(m, l);
        g.ldb = layer_in(m, l);
        g.bias = m->params + b_off(m, l);
        int rc;
        if (l < L - 1) {
            g.cf = Z ? Z[l] : nullptr;
            g.ldcf = m->hidden;
            g.cb = Y[l];
            g.ldcb = m->hidden;
            rc = gemm<false, true, EPI_GELU>(g, st);
        } else {
            g.cf = out;
            g.ldcf = m->out_dim;
            rc = gemm<false, true, EPI_BIAS>(g, st);
        }
        if (rc) return rc;
    }
    return GM_OK;
}

size_t train_ws_bytes(const gm_mlp *m, int n)
{
    const int L = n_layers(m);
    size_t b = 0;
    auto add = [&](size_t bytes) { b += (bytes + 255) & ~(size_t)255; };
    for (int l = 0; l < L - 1; ++l) {
        add((size_t)n * m->hidden * 2);     // Y
        add((size_t)n * m->hidden * 4);     // Z
    }
    add((size_t)n * m->out_dim * 4);        // out
    add((size_t)n * m->out_dim * 2);        // dO
    add((size_t)n * m->hidden * 2 * 2);     // dZ ping-pong
    add((size_t)kColSlices * NWAVE * std::max(m->hidden, m->out_dim) * 4);
    add((size_t)((n + 15) / 16) * 8);       // loss partials
    size_t part = 0;                        // K-split partial sums of the weight gradients
    for (int l = 0; l < L; ++l) part = std::max(part, dw_part_floats(layer_out(m, l), layer_in(m, l), n));
    add(part * 4);
    return b + 256;
}

int backward_pass(gm_ctx *c, const gm_mlp *m, int n, const uint16_t *x, int64_t ldx, const int *rows,
                  const float *targets, double *loss_out, hipStream_t st)
{
    const int L = n_layers(m);
    int rc = ensure_ws(c, train_ws_bytes(m, n));
    if (rc) return rc;
    Carve cv{reinterpret_cast<char *>(c->mlp_ws)};
    uint16_t *Y[17];
    float *Z[17];
    for (int l = 0; l < L - 1; ++l) {
        Y[l] = cv.take<uint16_t>((size_t)n * m->hidden);
        Z[l] = cv.take<float>((size_t)n * m->hidden);
    }
    float *out = cv.take<float>((size_t)n * m->out_dim);
    uint16_t *dout = cv.take<uint16_t>((size_t)n * m->out_dim);
    uint16_t *dz[2] = {cv.take<uint16_t>((size_t)2 * n * m->hidden), nullptr};
    dz[1] = dz[0] + (size_t)n * m->hidden;
    float *cpart = cv.take<float>((size_t)kColSlices * NWAVE * std::max(m->hidden, m->out_dim));
    const int nblk = (n + 15) / 16;
    double *lpart = cv.take<double>((size_t)nblk);
    size_t npart = 0;
    for (int l = 0; l < L; ++l) npart = std::max(npart, dw_part_floats(layer_out(m, l), layer_in(m, l), n));
    float *dwpart = cv.take<float>(npart);
    rc = forward_pass(m, n, x, ldx, rows, Y, Z, out, st);
    if (rc) return rc;
    hipLaunchKernelGGL(mse_kernel, dim3(nblk), dim3(256), 0, st, n, m->out_dim, m->n_out, out, targets, rows, dout,
                       lpart);
    if (hipGetLastError() != hipSuccess) return GM_EHIP;
    if (loss_out) {
        hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, st, nblk, lpart,
                           1.0 / ((double)n * m->n_out), loss_out);
        if (hipGetLastError() != hipSuccess) return GM_EHIP;
    }
    const uint16_t *dcur = dout;
    int64_t ldd = m->out_dim;
    for (int l = L - 1; l >= 0; --l) {
        const int nin = layer_in(m, l), nout = layer_out(m, l);
        // dW_l[o][i] = sum_m dZ_l[m][o] X_l[m][i]
        GemmArgs g{};
        g.M = nout;
        g.N = nin;
        g.K = n;
        g.a = dcur;
        g.lda = ldd;
        g.b = l == 0 ? x : Y[l - 1];
        g.ldb = l == 0 ? ldx : m->hidden;
        g.bmap = l == 0 ? rows : nullptr;
        g.cf = m->grad + w_off(m, l);
        g.ldcf = nin;
        rc = gemm_dw(g, dwpart, st);
        if (rc) return rc;
        hipLaunchKernelGGL(colsum_part_kernel, dim3((nout + 63) / 64, kColSlices), dim3(256), 0, st, n, nout, dcur,
                           ldd, cpart);
        hipLaunchKernelGGL(colsum_final_kernel, dim3((nout + 255) / 256), dim3(256), 0, st, nout, cpart,
                           m->grad + b_off(m, l));
        if (hipGetLastError() != hipSuccess) return GM_EHIP;
        if (l > 0) {
            // dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1})
            GemmArgs d{};
            d.M = n;
            d.N = nin;
            d.K = nout;
            d.a = dcur;
            d.lda = ldd;
            d.b = m->params_bf16 + w_off(m, l);
            d.ldb = nin;
            uint16_t *dnext = dz[l & 1];
            d.cb = dnext;
            d.ldcb = m->hidden;
            d.z = Z[l - 1];
            d.ldz = m->hidden;
            rc = gemm<false, false, EPI_DGELU>(d, st);
            if (rc) return rc;
            dcur = dnext;
            ldd = m->hidden;
        }
    }
    return GM_OK;
}

int adamw_step(const gm_mlp *m, int64_t step, const gm_adamw *o, hipStream_t st)
{
    if (!o || step < 1 || !(o->lr >= 0.0) || !(o->beta1 >= 0.0 && o->beta1 < 1.0) ||
        !(o->beta2 >= 0.0 && o->beta2 < 1.0) || !(o->eps > 0.0) || !(o->weight_decay >= 0.0))
        return GM_EINVAL;
    const double bc1 = 1.0 - std::pow(o->beta1, (double)step), bc2 = 1.0 - std::pow(o->beta2, (double)step);
    const int64_t cnt = count_params(m);
    hipLaunchKernelGGL(adamw_kernel, dim3(1024), dim3(256), 0, st, cnt, m->params, m->params_bf16, m->grad, m->adam_m,
                       m->adam_v, (float)o->lr, (float)o->beta1, (float)o->beta2, (float)o->eps,
                       (float)o->weight_decay, (float)bc1, (float)bc2);
    return hipGetLastError() == hipSuccess ? GM_OK : GM_EHIP;
}

// A single Sersic component plus sky with every slot a column: the model the
// proposal encodes.
int check_proposal_model(const Match &mt)
{
    if (mt.single_type != GM_SERSIC || !mt.has_sky || mt.tilt || mt.box) return GM_EUNSUPPORTED;
    for (int k = 0; k < 8; ++k)
        if (mt.ci.ma.col[k] < 0) return GM_EUNSUPPORTED;
    return GM_OK;
}

int check_proposal_mlp(const gm_mlp *m)
{
    if (m->in_dim != kInDim || m->n_out != kNOut) return GM_EINVAL;
    return GM_OK;
}

// meta for a batch (host sizes -> device), through the shared staging path
int stage_meta(gm_ctx *c, const Match &mt, hipStream_t st, Staged *sg) { return stage(c, mt.ci, nullptr, 0, st, sg); }

int features_launch(gm_ctx *c, const Match &mt, uint16_t *x, int64_t ldx, double *mom8, double *pk,
                    hipStream_t st)
{
    Staged sg;
    int rc = stage_meta(c, mt, st, &sg);
    if (rc) return rc;
    const gm_batch *b = mt.ci.b;
    BatchArgs ba{sg.meta, b->data, b->sigma, nullptr, b->omega};
    const int grid = std::min(b->n_gal, std::max(c->num_cu, 1) * 8);
    hipLaunchKernelGGL(features_kernel, dim3(grid), dim3(NT), 0, st, ba, mt.ci.ma.m0, b->n_gal, x, ldx, mom8, pk);
    return hipGetLastError() == hipSuccess ? GM_OK : GM_EHIP;
}

int decode_launch(gm_ctx *c, const Match &mt, const float *out, int out_dim, const double *mom8, double *params,
                  int *valid, hipStream_t st)
{
    Staged sg;
    int rc = stage_meta(c, mt, st, &sg);
    if (rc) return rc;
    const int n = mt.ci.b->n_gal;
    hipLaunchKernelGGL(decode_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, mt.ci.ma, sg.meta, out, out_dim,
                       mom8, params, valid);
    return hipGetLastError() == hipSuccess ? GM_OK : GM_EHIP;
}


int learned_checks(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_mlp *mlp,
                   const gm_fit_opts *opts, Match &mt)
{
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if ((rc = check_proposal_model(mt))) return rc;
    if ((rc = check_mlp(mlp, false))) return rc;
    if ((rc = check_proposal_mlp(mlp))) return rc;
    if (opts && (opts->max_iter < 0 || !(opts->lambda0 > 0.0) || !(opts->step_tol > 0.0) ||
                 opts->proposal_max_iter < 0))
        return GM_EINVAL;
    return GM_OK;
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t learned_ws_bytes(const gm_mlp *mlp, int n, int p)
{
    return al256((size_t)n * kInDim * 2) + al256((size_t)n * 8 * 8) + al256((size_t)n * mlp->out_dim * 4) +
           2 * al256((size_t)n * mlp->hidden * 2) + al256((size_t)n * p * 8) + al256((size_t)n * 4) +
           al256((size_t)n * 8) + 256;
}

// The learned-start fit on the context's MLP workspace (already sized by
// learned_ws_bytes): features and image moments, the moment guess from them,
// network, decoding, then one LM launch from the valid proposals in which
// every galaxy whose proposal is invalid or whose fit from it does not
// converge within the trial budget is refitted from the moment guess by the
// same workgroup.  events (nullable): before the features, before and after
// the LM launch, at the end.
int learned_seq(gm_ctx *ctx, const Match &mt, const Variant *var, const gm_mlp *mlp, const gm_fit_opts *opts,
                double *params_out, double *chi2_out, int32_t *niter_out, int32_t *status_out, int32_t *fallback_out,
                void *const *events, hipStream_t st)
{
    const int n = mt.ci.b->n_gal, p = mt.ci.ma.p;
    Carve cv{reinterpret_cast<char *>(ctx->mlp_ws)};
    uint16_t *x = cv.take<uint16_t>((size_t)n * kInDim);
    double *mom8 = cv.take<double>((size_t)n * 8);
    float *out = cv.take<float>((size_t)n * mlp->out_dim);
    uint16_t *act0 = cv.take<uint16_t>((size_t)n * mlp->hidden);
    uint16_t *act1 = cv.take<uint16_t>((size_t)n * mlp->hidden);
    double *pdef = cv.take<double>((size_t)n * p);
    int *valid = cv.take<int>(n);
    double *pk = cv.take<double>(n);
    int rc = mark_event(ctx, events, 0, st);
    if (rc) return rc;
    // features, the default guess (the refit start) from the same moments, proposal
    rc = features_launch(ctx, mt, x, kInDim, mom8, pk, st);
    if (rc) return rc;
    rc = var->guess_stored(ctx, mt.ci, mom8, pk, pdef, st);
    if (rc) return rc;
    uint16_t *Y[17];
    for (int l = 0; l < mlp->n_hidden; ++l) Y[l] = (l & 1) ? act1 : act0;
    rc = forward_pass(mlp, n, x, kInDim, nullptr, Y, nullptr, out, st);
    if (rc) return rc;
    rc = decode_launch(ctx, mt, out, mlp->out_dim, mom8, params_out, valid, st);
    if (rc) return rc;
    // LM from the valid proposals, refits from the moment guess in place
    gm_fit_opts o = opts ? *opts : gm_fit_opts{100, 1e-3, 1e-4, nullptr, 0, nullptr};
    o.active = nullptr;
    FitExtra rf;
    rf.refit_start = pdef;
    rf.valid = valid;
    rf.refit_code = fallback_out;
    rf.first_max_iter =
        (o.proposal_max_iter > 0 && o.proposal_max_iter < o.max_iter) ? o.proposal_max_iter : o.max_iter;
    if ((rc = mark_event(ctx, events, 1, st))) return rc;
    rc = var->fit(ctx, mt.ci, &o, params_out, chi2_out, niter_out, status_out, &rf, st);
    if (rc) return rc;
    if ((rc = mark_event(ctx, events, 2, st))) return rc;
    return mark_event(ctx, events, 3, st);
}

}  // namespace

extern "C" {

int64_t gm_mlp_param_count(const gm_mlp *mlp)
{
    gm_mlp m = mlp ? *mlp : gm_mlp{};
    if (!mlp) return -1;
    // sizes only: pointers are not needed to count
    if (m.in_dim < 8 || m.hidden < 8 || m.n_hidden < 1 || m.n_hidden > 16 || m.out_dim < 8 || m.in_dim % 8 ||
        m.hidden % 8 || m.out_dim % 8)
        return -1;
    return count_params(&m);
}

int gm_mlp_sync(gm_ctx *ctx, const gm_mlp *mlp, void *stream)
{
    if (!ctx) return GM_EINVAL;
    int rc = check_mlp(mlp, false);
    if (rc) return rc;
    Scoped sd(ctx->device);
    hipLaunchKernelGGL(sync_bf16_kernel, dim3(1024), dim3(256), 0, (hipStream_t)stream, count_params(mlp),
                       mlp->params, mlp->params_bf16);
    return hipGetLastError() == hipSuccess ? GM_OK : GM_EHIP;
}

int gm_mlp_forward(gm_ctx *ctx, const gm_mlp *mlp, int32_t n, const uint16_t *x, int64_t ldx, float *out,
                   void *stream)
{
    if (!ctx || n < 0) return GM_EINVAL;
    int rc = check_mlp(mlp, false);
    if (rc) return rc;
    if (n == 0) return GM_OK;
    if (!x || !out || ldx < mlp->in_dim || ldx % 8 || !aligned16(x)) return GM_EINVAL;
    Scoped sd(ctx->device);
    const size_t act = (((size_t)n * mlp->hidden * 2 + 255) & ~(size_t)255);
    rc = ensure_ws(ctx, 2 * act + 256);
    if (rc) return rc;
    uint16_t *buf[2] = {reinterpret_cast<uint16_t *>(ctx->mlp_ws),
                        reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(ctx->mlp_ws) + act)};
    uint16_t *Y[17];
    for (int l = 0; l < mlp->n_hidden; ++l) Y[l] = buf[l & 1];
    return forward_pass(mlp, n, x, ldx, nullptr, Y, nullptr, out, (hipStream_t)stream);
}

int gm_mlp_gemm(gm_ctx *ctx, int32_t op, int32_t m, int32_t n, int32_t k, const uint16_t *a, int64_t lda,
                const int32_t *a_rows, const uint16_t *b, int64_t ldb, const int32_t *b_rows, float *c,
                int64_t ldc, void *stream)
{
    if (!ctx || m < 0 || n < 0 || k < 0 || op < GM_GEMM_NT || op > GM_GEMM_TN) return GM_EINVAL;
    if (m == 0 || n == 0) return GM_OK;
    if (!c || ldc < n || lda % 8 || ldb % 8) return GM_EINVAL;
    if (k > 0 && (!a || !b || !aligned16(a) || !aligned16(b))) return GM_EINVAL;     // k = 0: C = 0, no reads
    hipStream_t st = (hipStream_t)stream;
    Scoped sd(ctx->device);
    GemmArgs g{};
    g.M = m;
    g.N = n;
    g.K = k;
    g.a = a;
    g.lda = lda;
    g.b = b;
    g.ldb = ldb;
    g.cf = c;
    g.ldcf = ldc;
    if (op == GM_GEMM_NT) {
        if (k % 8 || lda < k || ldb < k || b_rows) return GM_EINVAL;
        g.amap = a_rows;
        return gemm<false, true, EPI_F32>(g, st);
    }
    if (op == GM_GEMM_NN) {
        if (k % 8 || n % 8 || lda < k || ldb < n || b_rows) return GM_EINVAL;
        g.amap = a_rows;
        return gemm<false, false, EPI_F32>(g, st);
    }
    if (m % 8 || n % 8 || lda < m || ldb < n || a_rows) return GM_EINVAL;
    g.bmap = b_rows;
    const size_t part = dw_part_floats(m, n, k);
    int rc = ensure_ws(ctx, part * 4 + 256);
    if (rc) return rc;
    return gemm_dw(g, reinterpret_cast<float *>(ctx->mlp_ws), st);
}

int gm_mlp_backward(gm_ctx *ctx, const gm_mlp *mlp, int32_t n, const uint16_t *x, int64_t ldx, const int32_t *rows,
                    const float *targets, double *loss_out, void *stream)
{
    if (!ctx || n < 0) return GM_EINVAL;
    int rc = check_mlp(mlp, true);
    if (rc) return rc;
    if (n == 0) return GM_OK;
    if (!x || !targets || ldx < mlp->in_dim || ldx % 8 || !aligned16(x)) return GM_EINVAL;
    Scoped sd(ctx->device);
    return backward_pass(ctx, mlp, n, x, ldx, rows, targets, loss_out, (hipStream_t)stream);
}

int gm_mlp_adamw(gm_ctx *ctx, const gm_mlp *mlp, int64_t step, const gm_adamw *opt, void *stream)
{
    if (!ctx) return GM_EINVAL;
    int rc = check_mlp(mlp, true);
    if (rc) return rc;
    Scoped sd(ctx->device);
    return adamw_step(mlp, step, opt, (hipStream_t)stream);
}

int gm_mlp_train_step(gm_ctx *ctx, const gm_mlp *mlp, int32_t n, const uint16_t *x, int64_t ldx,
                      const int32_t *rows, const float *targets, int64_t step, const gm_adamw *opt, double *loss_out,
                      void *stream)
{
    if (!ctx || n < 1) return GM_EINVAL;
    int rc = check_mlp(mlp, true);
    if (rc) return rc;
    if (!x || !targets || ldx < mlp->in_dim || ldx % 8 || !aligned16(x) || !opt || step < 1) return GM_EINVAL;
    Scoped sd(ctx->device);
    rc = backward_pass(ctx, mlp, n, x, ldx, rows, targets, loss_out, (hipStream_t)stream);
    if (rc) return rc;
    return adamw_step(mlp, step, opt, (hipStream_t)stream);
}

int gm_features(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, uint16_t *x_out, int64_t ldx,
                double *moments_out, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (batch->n_gal == 0) return GM_OK;
    if (!x_out || ldx < kInDim || ldx % 8 || !aligned16(x_out)) return GM_EINVAL;
    Scoped sd(ctx->device);
    return features_launch(ctx, mt, x_out, ldx, moments_out, nullptr, (hipStream_t)stream);
}

int gm_proposal_targets(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const double *truth,
                        const double *moments, float *targets_out, int32_t out_dim, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    rc = check_proposal_model(mt);
    if (rc) return rc;
    if (batch->n_gal == 0) return GM_OK;
    if (!truth || !moments || !targets_out || out_dim < kNOut) return GM_EINVAL;
    Scoped sd(ctx->device);
    const int n = batch->n_gal;
    hipLaunchKernelGGL(targets_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n, mt.ci.ma, truth,
                       moments, targets_out, (int)out_dim);
    return hipGetLastError() == hipSuccess ? GM_OK : GM_EHIP;
}

int gm_proposal_decode(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const float *out, int32_t out_dim,
                       const double *moments, double *params_out, int32_t *valid_out, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    rc = check_proposal_model(mt);
    if (rc) return rc;
    if (batch->n_gal == 0) return GM_OK;
    if (!out || !moments || !params_out || !valid_out || out_dim < kNOut) return GM_EINVAL;
    Scoped sd(ctx->device);
    return decode_launch(ctx, mt, out, out_dim, moments, params_out, valid_out, (hipStream_t)stream);
}

int gm_fit_learned(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_mlp *mlp,
                   const gm_fit_opts *opts, double *params_out, double *chi2_out, int32_t *niter_out,
                   int32_t *status_out, int32_t *fallback_out, void *const *events, void *stream)
{
    Match mt;
    int rc = learned_checks(ctx, model, batch, mlp, opts, mt);
    if (rc) return rc;
    if (batch->n_gal == 0) return GM_OK;
    if (!params_out || !chi2_out || !niter_out || !status_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    const Variant *var;
    if ((rc = pick_variant(ctx, mt, &var))) return rc;
    if ((rc = ensure_ws(ctx, learned_ws_bytes(mlp, batch->n_gal, model->p)))) return rc;
    return learned_seq(ctx, mt, var, mlp, opts, params_out, chi2_out, niter_out, status_out, fallback_out, events,
                       (hipStream_t)stream);
}

int gm_plan_fit_learned(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_mlp *mlp,
                        const gm_fit_opts *opts, double *params_out, double *chi2_out, int32_t *niter_out,
                        int32_t *status_out, int32_t *fallback_out, double *err_out, int32_t timing,
                        gm_plan **out)
{
    if (!out) return GM_EINVAL;
    *out = nullptr;
    Match mt;
    int rc = learned_checks(ctx, model, batch, mlp, opts, mt);
    if (rc) return rc;
    if (batch->n_gal == 0 || !params_out || !chi2_out || !niter_out || !status_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    gm_plan *p;
    // stagings: guess, features, decode, two fits, errors
    if ((rc = plan_open(ctx, batch->n_gal, 6, timing != 0, &p))) return rc;
    gm_ctx *pc = &p->ctx;
    void *const *events = timing ? p->ev : nullptr;
    const Variant *var = nullptr;
    rc = pick_variant(pc, mt, &var);
    // the workspace is sized before the capture, which then allocates nothing
    if (!rc) rc = ensure_ws(pc, learned_ws_bytes(mlp, batch->n_gal, model->p));
    if (!rc) rc = plan_begin(p);
    gm_fit_opts o = opts ? *opts : gm_fit_opts{100, 1e-3, 1e-4, nullptr, 0, nullptr};
    o.err_out = err_out;
    if (!rc)
        rc = learned_seq(pc, mt, var, mlp, &o, params_out, chi2_out, niter_out, status_out, fallback_out, events,
                         p->stream);
    return plan_end(p, rc, out);
}

int gm_synth_noise(gm_ctx *ctx, int32_t n_gal, const int32_t *h, const int32_t *w, const int64_t *img_off,
                   const float *unit, const double *snr, const double *sky, float sigma, double m0, uint64_t seed,
                   int64_t first_index, float *data_out, float *sigma_out, double *mag_out, int32_t mag_stride,
                   void *stream)
{
    if (!ctx || n_gal < 0 || !(sigma > 0.0f) || !std::isfinite(m0) || first_index < 0) return GM_EINVAL;
    if (n_gal == 0) return GM_OK;
    if (!h || !w || !img_off || !unit || !snr || !sky || !data_out || (mag_out && mag_stride < 1)) return GM_EINVAL;
    gm_batch b{};
    b.n_gal = n_gal;
    b.h = h;
    b.w = w;
    b.img_off = img_off;
    b.data = unit;
    b.sigma = unit;
    int rc = check_batch(&b, false);
    if (rc) return rc;
    Scoped sd(ctx->device);
    Match mt;
    mt.ci.b = &b;
    mt.ci.convolved = false;
    Staged sg;
    hipStream_t st = (hipStream_t)stream;
    rc = stage(ctx, mt.ci, nullptr, 0, st, &sg);
    if (rc) return rc;
    const int grid = std::min(n_gal, std::max(ctx->num_cu, 1) * 8);
    hipLaunchKernelGGL(synth_kernel, dim3(grid), dim3(NT), 0, st, sg.meta, n_gal, unit, snr, sky, sigma, m0,
                       (uint32_t)seed, (uint32_t)(seed >> 32), first_index, data_out, sigma_out, mag_out,
                       (int)mag_stride);
    return hipGetLastError() == hipSuccess ? GM_OK : GM_EHIP;
}

}  // extern "C"
