// gm_adam.h -- the gradient-descent fitter (Adam on chi^2, the paper's own
// fitter of Sec. 5.1): its gradient evaluation by the adjoint, its persistent
// kernel and its launch driver.  Included at the end of gm_launch.h.
#pragma once

namespace gm {

// One gradient evaluation at u for the gradient-descent fitter: chi^2 and
// g = J^T W r by the adjoint, two convolutions per evaluation whatever the
// number of variables.  Pass 1 convolves the light plane (FP64), forms the
// residual and stores the weighted residual R = w r (FP32) of every pixel in
// rb; the magnitude (DER) and analytic (sky) columns take their products
// from the convolved light and the pixel position there.  Pass 2 correlates R
// with the PSF -- a convolution with the flipped PSF psf_t, zero padding as in
// the forward model -- into Q and adds Q dI/du_k with the unconvolved,
// pixel-integrated derivatives of the light: sum_pixels R (PSF x D_k) =
// sum_pixels (PSF-correlated R) D_k.  rb holds H W floats; it is read back
// through L2 (agent-scope loads) after the workgroup barrier.
__device__ inline float load_l2(const float *p)
{
    return __uint_as_float(__hip_atomic_load(reinterpret_cast<const unsigned int *>(p), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT));
}

template <class F, int KT, int NG>
__device__ void evaluate_grad(const double *u, const ModelArgs &ma, const BatchArgs &ba, const Meta &me,
                              EvalShared<F> &sh, float *planes, const cfloat *psf_t, float *rb, double *out_chi2,
                              double *out_g)
{
    constexpr int P = F::P;
    constexpr int NR = 1 + P;
    const int H = me.h, W = me.w, K = me.k;
    const int tid = threadIdx.x;
    eval_prologue<F>(u, ma, H, W, sh, planes);
    const cfloat *psf = (const cfloat *)(ba.psf + uniform64(me.psf_off));
    const int IH = region_h(K), IWP = region_wp(K), IW = TILE + K - 1, c = (K - 1) / 2;
    double c2 = 0.0;
    float red[P];
#pragma unroll
    for (int q = 0; q < P; ++q) red[q] = 0.0f;
    int r, cg;
    strip_of(tid, K, r, cg);
    const int nty = (H + TILE - 1) / TILE, ntx = (W + TILE - 1) / TILE;
    // pass 1: model, residual, chi^2, R; columns from the convolved light
    for (int ty = 0; ty < nty; ++ty) {
        for (int tx = 0; tx < ntx; ++tx) {
            const int ti0 = ty * TILE, tj0 = tx * TILE;
            fill_region<F, 0, 1>(sh, planes, H, W, K, ti0, tj0);
            __syncthreads();
            double acc0[4];
            const double *base = reinterpret_cast<const double *>(planes) + 4 * cg;
            if constexpr (KT > 0) conv_plane<KT, double>(base, r, IWP, psf, acc0);
            else conv_plane_any<double>(base, r, K, IWP, psf, acc0);
            __syncthreads();
            const int i = ti0 + r;
            if (i >= H) continue;
            float dv[4], wv[4];
            strip_weights(ba, me.img_off + (int64_t)i * W, tj0 + 4 * cg, W, dv, wv);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int j = tj0 + 4 * cg + t;
                if (j >= W) continue;
                const float d = dv[t];
                const float wgt = wv[t];
                float R = 0.0f;
                if (wgt != 0.0f) {
                    const double pdx = ((double)j + 0.5) - 0.5 * W, pdy = 0.5 * H - ((double)i + 0.5);
                    const double res = (double)d - (acc0[t] + F::sky_at(sh.prep, pdx, pdy));
                    c2 = fma((double)wgt * res, res, c2);
                    R = wgt * (float)res;
                    const float fdx = (float)pdx, fdy = (float)pdy;
                    float none[F::NPL] = {};
#pragma unroll
                    for (int k = 0; k < P; ++k) {
                        if (F::analytic(k)) red[k] = fmaf(R, F::analytic_value(k, fdx, fdy), red[k]);
                        else if (k == F::DER) red[k] = fmaf(R, F::derived(acc0[t], none), red[k]);
                    }
                }
                rb[i * W + j] = R;
            }
        }
    }
    __syncthreads();
    // pass 2: Q = R correlated with the PSF, contracted with the derivatives
    for (int ty = 0; ty < nty; ++ty) {
        for (int tx = 0; tx < ntx; ++tx) {
            const int ti0 = ty * TILE, tj0 = tx * TILE;
            for (int t = tid; t < IH * IW; t += NT) {
                const int ri = t / IW, ci = t - ri * IW;
                const int gi = ti0 - c + ri, gj = tj0 - c + ci;
                planes[ri * IWP + ci] = (gi >= 0 && gi < H && gj >= 0 && gj < W) ? load_l2(rb + gi * W + gj) : 0.0f;
            }
            __syncthreads();
            float q4[4];
            if constexpr (KT > 0) conv_plane<KT, float>(planes + 4 * cg, r, IWP, psf_t, q4);
            else conv_plane_any<float>(planes + 4 * cg, r, K, IWP, psf_t, q4);
            __syncthreads();
            const int i = ti0 + r;
            if (i >= H) continue;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int j = tj0 + 4 * cg + t;
                if (j >= W) continue;
                double v0;
                float dp[F::NPL - 1];
                planes_at<F, false>(sh, i, j, H, v0, dp);
#pragma unroll
                for (int k = 0; k < P; ++k)
                    if (!F::analytic(k) && k != F::DER) red[k] = fmaf(q4[t], dp[F::plane(k) - 1], red[k]);
            }
        }
    }
    // fixed-order reduction in FP64, as in evaluate
    double *sred = reinterpret_cast<double *>(planes);
    const int lane = tid & 63, wave = tid >> 6;
    {
        double v = wave_sum(c2);
        if (lane == 0) sred[wave * NR] = v;
    }
#pragma unroll
    for (int q = 1; q < NR; ++q) {
        double v = wave_sum((double)red[q - 1]);
        if (lane == 0) sred[wave * NR + q] = v;
    }
    __syncthreads();
    for (int q = tid; q < NR; q += NT) {
        double sm = sred[q];
        for (int wv = 1; wv < NWAVE; ++wv) sm += sred[wv * NR + q];
        if (q == 0) *out_chi2 = sm;
        else out_g[q - 1] = sm;
    }
    __syncthreads();
}

// The PSF of every galaxy flipped in both axes (the correlation kernel of the
// adjoint): psf_t[off + (K-1-a) K + (K-1-b)] = psf[off + a K + b].  One
// workgroup per galaxy; galaxies that share a PSF write the same values.
static __global__ void flip_psf_kernel(const Meta *meta, int n_gal, const float *psf, float *psf_t)
{
    const int g = blockIdx.x;
    if (g >= n_gal) return;
    const Meta me = meta[g];
    const int K = me.k, n = K * K;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int a = e / K, b = e - a * K;
        psf_t[me.psf_off + (int64_t)(K - 1 - a) * K + (K - 1 - b)] = psf[me.psf_off + e];
    }
}

// ---------------------------------------------------------------- gradient descent (Adam)
// The paper's own fitter (Sec. 5.1: gradient descent, Adam in its examples)
// on the same model: chi^2 and g = J^T W r at u (evaluate_grad: the forward
// model and one adjoint correlation) give the gradient d chi^2 / d u = -2 g in
// the LM variables; Adam (Kingma and Ba 2015) takes
// `steps` steps with bias-corrected moments, the iterate clamped to the LM
// bounds after each, fixed slots untouched.  The reported chi^2 is that of a
// last evaluation at the final iterate; status GM_ST_MAXITER (all steps
// taken) or GM_ST_NONFINITE.
struct AdamArgs {
    const int *order;
    int n_gal;
    int *queue;
    double *params, *chi2;
    int *status;
    int steps;
    double lr, beta1, beta2, eps;
    const float *psf_t;     // flipped PSFs, same offsets as the PSFs
    float *rbuf;            // weighted residuals: rstride floats per workgroup
    int64_t rstride;
};

template <class F, int KT, int NG>
__global__ __launch_bounds__(NT, (min_wg<F, KT, NG>())) void adam_fit_kernel(ModelArgs ma, BatchArgs ba, AdamArgs aa)
{
    extern __shared__ float4 dyn_lds[];
    float *planes = reinterpret_cast<float *>(dyn_lds);
    __shared__ EvalShared<F> esh;
    __shared__ LMShared<F> s;
    constexpr int P = F::P;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s.gal = atomicAdd(aa.queue, 1);
        __syncthreads();
        const int qi = uniform(s.gal);
        if (qi >= aa.n_gal) break;
        const int g = uniform(aa.order[qi]);
        const Meta me = ba.meta[g];
        if (tid == 0) {
            load_u<F>(s, ma, aa.params + (int64_t)g * ma.p);
            clamp_u<F>(s.u, me.h, me.w);
        }
        __syncthreads();
        const cfloat *psf_t = (const cfloat *)(aa.psf_t + uniform64(me.psf_off));
        float *rb = aa.rbuf + (int64_t)blockIdx.x * aa.rstride;
        // moments of lane k (k < P): registers of the first wave
        double m1 = 0.0, m2 = 0.0, b1t = 1.0, b2t = 1.0;
        bool bad = false;
        for (int t = 1; t <= aa.steps && !bad; ++t) {
            evaluate_grad<F, KT, NG>(s.u, ma, ba, me, esh, planes, psf_t, rb, &s.chi2, s.g);
            bad = !isfinite(s.chi2);
            if (!bad && tid < P && s.freev[tid]) {
                const double grad = -2.0 * s.g[tid];
                m1 = aa.beta1 * m1 + (1.0 - aa.beta1) * grad;
                m2 = aa.beta2 * m2 + (1.0 - aa.beta2) * grad * grad;
                b1t *= aa.beta1;
                b2t *= aa.beta2;
                const double mh = m1 / (1.0 - b1t), vh = m2 / (1.0 - b2t);
                s.u[tid] = clamp_var<F>(tid, s.u[tid] - aa.lr * mh / (sqrt(vh) + aa.eps), me.h, me.w);
            }
            __syncthreads();
        }
        if (!bad) evaluate_grad<F, KT, NG>(s.u, ma, ba, me, esh, planes, psf_t, rb, &s.chi2, s.g);
        if (tid == 0) {
            double nat[P];
            canonical_nat<F>(s.u, s.freev, nat);
            double *out = aa.params + (int64_t)g * ma.p;
            for (int k = 0; k < P; ++k)
                if (ma.col[k] >= 0) out[ma.col[k]] = nat[k];
            aa.chi2[g] = s.chi2;
            aa.status[g] = (bad || !isfinite(s.chi2)) ? GM_ST_NONFINITE : GM_ST_MAXITER;
        }
        __syncthreads();
    }
}

// psf_len: floats of the PSF array the batch reads (0 for an unconvolved
// model, which runs with the unit PSF); max_px: the largest cutout.  The
// context's scratch holds the flipped PSFs, then one residual image of max_px
// floats per workgroup of the grid.
template <class F, int NG, int KT>
int launch_adam(gm_ctx *c, const ModelArgs &ma, const BatchArgs &ba, AdamArgs aa, size_t lds, int wpc,
                int64_t psf_len, int64_t max_px, hipStream_t st)
{
    auto kern = adam_fit_kernel<F, KT, NG>;
    int per_cu;
    int rc = prepare(kern, lds, &per_cu);
    if (rc) return rc;
    if (wpc > 0) per_cu = std::min(per_cu, wpc);
    int grid = std::min(aa.n_gal, per_cu * c->num_cu);
    const int64_t psf_al = (psf_len + 63) / 64 * 64;
    aa.rstride = (max_px + 63) / 64 * 64;
    void *ws;
    if ((rc = ensure_aux(c, sizeof(float) * (size_t)(psf_al + aa.rstride * grid), &ws))) return rc;
    float *wsf = reinterpret_cast<float *>(ws);
    if (psf_len > 0) {
        hipLaunchKernelGGL(flip_psf_kernel, dim3(aa.n_gal), dim3(256), 0, st, ba.meta, aa.n_gal, ba.psf, wsf);
        if ((rc = hip_rc(hipGetLastError()))) return rc;
        aa.psf_t = wsf;
    } else {
        aa.psf_t = ba.psf;      // the unit PSF is its own flip
    }
    aa.rbuf = wsf + psf_al;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, ma, ba, aa);
    return hip_rc(hipGetLastError());
}

template <class F, int NG, int... KTS>
int run_adam(gm_ctx *c, const CallInfo &ci, const gm_adam_opts *o, double *params, double *chi2, int32_t *status,
             hipStream_t st)
{
    const gm_batch *b = ci.b;
    size_t lds;
    int rc = check_lds<F, NG>(max_k(ci), &lds);
    if (rc) return rc;
    std::vector<int> order(b->n_gal);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> cost(b->n_gal);
    for (int g = 0; g < b->n_gal; ++g) {
        double k = ci.convolved ? b->psf_k[g] : 1.0;
        cost[g] = (double)b->h[g] * b->w[g] * k * k;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    Staged sg;
    rc = stage(c, ci, order.data(), sizeof(int) * (size_t)b->n_gal, st, &sg);
    if (rc) return rc;
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, st, sg.queue, 0);
    if (hipGetLastError() != hipSuccess) return GM_EHIP;
    AdamArgs aa{};
    aa.order = reinterpret_cast<const int *>(sg.extra);
    aa.n_gal = b->n_gal;
    aa.queue = sg.queue;
    aa.params = params;
    aa.chi2 = chi2;
    aa.status = status;
    aa.steps = o->steps;
    aa.lr = o->lr;
    aa.beta1 = o->beta1;
    aa.beta2 = o->beta2;
    aa.eps = o->eps;
    int64_t psf_len = 0, max_px = 0;
    for (int g = 0; g < b->n_gal; ++g) {
        if (ci.convolved) psf_len = std::max(psf_len, b->psf_off[g] + (int64_t)b->psf_k[g] * b->psf_k[g]);
        max_px = std::max(max_px, (int64_t)b->h[g] * b->w[g]);
    }
    return Dispatch<F, NG, KTS...>::adam(batch_kt(ci), c, ci.ma, batch_args(c, ci, sg), aa, lds, ci.wpc, psf_len,
                                         max_px, st);
}

}  // namespace gm
