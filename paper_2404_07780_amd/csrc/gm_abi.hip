// gm_abi.hip -- host side of libgmfit: the C ABI declared in include/gmfit.h.
//
// Every call validates its arguments, matches the caller's gm_model against
// a compiled model family (mapping the family's internal LM vector onto the
// caller's parameter columns), stages the host-side size metadata into a
// grow-only device workspace of the context and launches one kernel on the
// caller's stream.  Nothing is allocated once the workspace has grown to the
// largest batch seen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "gm_kernels.h"

using namespace gm;

namespace {

constexpr size_t kMaxLds = 160 * 1024;

enum FamilyId { FAM_NONE = 0, FAM_SERSIC = 1, FAM_BULGEDISK = 2 };

struct Workspace {
    void *dev = nullptr;
    size_t dev_bytes = 0;
    void *host = nullptr;        // pinned staging
    size_t host_bytes = 0;
    hipEvent_t staged = nullptr; // last copy out of the staging buffer
    bool pending = false;
};

}  // namespace

struct gm_ctx {
    int device = 0;
    int num_cu = 0;
    Workspace ws;
};

namespace {

int hip_fail(hipError_t e) { return e == hipSuccess ? GM_OK : GM_EHIP; }

struct Scoped {
    int prev = -1;
    explicit Scoped(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~Scoped()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int ensure_dev(gm_ctx *c, size_t bytes)
{
    if (c->ws.dev_bytes >= bytes) return GM_OK;
    if (c->ws.dev) {
        if (hipDeviceSynchronize() != hipSuccess) return GM_EHIP;
        (void)hipFree(c->ws.dev);
        c->ws.dev = nullptr;
        c->ws.dev_bytes = 0;
    }
    size_t nb = std::max(bytes, (size_t)1 << 20);
    if (hipMalloc(&c->ws.dev, nb) != hipSuccess) return GM_ENOMEM;
    c->ws.dev_bytes = nb;
    return GM_OK;
}

int ensure_host(gm_ctx *c, size_t bytes)
{
    if (c->ws.pending) {
        if (hipEventSynchronize(c->ws.staged) != hipSuccess) return GM_EHIP;
        c->ws.pending = false;
    }
    if (c->ws.host_bytes >= bytes) return GM_OK;
    if (c->ws.host) (void)hipHostFree(c->ws.host);
    c->ws.host = nullptr;
    c->ws.host_bytes = 0;
    size_t nb = std::max(bytes, (size_t)1 << 20);
    if (hipHostMalloc(&c->ws.host, nb, hipHostMallocDefault) != hipSuccess) return GM_ENOMEM;
    c->ws.host_bytes = nb;
    return GM_OK;
}

// ---------------------------------------------------------------- model matching
// Natural slot counts per profile type (index = type).
const int kSlots[8] = {0, 7, 6, 8, 8, 6, 7, 1};

bool comp_ok(const gm_component &c, int p)
{
    if (c.type < GM_SERSIC || c.type > GM_SKY) return false;
    for (int s = 0; s < 8; ++s) {
        int k = c.param_index[s];
        if (s >= kSlots[c.type]) {
            if (k >= 0) return false;
        } else if (k >= p) {
            return false;
        }
    }
    return true;
}

struct Match {
    FamilyId fam = FAM_NONE;
    ModelArgs ma{};
};

// internal index k <- slot s of component c
void take(const gm_component &c, int s, int k, ModelArgs &ma)
{
    ma.col[k] = c.param_index[s];
    ma.fixedv[k] = c.fixed[s];
}

int match_model(const gm_model *m, Match &out)
{
    if (!m || m->n_comp < 1 || m->n_comp > 4 || m->p < 1 || m->p > MAXP) return GM_EINVAL;
    if (m->oversample < 1 || m->oversample > 16 || m->os_window < 0 || m->os_window > 5 ||
        (m->os_window > 0 && (m->os_window & 1) == 0) || !std::isfinite(m->m0))
        return GM_EINVAL;
    const gm_component *ser = nullptr, *exd = nullptr, *sky = nullptr;
    int nother = 0;
    for (int i = 0; i < m->n_comp; ++i) {
        const gm_component &c = m->comp[i];
        if (!comp_ok(c, m->p)) return GM_EINVAL;
        if (c.type == GM_SKY) {
            if (c.convolve) return GM_EINVAL;
            if (sky) return GM_EUNSUPPORTED;
            sky = &c;
        } else if (c.type == GM_SERSIC && c.convolve && !ser) {
            ser = &c;
        } else if (c.type == GM_EXPDISK && c.convolve && !exd) {
            exd = &c;
        } else {
            nother++;
        }
    }
    // every column must be referenced by some slot
    std::vector<int> seen(m->p, 0);
    for (int i = 0; i < m->n_comp; ++i)
        for (int s = 0; s < kSlots[m->comp[i].type]; ++s)
            if (m->comp[i].param_index[s] >= 0) seen[m->comp[i].param_index[s]] = 1;
    for (int k = 0; k < m->p; ++k)
        if (!seen[k]) return GM_EINVAL;
    if (nother || !ser) return GM_EUNSUPPORTED;
    ModelArgs ma{};
    ma.p = m->p;
    ma.m0 = m->m0;
    ma.osf = m->oversample;
    ma.osw = m->oversample > 1 ? m->os_window : 0;
    for (int k = 0; k < MAXP; ++k) {
        ma.col[k] = -1;
        ma.fixedv[k] = 0.0;
    }
    FamilyId fam;
    int nint;
    if (!exd) {
        fam = FAM_SERSIC;
        nint = FamSersic::P;
        for (int s = 0; s < 7; ++s) take(*ser, s, s, ma);
        if (sky) take(*sky, 0, 7, ma);
    } else {
        // bulge + disk: the disk's centre must be tied to the bulge's
        for (int s = 0; s < 2; ++s) {
            int a = ser->param_index[s], b = exd->param_index[s];
            if (a != b) return GM_EUNSUPPORTED;
            if (a < 0 && ser->fixed[s] != exd->fixed[s]) return GM_EUNSUPPORTED;
        }
        fam = FAM_BULGEDISK;
        nint = FamBulgeDisk::P;
        for (int s = 0; s < 7; ++s) take(*ser, s, s, ma);
        for (int s = 2; s < 6; ++s) take(*exd, s, 5 + s, ma);
        if (sky) take(*sky, 0, 11, ma);
    }
    // a column used by two internal variables would be an unsupported tie
    std::vector<int> used(m->p, 0);
    for (int k = 0; k < nint; ++k)
        if (ma.col[k] >= 0 && used[ma.col[k]]++) return GM_EUNSUPPORTED;
    out.fam = fam;
    out.ma = ma;
    return GM_OK;
}

int check_batch(const gm_batch *b)
{
    if (!b || b->n_gal < 0) return GM_EINVAL;
    if (b->n_gal == 0) return GM_OK;
    if (!b->h || !b->w || !b->img_off || !b->psf_k || !b->psf_off || !b->psf) return GM_EINVAL;
    for (int g = 0; g < b->n_gal; ++g) {
        if (b->h[g] < 1 || b->w[g] < 1 || b->h[g] > 1024 || b->w[g] > 1024) return GM_EINVAL;
        if (b->psf_k[g] < 1 || (b->psf_k[g] & 1) == 0) return GM_EINVAL;
        if (b->img_off[g] < 0 || b->psf_off[g] < 0) return GM_EINVAL;
    }
    return GM_OK;
}

// Compile-time PSF side shared by the whole batch (15 or 25), else 0.
int batch_kt(const gm_batch *b)
{
    int k0 = b->n_gal ? b->psf_k[0] : 0;
    for (int g = 1; g < b->n_gal; ++g)
        if (b->psf_k[g] != k0) return 0;
    return (k0 == 15 || k0 == 25) ? k0 : 0;
}

int max_k(const gm_batch *b)
{
    int k = 1;
    for (int g = 0; g < b->n_gal; ++g) k = std::max(k, b->psf_k[g]);
    return k;
}

// Device workspace of one call: [meta | extra | queue counter].
struct Staged {
    Meta *meta;
    void *extra;
    int *queue;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Stage meta [+ extra bytes] into the device workspace.
int stage(gm_ctx *c, const gm_batch *b, const void *extra, size_t extra_bytes, hipStream_t st, Staged *out)
{
    size_t mb_al = align256(sizeof(Meta) * (size_t)b->n_gal);
    size_t ex_al = align256(extra_bytes);
    size_t q_off = mb_al + ex_al;
    size_t total = q_off + 256;
    int rc = ensure_host(c, mb_al + ex_al);
    if (rc) return rc;
    rc = ensure_dev(c, total);
    if (rc) return rc;
    Meta *hm = reinterpret_cast<Meta *>(c->ws.host);
    for (int g = 0; g < b->n_gal; ++g) {
        hm[g].h = b->h[g];
        hm[g].w = b->w[g];
        hm[g].k = b->psf_k[g];
        hm[g].pad = 0;
        hm[g].img_off = b->img_off[g];
        hm[g].psf_off = b->psf_off[g];
    }
    char *hp = reinterpret_cast<char *>(c->ws.host);
    if (extra_bytes) memcpy(hp + mb_al, extra, extra_bytes);
    if (hipMemcpyAsync(c->ws.dev, c->ws.host, mb_al + ex_al, hipMemcpyHostToDevice, st) != hipSuccess)
        return GM_EHIP;
    if (hipEventRecord(c->ws.staged, st) != hipSuccess) return GM_EHIP;
    c->ws.pending = true;
    char *dp = reinterpret_cast<char *>(c->ws.dev);
    out->meta = reinterpret_cast<Meta *>(dp);
    out->extra = dp + mb_al;
    out->queue = reinterpret_cast<int *>(dp + q_off);
    return GM_OK;
}

template <class F>
size_t static_lds()
{
    return sizeof(EvalShared<F>) + sizeof(LMShared<F>) + 64;
}

// Dynamic LDS of a kernel with NG plane groups for PSF side K: the plane
// buffer, which also hosts the window partial sums, the wave partial sums of
// the normal equations and the thread-0 solver temporaries.
template <class F, int NG>
size_t lds_bytes(int K)
{
    return std::max({planes_bytes<F, NG>(K), (size_t)NWAVE * (1 + F::P + F::P * (F::P + 1) / 2) * 8,
                     (size_t)3 * F::P * F::P * 8, window_scratch_bytes<F>()});
}

// Plane-group variants compiled per family (the first is the default).
template <class F> struct Groups;
template <> struct Groups<FamSersic> { static constexpr int a = 1, b = 2; };
template <> struct Groups<FamBulgeDisk> { static constexpr int a = 2, b = 3; };

// Fewest groups that let two workgroups share a CU, else fewest that fit.
template <class F>
int pick_groups(int K, int *ng, size_t *lds)
{
    constexpr int A = Groups<F>::a, B = Groups<F>::b;
    size_t la = lds_bytes<F, A>(K) + static_lds<F>(), lb = lds_bytes<F, B>(K) + static_lds<F>();
    if (2 * la <= kMaxLds) { *ng = A; *lds = lds_bytes<F, A>(K); return GM_OK; }
    if (2 * lb <= kMaxLds) { *ng = B; *lds = lds_bytes<F, B>(K); return GM_OK; }
    if (la <= kMaxLds) { *ng = A; *lds = lds_bytes<F, A>(K); return GM_OK; }
    if (lb <= kMaxLds) { *ng = B; *lds = lds_bytes<F, B>(K); return GM_OK; }
    return GM_EUNSUPPORTED;
}

template <typename Kern>
int prepare(Kern kern, size_t lds, int *blocks_per_cu)
{
    if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return GM_EHIP;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, NT, lds) != hipSuccess) return GM_EHIP;
    *blocks_per_cu = std::max(nb, 1);
    return GM_OK;
}

template <class F, int KT, int NG>
int launch_fit_k(gm_ctx *c, const ModelArgs &ma, const BatchArgs &ba, const FitArgs &fa, size_t lds, hipStream_t st)
{
    auto kern = lm_fit_kernel<F, KT, NG>;
    int per_cu;
    int rc = prepare(kern, lds, &per_cu);
    if (rc) return rc;
    int grid = std::min(fa.n_gal, per_cu * c->num_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, ma, ba, fa);
    return hip_fail(hipGetLastError());
}

template <class F, int KT, int NG>
int launch_err_k(gm_ctx *c, const ModelArgs &ma, const BatchArgs &ba, const ErrArgs &ea, size_t lds, hipStream_t st)
{
    auto kern = errors_kernel<F, KT, NG>;
    int per_cu;
    int rc = prepare(kern, lds, &per_cu);
    if (rc) return rc;
    int grid = std::min(ea.n_gal, per_cu * c->num_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, ma, ba, ea);
    return hip_fail(hipGetLastError());
}

template <class F, int KT, int NG>
int launch_img_k(gm_ctx *c, const ModelArgs &ma, const BatchArgs &ba, const ImageArgs &ia, size_t lds, hipStream_t st)
{
    auto kern = image_kernel<F, KT, NG>;
    int per_cu;
    int rc = prepare(kern, lds, &per_cu);
    if (rc) return rc;
    int grid = std::min(ia.n_tiles, 4 * per_cu * c->num_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, ma, ba, ia);
    return hip_fail(hipGetLastError());
}

// Dispatch on the compile-time PSF side and the plane-group count.
#define GM_KT_NG_DISPATCH(LAUNCH, F, kt, ng, ...)                                              \
    ((kt) == 15 ? ((ng) == Groups<F>::a ? LAUNCH<F, 15, Groups<F>::a>(__VA_ARGS__)             \
                                        : LAUNCH<F, 15, Groups<F>::b>(__VA_ARGS__))            \
     : (kt) == 25 ? ((ng) == Groups<F>::a ? LAUNCH<F, 25, Groups<F>::a>(__VA_ARGS__)           \
                                          : LAUNCH<F, 25, Groups<F>::b>(__VA_ARGS__))          \
                  : ((ng) == Groups<F>::a ? LAUNCH<F, 0, Groups<F>::a>(__VA_ARGS__)            \
                                          : LAUNCH<F, 0, Groups<F>::b>(__VA_ARGS__)))

// ---------------------------------------------------------------- per-call drivers
template <class F>
int run_fit(gm_ctx *c, const ModelArgs &ma, const gm_batch *b, const gm_fit_opts *o, double *params, double *chi2,
            int32_t *niter, int32_t *status, hipStream_t st)
{
    int ng;
    size_t lds;
    int rc = pick_groups<F>(max_k(b), &ng, &lds);
    if (rc) return rc;
    // longest-processing-time order: biggest cutouts (times PSF area) first
    std::vector<int> order(b->n_gal);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> cost(b->n_gal);
    for (int g = 0; g < b->n_gal; ++g) cost[g] = (double)b->h[g] * b->w[g] * b->psf_k[g] * b->psf_k[g];
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    Staged sg;
    rc = stage(c, b, order.data(), sizeof(int) * (size_t)b->n_gal, st, &sg);
    if (rc) return rc;
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, st, sg.queue, 0);
    if (hipGetLastError() != hipSuccess) return GM_EHIP;
    BatchArgs ba{sg.meta, b->data, b->sigma, b->psf, b->omega};
    FitArgs fa{};
    fa.order = reinterpret_cast<const int *>(sg.extra);
    fa.n_gal = b->n_gal;
    fa.queue = sg.queue;
    fa.params = params;
    fa.chi2 = chi2;
    fa.niter = niter;
    fa.status = status;
    fa.max_iter = o ? o->max_iter : 100;
    fa.lambda0 = o ? o->lambda0 : 1e-3;
    fa.tol = o ? o->step_tol : 1e-4;
    return GM_KT_NG_DISPATCH(launch_fit_k, F, batch_kt(b), ng, c, ma, ba, fa, lds, st);
}

template <class F>
int run_errors(gm_ctx *c, const ModelArgs &ma, const gm_batch *b, const double *params, double *err, double *cov,
               hipStream_t st)
{
    int ng;
    size_t lds;
    int rc = pick_groups<F>(max_k(b), &ng, &lds);
    if (rc) return rc;
    Staged sg;
    rc = stage(c, b, nullptr, 0, st, &sg);
    if (rc) return rc;
    BatchArgs ba{sg.meta, b->data, b->sigma, b->psf, b->omega};
    ErrArgs ea{params, err, cov, b->n_gal};
    return GM_KT_NG_DISPATCH(launch_err_k, F, batch_kt(b), ng, c, ma, ba, ea, lds, st);
}

template <class F>
int run_image(gm_ctx *c, const ModelArgs &ma, const gm_batch *b, const double *params, float *out, int mode,
              hipStream_t st)
{
    int ng;
    size_t lds;
    int rc = pick_groups<F>(max_k(b), &ng, &lds);
    if (rc) return rc;
    std::vector<TileItem> tiles;
    for (int g = 0; g < b->n_gal; ++g)
        for (int ty = 0; ty < (b->h[g] + TILE - 1) / TILE; ++ty)
            for (int tx = 0; tx < (b->w[g] + TILE - 1) / TILE; ++tx) tiles.push_back({g, ty, tx, 0});
    Staged sg;
    rc = stage(c, b, tiles.data(), sizeof(TileItem) * tiles.size(), st, &sg);
    if (rc) return rc;
    BatchArgs ba{sg.meta, b->data, b->sigma, b->psf, b->omega};
    ImageArgs ia{reinterpret_cast<const TileItem *>(sg.extra), (int)tiles.size(), params, out, mode};
    return GM_KT_NG_DISPATCH(launch_img_k, F, batch_kt(b), ng, c, ma, ba, ia, lds, st);
}

template <class F>
int run_guess(gm_ctx *c, const ModelArgs &ma, const gm_batch *b, double *params, double *moments, hipStream_t st)
{
    Staged sg;
    int rc = stage(c, b, nullptr, 0, st, &sg);
    if (rc) return rc;
    BatchArgs ba{sg.meta, b->data, b->sigma, b->psf, b->omega};
    GuessArgs ga{params, moments, b->n_gal};
    int grid = std::min(b->n_gal, 8 * c->num_cu);
    hipLaunchKernelGGL(guess_kernel<F>, dim3(grid), dim3(NT), 0, st, ma, ba, ga);
    return hip_fail(hipGetLastError());
}

int prologue(gm_ctx *c, const gm_model *m, const gm_batch *b, Match &mt)
{
    if (!c) return GM_EINVAL;
    int rc = match_model(m, mt);
    if (rc) return rc;
    rc = check_batch(b);
    if (rc) return rc;
    if (b->n_gal > 0 && (!b->data || !b->sigma)) return GM_EINVAL;
    return GM_OK;
}

}  // namespace

extern "C" {

int gm_create(gm_ctx **out, int hip_device)
{
    if (!out) return GM_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return GM_EHIP;
    if (hip_device < 0 || hip_device >= n) return GM_EINVAL;
    Scoped sd(hip_device);
    gm_ctx *c = new (std::nothrow) gm_ctx();
    if (!c) return GM_ENOMEM;
    c->device = hip_device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess ||
        hipEventCreateWithFlags(&c->ws.staged, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return GM_EHIP;
    }
    c->num_cu = prop.multiProcessorCount;
    *out = c;
    return GM_OK;
}

void gm_destroy(gm_ctx *c)
{
    if (!c) return;
    Scoped sd(c->device);
    (void)hipDeviceSynchronize();
    if (c->ws.dev) (void)hipFree(c->ws.dev);
    if (c->ws.host) (void)hipHostFree(c->ws.host);
    if (c->ws.staged) (void)hipEventDestroy(c->ws.staged);
    delete c;
}

const char *gm_error_string(int code)
{
    switch (code) {
    case GM_OK: return "success";
    case GM_EINVAL: return "invalid argument";
    case GM_EHIP: return "HIP runtime call failed";
    case GM_ENOMEM: return "out of memory";
    case GM_EUNSUPPORTED: return "model or size not supported by the compiled kernels";
    default: return "unknown error";
    }
}

#define GM_DISPATCH(call_sersic, call_bd) \
    (mt.fam == FAM_SERSIC ? (call_sersic) : (call_bd))

int gm_model_image(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const double *params,
                   float *model_out, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (batch->n_gal == 0) return GM_OK;
    if (!params || !model_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    return GM_DISPATCH(run_image<FamSersic>(ctx, mt.ma, batch, params, model_out, 0, st),
                       run_image<FamBulgeDisk>(ctx, mt.ma, batch, params, model_out, 0, st));
}

int gm_jacobian(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const double *params, float *jac_out,
                void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (batch->n_gal == 0) return GM_OK;
    if (!params || !jac_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    return GM_DISPATCH(run_image<FamSersic>(ctx, mt.ma, batch, params, jac_out, 1, st),
                       run_image<FamBulgeDisk>(ctx, mt.ma, batch, params, jac_out, 1, st));
}

int gm_default_guess(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, double *params_out,
                     double *moments_out, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (batch->n_gal == 0) return GM_OK;
    if (!params_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    return GM_DISPATCH(run_guess<FamSersic>(ctx, mt.ma, batch, params_out, moments_out, st),
                       run_guess<FamBulgeDisk>(ctx, mt.ma, batch, params_out, moments_out, st));
}

int gm_fit_batch(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_fit_opts *opts,
                 double *params_inout, double *chi2_out, int32_t *niter_out, int32_t *status_out, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (opts && (opts->max_iter < 0 || !(opts->lambda0 > 0.0) || !(opts->step_tol > 0.0))) return GM_EINVAL;
    if (batch->n_gal == 0) return GM_OK;
    if (!params_inout || !chi2_out || !niter_out || !status_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    return GM_DISPATCH(
        run_fit<FamSersic>(ctx, mt.ma, batch, opts, params_inout, chi2_out, niter_out, status_out, st),
        run_fit<FamBulgeDisk>(ctx, mt.ma, batch, opts, params_inout, chi2_out, niter_out, status_out, st));
}

int gm_param_errors(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const double *params,
                    double *err_out, double *cov_out, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (batch->n_gal == 0) return GM_OK;
    if (!params || !err_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    return GM_DISPATCH(run_errors<FamSersic>(ctx, mt.ma, batch, params, err_out, cov_out, st),
                       run_errors<FamBulgeDisk>(ctx, mt.ma, batch, params, err_out, cov_out, st));
}

}  // extern "C"
