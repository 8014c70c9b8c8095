// gm_launch.h -- host-side drivers of the kernels, templated on the model
// family.  Each family is instantiated in a translation unit of its own
// (gm_fam_*.hip) so that the families compile in parallel; gm_abi.hip reaches
// them through a table of FamilyOps.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "gm_kernels.h"

struct gm_ctx {
    int device = 0;
    int num_cu = 0;
    void *dev = nullptr;          // grow-only device workspace
    size_t dev_bytes = 0;
    void *host = nullptr;         // pinned staging buffer
    size_t host_bytes = 0;
    hipEvent_t staged = nullptr;  // last copy out of the staging buffer
    bool pending = false;
    float *unit_psf = nullptr;    // device 1x1 kernel {1.0}: runs unconvolved models
    void *mlp_ws = nullptr;       // grow-only device workspace of the learned proposal
    size_t mlp_ws_bytes = 0;
    void *aux = nullptr;          // grow-only device scratch (adjoint partial sums)
    size_t aux_bytes = 0;
    void *team = nullptr;         // grow-only device scratch of fits shared by teams of workgroups
    size_t team_bytes = 0;
    int64_t wall_hz = 0;          // rate of the device's wall clock (team waits)
    struct Sched {
        int family, k, ng, wpc, team, team_min, team_wait_us;
    };
    std::vector<Sched> sched;     // gm_set_schedule entries
    // Set while a plan is being captured into a graph: staging then carves the
    // plan's own device arena and writes the bytes to a host image of it,
    // uploaded once the capture has ended (no copy or event enters the graph).
    struct Capture {
        char *arena = nullptr;
        size_t bytes = 0;
        size_t used = 0;
        std::vector<char> image;
    };
    Capture *capture = nullptr;
};

// A captured call sequence (gm_plan_fit, gm_plan_fit_learned): a private
// context whose workspaces only the graph's kernels use, the staging arena,
// the capture stream and the instantiated graph.
struct gm_plan {
    gm_ctx ctx;
    gm_ctx::Capture cap;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *ev[4] = {};       // timing events recorded as graph nodes (gm_plan_elapsed)
    bool launched = false;
};

namespace gm {

constexpr size_t kMaxLds = 160 * 1024;

// Everything a driver needs besides the family: the caller's batch (host
// metadata, device pixels), the matched model and whether the model is
// convolved (an unconvolved model runs with the 1x1 unit PSF).
struct CallInfo {
    const gm_batch *b;
    ModelArgs ma;
    bool convolved;
    int wpc = 0;          // persistent workgroups per CU (0: as many as are resident)
    int team = 0;         // workgroups per fit: 0 automatic, 1 one, k > 1 up to k (gm_schedule)
    int team_min = 1;     // fits with fewer tiles keep one workgroup when team > 1
    int team_wait_us = 0; // bound of a team's waits (0: 20 s)
};

// Device workspace of one call: [meta | extra | queue counter].
struct Staged {
    Meta *meta;
    void *extra;
    int *queue;
};

// Optional parts of a fit launch (FitArgs): the refit of galaxies whose first
// fit does not converge, bootstrap replicas, and metadata already on the
// device.
struct FitExtra {
    // non-null: meta, fit order (extra) and a zeroed queue counter already on
    // the device (gm_fit_batch_noalloc); no host ordering and no staging
    const Staged *pre = nullptr;
    const double *refit_start = nullptr;   // [n_gal][p] start of the refit
    const int *valid = nullptr;            // nullable: 0 = the first start is unusable
    int *refit_code = nullptr;             // nullable: 0 / 1 / 2 per galaxy
    int first_max_iter = 0;                // trials of the first fit
    int n_boot = 0;                        // > 0: n_boot replicas of each galaxy
    uint64_t boot_seed = 0;
};

// defined in gm_abi.hip
int stage(gm_ctx *c, const CallInfo &ci, const void *extra, size_t extra_bytes, hipStream_t st, Staged *out);
int batch_kt(const CallInfo &ci);
int max_k(const CallInfo &ci);
// grow-only device scratch of the context (stream-ordered reuse)
int ensure_aux(gm_ctx *c, size_t bytes, void **out);
int ensure_team(gm_ctx *c, size_t bytes, void **out);
// context set-up and release (gm_create, gm_destroy and plans)
int ctx_init(gm_ctx *c, int device);
void ctx_release(gm_ctx *c);
// records events[i] (if events is not null) on st; inside a capture as an
// event node of the graph
int mark_event(const gm_ctx *c, void *const *events, int i, hipStream_t st);
// Plans: plan_open makes the private context (the parent's schedule copied),
// an arena for `stages` stagings of n_gal galaxies and, when timing, the
// plan's four events (p->ev, NULL otherwise); plan_begin starts the
// capture on the plan's stream; plan_end ends it, uploads the arena and
// instantiates the graph when rc is GM_OK, and on any failure destroys the plan.
int plan_open(gm_ctx *parent, int n_gal, int stages, bool timing, gm_plan **out);
int plan_begin(gm_plan *p);
int plan_end(gm_plan *p, int rc, gm_plan **out);

inline int hip_rc(hipError_t e) { return e == hipSuccess ? GM_OK : GM_EHIP; }

inline BatchArgs batch_args(gm_ctx *c, const CallInfo &ci, const Staged &sg)
{
    return BatchArgs{sg.meta, ci.b->data, ci.b->sigma, ci.convolved ? ci.b->psf : c->unit_psf, ci.b->omega};
}

template <class F>
size_t static_lds()
{
    return sizeof(EvalShared<F>) + sizeof(LMShared<F>) + 64;
}

// Dynamic LDS for NG plane groups and PSF side K (lds_total_bytes).
template <class F, int NG>
size_t lds_bytes(int K)
{
    return lds_total_bytes<F, NG>(K);
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

// Workgroups of lm_fit_kernel<F, KT, NG> resident per CU at `lds` bytes of
// dynamic LDS.
template <class F, int NG, int KT>
int resident_fit(size_t lds, int *per_cu)
{
    return prepare(lm_fit_kernel<F, KT, NG>, lds, per_cu);
}

template <class F, int NG, int KT>
int launch_fit(gm_ctx *c, const ModelArgs &ma, const BatchArgs &ba, const FitArgs &fa, size_t lds, int wpc,
               hipStream_t st)
{
    auto kern = lm_fit_kernel<F, KT, NG>;
    int per_cu;
    int rc = prepare(kern, lds, &per_cu);
    if (rc) return rc;
    if (wpc > 0) per_cu = std::min(per_cu, wpc);
    int grid = std::min(fa.n_gal, per_cu * c->num_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, ma, ba, fa);
    return hip_rc(hipGetLastError());
}

// Gradient-descent fitter (gm_adam.h, included at the end)
struct AdamArgs;
template <class F, int NG, int KT>
int launch_adam(gm_ctx *c, const ModelArgs &ma, const BatchArgs &ba, AdamArgs aa, size_t lds, int wpc,
                int64_t psf_len, int64_t max_px, hipStream_t st);
template <class F, int NG, int... KTS>
int run_adam(gm_ctx *c, const CallInfo &ci, const gm_adam_opts *o, double *params, double *chi2, int32_t *status,
             hipStream_t st);

template <class F, int NG, int KT>
int launch_err(gm_ctx *c, const ModelArgs &ma, const BatchArgs &ba, const ErrArgs &ea, size_t lds, int wpc,
               hipStream_t st)
{
    auto kern = errors_kernel<F, KT, NG>;
    int per_cu;
    int rc = prepare(kern, lds, &per_cu);
    if (rc) return rc;
    if (wpc > 0) per_cu = std::min(per_cu, wpc);
    int grid = std::min(ea.n_gal, per_cu * c->num_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, ma, ba, ea);
    return hip_rc(hipGetLastError());
}

template <class F, int NG, int KT>
int launch_img(gm_ctx *c, const ModelArgs &ma, const BatchArgs &ba, const ImageArgs &ia, size_t lds, hipStream_t st)
{
    auto kern = image_kernel<F, KT, NG>;
    int per_cu;
    int rc = prepare(kern, lds, &per_cu);
    if (rc) return rc;
    int grid = std::min(ia.n_tiles, 4 * per_cu * c->num_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, ma, ba, ia);
    return hip_rc(hipGetLastError());
}

// Dispatch on the batch's compile-time PSF side: KT0 first, then the others.
template <class F, int NG, int... KTS>
struct Dispatch;
template <class F, int NG>
struct Dispatch<F, NG> {
    static int resident(int, size_t lds, int *per_cu) { return resident_fit<F, NG, 0>(lds, per_cu); }
    template <class... A> static int fit(int, A &&...a) { return launch_fit<F, NG, 0>(a...); }
    template <class... A> static int adam(int, A &&...a) { return launch_adam<F, NG, 0>(a...); }
    template <class... A> static int err(int, A &&...a) { return launch_err<F, NG, 0>(a...); }
    template <class... A> static int img(int, A &&...a) { return launch_img<F, NG, 0>(a...); }
};
template <class F, int NG, int K0, int... KR>
struct Dispatch<F, NG, K0, KR...> {
    static int resident(int kt, size_t lds, int *per_cu)
    {
        return kt == K0 ? resident_fit<F, NG, K0>(lds, per_cu) : Dispatch<F, NG, KR...>::resident(kt, lds, per_cu);
    }
    template <class... A> static int fit(int kt, A &&...a)
    {
        return kt == K0 ? launch_fit<F, NG, K0>(a...) : Dispatch<F, NG, KR...>::fit(kt, a...);
    }
    template <class... A> static int adam(int kt, A &&...a)
    {
        return kt == K0 ? launch_adam<F, NG, K0>(a...) : Dispatch<F, NG, KR...>::adam(kt, a...);
    }
    template <class... A> static int err(int kt, A &&...a)
    {
        return kt == K0 ? launch_err<F, NG, K0>(a...) : Dispatch<F, NG, KR...>::err(kt, a...);
    }
    template <class... A> static int img(int kt, A &&...a)
    {
        return kt == K0 ? launch_img<F, NG, K0>(a...) : Dispatch<F, NG, KR...>::img(kt, a...);
    }
};

template <class F, int NG>
int check_lds(int K, size_t *lds)
{
    *lds = lds_bytes<F, NG>(K);
    return (*lds + static_lds<F>() <= kMaxLds) ? GM_OK : GM_EUNSUPPORTED;
}

template <class F, int NG, int... KTS>
int run_fit(gm_ctx *c, const CallInfo &ci, const gm_fit_opts *o, double *params, double *chi2, int32_t *niter,
            int32_t *status, const FitExtra *ex, hipStream_t st)
{
    const gm_batch *b = ci.b;
    size_t lds;
    int rc = check_lds<F, NG>(max_k(ci), &lds);
    if (rc) return rc;
    // fit indices: the galaxies, or n_boot replicas of each (i -> galaxy i / n_boot)
    const int nb = (ex && ex->n_boot > 0) ? ex->n_boot : 1;
    const int nfit = b->n_gal * nb;
    Staged sg;
    const int kt = batch_kt(ci);
    int n_items = nfit;
    TeamItem *teams_items = nullptr;
    TeamCtl *team_ctl = nullptr;
    double *team_part = nullptr;
    int64_t part_stride = 0;
    if (ex && ex->pre) {
        if (nb != 1) return GM_EINVAL;
        sg = *ex->pre;
    } else {
        // longest-processing-time order: biggest cutouts (times PSF area) first
        std::vector<int> order(nfit);
        std::iota(order.begin(), order.end(), 0);
        std::vector<double> cost(b->n_gal);
        for (int g = 0; g < b->n_gal; ++g) {
            double k = ci.convolved ? b->psf_k[g] : 1.0;
            cost[g] = (double)b->h[g] * b->w[g] * k * k;
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x / nb] > cost[y / nb]; });
        // workgroups per fit (gm_schedule.team); a team is never larger than 32, so
        // that its workgroups are resident together whatever else runs on the GPU
        std::vector<int> tsz(nfit, 1);
        int gmax = 1, n_teams = 0;
        if (ci.team != 1) {
            int per_cu = 1;
            if ((rc = Dispatch<F, NG, KTS...>::resident(kt, lds, &per_cu))) return rc;
            if (ci.wpc > 0) per_cu = std::min(per_cu, ci.wpc);
            const int R = per_cu * std::max(c->num_cu, 1);
            for (int i = 0; i < nfit; ++i) {
                const int g = i / nb;
                const int tiles = ((b->h[g] + TILE - 1) / TILE) * ((b->w[g] + TILE - 1) / TILE);
                int G = 1;
                if (ci.team == 0)
                    G = nfit < R ? std::min({32, R / nfit, tiles}) : 1;
                else if (tiles >= ci.team_min)
                    G = std::min({ci.team, 32, tiles});
                tsz[i] = std::max(1, std::min(G, R));
                gmax = std::max(gmax, tsz[i]);
            }
        }
        if (gmax > 1) {
            std::vector<TeamItem> items;
            items.reserve(nfit);
            for (int i : order) {
                const int G = tsz[i];
                const int team = G > 1 ? n_teams++ : 0;
                for (int r = 0; r < G; ++r) items.push_back(TeamItem{i, r, G, team});
            }
            n_items = (int)items.size();
            constexpr int NR = 1 + F::P + F::P * (F::P + 1) / 2;
            part_stride = (int64_t)gmax * NR;
            const size_t ctl_bytes = (sizeof(TeamCtl) * (size_t)n_teams + 255) & ~(size_t)255;
            void *tw = nullptr;
            if ((rc = ensure_team(c, ctl_bytes + sizeof(double) * (size_t)part_stride * n_teams, &tw))) return rc;
            team_ctl = reinterpret_cast<TeamCtl *>(tw);
            team_part = reinterpret_cast<double *>(reinterpret_cast<char *>(tw) + ctl_bytes);
            rc = stage(c, ci, items.data(), sizeof(TeamItem) * items.size(), st, &sg);
            if (rc) return rc;
            teams_items = reinterpret_cast<TeamItem *>(sg.extra);
            const int nwords = (int)(sizeof(TeamCtl) / sizeof(int)) * n_teams;
            hipLaunchKernelGGL(fill_ints_kernel, dim3((nwords + 255) / 256), dim3(256), 0, st,
                               reinterpret_cast<int *>(team_ctl), nwords, 0);
            if (hipGetLastError() != hipSuccess) return GM_EHIP;
        } else {
            rc = stage(c, ci, order.data(), sizeof(int) * (size_t)nfit, st, &sg);
            if (rc) return rc;
        }
        hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, st, sg.queue, 0);
        if (hipGetLastError() != hipSuccess) return GM_EHIP;
    }
    FitArgs fa{};
    fa.order = teams_items ? nullptr : reinterpret_cast<const int *>(sg.extra);
    fa.items = teams_items;
    fa.ctl = team_ctl;
    fa.part = team_part;
    fa.part_stride = part_stride;
    const int64_t hz = std::max<int64_t>(c->wall_hz, 1000000);
    fa.spin_limit = ci.team_wait_us > 0 ? std::max<int64_t>(1, hz * ci.team_wait_us / 1000000) : 20 * hz;
    fa.active = o ? o->active : nullptr;
    fa.n_gal = n_items;
    fa.queue = sg.queue;
    fa.params = params;
    fa.chi2 = chi2;
    fa.niter = niter;
    fa.status = status;
    fa.err = o ? o->err_out : nullptr;
    fa.max_iter = o ? o->max_iter : 100;
    fa.lambda0 = o ? o->lambda0 : 1e-3;
    fa.tol = o ? o->step_tol : 1e-4;
    if (ex) {
        fa.refit_start = ex->refit_start;
        fa.valid = ex->valid;
        fa.refit_code = ex->refit_code;
        fa.first_max_iter = ex->first_max_iter;
        fa.n_boot = ex->n_boot;
        fa.boot_k0 = (uint32_t)ex->boot_seed;
        fa.boot_k1 = (uint32_t)(ex->boot_seed >> 32);
    }
    return Dispatch<F, NG, KTS...>::fit(kt, c, ci.ma, batch_args(c, ci, sg), fa, lds, ci.wpc, st);
}

template <class F, int NG, int... KTS>
int run_errors(gm_ctx *c, const CallInfo &ci, const double *params, double *err, double *cov, hipStream_t st)
{
    size_t lds;
    int rc = check_lds<F, NG>(max_k(ci), &lds);
    if (rc) return rc;
    Staged sg;
    rc = stage(c, ci, nullptr, 0, st, &sg);
    if (rc) return rc;
    ErrArgs ea{params, err, cov, ci.b->n_gal};
    return Dispatch<F, NG, KTS...>::err(batch_kt(ci), c, ci.ma, batch_args(c, ci, sg), ea, lds, ci.wpc, st);
}

template <class F, int NG, int... KTS>
int run_image(gm_ctx *c, const CallInfo &ci, const double *params, float *out, int mode, hipStream_t st)
{
    const gm_batch *b = ci.b;
    size_t lds;
    int rc = check_lds<F, NG>(max_k(ci), &lds);
    if (rc) return rc;
    std::vector<TileItem> tiles;
    for (int g = 0; g < b->n_gal; ++g)
        for (int ty = 0; ty < (b->h[g] + TILE - 1) / TILE; ++ty)
            for (int tx = 0; tx < (b->w[g] + TILE - 1) / TILE; ++tx) tiles.push_back({g, ty, tx, 0});
    Staged sg;
    rc = stage(c, ci, tiles.data(), sizeof(TileItem) * tiles.size(), st, &sg);
    if (rc) return rc;
    ImageArgs ia{reinterpret_cast<const TileItem *>(sg.extra), (int)tiles.size(), params, out, mode, nullptr, nullptr};
    return Dispatch<F, NG, KTS...>::img(batch_kt(ci), c, ci.ma, batch_args(c, ci, sg), ia, lds, st);
}

// Adjoint of the model image: grad[g][c] = sum_pixels dM/dp_c * gin (natural
// units), per-tile FP64 partials then a per-galaxy sum in tile order.
template <class F, int NG, int... KTS>
int run_vjp(gm_ctx *c, const CallInfo &ci, const double *params, const float *gin, double *grad, hipStream_t st)
{
    const gm_batch *b = ci.b;
    size_t lds;
    int rc = check_lds<F, NG>(max_k(ci), &lds);
    if (rc) return rc;
    std::vector<TileItem> tiles;
    std::vector<int> tstart(b->n_gal + 1, 0);
    for (int g = 0; g < b->n_gal; ++g) {
        tstart[g] = (int)tiles.size();
        for (int ty = 0; ty < (b->h[g] + TILE - 1) / TILE; ++ty)
            for (int tx = 0; tx < (b->w[g] + TILE - 1) / TILE; ++tx) tiles.push_back({g, ty, tx, 0});
    }
    tstart[b->n_gal] = (int)tiles.size();
    const size_t tb = sizeof(TileItem) * tiles.size();
    std::vector<char> blob(tb + sizeof(int) * tstart.size());
    memcpy(blob.data(), tiles.data(), tb);
    memcpy(blob.data() + tb, tstart.data(), sizeof(int) * tstart.size());
    double *part = nullptr;
    rc = ensure_aux(c, sizeof(double) * F::P * tiles.size(), reinterpret_cast<void **>(&part));
    if (rc) return rc;
    Staged sg;
    rc = stage(c, ci, blob.data(), blob.size(), st, &sg);
    if (rc) return rc;
    ImageArgs ia{reinterpret_cast<const TileItem *>(sg.extra), (int)tiles.size(), params, nullptr, 2, gin, part};
    rc = Dispatch<F, NG, KTS...>::img(batch_kt(ci), c, ci.ma, batch_args(c, ci, sg), ia, lds, st);
    if (rc) return rc;
    const int *ts = reinterpret_cast<const int *>(reinterpret_cast<const char *>(sg.extra) + tb);
    hipLaunchKernelGGL(vjp_reduce_kernel, dim3((b->n_gal + 255) / 256), dim3(256), 0, st, b->n_gal, F::P, ci.ma, ts,
                       part, grad);
    return hip_rc(hipGetLastError());
}

template <class F>
int run_guess(gm_ctx *c, const CallInfo &ci, double *params, double *moments, hipStream_t st)
{
    Staged sg;
    int rc = stage(c, ci, nullptr, 0, st, &sg);
    if (rc) return rc;
    GuessArgs ga{params, moments, ci.b->n_gal};
    int grid = std::min(ci.b->n_gal, 8 * c->num_cu);
    hipLaunchKernelGGL(guess_kernel<F>, dim3(grid), dim3(NT), 0, st, ci.ma, batch_args(c, ci, sg), ga);
    return hip_rc(hipGetLastError());
}

// Default starts from moments already stored by the feature pass (mom8, pk:
// device arrays of n_gal x 8 and n_gal doubles).
template <class F>
int run_guess_stored(gm_ctx *, const CallInfo &ci, const double *mom8, const double *pk, double *params,
                     hipStream_t st)
{
    const int n = ci.b->n_gal;
    if (n <= 0) return GM_OK;
    hipLaunchKernelGGL(guess_stored_kernel<F>, dim3((n + 255) / 256), dim3(256), 0, st, ci.ma, n, mom8, pk, params);
    return hip_rc(hipGetLastError());
}

template <class F, int NG>
size_t variant_lds(int K)
{
    return lds_bytes<F, NG>(K) + static_lds<F>();
}

// Entry points of one family compiled with NG plane groups.
struct Variant {
    int ng = 0;
    size_t (*lds)(int K) = nullptr;     // LDS bytes per workgroup at PSF side K
    int (*fit)(gm_ctx *, const CallInfo &, const gm_fit_opts *, double *, double *, int32_t *, int32_t *,
               const FitExtra *, hipStream_t) = nullptr;
    int (*errors)(gm_ctx *, const CallInfo &, const double *, double *, double *, hipStream_t) = nullptr;
    int (*image)(gm_ctx *, const CallInfo &, const double *, float *, int, hipStream_t) = nullptr;
    int (*guess)(gm_ctx *, const CallInfo &, double *, double *, hipStream_t) = nullptr;
    int (*guess_stored)(gm_ctx *, const CallInfo &, const double *, const double *, double *, hipStream_t) = nullptr;
    int (*vjp)(gm_ctx *, const CallInfo &, const double *, const float *, double *, hipStream_t) = nullptr;
    int (*adam)(gm_ctx *, const CallInfo &, const gm_adam_opts *, double *, double *, int32_t *,
                hipStream_t) = nullptr;
};

template <class F, int NG, int... KTS>
Variant make_variant()
{
    Variant v;
    v.ng = NG;
    v.lds = variant_lds<F, NG>;
    v.fit = run_fit<F, NG, KTS...>;
    v.errors = run_errors<F, NG, KTS...>;
    v.image = run_image<F, NG, KTS...>;
    v.guess = run_guess<F>;
    v.guess_stored = run_guess_stored<F>;
    v.vjp = run_vjp<F, NG, KTS...>;
    v.adam = run_adam<F, NG, KTS...>;
    return v;
}

// A model family: its compiled variants in order of preference (the first
// whose LDS fits is the default schedule).
constexpr int kMaxVariants = 3;
struct FamilyOps {
    int id = 0;
    int n = 0;
    Variant v[kMaxVariants];
};

// variants, one per translation unit (gm_fam_*.hip)
Variant var_sersic_1();
Variant var_sersic_2();
Variant var_bulgedisk_2();
Variant var_bulgedisk_3();
Variant var_sersicbar_2();
Variant var_sersicbar_3();
Variant var_expdisk_1();
Variant var_expdisk_2();
Variant var_ferrer_1();
Variant var_ferrer_2();
Variant var_king_1();
Variant var_king_2();
Variant var_gaussian_1();
Variant var_gaussian_2();
Variant var_moffat_2();
Variant var_sersictilt_1();
Variant var_sersictilt_2();
Variant var_sersicbox_1();
Variant var_sersicbox_2();
Variant var_ferrerfree_1();
Variant var_ferrerfree_2();
Variant var_kingfree_1();
Variant var_kingfree_2();

// A caller's gm_model matched against the compiled families (gm_abi.hip).
struct Match {
    const FamilyOps *ops = nullptr;
    CallInfo ci{};
    int single_type = 0;      // profile type of a one-component model, else 0
    bool has_sky = false;
    bool tilt = false;        // the sky is the tilted plane
    bool box = false;         // a Sersic with boxiness (B free or not 0)
};
int match_model(const gm_model *m, Match &out);
int check_batch(const gm_batch *b, bool convolved);
// validate context, model and batch; fills mt (mt.ci.b = b)
int prologue(gm_ctx *c, const gm_model *m, const gm_batch *b, Match &mt);
// the variant a call runs with (context schedule, else the family default);
// sets mt.ci.wpc.  GM_EUNSUPPORTED when no variant fits the batch's PSF side.
int pick_variant(gm_ctx *c, Match &mt, const Variant **out);

// makes the context's device current for the scope of a call
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

}  // namespace gm

#include "gm_adam.h"
