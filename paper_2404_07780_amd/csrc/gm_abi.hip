// gm_abi.hip -- host side of libgmfit: the C ABI declared in include/gmfit.h.
//
// Every call validates its arguments, matches the caller's gm_model against a
// compiled model family (mapping the family's internal LM vector onto the
// caller's parameter columns), stages the host-side size metadata into the
// context's grow-only device workspace and launches one kernel on the caller's
// stream.  Nothing is allocated once the workspace has grown to the largest
// batch seen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "gm_launch.h"

using namespace gm;

// Device scratch of gm_fit_batch_noalloc, for callers that cannot allocate:
// per galaxy its Meta record (32 B), its fit order (4 B) and the raw size
// metadata copied from the caller's host arrays (h, w, PSF side: 4 B each;
// image and PSF offsets: 8 B each), plus the work-queue counter.  Every GPU
// holds its own copy until the process ends; host code reaches it only
// through the address resolved per device at context set-up.
constexpr int kNoAllocMaxGal = GM_NOALLOC_MAX_GAL;
constexpr size_t kNaMeta = (size_t)kNoAllocMaxGal * sizeof(Meta);
constexpr size_t kNaOrder = (size_t)kNoAllocMaxGal * sizeof(int32_t);
constexpr size_t kNaQueue = 256;
constexpr size_t kNaRaw32 = (size_t)kNoAllocMaxGal * sizeof(int32_t);
constexpr size_t kNaRaw64 = (size_t)kNoAllocMaxGal * sizeof(int64_t);
constexpr size_t kNoAllocBytes = kNaMeta + kNaOrder + kNaQueue + 3 * kNaRaw32 + 2 * kNaRaw64;
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices];        // device address of `scratch` on each GPU
std::mutex g_scratch_mu;

// With `device` current: resolve the device address of `scratch` once.
int resolve_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return GM_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return GM_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GM_EHIP;
    g_scratch[device] = ptr;
    return GM_OK;
}

void *scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[device];
}

// Meta records of the raw host-copied sizes, the identity fit order and a
// zero work-queue counter (a kernel, not a memset: callers may capture it).
__global__ void noalloc_pack_kernel(int n, int convolved, const int32_t *h, const int32_t *w, const int32_t *k,
                                    const int64_t *img_off, const int64_t *psf_off, Meta *meta, int *order,
                                    int *queue)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *queue = 0;
    if (i >= n) return;
    Meta m;
    m.h = h[i];
    m.w = w[i];
    m.k = convolved ? k[i] : 1;
    m.pad = 0;
    m.img_off = img_off[i];
    m.psf_off = convolved ? psf_off[i] : 0;
    meta[i] = m;
    order[i] = i;
}

}  // namespace

namespace gm {

namespace {

int ensure_dev(gm_ctx *c, size_t bytes)
{
    if (c->dev_bytes >= bytes) return GM_OK;
    if (c->dev) {
        if (hipDeviceSynchronize() != hipSuccess) return GM_EHIP;
        (void)hipFree(c->dev);
        c->dev = nullptr;
        c->dev_bytes = 0;
    }
    size_t nb = std::max(bytes, (size_t)1 << 20);
    if (hipMalloc(&c->dev, nb) != hipSuccess) return GM_ENOMEM;
    c->dev_bytes = nb;
    return GM_OK;
}

int ensure_host(gm_ctx *c, size_t bytes)
{
    if (c->pending) {
        if (hipEventSynchronize(c->staged) != hipSuccess) return GM_EHIP;
        c->pending = false;
    }
    if (c->host_bytes >= bytes) return GM_OK;
    if (c->host) (void)hipHostFree(c->host);
    c->host = nullptr;
    c->host_bytes = 0;
    size_t nb = std::max(bytes, (size_t)1 << 20);
    if (hipHostMalloc(&c->host, nb, hipHostMallocDefault) != hipSuccess) return GM_ENOMEM;
    c->host_bytes = nb;
    return GM_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int ensure_aux(gm_ctx *c, size_t bytes, void **out)
{
    if (c->aux_bytes < bytes) {
        if (c->aux) {
            if (hipDeviceSynchronize() != hipSuccess) return GM_EHIP;
            (void)hipFree(c->aux);
            c->aux = nullptr;
            c->aux_bytes = 0;
        }
        size_t nb = std::max(bytes, (size_t)1 << 20);
        if (hipMalloc(&c->aux, nb) != hipSuccess) return GM_ENOMEM;
        c->aux_bytes = nb;
    }
    *out = c->aux;
    return GM_OK;
}

int ensure_team(gm_ctx *c, size_t bytes, void **out)
{
    if (c->team_bytes < bytes) {
        if (c->team) {
            if (hipDeviceSynchronize() != hipSuccess) return GM_EHIP;
            (void)hipFree(c->team);
            c->team = nullptr;
            c->team_bytes = 0;
        }
        size_t nb = std::max(bytes, (size_t)1 << 20);
        if (hipMalloc(&c->team, nb) != hipSuccess) return GM_ENOMEM;
        c->team_bytes = nb;
    }
    *out = c->team;
    return GM_OK;
}

int stage(gm_ctx *c, const CallInfo &ci, const void *extra, size_t extra_bytes, hipStream_t st, Staged *out)
{
    const gm_batch *b = ci.b;
    size_t mb_al = align256(sizeof(Meta) * (size_t)b->n_gal);
    size_t ex_al = align256(extra_bytes);
    size_t q_off = mb_al + ex_al;
    char *hp, *dp;
    gm_ctx::Capture *cap = c->capture;
    if (cap) {
        // plan capture: a fresh piece of the plan's arena, filled on the host now
        // and uploaded after the capture
        if (cap->used + q_off + 256 > cap->bytes) return GM_ENOMEM;
        hp = cap->image.data() + cap->used;
        dp = cap->arena + cap->used;
        cap->used += q_off + 256;
    } else {
        int rc = ensure_host(c, mb_al + ex_al);
        if (rc) return rc;
        rc = ensure_dev(c, q_off + 256);
        if (rc) return rc;
        hp = reinterpret_cast<char *>(c->host);
        dp = reinterpret_cast<char *>(c->dev);
    }
    Meta *hm = reinterpret_cast<Meta *>(hp);
    for (int g = 0; g < b->n_gal; ++g) {
        hm[g].h = b->h[g];
        hm[g].w = b->w[g];
        hm[g].k = ci.convolved ? b->psf_k[g] : 1;
        hm[g].pad = 0;
        hm[g].img_off = b->img_off[g];
        hm[g].psf_off = ci.convolved ? b->psf_off[g] : 0;
    }
    if (extra_bytes) memcpy(hp + mb_al, extra, extra_bytes);
    if (!cap) {
        if (hipMemcpyAsync(c->dev, c->host, mb_al + ex_al, hipMemcpyHostToDevice, st) != hipSuccess) return GM_EHIP;
        if (hipEventRecord(c->staged, st) != hipSuccess) return GM_EHIP;
        c->pending = true;
    }
    out->meta = reinterpret_cast<Meta *>(dp);
    out->extra = dp + mb_al;
    out->queue = reinterpret_cast<int *>(dp + q_off);
    return GM_OK;
}

int mark_event(const gm_ctx *c, void *const *events, int i, hipStream_t st)
{
    if (!events) return GM_OK;
    if (!c->capture) return hip_rc(hipEventRecord((hipEvent_t)events[i], st));
    // inside a capture: an event-record node after the nodes captured so far,
    // made the stream's capture dependency so that later work follows it
    hipStreamCaptureStatus cs;
    unsigned long long id;
    hipGraph_t g;
    const hipGraphNode_t *deps;
    size_t nd;
    if (hipStreamGetCaptureInfo_v2(st, &cs, &id, &g, &deps, &nd) != hipSuccess ||
        cs != hipStreamCaptureStatusActive)
        return GM_EHIP;
    hipGraphNode_t node;
    if (hipGraphAddEventRecordNode(&node, g, deps, nd, (hipEvent_t)events[i]) != hipSuccess) return GM_EHIP;
    return hip_rc(hipStreamUpdateCaptureDependencies(st, &node, 1, hipStreamSetCaptureDependencies));
}

int ctx_init(gm_ctx *c, int device)
{
    c->device = device;
    hipDeviceProp_t prop;
    const float one = 1.0f;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess ||
        hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&c->unit_psf, sizeof(float)) != hipSuccess ||
        hipMemcpy(c->unit_psf, &one, sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        ctx_release(c);
        return GM_EHIP;
    }
    c->num_cu = prop.multiProcessorCount;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0) khz = 100000;
    c->wall_hz = (int64_t)khz * 1000;
    if (resolve_scratch(device) != GM_OK) {
        ctx_release(c);
        return GM_EHIP;
    }
    return GM_OK;
}

void ctx_release(gm_ctx *c)
{
    if (c->dev) (void)hipFree(c->dev);
    if (c->host) (void)hipHostFree(c->host);
    if (c->unit_psf) (void)hipFree(c->unit_psf);
    if (c->mlp_ws) (void)hipFree(c->mlp_ws);
    if (c->aux) (void)hipFree(c->aux);
    if (c->team) (void)hipFree(c->team);
    if (c->staged) (void)hipEventDestroy(c->staged);
    c->dev = c->host = c->mlp_ws = c->aux = c->team = nullptr;
    c->unit_psf = nullptr;
    c->staged = nullptr;
    c->dev_bytes = c->host_bytes = c->mlp_ws_bytes = c->aux_bytes = c->team_bytes = 0;
}

namespace {

void plan_free(gm_plan *p)
{
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->stream) (void)hipStreamDestroy(p->stream);
    if (p->cap.arena) (void)hipFree(p->cap.arena);
    for (void *e : p->ev)
        if (e) (void)hipEventDestroy((hipEvent_t)e);
    ctx_release(&p->ctx);
    delete p;
}

}  // namespace

int plan_open(gm_ctx *parent, int n_gal, int stages, bool timing, gm_plan **out)
{
    *out = nullptr;
    gm_plan *p = new (std::nothrow) gm_plan();
    if (!p) return GM_ENOMEM;
    int rc = ctx_init(&p->ctx, parent->device);
    if (rc) {
        delete p;
        return rc;
    }
    p->ctx.sched = parent->sched;
    // per staging: metadata, the largest extra a plan stages (the LPT order, or
    // the queue entries of fits shared by teams of workgroups: at most the
    // largest team size of the schedules per fit, or fits + 4096 in the
    // automatic mode, which forms teams only below the resident workgroups)
    // and the queue counter
    size_t team_cap = 1;
    for (const auto &e : parent->sched)
        if (e.team > 1) team_cap = std::max(team_cap, (size_t)std::min(e.team, 32));
    const size_t items = std::max((size_t)n_gal * team_cap, (size_t)n_gal + 4096);
    const size_t extra = std::max(sizeof(int) * (size_t)n_gal, sizeof(TeamItem) * items);
    const size_t per = align256(sizeof(Meta) * (size_t)n_gal) + align256(extra) + 256;
    p->cap.bytes = per * (size_t)stages;
    try {
        p->cap.image.assign(p->cap.bytes, 0);
    } catch (...) {
        plan_free(p);
        return GM_ENOMEM;
    }
    if (hipMalloc(&p->cap.arena, p->cap.bytes) != hipSuccess) {
        p->cap.arena = nullptr;
        plan_free(p);
        return GM_ENOMEM;
    }
    if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
        p->stream = nullptr;
        plan_free(p);
        return GM_EHIP;
    }
    for (int i = 0; timing && i < 4; ++i) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            plan_free(p);
            return GM_EHIP;
        }
        p->ev[i] = e;
    }
    *out = p;
    return GM_OK;
}

int plan_begin(gm_plan *p)
{
    if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeRelaxed) != hipSuccess) return GM_EHIP;
    p->ctx.capture = &p->cap;
    return GM_OK;
}

int plan_end(gm_plan *p, int rc, gm_plan **out)
{
    *out = nullptr;
    if (p->ctx.capture) {
        p->ctx.capture = nullptr;
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(p->stream, &g) != hipSuccess && rc == GM_OK) rc = GM_EHIP;
        p->graph = g;
        if (!g && rc == GM_OK) rc = GM_EHIP;
    }
    if (rc == GM_OK &&
        hipMemcpy(p->cap.arena, p->cap.image.data(), p->cap.used, hipMemcpyHostToDevice) != hipSuccess)
        rc = GM_EHIP;
    if (rc == GM_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
        p->exec = nullptr;
        rc = GM_EHIP;
    }
    if (rc != GM_OK) {
        (void)hipGetLastError();
        plan_free(p);
        return rc;
    }
    *out = p;
    return GM_OK;
}

// PSF side shared by the whole batch, else 0 (a family without a compile-time
// kernel for that side takes its generic kernel).
int batch_kt(const CallInfo &ci)
{
    const gm_batch *b = ci.b;
    if (!ci.convolved || b->n_gal == 0) return 0;
    int k0 = b->psf_k[0];
    for (int g = 1; g < b->n_gal; ++g)
        if (b->psf_k[g] != k0) return 0;
    return k0;
}

int max_k(const CallInfo &ci)
{
    int k = 1;
    if (ci.convolved)
        for (int g = 0; g < ci.b->n_gal; ++g) k = std::max(k, ci.b->psf_k[g]);
    return k;
}

}  // namespace gm

namespace {

// Natural slots per profile type (index = type), the LM slots among them in
// the plain families, and the first slot that is always fixed (Moffat beta).
// The Sersic's eighth slot, the boxiness B of eq. (r), runs in the boxy
// family when free or not 0; the shape exponents Ferrer a, b and King alpha
// are fixed constants of the plain families and, when any is a column, LM
// variables of the free-shape families.
const int kSlots[9] = {0, 8, 6, 8, 8, 6, 7, 1, 3};
const int kLmSlots[9] = {0, 7, 6, 6, 7, 6, 6, 1, 3};
const int kShape0[9] = {0, 8, 6, 8, 8, 6, 6, 1, 3};

bool boxy(const gm_component &c) { return c.type == GM_SERSIC && (c.param_index[7] >= 0 || c.fixed[7] != 0.0); }
bool free_shape(const gm_component &c)
{
    return (c.type == GM_FERRER && (c.param_index[6] >= 0 || c.param_index[7] >= 0)) ||
           (c.type == GM_KING && c.param_index[7] >= 0);
}

bool comp_ok(const gm_component &c, int p)
{
    if (c.type < GM_SERSIC || c.type > GM_SKYPLANE) return false;
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

// internal index k <- slot s of component c
void take(const gm_component &c, int s, int k, ModelArgs &ma)
{
    ma.col[k] = c.param_index[s];
    ma.fixedv[k] = c.fixed[s];
}

// Family tables (variants in order of preference), built once.
enum {
    FAM_SERSIC = 1, FAM_EXPDISK, FAM_FERRER, FAM_KING, FAM_GAUSSIAN, FAM_MOFFAT, FAM_BULGEDISK, FAM_SERSICBAR,
    FAM_SERSICTILT, FAM_SERSICBOX, FAM_FERRERFREE, FAM_KINGFREE
};

FamilyOps family(int id, Variant a, Variant b)
{
    FamilyOps f;
    f.id = id;
    f.n = 2;
    f.v[0] = a;
    f.v[1] = b;
    return f;
}

FamilyOps family(int id, Variant a)
{
    FamilyOps f;
    f.id = id;
    f.n = 1;
    f.v[0] = a;
    return f;
}

const FamilyOps *family_table(int id)
{
    static const FamilyOps tab[] = {
        family(FAM_SERSIC, var_sersic_1(), var_sersic_2()),
        family(FAM_EXPDISK, var_expdisk_1(), var_expdisk_2()),
        family(FAM_FERRER, var_ferrer_1(), var_ferrer_2()),
        family(FAM_KING, var_king_1(), var_king_2()),
        family(FAM_GAUSSIAN, var_gaussian_1(), var_gaussian_2()),
        // one plane group is not built for Moffat: that variant gave wrong images and then a
        // memory fault at PSF side 25 with no cause found in its source
        family(FAM_MOFFAT, var_moffat_2()),
        family(FAM_BULGEDISK, var_bulgedisk_2(), var_bulgedisk_3()),
        family(FAM_SERSICBAR, var_sersicbar_2(), var_sersicbar_3()),
        family(FAM_SERSICTILT, var_sersictilt_1(), var_sersictilt_2()),
        family(FAM_SERSICBOX, var_sersicbox_1(), var_sersicbox_2()),
        family(FAM_FERRERFREE, var_ferrerfree_1(), var_ferrerfree_2()),
        family(FAM_KINGFREE, var_kingfree_1(), var_kingfree_2()),
    };
    // indexed by id: the entries are in FAM_* order
    static_assert(sizeof(tab) / sizeof(tab[0]) == FAM_KINGFREE, "family table out of order");
    return &tab[id - 1];
}

const FamilyOps *single_ops(int type)
{
    switch (type) {
    case GM_SERSIC: return family_table(FAM_SERSIC);
    case GM_EXPDISK: return family_table(FAM_EXPDISK);
    case GM_FERRER: return family_table(FAM_FERRER);
    case GM_KING: return family_table(FAM_KING);
    case GM_GAUSSIAN: return family_table(FAM_GAUSSIAN);
    default: return family_table(FAM_MOFFAT);
    }
}

}  // namespace

namespace gm {

int match_model(const gm_model *m, Match &out)
{
    if (!m || m->n_comp < 1 || m->n_comp > 4 || m->p < 1 || m->p > MAXP) return GM_EINVAL;
    if (m->oversample < 1 || m->oversample > MAXOSF || m->os_window < 0 || m->os_window > 5 ||
        (m->os_window > 0 && (m->os_window & 1) == 0) || !std::isfinite(m->m0))
        return GM_EINVAL;
    const gm_component *rad[4], *sky = nullptr;
    int nrad = 0;
    for (int i = 0; i < m->n_comp; ++i) {
        const gm_component &c = m->comp[i];
        if (!comp_ok(c, m->p)) return GM_EINVAL;
        if (c.type == GM_SKY || c.type == GM_SKYPLANE) {
            if (c.convolve) return GM_EINVAL;
            if (sky) return GM_EUNSUPPORTED;
            sky = &c;
        } else {
            rad[nrad++] = &c;
        }
    }
    // every column must be referenced by some slot
    int seen[MAXP] = {};
    for (int i = 0; i < m->n_comp; ++i)
        for (int s = 0; s < kSlots[m->comp[i].type]; ++s)
            if (m->comp[i].param_index[s] >= 0) seen[m->comp[i].param_index[s]] = 1;
    for (int k = 0; k < m->p; ++k)
        if (!seen[k]) return GM_EINVAL;
    if (nrad < 1 || nrad > 2) return GM_EUNSUPPORTED;
    // shape constants (Ferrer a, b; King alpha; Moffat beta) must be fixed
    for (int i = 0; i < nrad; ++i)
        for (int s = kShape0[rad[i]->type]; s < kSlots[rad[i]->type]; ++s)
            if (rad[i]->param_index[s] >= 0) return GM_EUNSUPPORTED;
    ModelArgs ma{};
    ma.p = m->p;
    ma.m0 = m->m0;
    ma.osf = m->oversample;
    ma.osw = m->oversample > 1 ? m->os_window : 0;
    for (int k = 0; k < MAXP; ++k) {
        ma.col[k] = -1;
        ma.fixedv[k] = 0.0;
    }
    ma.nflux = 0;
    for (int i = 0; i < nrad; ++i)
        if (rad[i]->param_index[2] >= 0) ma.nflux++;
    int nint;
    bool convolved = true;
    const FamilyOps *ops;
    if (nrad == 1) {
        const gm_component &c = *rad[0];
        convolved = c.convolve != 0;
        const bool bx = boxy(c), fs = free_shape(c);
        int ns = (bx || fs) ? 8 : kLmSlots[c.type];
        for (int s = 0; s < ns; ++s) take(c, s, s, ma);
        for (int s = ns; s < kSlots[c.type]; ++s) ma.cst[s - ns] = c.fixed[s];
        if (bx || fs) {
            // the boxy Sersic and the free-shape Ferrer and King are compiled with a flat sky
            if (sky && sky->type == GM_SKYPLANE) return GM_EUNSUPPORTED;
            if (sky) take(*sky, 0, ns, ma);
            nint = ns + 1;
            ops = family_table(bx ? FAM_SERSICBOX : c.type == GM_FERRER ? FAM_FERRERFREE : FAM_KINGFREE);
        } else if (sky && sky->type == GM_SKYPLANE) {
            // the tilted-plane sky is compiled for a single Sersic
            if (c.type != GM_SERSIC) return GM_EUNSUPPORTED;
            for (int s = 0; s < 3; ++s) take(*sky, s, ns + s, ma);
            nint = ns + 3;
            ops = family_table(FAM_SERSICTILT);
        } else {
            if (sky) take(*sky, 0, ns, ma);
            nint = ns + 1;
            ops = single_ops(c.type);
        }
    } else {
        // Sersic + (exponential disk | Ferrer) with a shared centre, both convolved
        const gm_component *a = rad[0], *b = rad[1];
        if (sky && sky->type == GM_SKYPLANE) return GM_EUNSUPPORTED;
        if (boxy(*a) || boxy(*b) || free_shape(*a) || free_shape(*b)) return GM_EUNSUPPORTED;
        if (b->type == GM_SERSIC) std::swap(a, b);
        if (a->type != GM_SERSIC || !(b->type == GM_EXPDISK || b->type == GM_FERRER) || !a->convolve ||
            !b->convolve)
            return GM_EUNSUPPORTED;
        for (int s = 0; s < 2; ++s) {
            if (a->param_index[s] != b->param_index[s]) return GM_EUNSUPPORTED;
            if (a->param_index[s] < 0 && a->fixed[s] != b->fixed[s]) return GM_EUNSUPPORTED;
        }
        for (int s = 0; s < 7; ++s) take(*a, s, s, ma);
        int nb = kLmSlots[b->type];
        for (int s = 2; s < nb; ++s) take(*b, s, 5 + s, ma);
        for (int s = nb; s < kSlots[b->type]; ++s) ma.cst[2 + s - nb] = b->fixed[s];
        nint = 7 + nb - 2 + 1;
        if (sky) take(*sky, 0, nint - 1, ma);
        ops = family_table(b->type == GM_EXPDISK ? FAM_BULGEDISK : FAM_SERSICBAR);
    }
    // a column used by two internal variables would be an unsupported tie
    int used[MAXP] = {};
    for (int k = 0; k < nint; ++k)
        if (ma.col[k] >= 0 && used[ma.col[k]]++) return GM_EUNSUPPORTED;
    out.ops = ops;
    out.ci.ma = ma;
    out.ci.convolved = convolved;
    out.single_type = nrad == 1 ? rad[0]->type : 0;
    out.has_sky = sky != nullptr;
    out.tilt = sky != nullptr && sky->type == GM_SKYPLANE;
    out.box = nrad == 1 && boxy(*rad[0]);
    return GM_OK;
}

int check_batch(const gm_batch *b, bool convolved)
{
    if (!b || b->n_gal < 0) return GM_EINVAL;
    if (b->n_gal == 0) return GM_OK;
    if (!b->h || !b->w || !b->img_off || !b->data || !b->sigma) return GM_EINVAL;
    if (convolved && (!b->psf_k || !b->psf_off || !b->psf)) return GM_EINVAL;
    for (int g = 0; g < b->n_gal; ++g) {
        if (b->h[g] < 1 || b->w[g] < 1 || b->h[g] > 1024 || b->w[g] > 1024 || b->img_off[g] < 0) return GM_EINVAL;
        if (convolved && (b->psf_k[g] < 1 || (b->psf_k[g] & 1) == 0 || b->psf_off[g] < 0)) return GM_EINVAL;
    }
    return GM_OK;
}

int prologue(gm_ctx *c, const gm_model *m, const gm_batch *b, Match &mt)
{
    if (!c) return GM_EINVAL;
    int rc = match_model(m, mt);
    if (rc) return rc;
    rc = check_batch(b, mt.ci.convolved);
    if (rc) return rc;
    mt.ci.b = b;
    return GM_OK;
}

int pick_variant(gm_ctx *c, Match &mt, const Variant **out)
{
    const FamilyOps *f = mt.ops;
    const int K = max_k(mt.ci);
    // an explicit schedule for this PSF side, else one for every side
    const gm_ctx::Sched *hit = nullptr;
    for (const auto &e : c->sched)
        if (e.family == f->id && (e.k == K || (e.k == 0 && !hit))) hit = &e;
    mt.ci.wpc = 0;
    mt.ci.team = 0;
    mt.ci.team_min = 1;
    mt.ci.team_wait_us = 0;
    if (hit) {
        mt.ci.team = hit->team;
        mt.ci.team_min = std::max(hit->team_min, 1);
        mt.ci.team_wait_us = hit->team_wait_us;
        for (int i = 0; i < f->n; ++i)
            if (f->v[i].ng == hit->ng || hit->ng == 0) {
                if (f->v[i].lds(K) > kMaxLds) break;
                mt.ci.wpc = hit->wpc;
                *out = &f->v[i];
                return GM_OK;
            }
    }
    for (int i = 0; i < f->n; ++i)
        if (f->v[i].lds(K) <= kMaxLds) {
            if (hit) mt.ci.wpc = hit->wpc;
            *out = &f->v[i];
            return GM_OK;
        }
    return GM_EUNSUPPORTED;
}

}  // namespace gm

namespace {

__global__ void copy_f64_kernel(const double *src, double *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// dst[(g nb + r) p + k] = src[g p + k]: every replica starts at its galaxy's params
__global__ void replicate_kernel(const double *src, double *dst, int n_gal, int nb, int p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_gal * nb * p) return;
    const int64_t fit = i / p, k = i - fit * p;
    dst[i] = src[(fit / nb) * p + k];
}

// Bootstrap error of column k of galaxy g over its m replicas that converged:
// sigma^2 = (1/m) sum (p_r - mean)^2 (Sec. 5.2; two passes, replicas in order)
// of the differences from params[g][k], wrapped into (-90, 90] for position
// angles.
__global__ void boot_reduce_kernel(int n_gal, int nb, int p, uint32_t pa_mask, const double *params,
                                   const double *rep, const int *status, double *err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_gal * p) return;
    const int64_t g = i / p;
    const int k = (int)(i - g * p);
    const bool pa = (pa_mask >> k) & 1u;
    const double ref = params[i];
    auto diff = [&](int r) {
        double d = rep[(g * nb + r) * p + k] - ref;
        if (pa) {
            d = fmod(d, 180.0);
            if (d > 90.0) d -= 180.0;
            if (d <= -90.0) d += 180.0;
        }
        return d;
    };
    int m = 0;
    double sum = 0.0;
    for (int r = 0; r < nb; ++r)
        if (status[g * nb + r] == GM_ST_CONVERGED) {
            sum += diff(r);
            ++m;
        }
    if (m < 2) {
        err[i] = NAN;
        return;
    }
    const double mean = sum / m;
    double ss = 0.0;
    for (int r = 0; r < nb; ++r)
        if (status[g * nb + r] == GM_ST_CONVERGED) {
            const double e = diff(r) - mean;
            ss += e * e;
        }
    err[i] = sqrt(ss / m);
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
    int rc = ctx_init(c, hip_device);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return GM_OK;
}

void gm_destroy(gm_ctx *c)
{
    if (!c) return;
    Scoped sd(c->device);
    (void)hipDeviceSynchronize();
    ctx_release(c);
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

int gm_model_image(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const double *params,
                   float *model_out, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (batch->n_gal == 0) return GM_OK;
    if (!params || !model_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    const Variant *v;
    if ((rc = pick_variant(ctx, mt, &v))) return rc;
    return v->image(ctx, mt.ci, params, model_out, 0, (hipStream_t)stream);
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
    const Variant *v;
    if ((rc = pick_variant(ctx, mt, &v))) return rc;
    return v->image(ctx, mt.ci, params, jac_out, 1, (hipStream_t)stream);
}

int gm_set_schedule(gm_ctx *ctx, const gm_model *model, int32_t psf_k, const gm_schedule *sched)
{
    if (!ctx || !sched || psf_k < 0 || (psf_k > 0 && (psf_k & 1) == 0) || sched->plane_groups < 0 ||
        sched->wg_per_cu < 0 || sched->team < 0 || sched->team_min_tiles < 0 || sched->team_wait_us < 0)
        return GM_EINVAL;
    Match mt;
    int rc = match_model(model, mt);
    if (rc) return rc;
    if (sched->plane_groups > 0) {
        bool found = false;
        for (int i = 0; i < mt.ops->n; ++i) found = found || mt.ops->v[i].ng == sched->plane_groups;
        if (!found) return GM_EUNSUPPORTED;
    }
    const int k = mt.ci.convolved ? psf_k : 1;
    for (auto &e : ctx->sched)
        if (e.family == mt.ops->id && e.k == k) {
            e.ng = sched->plane_groups;
            e.wpc = sched->wg_per_cu;
            e.team = sched->team;
            e.team_min = sched->team_min_tiles;
            e.team_wait_us = sched->team_wait_us;
            return GM_OK;
        }
    ctx->sched.push_back({mt.ops->id, k, sched->plane_groups, sched->wg_per_cu, sched->team, sched->team_min_tiles,
                          sched->team_wait_us});
    return GM_OK;
}

int gm_schedule_options(const gm_model *model, int32_t psf_k, int32_t *plane_groups_out, int32_t cap,
                        int32_t *n_out)
{
    if (!n_out || psf_k < 1 || (psf_k & 1) == 0 || cap < 0 || (cap > 0 && !plane_groups_out)) return GM_EINVAL;
    Match mt;
    int rc = match_model(model, mt);
    if (rc) return rc;
    const int k = mt.ci.convolved ? psf_k : 1;
    int n = 0;
    for (int i = 0; i < mt.ops->n; ++i)
        if (mt.ops->v[i].lds(k) <= kMaxLds) {
            if (n < cap) plane_groups_out[n] = mt.ops->v[i].ng;
            ++n;
        }
    *n_out = n;
    return GM_OK;
}

int gm_model_vjp(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const double *params,
                 const float *grad_image, double *grad_params_out, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (batch->n_gal == 0) return GM_OK;
    if (!params || !grad_image || !grad_params_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    const Variant *v;
    if ((rc = pick_variant(ctx, mt, &v))) return rc;
    return v->vjp(ctx, mt.ci, params, grad_image, grad_params_out, (hipStream_t)stream);
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
    const Variant *v;
    if ((rc = pick_variant(ctx, mt, &v))) return rc;
    return v->guess(ctx, mt.ci, params_out, moments_out, (hipStream_t)stream);
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
    const Variant *v;
    if ((rc = pick_variant(ctx, mt, &v))) return rc;
    return v->fit(ctx, mt.ci, opts, params_inout, chi2_out, niter_out, status_out, nullptr, (hipStream_t)stream);
}

int gm_fit_batch_noalloc(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_fit_opts *opts,
                         double *params_inout, double *chi2_out, int32_t *niter_out, int32_t *status_out,
                         void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (opts && (opts->max_iter < 0 || !(opts->lambda0 > 0.0) || !(opts->step_tol > 0.0))) return GM_EINVAL;
    if (batch->n_gal > kNoAllocMaxGal) return GM_EINVAL;
    if (batch->n_gal == 0) return GM_OK;
    if (!params_inout || !chi2_out || !niter_out || !status_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    char *base = reinterpret_cast<char *>(scratch_of(ctx->device));
    if (!base) return GM_EHIP;
    const Variant *v;
    if ((rc = pick_variant(ctx, mt, &v))) return rc;
    const hipStream_t st = (hipStream_t)stream;
    const int n = batch->n_gal;
    Meta *meta = reinterpret_cast<Meta *>(base);
    int *order = reinterpret_cast<int *>(base + kNaMeta);
    int *queue = reinterpret_cast<int *>(base + kNaMeta + kNaOrder);
    char *raw = base + kNaMeta + kNaOrder + kNaQueue;
    int32_t *rh = reinterpret_cast<int32_t *>(raw);
    int32_t *rw = reinterpret_cast<int32_t *>(raw + kNaRaw32);
    int32_t *rk = reinterpret_cast<int32_t *>(raw + 2 * kNaRaw32);
    int64_t *rio = reinterpret_cast<int64_t *>(raw + 3 * kNaRaw32);
    int64_t *rpo = reinterpret_cast<int64_t *>(raw + 3 * kNaRaw32 + kNaRaw64);
    const size_t n4 = sizeof(int32_t) * (size_t)n, n8 = sizeof(int64_t) * (size_t)n;
    if (hipMemcpyAsync(rh, batch->h, n4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(rw, batch->w, n4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(rio, batch->img_off, n8, hipMemcpyHostToDevice, st) != hipSuccess)
        return GM_EHIP;
    if (mt.ci.convolved && (hipMemcpyAsync(rk, batch->psf_k, n4, hipMemcpyHostToDevice, st) != hipSuccess ||
                            hipMemcpyAsync(rpo, batch->psf_off, n8, hipMemcpyHostToDevice, st) != hipSuccess))
        return GM_EHIP;
    hipLaunchKernelGGL(noalloc_pack_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, mt.ci.convolved ? 1 : 0,
                       rh, rw, rk, rio, rpo, meta, order, queue);
    if ((rc = hip_rc(hipGetLastError()))) return rc;
    Staged sg;
    sg.meta = meta;
    sg.extra = order;
    sg.queue = queue;
    FitExtra ex;
    ex.pre = &sg;
    return v->fit(ctx, mt.ci, opts, params_inout, chi2_out, niter_out, status_out, &ex, st);
}

int gm_fit_adam(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_adam_opts *opts,
                double *params_inout, double *chi2_out, int32_t *status_out, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (!opts || opts->steps < 0 || !(opts->lr > 0.0) || !(opts->beta1 >= 0.0 && opts->beta1 < 1.0) ||
        !(opts->beta2 >= 0.0 && opts->beta2 < 1.0) || !(opts->eps > 0.0))
        return GM_EINVAL;
    if (batch->n_gal == 0) return GM_OK;
    if (!params_inout || !chi2_out || !status_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    const Variant *v;
    if ((rc = pick_variant(ctx, mt, &v))) return rc;
    return v->adam(ctx, mt.ci, opts, params_inout, chi2_out, status_out, (hipStream_t)stream);
}

int gm_bootstrap(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_fit_opts *opts,
                 const double *params, int32_t n_boot, uint64_t seed, double *err_out, double *rep_params_out,
                 int32_t *rep_status_out, int32_t *rep_niter_out, void *stream)
{
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (opts && (opts->max_iter < 0 || !(opts->lambda0 > 0.0) || !(opts->step_tol > 0.0))) return GM_EINVAL;
    if (n_boot < 2 || (int64_t)batch->n_gal * n_boot > (1 << 30)) return GM_EINVAL;
    if (batch->n_gal == 0) return GM_OK;
    if (!params || !err_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    const Variant *v;
    if ((rc = pick_variant(ctx, mt, &v))) return rc;
    const hipStream_t st = (hipStream_t)stream;
    const int n = batch->n_gal, p = model->p;
    const int64_t nfit = (int64_t)n * n_boot;
    // position-angle columns
    const int pa_slot[9] = {-1, 6, 5, 5, 6, 5, 5, -1, -1};
    uint32_t pa_mask = 0;
    for (int c = 0; c < model->n_comp; ++c) {
        const int sl = pa_slot[model->comp[c].type];
        if (sl >= 0 && model->comp[c].param_index[sl] >= 0) pa_mask |= 1u << model->comp[c].param_index[sl];
    }
    // replica parameters, chi^2, trials and status in the context's scratch
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t need = al(sizeof(double) * nfit * p) + al(sizeof(double) * nfit) + 2 * al(sizeof(int) * nfit);
    void *ws = nullptr;
    if ((rc = ensure_aux(ctx, need, &ws))) return rc;
    char *w8 = reinterpret_cast<char *>(ws);
    double *rp = rep_params_out ? rep_params_out : reinterpret_cast<double *>(w8);
    w8 += al(sizeof(double) * nfit * p);
    double *chi2 = reinterpret_cast<double *>(w8);
    w8 += al(sizeof(double) * nfit);
    int *niter = rep_niter_out ? rep_niter_out : reinterpret_cast<int *>(w8);
    w8 += al(sizeof(int) * nfit);
    int *rs = rep_status_out ? rep_status_out : reinterpret_cast<int *>(w8);
    const int64_t cnt = nfit * p;
    hipLaunchKernelGGL(replicate_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, params, rp, n,
                       (int)n_boot, p);
    if ((rc = hip_rc(hipGetLastError()))) return rc;
    gm_fit_opts o = opts ? *opts : gm_fit_opts{100, 1e-3, 1e-4, nullptr, 0, nullptr};
    o.active = nullptr;
    o.err_out = nullptr;
    FitExtra ex;
    ex.n_boot = n_boot;
    ex.boot_seed = seed;
    if ((rc = v->fit(ctx, mt.ci, &o, rp, chi2, niter, rs, &ex, st))) return rc;
    const int64_t ne = (int64_t)n * p;
    hipLaunchKernelGGL(boot_reduce_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, n, (int)n_boot, p,
                       pa_mask, params, rp, rs, err_out);
    return hip_rc(hipGetLastError());
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
    const Variant *v;
    if ((rc = pick_variant(ctx, mt, &v))) return rc;
    return v->errors(ctx, mt.ci, params, err_out, cov_out, (hipStream_t)stream);
}

int gm_plan_fit(gm_ctx *ctx, const gm_model *model, const gm_batch *batch, const gm_fit_opts *opts,
                const double *start, double *params_out, double *chi2_out, int32_t *niter_out,
                int32_t *status_out, double *err_out, int32_t timing, gm_plan **out)
{
    if (!out) return GM_EINVAL;
    *out = nullptr;
    Match mt;
    int rc = prologue(ctx, model, batch, mt);
    if (rc) return rc;
    if (opts && (opts->max_iter < 0 || !(opts->lambda0 > 0.0) || !(opts->step_tol > 0.0))) return GM_EINVAL;
    if (batch->n_gal == 0 || !params_out || !chi2_out || !niter_out || !status_out) return GM_EINVAL;
    Scoped sd(ctx->device);
    gm_plan *p;
    if ((rc = plan_open(ctx, batch->n_gal, 3, timing != 0, &p))) return rc;
    gm_ctx *pc = &p->ctx;
    void *const *events = timing ? p->ev : nullptr;
    const hipStream_t st = p->stream;
    const Variant *v = nullptr;
    rc = pick_variant(pc, mt, &v);
    if (!rc) rc = plan_begin(p);
    if (!rc) rc = mark_event(pc, events, 0, st);
    if (!rc) {
        if (start) {
            const int64_t cnt = (int64_t)batch->n_gal * model->p;
            hipLaunchKernelGGL(copy_f64_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, start,
                               params_out, cnt);
            rc = hip_rc(hipGetLastError());
        } else {
            rc = v->guess(pc, mt.ci, params_out, nullptr, st);
        }
    }
    gm_fit_opts o = opts ? *opts : gm_fit_opts{100, 1e-3, 1e-4, nullptr, 0, nullptr};
    o.err_out = err_out;
    if (!rc) rc = mark_event(pc, events, 1, st);
    if (!rc) rc = v->fit(pc, mt.ci, &o, params_out, chi2_out, niter_out, status_out, nullptr, st);
    if (!rc) rc = mark_event(pc, events, 2, st);
    if (!rc) rc = mark_event(pc, events, 3, st);
    return plan_end(p, rc, out);
}

int gm_plan_launch(gm_plan *plan, void *stream)
{
    if (!plan || !plan->exec) return GM_EINVAL;
    Scoped sd(plan->ctx.device);
    int rc = hip_rc(hipGraphLaunch(plan->exec, (hipStream_t)stream));
    if (!rc) plan->launched = true;
    return rc;
}

int gm_plan_elapsed(gm_plan *plan, float *ms_out)
{
    if (!plan || !ms_out || !plan->ev[0] || !plan->launched) return GM_EINVAL;
    Scoped sd(plan->ctx.device);
    hipEvent_t *e = reinterpret_cast<hipEvent_t *>(plan->ev);
    if (hipEventSynchronize(e[3]) != hipSuccess) return GM_EHIP;
    for (int i = 0; i < 3; ++i)
        if (hipEventElapsedTime(&ms_out[i], e[i], e[i + 1]) != hipSuccess) return GM_EHIP;
    return GM_OK;
}

void gm_plan_destroy(gm_plan *plan)
{
    if (!plan) return;
    Scoped sd(plan->ctx.device);
    plan_free(plan);
}

}  // extern "C"
