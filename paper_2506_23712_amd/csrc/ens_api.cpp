// ens_api.cpp -- host side of libensdns: the C ABI declared in include/ens.h,
// member registry, per-member-set step plans, HIP graph capture and replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <tuple>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ens_internal.h"
#include "ens_diag.h"
#include "ens_lambda.h"

#define ENS_API extern "C" __attribute__((visibility("default")))

namespace {

using namespace ens;

thread_local std::string g_err;

ens_status fail(ens_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

bool pow2_supported(int n) { return n == 16 || n == 32 || n == 64 || n == 128 || n == 256 || n == 512 || n == 1024; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------------------------ twiddles
// tw[j] = exp(-2 pi i j / n), j < n, evaluated in FP64 on the first octant and
// mapped by symmetry so that quarter/eighth turns are exact.
void twiddles_fp64(int n, std::vector<double> &out) {
    out.resize(2 * (size_t)n);
    const int q4 = n / 4, q8 = n / 8;
    for (int j = 0; j < n; j++) {
        int quad = j / q4, r = j % q4;
        double c, s;
        if (q8 > 0 && r > q8) {
            const double a = 2.0 * M_PI * (double)(q4 - r) / (double)n;
            c = std::sin(a); s = std::cos(a);
        } else {
            const double a = 2.0 * M_PI * (double)r / (double)n;
            c = std::cos(a); s = std::sin(a);
        }
        double cc, ss;   // rotate by quad quarter turns
        switch (quad) {
        case 0: cc = c; ss = s; break;
        case 1: cc = -s; ss = c; break;
        case 2: cc = -c; ss = -s; break;
        default: cc = s; ss = -c; break;
        }
        out[2 * j] = cc;
        out[2 * j + 1] = -ss;
    }
}

std::mutex g_tw_mu;
std::map<std::tuple<int, int, int>, void *> g_tw;   // (device, n, prec) -> device table

hipError_t get_twiddles(int device, int n, int prec, const void **out) {
    std::lock_guard<std::mutex> lk(g_tw_mu);
    auto key = std::make_tuple(device, n, prec);
    auto it = g_tw.find(key);
    if (it != g_tw.end()) { *out = it->second; return hipSuccess; }
    std::vector<double> d;
    twiddles_fp64(n, d);
    void *p = nullptr;
    hipError_t e;
    if (prec == ENS_FP32) {
        std::vector<float> f(d.size());
        for (size_t i = 0; i < d.size(); i++) f[i] = (float)d[i];
        e = hipMalloc(&p, f.size() * sizeof(float));
        if (e != hipSuccess) return e;
        e = hipMemcpy(p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
    } else {
        e = hipMalloc(&p, d.size() * sizeof(double));
        if (e != hipSuccess) return e;
        e = hipMemcpy(p, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return e;
    g_tw[key] = p;
    *out = p;
    return hipSuccess;
}

// ------------------------------------------------------------ member layout
struct Layout {
    size_t off_st, off_uh, off_q, off_a, off_b, off_part, off_counts, off_mom, total;
};

Layout member_layout(const ens_member_desc &d, const HistGeom *hg) {
    const Geom g = make_geom(d.n, d.precision);
    const size_t cs = d.precision == ENS_FP32 ? 8 : 16;
    const long long n = d.n;
    Layout L;
    size_t o = 0;
    L.off_st = o; o += align256(sizeof(DevState));
    L.off_uh = o; o += align256(3 * (size_t)g.S * cs);
    L.off_q = o; o += align256(3 * (size_t)g.S * cs);
    // bufA: statistics z-inverse out, z-inverse out, x-pass out;
    // bufB: statistics y-inverse out, y-inverse out, y-forward out
    const size_t a_elems = std::max({(size_t)6 * n * g.nzl, (size_t)5 * n * g.zp, (size_t)3 * n * g.nyl});
    const size_t b_elems = std::max({(size_t)9 * n * n * g.px, (size_t)6 * n * g.nyl, (size_t)3 * (2 * g.K + 1) * g.nyl});
    L.off_a = o; o += align256(a_elems * cs);
    L.off_b = o; o += align256(b_elems * cs);
    const size_t nparts = std::max({(size_t)(2 * zfwd_blocks(d.n, d.precision)), (size_t)init_blocks(d.n),
                                    (size_t)(ENS_NMOM * xstats_blocks(d.n)), (size_t)scales_partials(g.K),
                                    (size_t)spectrum_partials(g.K)});
    L.off_part = o; o += align256(nparts * sizeof(double));
    const size_t ncounts = hg ? (size_t)hg->n_counts : 0;
    L.off_counts = o; o += align256(ncounts * sizeof(unsigned long long));
    L.off_mom = o; o += align256(ENS_NMOM * sizeof(double));
    L.total = o;
    return L;
}

struct Member {
    ens_member_desc d;
    Geom g;
    Layout lay;
    void *ws = nullptr;
    MemberDev md;            // host copy
    MemberDev *dev = nullptr;   // device copy (library-owned, one element)
    hipStream_t last = nullptr;
};

struct Group {
    int n = 0, prec = 0;
    std::vector<int> ids;
    MemberDev *dev = nullptr;   // device array of the group's MemberDev
    const void *tw = nullptr;
};

// What a step takes from and leaves to its neighbours in one ens_step call
// (with the fused z forward): every step but the call's first finds its first
// z inverse already done by the previous step's last z forward, and every
// step but the call's last does that for the next one.
struct StepKind {
    bool zinv0_done;   // stage 0's z inverse was performed by the previous step
    bool fuse_last;    // the last stage's z forward performs the next step's first z inverse
    int index() const { return (zinv0_done ? 2 : 0) + (fuse_last ? 1 : 0); }
};
constexpr StepKind kLoneStep{false, false};

struct Plan {
    std::vector<Group> groups;
    hipGraphExec_t exec[4] = {};     // one captured step per StepKind::index()
    hipGraph_t graph[4] = {};
};

void free_graphs(Plan &pl) {
    for (int i = 0; i < 4; i++) {
        if (pl.exec[i]) (void)hipGraphExecDestroy(pl.exec[i]);
        if (pl.graph[i]) (void)hipGraphDestroy(pl.graph[i]);
        pl.exec[i] = nullptr;
        pl.graph[i] = nullptr;
    }
}

}  // namespace

struct ens_ctx {
    int device = 0;
    bool poisoned = false;
    int graphs = 1;                   // 0 direct launches, 1 one graph per step, 2 ... with a branch per group
    bool has_hist = false;
    ens_hist_desc hist{};
    HistGeom hg{};
    double *ledge = nullptr;          // log-histogram edges 10^(lo + b (hi - lo) / bins), b = 0..bins
    hipStream_t cap = nullptr;   // private stream used for graph capture
    std::vector<hipStream_t> side;    // capture streams of the per-group branches (graph mode 2)
    std::vector<hipEvent_t> fork;     // fork / join events of those branches
    std::vector<std::unique_ptr<Member>> members;
    std::map<std::vector<int>, std::unique_ptr<Plan>> plans;
    std::vector<void *> dev_allocs;   // library-owned small device tables
    void *mix_scratch = nullptr;      // member table of ens_mix (library-owned)
    size_t mix_scratch_bytes = 0;
    std::map<std::tuple<int, int, int>, int> variant;   // (pass, n, precision) -> kernel variant
};

namespace {

#define HIPCK(ctx, expr)                                                                   \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) {                                                            \
            if (ctx) (ctx)->poisoned = true;                                               \
            return fail(ENS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));      \
        }                                                                                  \
    } while (0)

ens_status check_ctx(const ens_ctx *ctx) {
    if (!ctx) return fail(ENS_E_INVALID, "null context");
    if (ctx->poisoned) return fail(ENS_E_STATE, "context poisoned by an earlier HIP failure");
    return ENS_OK;
}

ens_status validate_desc(const ens_member_desc *d) {
    if (!d) return fail(ENS_E_INVALID, "null member descriptor");
    if (!pow2_supported(d->n)) return fail(ENS_E_UNSUPPORTED, "n must be one of 16, 32, 64, 128, 256, 512, 1024");
    if (d->precision != ENS_FP64 && d->precision != ENS_FP32) return fail(ENS_E_INVALID, "precision must be 0 or 1");
    if (d->n == 1024 && d->precision != ENS_FP32) return fail(ENS_E_UNSUPPORTED, "n = 1024 is supported in FP32 only");
    if (!(d->box > 0) || !std::isfinite(d->box)) return fail(ENS_E_INVALID, "box must be positive");
    if (!(d->nu >= 0) || !std::isfinite(d->nu)) return fail(ENS_E_INVALID, "nu must be >= 0");
    if (!(d->eps_ref >= 0) || !std::isfinite(d->eps_ref)) return fail(ENS_E_INVALID, "eps_ref must be >= 0");
    if (!std::isfinite(d->lambda)) return fail(ENS_E_INVALID, "lambda must be finite");
    if (!(d->kf_lo >= 0) || !(d->kf_hi >= d->kf_lo) || !std::isfinite(d->kf_hi))
        return fail(ENS_E_INVALID, "need 0 <= kf_lo <= kf_hi");
    if (!(d->dt > 0) && !(d->cfl > 0)) return fail(ENS_E_INVALID, "need dt > 0 or cfl > 0");
    if (!std::isfinite(d->dt) || !std::isfinite(d->cfl)) return fail(ENS_E_INVALID, "dt/cfl must be finite");
    if (!(d->k_peak > 0) || !(d->e0 >= 0) || !std::isfinite(d->e0)) return fail(ENS_E_INVALID, "need k_peak > 0, e0 >= 0");
    if (d->visc_mode != 0 && d->visc_mode != 1) return fail(ENS_E_INVALID, "visc_mode must be 0 or 1");
    if (d->reserved != 0) return fail(ENS_E_INVALID, "reserved must be 0");
    return ENS_OK;
}

ens_status validate_hist(const ens_hist_desc *h) {
    if (h->qr_bins <= 0 || h->log_bins <= 0 || h->a_bins <= 0) return fail(ENS_E_INVALID, "histogram bin counts must be positive");
    if (h->qr_bins > 4096 || h->log_bins > (1 << 20) || h->a_bins > (1 << 20)) return fail(ENS_E_INVALID, "too many bins");
    for (double v : {h->q_lo, h->q_hi, h->r_lo, h->r_hi, h->log10_lo, h->log10_hi, h->a_lo, h->a_hi, h->eps_ref, h->nu_ref})
        if (!std::isfinite(v)) return fail(ENS_E_INVALID, "histogram ranges and reference scales must be finite");
    if (!(h->q_hi > h->q_lo) || !(h->r_hi > h->r_lo) || !(h->log10_hi > h->log10_lo) || !(h->a_hi > h->a_lo))
        return fail(ENS_E_INVALID, "histogram ranges need hi > lo");
    if (!(h->eps_ref > 0) || !(h->nu_ref > 0)) return fail(ENS_E_INVALID, "eps_ref and nu_ref must be positive");
    if (!stats_hist_fits(*h)) return fail(ENS_E_UNSUPPORTED, "log_bins + a_bins too large for the statistics kernel");
    return ENS_OK;
}

ens_status member_of(ens_ctx *ctx, int32_t m, Member **out) {
    if (m < 0 || m >= (int32_t)ctx->members.size() || !ctx->members[m]) return fail(ENS_E_INVALID, "bad member id");
    *out = ctx->members[m].get();
    return ENS_OK;
}

ens_status make_plan(ens_ctx *ctx, const std::vector<int> &ids, Plan **out) {
    auto it = ctx->plans.find(ids);
    if (it != ctx->plans.end()) { *out = it->second.get(); return ENS_OK; }
    auto plan = std::make_unique<Plan>();
    std::map<std::pair<int, int>, std::vector<int>> by;
    for (int id : ids) {
        Member *m = ctx->members[id].get();
        by[{m->d.n, m->d.precision}].push_back(id);
    }
    for (auto &kv : by) {
        Group g;
        g.n = kv.first.first; g.prec = kv.first.second; g.ids = kv.second;
        std::vector<MemberDev> host;
        for (int id : g.ids) host.push_back(ctx->members[id]->md);
        void *p = nullptr;
        HIPCK(ctx, hipMalloc(&p, host.size() * sizeof(MemberDev)));
        ctx->dev_allocs.push_back(p);
        HIPCK(ctx, hipMemcpy(p, host.data(), host.size() * sizeof(MemberDev), hipMemcpyHostToDevice));
        g.dev = (MemberDev *)p;
        HIPCK(ctx, get_twiddles(ctx->device, g.n, g.prec, &g.tw));
        plan->groups.push_back(g);
    }
    *out = plan.get();
    ctx->plans[ids] = std::move(plan);
    return ENS_OK;
}

// Enqueue one RK step of every group of the plan.  With `ev` (profiling),
// events are recorded around each launch and times are added to ms[pass].
struct Prof {
    std::vector<hipEvent_t> ev;
    std::vector<int> pass;
};

int variant_of(const ens_ctx *ctx, int pass, int n, int prec) {
    auto it = ctx->variant.find(std::make_tuple(pass, n, prec));
    return it != ctx->variant.end() ? it->second : default_variant(pass, n, prec);
}

// One RK step of one group (three stages, then the end-of-step reduction) on
// stream s; the groups of a plan are independent of each other.
// With the fused z forward (variant 1) the z forward of stages 0 and 1 also
// performs the next stage's z inverse, which is then not launched; so is
// stage 0's when the previous step of the same call performed it.
bool zinv_fused(const ens_ctx *ctx, int pass, int stage, int n, int prec, StepKind k) {
    return pass == P_ZINV && variant_of(ctx, P_ZFWD, n, prec) == 1 && (stage > 0 || k.zinv0_done);
}

// The variant launched for a pass: the fused z forward's last stage runs as
// the internal variant 2 when the next step of the call takes its z inverse.
int launch_variant(const ens_ctx *ctx, int pass, int stage, int n, int prec, StepKind k) {
    const int v = variant_of(ctx, pass, n, prec);
    return (pass == P_ZFWD && v == 1 && stage == 2 && k.fuse_last) ? 2 : v;
}

hipError_t enqueue_group(const ens_ctx *ctx, const Group &g, hipStream_t s, StepKind k) {
    const int cnt = (int)g.ids.size();
    hipError_t e;
    for (int stage = 0; stage < 3; stage++)
        for (int pass = P_BAND; pass <= P_ZFWD; pass++) {
            if (zinv_fused(ctx, pass, stage, g.n, g.prec, k)) continue;
            if ((e = launch_pass(pass, launch_variant(ctx, pass, stage, g.n, g.prec, k), g.n, g.prec, g.dev, cnt,
                                 stage, g.tw, s)))
                return e;
        }
    return launch_pass(P_END, 0, g.n, g.prec, g.dev, cnt, 0, g.tw, s);
}

// Graph mode 2: inside the capture on ctx->cap, fork one branch per group onto
// its own stream and join them again, so that the captured graph lets the
// groups' kernels run side by side.  Streams and events exist before capture.
hipError_t enqueue_step_branches(const ens_ctx *ctx, const Plan &pl, StepKind k) {
    hipError_t e = hipEventRecord(ctx->fork[0], ctx->cap);
    for (size_t i = 0; i < pl.groups.size() && e == hipSuccess; i++) {
        if ((e = hipStreamWaitEvent(ctx->side[i], ctx->fork[0], 0))) break;
        if ((e = enqueue_group(ctx, pl.groups[i], ctx->side[i], k))) break;
        if ((e = hipEventRecord(ctx->fork[i + 1], ctx->side[i]))) break;
        e = hipStreamWaitEvent(ctx->cap, ctx->fork[i + 1], 0);
    }
    return e;
}

hipError_t enqueue_step(const ens_ctx *ctx, const Plan &pl, hipStream_t s, Prof *prof, StepKind k) {
    hipError_t e = hipSuccess;
    auto rec = [&](int pass, auto &&fn) -> hipError_t {
        if (prof) {
            // events belong to prof as soon as they exist: the caller destroys
            // them whatever fails later
            hipEvent_t a, b;
            hipError_t r = hipEventCreate(&a);
            if (r != hipSuccess) return r;
            prof->ev.push_back(a);
            r = hipEventCreate(&b);
            if (r != hipSuccess) return r;
            prof->ev.push_back(b);
            prof->pass.push_back(pass);
            r = hipEventRecord(a, s);
            if (r != hipSuccess) return r;
            r = fn();
            if (r != hipSuccess) return r;
            return hipEventRecord(b, s);
        }
        return fn();
    };
    for (int stage = 0; stage < 3; stage++) {
        for (const Group &g : pl.groups) {
            const int cnt = (int)g.ids.size();
            for (int pass = P_BAND; pass <= P_ZFWD; pass++) {
                if (zinv_fused(ctx, pass, stage, g.n, g.prec, k)) continue;
                const int v = launch_variant(ctx, pass, stage, g.n, g.prec, k);
                if ((e = rec(pass, [&] { return launch_pass(pass, v, g.n, g.prec, g.dev, cnt, stage, g.tw, s); }))) return e;
            }
        }
    }
    for (const Group &g : pl.groups) {
        const int cnt = (int)g.ids.size();
        if ((e = rec(P_END, [&] { return launch_pass(P_END, 0, g.n, g.prec, g.dev, cnt, 0, g.tw, s); }))) return e;
    }
    return hipSuccess;
}

ens_status collect_ids(ens_ctx *ctx, const int32_t *members, int32_t count, std::vector<int> &ids) {
    if (count <= 0 || !members) return fail(ENS_E_INVALID, "empty member list");
    ids.assign(members, members + count);
    std::vector<int> sorted = ids;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return fail(ENS_E_INVALID, "duplicate member id");
    for (int id : ids) {
        Member *m;
        ens_status st = member_of(ctx, id, &m);
        if (st) return st;
    }
    return ENS_OK;
}

}  // namespace

// ======================================================================= ABI
ENS_API const char *ens_last_error(void) { return g_err.c_str(); }

ENS_API ens_status ens_create(ens_ctx **out, int device, const ens_hist_desc *h) {
    if (!out) return fail(ENS_E_INVALID, "null output pointer");
    *out = nullptr;
    if (h) {
        ens_status st = validate_hist(h);
        if (st) return st;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(ENS_E_HIP, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(ENS_E_INVALID, "device index out of range");
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(ENS_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    // device address of the static mixture table (ens_mix_noalloc), once per device
    e = mix_static_setup(device);
    if (e != hipSuccess) return fail(ENS_E_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    auto ctx = std::make_unique<ens_ctx>();
    ctx->device = device;
    if (h) {
        ctx->has_hist = true;
        ctx->hist = *h;
        ctx->hg = make_hist_geom(*h);
        std::vector<double> edges((size_t)h->log_bins + 1);
        const double w = (h->log10_hi - h->log10_lo) / (double)h->log_bins;
        for (size_t b = 0; b < edges.size(); b++) edges[b] = std::pow(10.0, h->log10_lo + (double)b * w);
        e = hipMalloc(&ctx->ledge, edges.size() * sizeof(double));
        if (e != hipSuccess) return fail(ENS_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
        ctx->dev_allocs.push_back(ctx->ledge);
        e = hipMemcpy(ctx->ledge, edges.data(), edges.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(ctx->ledge);
            return fail(ENS_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
    }
    e = hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (ctx->ledge) (void)hipFree(ctx->ledge);
        return fail(ENS_E_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    *out = ctx.release();
    return ENS_OK;
}

ENS_API ens_status ens_destroy(ens_ctx *ctx) {
    if (!ctx) return fail(ENS_E_INVALID, "null context");
    // Teardown is best effort: every handle is released even if an earlier
    // release (or a sticky error of the device) fails.
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : ctx->plans) free_graphs(*kv.second);
    for (auto &m : ctx->members)
        if (m && m->dev) (void)hipFree(m->dev);
    for (void *p : ctx->dev_allocs) (void)hipFree(p);
    if (ctx->mix_scratch) (void)hipFree(ctx->mix_scratch);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    for (hipStream_t st : ctx->side) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : ctx->fork) (void)hipEventDestroy(ev);
    delete ctx;
    return ENS_OK;
}

ENS_API ens_status ens_set_graphs(ens_ctx *ctx, int32_t mode) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (mode < 0 || mode > 2) return fail(ENS_E_INVALID, "graph mode must be 0, 1 or 2");
    if (mode != ctx->graphs) {
        HIPCK(ctx, hipSetDevice(ctx->device));
        HIPCK(ctx, hipDeviceSynchronize());
        for (auto &kv : ctx->plans) free_graphs(*kv.second);   // captured with the other mode
    }
    ctx->graphs = mode;
    return ENS_OK;
}

ENS_API ens_status ens_member_workspace_bytes(const ens_ctx *ctx, const ens_member_desc *d, size_t *bytes) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!bytes) return fail(ENS_E_INVALID, "null output pointer");
    if (ens_status st = validate_desc(d)) return st;
    *bytes = member_layout(*d, ctx->has_hist ? &ctx->hg : nullptr).total;
    return ENS_OK;
}

ENS_API ens_status ens_member_init(ens_ctx *ctx, const ens_member_desc *d, void *dev_workspace, size_t bytes,
                                   void *stream, int32_t *member_id) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (ens_status st = validate_desc(d)) return st;
    if (!member_id) return fail(ENS_E_INVALID, "null member_id");
    if (!dev_workspace || ((uintptr_t)dev_workspace & 255)) return fail(ENS_E_INVALID, "workspace must be 256-byte aligned device memory");
    const Layout lay = member_layout(*d, ctx->has_hist ? &ctx->hg : nullptr);
    if (bytes < lay.total) return fail(ENS_E_OOM, "workspace too small: need " + std::to_string(lay.total) + " bytes");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, dev_workspace) != hipSuccess || attr.type != hipMemoryTypeDevice)
        return fail(ENS_E_INVALID, "workspace is not device memory");
    HIPCK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    auto m = std::make_unique<Member>();
    m->d = *d;
    m->g = make_geom(d->n, d->precision);
    m->lay = lay;
    m->ws = dev_workspace;
    char *base = (char *)dev_workspace;
    MemberDev &md = m->md;
    md.st = (DevState *)(base + lay.off_st);
    md.uh = base + lay.off_uh;
    md.q = base + lay.off_q;
    md.bufA = base + lay.off_a;
    md.bufB = base + lay.off_b;
    md.partials = (double *)(base + lay.off_part);
    md.counts = (unsigned long long *)(base + lay.off_counts);
    md.moments = (double *)(base + lay.off_mom);
    md.nu = d->nu;
    md.eps_m = std::exp(d->lambda) * d->eps_ref;
    md.kf_lo2 = d->kf_lo * d->kf_lo;
    md.kf_hi2 = d->kf_hi * d->kf_hi;
    md.dt_fixed = d->dt > 0 ? d->dt : 0.0;
    md.cfl = d->cfl;
    md.box = d->box;
    md.dk = 2.0 * M_PI / d->box;
    md.n = d->n; md.K = d->n / 3; md.prec = d->precision; md.visc_mode = d->visc_mode;
    md.px = m->g.px; md.zp = (int)m->g.zp;
    void *p = nullptr;
    HIPCK(ctx, hipMalloc(&p, sizeof(MemberDev)));
    m->dev = (MemberDev *)p;
    HIPCK(ctx, hipMemcpy(m->dev, &md, sizeof(MemberDev), hipMemcpyHostToDevice));
    // the pad entries of the state planes are never read; zero them anyway
    const long long state_doubles = 3 * m->g.S * (d->precision == ENS_FP32 ? 1 : 2);
    HIPCK(ctx, launch_fill_f64((double *)md.uh, state_doubles, 0.0, s));
    HIPCK(ctx, launch_fill_f64((double *)md.q, state_doubles, 0.0, s));
    HIPCK(ctx, launch_init_field(d->n, d->precision, m->dev, d->seed, d->k_peak, d->e0, s));
    if (ctx->has_hist) {
        HIPCK(ctx, launch_fill_u64(md.counts, ctx->hg.n_counts, 0ull, s));
        HIPCK(ctx, launch_fill_f64(md.moments, ENS_NMOM, 0.0, s));
    }
    m->last = s;
    *member_id = (int32_t)ctx->members.size();
    ctx->members.push_back(std::move(m));
    return ENS_OK;
}

ENS_API ens_status ens_member_set_state(ens_ctx *ctx, int32_t mid, const double *dev_uhat, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    Member *m;
    if (ens_status st = member_of(ctx, mid, &m)) return st;
    if (!dev_uhat) return fail(ENS_E_INVALID, "null state pointer");
    HIPCK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    HIPCK(ctx, launch_set_state(m->d.n, m->d.precision, m->dev, dev_uhat, s));
    HIPCK(ctx, launch_refresh_energy(m->d.precision, m->dev, m->md.st, m->g.K, s));
    m->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_member_get_state(ens_ctx *ctx, int32_t mid, double *dev_uhat, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    Member *m;
    if (ens_status st = member_of(ctx, mid, &m)) return st;
    if (!dev_uhat) return fail(ENS_E_INVALID, "null state pointer");
    HIPCK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    HIPCK(ctx, launch_get_state(m->d.n, m->d.precision, m->dev, dev_uhat, s));
    m->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_step(ens_ctx *ctx, const int32_t *members, int32_t count, int32_t nsteps, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (nsteps < 0) return fail(ENS_E_INVALID, "nsteps must be >= 0");
    std::vector<int> ids;
    if (ens_status st = collect_ids(ctx, members, count, ids)) return st;
    HIPCK(ctx, hipSetDevice(ctx->device));
    Plan *pl;
    if (ens_status st = make_plan(ctx, ids, &pl)) return st;
    hipStream_t s = (hipStream_t)stream;
    if (nsteps == 0) return ENS_OK;
    // step i of the call: its first z inverse done by step i - 1 (i > 0), the
    // next step's done by its last z forward (i < nsteps - 1)
    auto kind_of = [&](int i) { return StepKind{i > 0, i + 1 < nsteps}; };
    if (ctx->graphs) {
        for (int i = 0; i < nsteps; i++) {
            const StepKind k = kind_of(i);
            hipGraphExec_t &exec = pl->exec[k.index()];
            if (exec) {
                HIPCK(ctx, hipGraphLaunch(exec, s));
                continue;
            }
            const bool branches = ctx->graphs == 2 && pl->groups.size() > 1;
            if (branches) {
                while (ctx->side.size() < pl->groups.size()) {
                    hipStream_t st;
                    HIPCK(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
                    ctx->side.push_back(st);
                }
                while (ctx->fork.size() < pl->groups.size() + 1) {
                    hipEvent_t ev;
                    HIPCK(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
                    ctx->fork.push_back(ev);
                }
            }
            HIPCK(ctx, hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
            hipError_t e = branches ? enqueue_step_branches(ctx, *pl, k) : enqueue_step(ctx, *pl, ctx->cap, nullptr, k);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(ctx->cap, &g);
            HIPCK(ctx, e);
            HIPCK(ctx, e2);
            pl->graph[k.index()] = g;
            HIPCK(ctx, hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
            HIPCK(ctx, hipGraphLaunch(exec, s));
        }
    } else {
        for (int i = 0; i < nsteps; i++) HIPCK(ctx, enqueue_step(ctx, *pl, s, nullptr, kind_of(i)));
    }
    for (int id : ids) ctx->members[id]->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_profile_step(ens_ctx *ctx, const int32_t *members, int32_t count, void *stream, double *ms_out) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!ms_out) return fail(ENS_E_INVALID, "null output pointer");
    std::vector<int> ids;
    if (ens_status st = collect_ids(ctx, members, count, ids)) return st;
    HIPCK(ctx, hipSetDevice(ctx->device));
    Plan *pl;
    if (ens_status st = make_plan(ctx, ids, &pl)) return st;
    hipStream_t s = (hipStream_t)stream;
    Prof prof;
    hipError_t e = enqueue_step(ctx, *pl, s, &prof, kLoneStep);
    hipError_t e2 = hipStreamSynchronize(s);
    for (int p = 0; p < ENS_NPASS; p++) ms_out[p] = 0.0;
    for (size_t i = 0; i < prof.pass.size(); i++) {
        float ms = 0.f;
        if (e == hipSuccess && e2 == hipSuccess && hipEventElapsedTime(&ms, prof.ev[2 * i], prof.ev[2 * i + 1]) == hipSuccess)
            ms_out[prof.pass[i]] += ms;
    }
    for (hipEvent_t ev : prof.ev) (void)hipEventDestroy(ev);
    HIPCK(ctx, e);
    HIPCK(ctx, e2);
    for (int id : ids) ctx->members[id]->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_get_diag(ens_ctx *ctx, int32_t mid, ens_diag *out) {
    if (ens_status st = check_ctx(ctx)) return st;
    Member *m;
    if (ens_status st = member_of(ctx, mid, &m)) return st;
    if (!out) return fail(ENS_E_INVALID, "null output pointer");
    HIPCK(ctx, hipSetDevice(ctx->device));
    HIPCK(ctx, hipStreamSynchronize(m->last));
    HIPCK(ctx, hipMemcpy(out, &m->md.st->diag, sizeof(ens_diag), hipMemcpyDeviceToHost));
    return out->flags & 5 ? fail(ENS_E_DIVERGED, "member diverged (non-finite energy or no CFL velocity)") : ENS_OK;
}

ENS_API ens_status ens_stats_len(const ens_ctx *ctx, size_t *n_counts) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!n_counts) return fail(ENS_E_INVALID, "null output pointer");
    if (!ctx->has_hist) return fail(ENS_E_STATE, "context has no histogram descriptor");
    *n_counts = (size_t)ctx->hg.n_counts;
    return ENS_OK;
}

ENS_API ens_status ens_accumulate_stats(ens_ctx *ctx, const int32_t *members, int32_t count, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!ctx->has_hist) return fail(ENS_E_STATE, "context has no histogram descriptor");
    std::vector<int> ids;
    if (ens_status st = collect_ids(ctx, members, count, ids)) return st;
    HIPCK(ctx, hipSetDevice(ctx->device));
    Plan *pl;
    if (ens_status st = make_plan(ctx, ids, &pl)) return st;
    hipStream_t s = (hipStream_t)stream;
    for (const Group &g : pl->groups) {
        const int cnt = (int)g.ids.size();
        HIPCK(ctx, launch_grad_zinv(g.n, g.prec, g.dev, cnt, g.tw, s));
        HIPCK(ctx, launch_grad_yinv(g.n, g.prec, g.dev, cnt, g.tw, s));
        HIPCK(ctx, launch_grad_xstats(g.n, g.prec, g.dev, cnt, ctx->hist, ctx->ledge, g.tw, s));
        HIPCK(ctx, launch_stats_reduce(g.n, g.prec, g.dev, cnt, s));
    }
    for (int id : ids) ctx->members[id]->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_get_stats(ens_ctx *ctx, int32_t mid, uint64_t *counts, double *moments, uint64_t *n_points) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!ctx->has_hist) return fail(ENS_E_STATE, "context has no histogram descriptor");
    Member *m;
    if (ens_status st = member_of(ctx, mid, &m)) return st;
    HIPCK(ctx, hipSetDevice(ctx->device));
    HIPCK(ctx, hipStreamSynchronize(m->last));
    if (counts) HIPCK(ctx, hipMemcpy(counts, m->md.counts, ctx->hg.n_counts * sizeof(uint64_t), hipMemcpyDeviceToHost));
    if (moments) HIPCK(ctx, hipMemcpy(moments, m->md.moments, ENS_NMOM * sizeof(double), hipMemcpyDeviceToHost));
    if (n_points) {
        // every snapshot adds n^3 samples to the QR histogram (bins + specials)
        std::vector<uint64_t> c(ctx->hg.n_counts);
        HIPCK(ctx, hipMemcpy(c.data(), m->md.counts, c.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
        uint64_t s = 0;
        for (long long i = 0; i < ctx->hg.off_le; i++) s += c[i];
        *n_points = s;
    }
    return ENS_OK;
}

static_assert(offsetof(DevState, diag) == 0, "ens_member_set_diag writes the record at the start of DevState");

ENS_API ens_status ens_member_set_diag(ens_ctx *ctx, int32_t mid, const ens_diag *d, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    Member *m;
    if (ens_status st = member_of(ctx, mid, &m)) return st;
    if (!d) return fail(ENS_E_INVALID, "null diagnostics record");
    if (!(d->t >= 0.0) || !std::isfinite(d->t)) return fail(ENS_E_INVALID, "time must be finite and >= 0");
    if (d->step < 0) return fail(ENS_E_INVALID, "step count must be >= 0");
    if (d->reserved != 0) return fail(ENS_E_INVALID, "reserved must be 0");
    HIPCK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const ens_diag rec = *d;
    // DevState begins with the ens_diag record
    HIPCK(ctx, hipMemcpyAsync(m->md.st, &rec, sizeof(ens_diag), hipMemcpyHostToDevice, s));
    HIPCK(ctx, hipStreamSynchronize(s));
    m->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_set_stats(ens_ctx *ctx, int32_t mid, const uint64_t *counts, const double *moments, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!ctx->has_hist) return fail(ENS_E_STATE, "context has no histogram descriptor");
    Member *m;
    if (ens_status st = member_of(ctx, mid, &m)) return st;
    HIPCK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (counts)
        HIPCK(ctx, hipMemcpyAsync(m->md.counts, counts, ctx->hg.n_counts * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    if (moments)
        HIPCK(ctx, hipMemcpyAsync(m->md.moments, moments, ENS_NMOM * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCK(ctx, hipStreamSynchronize(s));
    m->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_reset_stats(ens_ctx *ctx, int32_t mid, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!ctx->has_hist) return fail(ENS_E_STATE, "context has no histogram descriptor");
    Member *m;
    if (ens_status st = member_of(ctx, mid, &m)) return st;
    HIPCK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    HIPCK(ctx, launch_fill_u64(m->md.counts, ctx->hg.n_counts, 0ull, s));
    HIPCK(ctx, launch_fill_f64(m->md.moments, ENS_NMOM, 0.0, s));
    m->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_mix_len(const ens_ctx *ctx, int32_t count, size_t *n_out) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!ctx->has_hist) return fail(ENS_E_STATE, "context has no histogram descriptor");
    if (count <= 0 || !n_out) return fail(ENS_E_INVALID, "bad arguments");
    const HistGeom &g = ctx->hg;
    *n_out = (size_t)count + (size_t)g.qb * g.qb + 2 * (size_t)g.lb + 2 * (size_t)g.ab + ENS_NMOM + 8;
    return ENS_OK;
}

ENS_API ens_status ens_mix(ens_ctx *ctx, const int32_t *members, int32_t count, double c, double Z,
                           int32_t weight_mode, double q_sigma, double *dev_out, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!ctx->has_hist) return fail(ENS_E_STATE, "context has no histogram descriptor");
    std::vector<int> ids;
    if (ens_status st = collect_ids(ctx, members, count, ids)) return st;
    if (!dev_out) return fail(ENS_E_INVALID, "null output pointer");
    if (count > mix_max_members()) return fail(ENS_E_INVALID, "too many members for one mixture call");
    if (!(c > 0) || !(Z >= 0) || !std::isfinite(Z)) return fail(ENS_E_INVALID, "need c > 0 and Z >= 0");
    if (weight_mode < 0 || weight_mode > 3) return fail(ENS_E_INVALID, "weight_mode must be 0, 1, 2 or 3");
    if (weight_mode == 2 && (!(q_sigma > 0) || !(Z > 0))) return fail(ENS_E_INVALID, "mode 2 needs q_sigma > 0 and Z > 0");
    HIPCK(ctx, hipSetDevice(ctx->device));
    std::vector<const MemberDev *> mds;
    std::vector<double> lam;
    for (int id : ids) {
        mds.push_back(&ctx->members[id]->md);
        lam.push_back(ctx->members[id]->d.lambda);
    }
    hipStream_t s = (hipStream_t)stream;
    for (int id : ids) HIPCK(ctx, hipStreamSynchronize(ctx->members[id]->last));
    const size_t need = mix_scratch_bytes(count);
    if (need > ctx->mix_scratch_bytes) {
        // an earlier mixture's kernels may still read the old table
        if (ctx->mix_scratch) HIPCK(ctx, hipDeviceSynchronize());
        if (ctx->mix_scratch) HIPCK(ctx, hipFree(ctx->mix_scratch));
        ctx->mix_scratch = nullptr;
        HIPCK(ctx, hipMalloc(&ctx->mix_scratch, need));
        ctx->mix_scratch_bytes = need;
    }
    HIPCK(ctx, launch_mix(mds.data(), lam.data(), count, ctx->hist, c, Z, weight_mode, q_sigma, dev_out,
                          ctx->mix_scratch, s));
    return ENS_OK;
}

ENS_API ens_status ens_mix_noalloc(ens_ctx *ctx, const int32_t *members, int32_t count, double c, double Z,
                                   int32_t weight_mode, double q_sigma, double *dev_out, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!ctx->has_hist) return fail(ENS_E_STATE, "context has no histogram descriptor");
    if (!members || count <= 0) return fail(ENS_E_INVALID, "empty member list");
    if (count > ENS_MIX_STATIC_MAX)
        return fail(ENS_E_INVALID, "too many members for the static mixture table (at most " +
                                       std::to_string(ENS_MIX_STATIC_MAX) + ")");
    if (!dev_out) return fail(ENS_E_INVALID, "null output pointer");
    if (!(c > 0) || !(Z >= 0) || !std::isfinite(Z)) return fail(ENS_E_INVALID, "need c > 0 and Z >= 0");
    if (weight_mode < 0 || weight_mode > 3) return fail(ENS_E_INVALID, "weight_mode must be 0, 1, 2 or 3");
    if (weight_mode == 2 && (!(q_sigma > 0) || !(Z > 0))) return fail(ENS_E_INVALID, "mode 2 needs q_sigma > 0 and Z > 0");
    // ids checked without heap allocation: bounds, then duplicates on a sorted copy
    int32_t sorted[ENS_MIX_STATIC_MAX];
    const MemberDev *mds[ENS_MIX_STATIC_MAX];
    double lam[ENS_MIX_STATIC_MAX];
    for (int32_t i = 0; i < count; i++) {
        Member *m;
        if (ens_status st = member_of(ctx, members[i], &m)) return st;
        sorted[i] = members[i];
        mds[i] = &m->md;
        lam[i] = m->d.lambda;
    }
    std::sort(sorted, sorted + count);
    if (std::adjacent_find(sorted, sorted + count) != sorted + count) return fail(ENS_E_INVALID, "duplicate member id");
    HIPCK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    for (int32_t i = 0; i < count; i++) HIPCK(ctx, hipStreamSynchronize(ctx->members[members[i]]->last));
    HIPCK(ctx, launch_mix_static(ctx->device, mds, lam, count, ctx->hist, c, Z, weight_mode, q_sigma, dev_out, s));
    return ENS_OK;
}

ENS_API ens_status ens_mix_table(ens_ctx *ctx, const int32_t *members, int32_t count, const double *dev_pdf,
                                 int32_t table_len, double lam0, double dlam, double *dev_out, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!ctx->has_hist) return fail(ENS_E_STATE, "context has no histogram descriptor");
    std::vector<int> ids;
    if (ens_status st = collect_ids(ctx, members, count, ids)) return st;
    if (!dev_out || !dev_pdf) return fail(ENS_E_INVALID, "null pointer");
    if (count > mix_max_members()) return fail(ENS_E_INVALID, "too many members for one mixture call");
    if (table_len < 2 || !(dlam > 0) || !std::isfinite(lam0) || !std::isfinite(dlam))
        return fail(ENS_E_INVALID, "need table_len >= 2, dlam > 0 and a finite grid");
    HIPCK(ctx, hipSetDevice(ctx->device));
    std::vector<const MemberDev *> mds;
    std::vector<double> lam;
    for (int id : ids) {
        mds.push_back(&ctx->members[id]->md);
        lam.push_back(ctx->members[id]->d.lambda);
    }
    hipStream_t s = (hipStream_t)stream;
    for (int id : ids) HIPCK(ctx, hipStreamSynchronize(ctx->members[id]->last));
    const size_t need = mix_scratch_bytes(count);
    if (need > ctx->mix_scratch_bytes) {
        // an earlier mixture's kernels may still read the old table
        if (ctx->mix_scratch) HIPCK(ctx, hipDeviceSynchronize());
        if (ctx->mix_scratch) HIPCK(ctx, hipFree(ctx->mix_scratch));
        ctx->mix_scratch = nullptr;
        HIPCK(ctx, hipMalloc(&ctx->mix_scratch, need));
        ctx->mix_scratch_bytes = need;
    }
    HIPCK(ctx, launch_mix_table(mds.data(), lam.data(), count, ctx->hist, 1.0, 0.0, 4, 1.0, dev_pdf, table_len, lam0,
                                dlam, dev_out, ctx->mix_scratch, s));
    return ENS_OK;
}

ENS_API ens_status ens_lambda_pdf_from_cf(const double *dev_phi, int32_t table_len, double lam0, double dlam,
                                          double *dev_pdf, void *stream) {
    if (!dev_phi || !dev_pdf) return fail(ENS_E_INVALID, "null pointer");
    if (table_len < 2 || table_len > kMaxCfTable || !(dlam > 0) || !std::isfinite(lam0) || !std::isfinite(dlam))
        return fail(ENS_E_INVALID, "need 2 <= table_len <= 65536, dlam > 0 and a finite grid");
    const hipError_t e = launch_cf_invert(dev_phi, table_len, lam0, dlam, dev_pdf, (hipStream_t)stream);
    if (e != hipSuccess) return fail(ENS_E_HIP, hipGetErrorString(e));
    return ENS_OK;
}

ENS_API ens_status ens_scale_gap(ens_ctx *ctx, const int32_t *members, int32_t count, double rlambda_ref,
                                 double *Z_out, double *prefactor_out, double *rlambda_out) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!ctx->has_hist) return fail(ENS_E_STATE, "context has no histogram descriptor");
    std::vector<int> ids;
    if (ens_status st = collect_ids(ctx, members, count, ids)) return st;
    if (!Z_out || !prefactor_out) return fail(ENS_E_INVALID, "null output pointer");
    if (!(rlambda_ref > 0) || !std::isfinite(rlambda_ref)) return fail(ENS_E_INVALID, "need R_lambda,ref > 0");
    HIPCK(ctx, hipSetDevice(ctx->device));
    std::vector<double> rl(ids.size());
    double acc = 0.0;
    int used = 0;
    for (size_t i = 0; i < ids.size(); i++) {
        Member *m = ctx->members[ids[i]].get();
        HIPCK(ctx, hipStreamSynchronize(m->last));
        double mom[3];
        HIPCK(ctx, hipMemcpy(mom, m->md.moments + 26, sizeof(mom), hipMemcpyDeviceToHost));
        if (!(mom[2] > 0)) return fail(ENS_E_STATE, "a member has no statistics snapshot");
        const double E = mom[0] / mom[2], D = mom[1] / mom[2];
        if (!(E > 0) || !(D > 0)) return fail(ENS_E_STATE, "a member has no positive mean energy and dissipation");
        rl[i] = (2.0 * E / 3.0) * std::sqrt(15.0 / (m->d.nu * D));
        if (m->d.lambda >= 0.0) {
            acc += std::log(rl[i]) - m->d.lambda / 6.0;
            used++;
        }
    }
    if (!used) return fail(ENS_E_INVALID, "no member with lambda >= 0");
    const double A = std::exp(acc / used);
    *prefactor_out = A;
    *Z_out = 1.5 * std::log(rlambda_ref / A);
    if (rlambda_out) std::copy(rl.begin(), rl.end(), rlambda_out);
    return ENS_OK;
}

ENS_API ens_status ens_spectrum(ens_ctx *ctx, int32_t mid, int32_t nshell, double *dev_out, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    Member *m;
    if (ens_status st = member_of(ctx, mid, &m)) return st;
    if (nshell < 1) return fail(ENS_E_INVALID, "nshell must be >= 1");
    if (!dev_out) return fail(ENS_E_INVALID, "null output pointer");
    HIPCK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    HIPCK(ctx, launch_spectrum(m->d.precision, m->dev, m->g.K, nshell, dev_out, s));
    m->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_integral_scales(ens_ctx *ctx, int32_t mid, double *dev_out, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    Member *m;
    if (ens_status st = member_of(ctx, mid, &m)) return st;
    if (!dev_out) return fail(ENS_E_INVALID, "null output pointer");
    HIPCK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    HIPCK(ctx, launch_scales(m->d.precision, m->dev, m->g.K, dev_out, s));
    m->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_member_refine(ens_ctx *ctx, int32_t src, int32_t dst, void *stream) {
    if (ens_status st = check_ctx(ctx)) return st;
    Member *a, *b;
    if (ens_status st = member_of(ctx, src, &a)) return st;
    if (ens_status st = member_of(ctx, dst, &b)) return st;
    if (src == dst) return fail(ENS_E_INVALID, "refinement needs two members");
    if (b->d.n < a->d.n) return fail(ENS_E_INVALID, "refinement needs n_dst >= n_src");
    if (std::fabs(a->d.box - b->d.box) > 1e-12 * a->d.box) return fail(ENS_E_INVALID, "refinement needs the same box");
    HIPCK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    HIPCK(ctx, launch_refine(a->d.precision, b->d.precision, a->dev, b->dev, b->d.n, s));
    a->last = s;
    b->last = s;
    return ENS_OK;
}

ENS_API ens_status ens_fft_pencils(int32_t n, int32_t precision, int32_t sign, int64_t lines, const void *dev_in,
                                   void *dev_out, void *stream) {
    if (!pow2_supported(n)) return fail(ENS_E_UNSUPPORTED, "n must be one of 16, 32, 64, 128, 256, 512, 1024");
    if (precision != ENS_FP64 && precision != ENS_FP32) return fail(ENS_E_INVALID, "bad precision");
    if (sign != 1 && sign != -1) return fail(ENS_E_INVALID, "sign must be +1 or -1");
    if (lines < 0) return fail(ENS_E_INVALID, "lines must be >= 0");
    if (lines == 0) return ENS_OK;
    if (!dev_in || !dev_out) return fail(ENS_E_INVALID, "null data pointer");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(ENS_E_HIP, hipGetErrorString(e));
    const void *tw;
    e = get_twiddles(dev, n, precision, &tw);
    if (e != hipSuccess) return fail(ENS_E_HIP, hipGetErrorString(e));
    e = launch_fft_pencils(n, precision, sign, lines, dev_in, dev_out, tw, (hipStream_t)stream);
    if (e != hipSuccess) return fail(ENS_E_HIP, hipGetErrorString(e));
    return ENS_OK;
}

namespace {

const char *pass_name(int p) {
    static const char *names[ENS_NPASS] = {"band", "zinv", "yinv", "xpass", "yfwd", "zfwd_update", "end_step"};
    return (p >= 0 && p < ENS_NPASS) ? names[p] : "?";
}

std::string variant_key(int pass, int n, int prec) {
    return std::string(pass_name(pass)) + ":" + std::to_string(n) + ":" + (prec == ENS_FP32 ? "fp32" : "fp64");
}

// cache file: one "key variant" pair per line, '#' comments
void read_cache(const char *path, std::map<std::string, int> &out) {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::string key;
        int v;
        if (is >> key >> v) out[key] = v;
    }
}

void drop_graphs(ens_ctx *ctx) {
    for (auto &kv : ctx->plans) free_graphs(*kv.second);
}

}  // namespace

ENS_API ens_status ens_set_variant(ens_ctx *ctx, int32_t pass, int32_t n, int32_t precision, int32_t variant) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (pass < 0 || pass >= ENS_NPASS || variant < 0 || variant >= pass_variants(pass))
        return fail(ENS_E_INVALID, "bad pass or variant");
    if (!pow2_supported(n) || (precision != ENS_FP32 && precision != ENS_FP64)) return fail(ENS_E_INVALID, "bad n or precision");
    ctx->variant[std::make_tuple(pass, n, precision)] = variant;
    drop_graphs(ctx);
    return ENS_OK;
}

ENS_API ens_status ens_get_variant(const ens_ctx *ctx, int32_t pass, int32_t n, int32_t precision, int32_t *variant) {
    if (ens_status st = check_ctx(ctx)) return st;
    if (!variant || pass < 0 || pass >= ENS_NPASS) return fail(ENS_E_INVALID, "bad arguments");
    *variant = variant_of(ctx, pass, n, precision);
    return ENS_OK;
}

ENS_API ens_status ens_autotune(ens_ctx *ctx, const int32_t *members, int32_t count, void *stream, const char *cache_path) {
    if (ens_status st = check_ctx(ctx)) return st;
    std::vector<int> ids;
    if (ens_status st = collect_ids(ctx, members, count, ids)) return st;
    HIPCK(ctx, hipSetDevice(ctx->device));
    Plan *pl;
    if (ens_status st = make_plan(ctx, ids, &pl)) return st;
    hipStream_t s = (hipStream_t)stream;
    std::map<std::string, int> cache;
    if (cache_path) read_cache(cache_path, cache);
    hipEvent_t a, b;
    HIPCK(ctx, hipEventCreate(&a));
    HIPCK(ctx, hipEventCreate(&b));
    // Only the transform passes are timed: they write nothing but their
    // scratch buffers, so the members' state is unchanged by tuning.
    for (const Group &g : pl->groups) {
        const int cnt = (int)g.ids.size();
        for (int pass : {P_ZINV, P_YINV, P_XPASS, P_YFWD}) {
            const std::string key = variant_key(pass, g.n, g.prec);
            auto hit = cache.find(key);
            if (hit != cache.end() && hit->second >= 0 && hit->second < pass_variants(pass)) {
                ctx->variant[std::make_tuple(pass, g.n, g.prec)] = hit->second;
                continue;
            }
            int best = 0;
            float best_ms = 1e30f;
            // each variant: warm-up, then three timed runs of five launches; the
            // fastest run counts (variants within a few per cent of each other
            // are otherwise decided by interference from the rest of the device)
            // The x pass is timed in its place in the stage, each launch after
            // the y inverse (already tuned) that writes its inputs: variants
            // within a few per cent of each other in isolation rank differently
            // there.
            const int prev = pass == P_XPASS ? variant_of(ctx, P_YINV, g.n, g.prec) : -1;
            auto launch = [&](int v) -> hipError_t {
                if (prev >= 0)
                    if (hipError_t e = launch_pass(P_YINV, prev, g.n, g.prec, g.dev, cnt, 1, g.tw, s)) return e;
                return launch_pass(pass, v, g.n, g.prec, g.dev, cnt, 1, g.tw, s);
            };
            for (int v = 0; v < pass_variants(pass); v++) {
                for (int w = 0; w < 2; w++) HIPCK(ctx, launch(v));
                float v_ms = 1e30f;
                for (int trial = 0; trial < 3; trial++) {
                    HIPCK(ctx, hipEventRecord(a, s));
                    const int reps = 5;
                    for (int r = 0; r < reps; r++) HIPCK(ctx, launch(v));
                    HIPCK(ctx, hipEventRecord(b, s));
                    HIPCK(ctx, hipEventSynchronize(b));
                    float ms = 0.f;
                    HIPCK(ctx, hipEventElapsedTime(&ms, a, b));
                    v_ms = ms < v_ms ? ms : v_ms;
                }
                if (v_ms < best_ms) { best_ms = v_ms; best = v; }
            }
            ctx->variant[std::make_tuple(pass, g.n, g.prec)] = best;
            cache[key] = best;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    drop_graphs(ctx);
    if (cache_path) {
        std::ofstream f(cache_path);
        f << "# libensdns kernel variants (pass:n:precision variant); 0 = 8, 1 = 16 values per thread, 2 and 3 = the same with twice the lines per workgroup (y/z passes) or the streamed x pass with 8 and 16, 4 to 6 = wave-private streamed x pass\n";
        for (auto &kv : cache) f << kv.first << " " << kv.second << "\n";
    }
    return ENS_OK;
}
