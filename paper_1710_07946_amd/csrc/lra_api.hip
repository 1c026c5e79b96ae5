// lra_api.hip -- host side of the C ABI declared in include/lra_cur.h:
// argument validation, launch geometry (team size, LDS budget), and the
// cached per-(device, stream) workspace.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>
#include <utility>
#include <vector>

#include "lra_internal.h"

namespace {

using lra::BlockDesc;
using lra::PtsDesc;
using lra::CAConfig;
using lra::kBlock;
using lra::kLMax;
using lra::kSMax;
using lra::kRMax;
using lra::TeamWs;

struct Workspace {
    int device = -1;
    unsigned *counters = nullptr;   // [1 ..] work queues of the batched launches
    uint64_t *xw = nullptr;         // team exchange words [2][kMaxTeam][kSlotWords]
    int64_t *init_cols = nullptr;   // [kRMax]
    unsigned char *desc = nullptr;  // batch descriptors, then the launch order (int32)
    size_t desc_cap = 0;            // bytes
    void *stage = nullptr;          // pinned host staging of the descriptors and the order
    size_t stage_cap = 0;           // bytes
    hipEvent_t stage_done = nullptr;  // the last copy out of `stage` has completed
    std::vector<unsigned char> staged;  // bytes of the last staged copy (equal bytes: no copy)
    int32_t *bidiag = nullptr;      // bidiagonal-multiplier column table (kBdTableInts)
    double *sketch = nullptr;       // global sketch panels when they do not fit LDS
    size_t sketch_cap = 0;          // bytes
    void *work = nullptr;           // residual / adjoint / leverage work arrays
    size_t work_cap = 0;            // bytes
};

// Grow-only work array of a workspace (the stream is drained before a reallocation).
lra_status ws_work(Workspace *w, hipStream_t stream, size_t bytes, void **out) {
    if (w->work_cap < bytes) {
        (void)hipStreamSynchronize(stream);
        (void)hipFree(w->work);
        w->work = nullptr;
        w->work_cap = 0;
        if (hipMalloc(&w->work, bytes) != hipSuccess) return LRA_ENOMEM;
        w->work_cap = bytes;
    }
    *out = w->work;
    return LRA_OK;
}

// Copy `bytes` of host descriptors to the workspace's device descriptor
// buffer without blocking the host: the bytes go through a pinned staging
// buffer, which is reused once the previous copy out of it has completed (an
// event), and a call whose bytes equal the last staged ones copies nothing.
lra_status stage_desc(Workspace *w, hipStream_t stream, const void *host, size_t bytes, unsigned char **dev_out) {
    if (w->desc_cap < bytes) {
        (void)hipStreamSynchronize(stream);
        (void)hipFree(w->desc);
        w->desc = nullptr;
        w->desc_cap = 0;
        w->staged.clear();
        if (hipMalloc((void **)&w->desc, bytes) != hipSuccess) return LRA_ENOMEM;
        w->desc_cap = bytes;
    }
    *dev_out = w->desc;
    if (w->staged.size() == bytes && memcmp(w->staged.data(), host, bytes) == 0) return LRA_OK;
    if (!w->stage_done && hipEventCreateWithFlags(&w->stage_done, hipEventDisableTiming) != hipSuccess)
        return LRA_EDEVICE;
    if (hipEventSynchronize(w->stage_done) != hipSuccess) return LRA_EDEVICE;
    if (w->stage_cap < bytes) {
        if (w->stage) (void)hipHostFree(w->stage);
        w->stage = nullptr;
        w->stage_cap = 0;
        if (hipHostMalloc(&w->stage, bytes, hipHostMallocDefault) != hipSuccess) return LRA_ENOMEM;
        w->stage_cap = bytes;
    }
    memcpy(w->stage, host, bytes);
    w->staged.clear();
    if (hipMemcpyAsync(w->desc, w->stage, bytes, hipMemcpyHostToDevice, stream) != hipSuccess) return LRA_EDEVICE;
    if (hipEventRecord(w->stage_done, stream) != hipSuccess) return LRA_EDEVICE;
    w->staged.assign(static_cast<const unsigned char *>(host), static_cast<const unsigned char *>(host) + bytes);
    return LRA_OK;
}

using lra::kMaxTeam;

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

struct DevInfo {
    int cus = 0;
    int lds = 0;
    int wall_khz = 0;  // rate of the device wall clock
};
std::map<int, DevInfo> g_dev;

lra_status query_dev(int dev, DevInfo *d);

lra_status dev_info(int dev, DevInfo *out) {
    auto it = g_dev.find(dev);
    if (it == g_dev.end()) {
        DevInfo d;
        lra_status st = query_dev(dev, &d);
        if (st != LRA_OK) return st;
        it = g_dev.emplace(dev, d).first;
    }
    *out = it->second;
    return LRA_OK;
}

lra_status get_ws(hipStream_t stream, Workspace **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LRA_EDEVICE;
    Workspace &w = g_ws[std::make_pair(dev, stream)];
    if (!w.counters) {
        w.device = dev;
        if (hipMalloc(&w.counters, 64 * sizeof(unsigned)) != hipSuccess) return LRA_ENOMEM;
        if (hipMalloc(&w.xw, (size_t)2 * kMaxTeam * lra::kSlotWords * sizeof(uint64_t)) != hipSuccess)
            return LRA_ENOMEM;
        if (hipMalloc(&w.init_cols, kRMax * sizeof(int64_t)) != hipSuccess) return LRA_ENOMEM;
    }
    *out = &w;
    return LRA_OK;
}

lra_status fill_config(const lra_opts *opts, int32_t r, int32_t sweeps, CAConfig *c, lra_opts *o_out) {
    lra_opts o;
    if (opts) o = *opts;
    else lra_default_opts(&o);
    if (!(o.delta >= 0.0) || !std::isfinite(o.delta)) return LRA_EINVAL;
    if (o.preprocess != LRA_PRE_NONE && o.preprocess != LRA_PRE_ASRHT && o.preprocess != LRA_PRE_BIDIAG &&
        o.preprocess != LRA_PRE_ASRFT)
        return LRA_EINVAL;
    if (o.max_swaps < 0) o.max_swaps = 16 * r;
    if (o.ah_samples <= 0) o.ah_samples = 2 * r;
    if (o.refine_steps < 0 || o.refine_steps > 16) return LRA_EINVAL;
    if (o.preprocess == LRA_PRE_ASRHT) {
        if (o.ah_depth < 0 || o.ah_depth > 20) return LRA_EINVAL;
        if (o.ah_samples < r || o.ah_samples > kLMax) return LRA_EINVAL;
    }
    if (o.preprocess == LRA_PRE_BIDIAG) {
        if (o.ah_depth < 0 || (1 << o.ah_depth) > lra::kBdTerms) return LRA_EINVAL;
        if (o.ah_samples < r || o.ah_samples > kLMax) return LRA_EINVAL;
    }
    if (o.preprocess == LRA_PRE_ASRFT) {
        // the coefficient table (l 2^d complex entries) lives in the LU
        // scratch of the workgroup, which the sketch does not use
        if (o.ah_depth < 0 || o.ah_depth > 3) return LRA_EINVAL;
        if (2 * o.ah_samples < r || 2 * o.ah_samples > kLMax || (o.ah_samples << o.ah_depth) > lra::kAftCoefs)
            return LRA_EINVAL;
    }
    c->r = r;
    c->sweeps = sweeps;
    c->delta = o.delta;
    c->max_swaps = o.max_swaps;
    c->pre = o.preprocess;
    c->ah_depth = o.ah_depth;
    c->ah_samples = o.ah_samples;
    c->refine_steps = o.refine_steps;
    c->panel_bytes = 0;
    c->init_cols = nullptr;
    c->sketch_ws = nullptr;
    c->bd_table = nullptr;
    c->margins = o.track_margin ? 1 : 0;
    *o_out = o;
    return LRA_OK;
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// LDS plan for a team of `team` workgroups: the C-A panel slice (largest of
// the column and row panels, r doubles per item) and the nucleus workspace
// (4 r^2 doubles) always live in LDS; the sketch slice (l doubles per item)
// joins them when it fits, else it goes to global memory.
struct LdsPlan {
    size_t panel_bytes = 0;  // dynamic LDS before the flag bytes
    size_t dyn_bytes = 0;    // total dynamic LDS
    bool sketch_global = false;
    int64_t ipw_s = 0;       // sketch items per workgroup
    bool fits = false;
};

LdsPlan plan_lds(int64_t m, int64_t n, int r, int pre, int l, int team, size_t budget) {
    LdsPlan p;
    const int64_t ipw = std::max((m + team - 1) / team, (n + team - 1) / team);
    // panels are slot-major with the slot stride rounded up to odd
    size_t cells = std::max((size_t)(ipw | 1) * r, (size_t)4 * r * r);
    int64_t flag_items = ipw;
    if (pre == LRA_PRE_ASRHT || pre == LRA_PRE_BIDIAG || pre == LRA_PRE_ASRFT) {
        p.ipw_s = ((m >= n) ? (n + team - 1) / team : (m + team - 1) / team);
        const size_t sk = (size_t)(p.ipw_s | 1) * l;
        const size_t with = align16(std::max(cells, sk) * sizeof(double)) + align16(std::max(ipw, p.ipw_s));
        if (with <= budget) {
            cells = std::max(cells, sk);
            flag_items = std::max(ipw, p.ipw_s);
        } else {
            p.sketch_global = true;
            flag_items = std::max(ipw, p.ipw_s);
        }
    }
    p.panel_bytes = align16(cells * sizeof(double));
    p.dyn_bytes = p.panel_bytes + align16((size_t)flag_items);
    p.fits = p.dyn_bytes <= budget;
    return p;
}

// Options, launch geometry and global sketch size of one lra_cur call (shared
// by lra_cur and lra_cur_noalloc).
struct CurPlan {
    CAConfig cfg;
    lra_opts o;
    int team = 0;
    LdsPlan lds;
    size_t sketch_bytes = 0;  // global sketch panel (0: the sketch slices live in LDS)
};

// Argument checks of lra_cur that need no device state.
lra_status check_cur(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r, int32_t sweeps,
                     const lra_opts *opts, const int64_t *I_out, const int64_t *J_out, const double *U_out,
                     CurPlan *cp) {
    if (!W || !I_out || !J_out || !U_out) return LRA_EINVAL;
    if (dt != LRA_F64 && dt != LRA_F32 && dt != LRA_BF16) return LRA_EINVAL;
    if (m < 1 || n < 1 || lda < n || r < 1 || r > kRMax || r > m || r > n || sweeps < 1) return LRA_EINVAL;
    if (m >= ((int64_t)1 << 39) || n >= ((int64_t)1 << 39)) return LRA_EINVAL;  // item ids travel in 40 bits
    lra_opts &o = cp->o;
    lra_status st = fill_config(opts, r, sweeps, &cp->cfg, &o);
    if (st != LRA_OK) return st;
    if (o.preprocess == LRA_PRE_ASRHT || o.preprocess == LRA_PRE_ASRFT) {
        const int64_t dim = (m >= n) ? m : n;  // the dimension the multiplier acts on
        const int64_t q2 = (int64_t)1 << o.ah_depth;
        const int64_t N = q2 * ((dim + q2 - 1) / q2);
        if (o.ah_samples > N) return LRA_EINVAL;
    }
    if (o.preprocess == LRA_PRE_BIDIAG) {
        const int64_t dim = (m >= n) ? m : n;  // the dimension the multiplier acts on
        if (dim < 2 || dim > (int64_t)INT32_MAX || o.ah_samples > dim) return LRA_EINVAL;
    }
    if (o.init_cols) {
        if (o.preprocess != LRA_PRE_NONE) return LRA_EINVAL;
        for (int a = 0; a < r; a++) {
            if (o.init_cols[a] < 0 || o.init_cols[a] >= n) return LRA_EINVAL;
            for (int b = 0; b < a; b++)
                if (o.init_cols[a] == o.init_cols[b]) return LRA_EINVAL;
        }
    }
    return LRA_OK;
}

// Team size and LDS plan of an lra_cur call.  Team size: the smallest number
// of workgroups whose panel slices fit in LDS, but at least one workgroup per
// 160 items (more workgroups shorten the per-decision scans, fewer make each
// team selection cheaper; 160 was the best trade-off measured on the
// 20000 x 20000 rank-50 workload).
lra_status plan_cur(const DevInfo &dinfo, int64_t m, int64_t n, int32_t r, CurPlan *cp) {
    const lra_opts &o = cp->o;
    const int max_team = std::min(dinfo.cus, kMaxTeam);
    const size_t lds_budget = (size_t)dinfo.lds - lra::static_lds_bytes() - 256;
    // real width of the sketch panel (the Fourier sketch keeps Re and Im)
    const int wsk = o.preprocess == LRA_PRE_ASRFT ? 2 * o.ah_samples : o.ah_samples;
    int team;
    LdsPlan plan;
    if (o.team_size > 0) {
        team = std::min(o.team_size, max_team);
        plan = plan_lds(m, n, r, o.preprocess, wsk, team, lds_budget);
    } else {
        team = (int)std::min<int64_t>(max_team, std::max<int64_t>(1, (std::max(m, n) + 159) / 160));
        plan = plan_lds(m, n, r, o.preprocess, wsk, team, lds_budget);
        while (!plan.fits && team < max_team) {
            team++;
            plan = plan_lds(m, n, r, o.preprocess, wsk, team, lds_budget);
        }
    }
    if (!plan.fits) return LRA_EUNSUPPORTED;
    cp->team = team;
    cp->lds = plan;
    cp->cfg.panel_bytes = (int32_t)plan.panel_bytes;
    cp->sketch_bytes = plan.sketch_global ? (size_t)team * (plan.ipw_s | 1) * wsk * sizeof(double) : 0;
    return LRA_OK;
}

lra_status query_dev(int dev, DevInfo *d) {
    if (hipDeviceGetAttribute(&d->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return LRA_EDEVICE;
    if (hipDeviceGetAttribute(&d->lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return LRA_EDEVICE;
    if (hipDeviceGetAttribute(&d->wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || d->wall_khz <= 0)
        d->wall_khz = 100000;
    return LRA_OK;
}

// ---- batched launches: size bins and their kernel variants
constexpr int kSrcPoints = 3;  // source code of the point-set form (beside the dtype codes)
constexpr int kMaxRules = 64;

// Built-in bin table (rank 16, the far-field workload's rank): blocks whose
// larger dimension is at most max_dim run on the register kernel with
// items_per_lane x waves x 64 >= max_dim item slots per workgroup; anything
// no rule covers runs on the LDS kernel.  A table measured by the tuner
// (tune_batched.py) replaces it at build time.
std::vector<lra_batch_rule> default_rules() {
#if __has_include("lra_tuned_rules.inc")
    static const lra_batch_rule tab[] = {
#include "lra_tuned_rules.inc"
    };
#else
    static const lra_batch_rule tab[] = {
        {128, 16, 2, 1}, {256, 16, 2, 2}, {512, 16, 2, 4}, {1024, 16, 2, 8},
    };
#endif
    std::vector<lra_batch_rule> v(tab, tab + sizeof(tab) / sizeof(tab[0]));
    std::stable_sort(v.begin(), v.end(),
                     [](const lra_batch_rule &a, const lra_batch_rule &b) { return a.max_dim < b.max_dim; });
    return v;
}

std::vector<lra_batch_rule> g_rules;
bool g_rules_set = false;

const std::vector<lra_batch_rule> &current_rules() {
    if (!g_rules_set) {
        g_rules = default_rules();
        g_rules_set = true;
    }
    return g_rules;
}

// Run a batch: bin the blocks by the rule table, stage the descriptors and the
// launch order (bins one after another, each largest first by m + n), then
// one persistent launch per bin on `stream`, the LDS bin and the bins of the
// largest blocks first.  desc points at `count` 32-byte descriptors
// (BlockDesc, or PtsDesc for src == kSrcPoints); dims holds (m, n) per block.
lra_status batched_run(int src, const void *base, const void *desc, const int64_t *dims, int64_t count,
                       CAConfig cfg, uint64_t seed, int64_t *I_out, int64_t *J_out, double *U_out, lra_info *infos,
                       hipStream_t stream) {
    const int r = cfg.r;
    std::lock_guard<std::mutex> lk(g_mu);
    const std::vector<lra_batch_rule> &rules = current_rules();
    struct Bin {
        int P, W;
        int64_t cap;   // item slots per workgroup (0: LDS kernel)
        std::vector<int32_t> ids;
        int64_t maxdim = 0;
    };
    std::vector<Bin> bins;
    auto bin_of = [&](int P, int W) -> Bin & {
        for (Bin &b : bins)
            if (b.P == P && b.W == W) return b;
        bins.push_back(Bin{P, W, (int64_t)64 * P * W, {}, 0});
        return bins.back();
    };
    for (int64_t b = 0; b < count; b++) {
        const int64_t d = std::max(dims[2 * b], dims[2 * b + 1]);
        int P = 0, W = 0;
        for (const lra_batch_rule &q : rules)
            if (q.r == r && d <= q.max_dim) {
                P = q.items_per_lane;
                W = q.waves;
                break;
            }
        Bin &bn = bin_of(P, W);
        bn.ids.push_back((int32_t)b);
        bn.maxdim = std::max(bn.maxdim, d);
    }
    // the LDS kernel's bin first (it holds the blocks too large for any
    // register variant), then by capacity, largest first
    std::stable_sort(bins.begin(), bins.end(), [](const Bin &a, const Bin &b) {
        if ((a.P == 0) != (b.P == 0)) return a.P == 0;
        return a.cap > b.cap;
    });
    if (bins.size() > 60) return LRA_EUNSUPPORTED;
    std::vector<unsigned char> host((size_t)count * 32 + (size_t)count * sizeof(int32_t));
    memcpy(host.data(), desc, (size_t)count * 32);
    int32_t *ord = reinterpret_cast<int32_t *>(host.data() + (size_t)count * 32);
    std::vector<int64_t> first(bins.size());
    int64_t at = 0;
    for (size_t i = 0; i < bins.size(); i++) {
        std::vector<int32_t> &ids = bins[i].ids;
        // longest blocks first (cost ~ (m + n) r^2 per sweep): the tail of
        // each persistent launch is then made of short blocks
        std::stable_sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) {
            return dims[2 * a] + dims[2 * a + 1] > dims[2 * b] + dims[2 * b + 1];
        });
        first[i] = at;
        for (int32_t id : ids) ord[at++] = id;
    }

    Workspace *ws = nullptr;
    lra_status st;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    DevInfo dinfo;
    if ((st = dev_info(ws->device, &dinfo)) != LRA_OK) return st;
    size_t lds_dyn = 0;
    for (const Bin &bn : bins) {
        if (bn.P != 0) continue;
        const size_t lds_budget = (size_t)dinfo.lds - lra::static_lds_bytes() - 256;
        const LdsPlan plan = plan_lds(bn.maxdim, bn.maxdim, r, LRA_PRE_NONE, 0, 1, lds_budget);
        if (!plan.fits) return LRA_EUNSUPPORTED;
        cfg.panel_bytes = (int32_t)plan.panel_bytes;
        lds_dyn = plan.dyn_bytes;
    }
    unsigned char *ddesc = nullptr;
    if ((st = stage_desc(ws, stream, host.data(), host.size(), &ddesc)) != LRA_OK) return st;
    const int32_t *dord = reinterpret_cast<const int32_t *>(ddesc + (size_t)count * 32);
    unsigned *queues = ws->counters + 1;
    hipLaunchKernelGGL(lra::zero_u32_kernel, dim3(1), dim3(64), 0, stream, queues, (int)bins.size());
    for (size_t i = 0; i < bins.size(); i++) {
        const Bin &bn = bins[i];
        const int64_t cnt = (int64_t)bn.ids.size();
        hipError_t e;
        if (bn.P == 0) {
            int occ = src == kSrcPoints ? lra::points_occupancy(lds_dyn) : lra::batched_occupancy(src, lds_dyn);
            if (occ < 1) occ = 1;
            const int grid = (int)std::min<int64_t>((int64_t)dinfo.cus * occ, cnt);
            if (src == kSrcPoints)
                e = lra::launch_points(static_cast<const double *>(base), reinterpret_cast<const PtsDesc *>(ddesc),
                                       dord + first[i], cnt, seed, cfg, queues + i, grid, lds_dyn, I_out, J_out, U_out,
                                       infos, stream);
            else
                e = lra::launch_batched(src, base, reinterpret_cast<const BlockDesc *>(ddesc), dord + first[i], cnt,
                                        seed, cfg, queues + i, grid, lds_dyn, I_out, J_out, U_out, infos, stream);
        } else {
            int occ = lra::reg_occupancy(r, bn.P, bn.W, src);
            if (occ < 1) occ = 1;
            const int grid = (int)std::min<int64_t>((int64_t)dinfo.cus * occ, cnt);
            e = lra::launch_reg(src, r, bn.P, bn.W, base, ddesc, dord + first[i], cnt, seed, cfg, queues + i, grid,
                                I_out, J_out, U_out, infos, stream);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return LRA_EDEVICE;
        }
    }
    return LRA_OK;
}

// Layout of the no-allocation scratch (byte offsets): the team exchange
// words for the largest team, the bidiagonal column table, then the global
// sketch panel, whose size bounds the shapes lra_cur_noalloc accepts.
constexpr size_t kNaXwOffset = 0;
constexpr size_t kNaXwBytes = (size_t)2 * kMaxTeam * lra::kSlotWords * sizeof(uint64_t);
constexpr size_t kNaBdOffset = kNaXwOffset + ((kNaXwBytes + 255) & ~size_t(255));
constexpr size_t kNaBdBytes = sizeof(int32_t) * lra::kBdTableInts;
constexpr size_t kNaSketchOffset = kNaBdOffset + ((kNaBdBytes + 255) & ~size_t(255));
constexpr size_t kNaSketchBytes = (size_t)8 << 20;
constexpr size_t kNaBytes = kNaSketchOffset + kNaSketchBytes;
static_assert(kNaBytes == LRA_NOALLOC_SCRATCH_BYTES, "the header states the scratch size");

}  // namespace

// Device scratch of lra_cur_noalloc: one copy per GPU, kept until the
// process ends.  In host code `scratch` only names the symbol; kernels get
// the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

// Per device: the address of `scratch` and the launch limits, set up once
// with the device current (fixed table: the no-allocation path allocates no
// host memory either).
constexpr int kNaMaxDev = 64;
struct NaDev {
    bool ready = false;
    unsigned char *ptr = nullptr;
    DevInfo info;
};
NaDev g_na[kNaMaxDev];

lra_status na_dev(NaDev **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LRA_EDEVICE;
    if (dev < 0 || dev >= kNaMaxDev) return LRA_EUNSUPPORTED;
    NaDev &d = g_na[dev];
    if (!d.ready) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return LRA_EDEVICE;
        }
        lra_status st = query_dev(dev, &d.info);
        if (st != LRA_OK) return st;
        d.ptr = static_cast<unsigned char *>(p);
        d.ready = true;
    }
    *out = &d;
    return LRA_OK;
}

}  // namespace

extern "C" {

void lra_default_opts(lra_opts *o) {
    if (!o) return;
    o->delta = 0.01;
    o->max_swaps = -1;
    o->preprocess = LRA_PRE_NONE;
    o->ah_depth = 3;
    o->ah_samples = 0;
    o->refine_steps = 0;
    o->team_size = 0;
    o->track_margin = 0;
    o->init_cols = nullptr;
}

const char *lra_strerror(lra_status s) {
    switch (s) {
    case LRA_OK: return "ok";
    case LRA_EINVAL: return "invalid argument or non-finite input entry";
    case LRA_ESINGULAR: return "rank-deficient panel (rank < r)";
    case LRA_EDEVICE: return "HIP runtime error";
    case LRA_ENOMEM: return "device workspace allocation failed";
    case LRA_EUNSUPPORTED: return "shape does not fit the on-chip panel layout";
    }
    return "unknown status";
}

lra_status lra_probe_exchange(int32_t rounds, double *ns_out, hipStream_t stream) {
    if (rounds < 2 || rounds > (1 << 24) || !ns_out) return LRA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    lra_status st;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    DevInfo dinfo;
    if ((st = dev_info(ws->device, &dinfo)) != LRA_OK) return st;
    void *scr = nullptr;
    if ((st = ws_work(ws, stream, 64, &scr)) != LRA_OK) return st;
    uint64_t *buf = static_cast<uint64_t *>(scr);
    uint64_t host[3] = {0, 0, 0};
    if (lra::launch_xlat(buf, rounds, (uint64_t)dinfo.wall_khz * 100ull, stream) != hipSuccess ||
        hipMemcpyAsync(host, buf, sizeof(host), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    if (host[2] || host[1] != (uint64_t)rounds) return LRA_EDEVICE;
    *ns_out = (double)host[0] * 1e6 / (double)dinfo.wall_khz / (double)rounds;
    return LRA_OK;
}

void lra_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_ws) {
        Workspace &w = kv.second;
        (void)hipSetDevice(w.device);
        (void)hipStreamSynchronize(kv.first.second);
        (void)hipFree(w.counters);
        (void)hipFree(w.xw);
        (void)hipFree(w.init_cols);
        (void)hipFree(w.desc);
        if (w.stage) (void)hipHostFree(w.stage);
        if (w.stage_done) (void)hipEventDestroy(w.stage_done);
        (void)hipFree(w.sketch);
        (void)hipFree(w.bidiag);
        (void)hipFree(w.work);
    }
    g_ws.clear();
    (void)hipSetDevice(cur);
}

lra_status lra_cur(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r, int32_t sweeps,
                   uint64_t seed, const lra_opts *opts, int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info,
                   hipStream_t stream) {
    CurPlan cp;
    lra_status st = check_cur(W, dt, m, n, lda, r, sweeps, opts, I_out, J_out, U_out, &cp);
    if (st != LRA_OK) return st;

    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    DevInfo dinfo;
    if ((st = dev_info(ws->device, &dinfo)) != LRA_OK) return st;
    if ((st = plan_cur(dinfo, m, n, r, &cp)) != LRA_OK) return st;
    CAConfig &cfg = cp.cfg;
    if (cp.sketch_bytes) {
        if (ws->sketch_cap < cp.sketch_bytes) {
            (void)hipStreamSynchronize(stream);
            (void)hipFree(ws->sketch);
            ws->sketch = nullptr;
            ws->sketch_cap = 0;
            if (hipMalloc(&ws->sketch, cp.sketch_bytes) != hipSuccess) return LRA_ENOMEM;
            ws->sketch_cap = cp.sketch_bytes;
        }
        cfg.sketch_ws = ws->sketch;
    }
    if (cp.o.init_cols) {
        if (hipMemcpyAsync(ws->init_cols, cp.o.init_cols, sizeof(int64_t) * r, hipMemcpyHostToDevice, stream) !=
            hipSuccess)
            return LRA_EDEVICE;
        cfg.init_cols = ws->init_cols;
    }
    if (cp.o.preprocess == LRA_PRE_BIDIAG) {
        if (!ws->bidiag && hipMalloc(&ws->bidiag, sizeof(int32_t) * lra::kBdTableInts) != hipSuccess)
            return LRA_ENOMEM;
        if (lra::launch_bidiag_table(seed, (m >= n) ? m : n, cp.o.ah_depth, cp.o.ah_samples, ws->bidiag, stream) !=
            hipSuccess) {
            (void)hipGetLastError();
            return LRA_EDEVICE;
        }
        cfg.bd_table = ws->bidiag;
    }
    // a team selection normally completes in microseconds; two seconds
    // without the expected word means the launch has failed
    TeamWs tws{ws->xw, (uint64_t)dinfo.wall_khz * 2000ull};
    hipError_t e = lra::launch_team(dt, W, m, n, lda, seed, cfg, tws, cp.team, cp.lds.dyn_bytes, I_out, J_out, U_out,
                                    info, stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

lra_status lra_cur_noalloc(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r, int32_t sweeps,
                           uint64_t seed, const lra_opts *opts, int64_t *I_out, int64_t *J_out, double *U_out,
                           lra_info *info, hipStream_t stream) {
    CurPlan cp;
    lra_status st = check_cur(W, dt, m, n, lda, r, sweeps, opts, I_out, J_out, U_out, &cp);
    if (st != LRA_OK) return st;
    if (cp.o.init_cols) return LRA_EINVAL;  // a host array would need a staging copy

    std::lock_guard<std::mutex> lk(g_mu);
    NaDev *nd = nullptr;
    if ((st = na_dev(&nd)) != LRA_OK) return st;
    if ((st = plan_cur(nd->info, m, n, r, &cp)) != LRA_OK) return st;
    if (cp.sketch_bytes > kNaSketchBytes) return LRA_EUNSUPPORTED;
    CAConfig &cfg = cp.cfg;
    uint64_t *xw = reinterpret_cast<uint64_t *>(nd->ptr + kNaXwOffset);
    if (cp.sketch_bytes) cfg.sketch_ws = reinterpret_cast<double *>(nd->ptr + kNaSketchOffset);
    if (cp.o.preprocess == LRA_PRE_BIDIAG) {
        int32_t *tab = reinterpret_cast<int32_t *>(nd->ptr + kNaBdOffset);
        if (lra::launch_bidiag_table(seed, (m >= n) ? m : n, cp.o.ah_depth, cp.o.ah_samples, tab, stream) !=
            hipSuccess) {
            (void)hipGetLastError();
            return LRA_EDEVICE;
        }
        cfg.bd_table = tab;
    }
    TeamWs tws{xw, (uint64_t)nd->info.wall_khz * 2000ull};
    hipError_t e = lra::launch_team(dt, W, m, n, lda, seed, cfg, tws, cp.team, cp.lds.dyn_bytes, I_out, J_out, U_out,
                                    info, stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

lra_status lra_cur_hadamard(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r,
                            int32_t sweeps, uint64_t seed, int32_t d, const lra_opts *opts, int64_t *I_out,
                            int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream) {
    if (!W || !I_out || !J_out || !U_out) return LRA_EINVAL;
    if (dt != LRA_F64 && dt != LRA_F32 && dt != LRA_BF16) return LRA_EINVAL;
    if (d < 0 || d > 6 || m < 1 || n < 1 || lda < n || r < 1 || r > kRMax || r > m || r > n || sweeps < 1)
        return LRA_EINVAL;
    const int64_t q2 = (int64_t)1 << d;
    const int64_t N = q2 * ((n + q2 - 1) / q2);  // order of the multiplier
    if (m >= ((int64_t)1 << 39) || N >= ((int64_t)1 << 39)) return LRA_EINVAL;  // item ids travel in 40 bits
    CAConfig cfg;
    lra_opts o;
    lra_status st = fill_config(opts, r, sweeps, &cfg, &o);
    if (st != LRA_OK) return st;
    if (o.preprocess != LRA_PRE_NONE || o.init_cols) return LRA_EINVAL;

    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    DevInfo dinfo;
    if ((st = dev_info(ws->device, &dinfo)) != LRA_OK) return st;
    const int max_team = std::min(dinfo.cus, kMaxTeam);
    const size_t lds_budget = (size_t)dinfo.lds - lra::static_lds_bytes() - 256;
    int team;
    LdsPlan plan;
    if (o.team_size > 0) {
        team = std::min(o.team_size, max_team);
        plan = plan_lds(m, N, r, LRA_PRE_NONE, 0, team, lds_budget);
    } else {
        team = (int)std::min<int64_t>(max_team, std::max<int64_t>(1, (std::max(m, N) + 159) / 160));
        plan = plan_lds(m, N, r, LRA_PRE_NONE, 0, team, lds_budget);
        while (!plan.fits && team < max_team) {
            team++;
            plan = plan_lds(m, N, r, LRA_PRE_NONE, 0, team, lds_budget);
        }
    }
    if (!plan.fits) return LRA_EUNSUPPORTED;
    cfg.panel_bytes = (int32_t)plan.panel_bytes;
    TeamWs tws{ws->xw, (uint64_t)dinfo.wall_khz * 2000ull};
    hipError_t e = lra::launch_hadamard(dt, W, m, n, lda, d, seed, cfg, tws, team, plan.dyn_bytes, I_out, J_out, U_out,
                                        info, stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

lra_status lra_cur_cynical(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r, int32_t k,
                           int32_t loops, int32_t sweeps, uint64_t seed, const lra_opts *opts, int64_t *I_out,
                           int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream) {
    if (!W || !I_out || !J_out || !U_out) return LRA_EINVAL;
    if (dt != LRA_F64 && dt != LRA_F32 && dt != LRA_BF16) return LRA_EINVAL;
    if (m < 1 || n < 1 || lda < n || r < 1 || k < r || k > kRMax || k > m || k > n || loops < 0 || sweeps < 1)
        return LRA_EINVAL;
    if (m >= ((int64_t)1 << 39) || n >= ((int64_t)1 << 39)) return LRA_EINVAL;  // item ids travel in 40 bits
    CAConfig ck, cr;
    lra_opts o, o2;
    lra_status st = fill_config(opts, k, std::max(loops, 1), &ck, &o);
    if (st != LRA_OK) return st;
    if ((st = fill_config(opts, r, sweeps, &cr, &o2)) != LRA_OK) return st;
    ck.margins = cr.margins = 0;  // the cynical CUR does not track decision margins
    if (o.preprocess != LRA_PRE_NONE || o.init_cols) return LRA_EINVAL;

    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    DevInfo dinfo;
    if ((st = dev_info(ws->device, &dinfo)) != LRA_OK) return st;
    const int max_team = std::min(dinfo.cus, kMaxTeam);
    const size_t lds_budget = (size_t)dinfo.lds - lra::static_lds_bytes() - 256;
    // without loops only the k x k sketch is solved, by one workgroup; with
    // loops the rank-k steps use the team rule of lra_cur
    int team = 1;
    LdsPlan plan;
    if (loops == 0) {
        plan = plan_lds(k, k, k, LRA_PRE_NONE, 0, 1, lds_budget);
    } else if (o.team_size > 0) {
        team = std::min(o.team_size, max_team);
        plan = plan_lds(m, n, k, LRA_PRE_NONE, 0, team, lds_budget);
    } else {
        team = (int)std::min<int64_t>(max_team, std::max<int64_t>(1, (std::max(m, n) + 159) / 160));
        plan = plan_lds(m, n, k, LRA_PRE_NONE, 0, team, lds_budget);
        while (!plan.fits && team < max_team) {
            team++;
            plan = plan_lds(m, n, k, LRA_PRE_NONE, 0, team, lds_budget);
        }
    }
    if (!plan.fits) return LRA_EUNSUPPORTED;
    ck.panel_bytes = cr.panel_bytes = (int32_t)plan.panel_bytes;
    TeamWs tws{ws->xw, (uint64_t)dinfo.wall_khz * 2000ull};
    hipError_t e = lra::launch_cynical(dt, W, m, n, lda, seed, loops, ck, cr, tws, team, plan.dyn_bytes, I_out, J_out,
                                       U_out, info, stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

lra_status lra_cur_projective(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r, int32_t k,
                              int32_t l, int32_t sweeps, uint64_t seed, const lra_opts *opts, int64_t *I_out,
                              int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream) {
    if (!W || !I_out || !J_out || !U_out) return LRA_EINVAL;
    if (dt != LRA_F64 && dt != LRA_F32 && dt != LRA_BF16) return LRA_EINVAL;
    if (m < 1 || n < 1 || lda < n || r < 1 || k < r || l < r || k > kRMax || l > kRMax || k > m || l > n ||
        sweeps < 1)
        return LRA_EINVAL;
    if (m >= ((int64_t)1 << 39) || n >= ((int64_t)1 << 39)) return LRA_EINVAL;  // item ids travel in 40 bits
    CAConfig cfg;
    lra_opts o;
    lra_status st = fill_config(opts, r, sweeps, &cfg, &o);
    if (st != LRA_OK) return st;
    cfg.margins = 0;  // the r-projective CUR does not track decision margins
    if (o.preprocess != LRA_PRE_NONE || o.init_cols) return LRA_EINVAL;

    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    DevInfo dinfo;
    if ((st = dev_info(ws->device, &dinfo)) != LRA_OK) return st;
    const int max_team = std::min(dinfo.cus, kMaxTeam);
    const size_t lds_budget = (size_t)dinfo.lds - lra::static_lds_bytes() - 256;
    // panels are items x max(k, l); the nucleus needs k l + l^2 <= 4 max(k, l)^2
    const int w = std::max(k, l);
    int team;
    LdsPlan plan;
    if (o.team_size > 0) {
        team = std::min(o.team_size, max_team);
        plan = plan_lds(m, n, w, LRA_PRE_NONE, 0, team, lds_budget);
    } else {
        team = (int)std::min<int64_t>(max_team, std::max<int64_t>(1, (std::max(m, n) + 159) / 160));
        plan = plan_lds(m, n, w, LRA_PRE_NONE, 0, team, lds_budget);
        while (!plan.fits && team < max_team) {
            team++;
            plan = plan_lds(m, n, w, LRA_PRE_NONE, 0, team, lds_budget);
        }
    }
    if (!plan.fits) return LRA_EUNSUPPORTED;
    cfg.panel_bytes = (int32_t)plan.panel_bytes;
    TeamWs tws{ws->xw, (uint64_t)dinfo.wall_khz * 2000ull};
    hipError_t e = lra::launch_projective(dt, W, m, n, lda, seed, k, l, cfg, tws, team, plan.dyn_bytes, I_out, J_out,
                                          U_out, info, stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

lra_status lra_cur_uniform_batched(const void *base, lra_dtype dt, const lra_block *blocks, int64_t count, int32_t r,
                                   int32_t k, int32_t l, uint64_t seed, int64_t *I_out, int64_t *J_out, double *U_out,
                                   lra_info *infos, hipStream_t stream) {
    if (!base || !blocks || count < 0 || !I_out || !J_out || !U_out) return LRA_EINVAL;
    if (dt != LRA_F64 && dt != LRA_F32 && dt != LRA_BF16) return LRA_EINVAL;
    if (r < 1 || k < r || l < r || k > kRMax || l > kRMax || count > (int64_t)INT32_MAX) return LRA_EINVAL;
    std::vector<BlockDesc> desc((size_t)count);
    for (int64_t b = 0; b < count; b++) {
        const lra_block &q = blocks[b];
        if (q.offset < 0 || q.m < 1 || q.n < 1 || q.lda < q.n) return LRA_EINVAL;
        desc[b] = BlockDesc{q.offset, q.m, q.n, q.lda};
    }
    if (count == 0) return LRA_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    lra_status st;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    DevInfo dinfo;
    if ((st = dev_info(ws->device, &dinfo)) != LRA_OK) return st;
    // the nucleus works on max(k, l) x min(k, l) and min(k, l)^2 doubles
    const size_t dyn = align16(sizeof(double) * (size_t)std::min(k, l) * (size_t)(k + l));
    unsigned char *ddesc = nullptr;
    if ((st = stage_desc(ws, stream, desc.data(), sizeof(BlockDesc) * count, &ddesc)) != LRA_OK) return st;
    int occ = lra::uniform_occupancy(dt, dyn);
    if (occ < 1) occ = 1;
    const int64_t grid = std::min<int64_t>((int64_t)dinfo.cus * occ, count);
    hipError_t e = lra::launch_uniform(dt, base, reinterpret_cast<const BlockDesc *>(ddesc), count, seed, r, k, l,
                                       (int)grid, dyn, I_out, J_out, U_out, infos, stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

lra_status lra_cur_dmm_batched(const void *base, lra_dtype dt, const lra_block *blocks, int64_t count, int32_t r,
                               int32_t k, int32_t l, int32_t iters, uint64_t seed, int64_t *I_out, int64_t *J_out,
                               double *U_out, lra_info *infos, hipStream_t stream) {
    if (!base || !blocks || count < 0 || !I_out || !J_out || !U_out) return LRA_EINVAL;
    if (dt != LRA_F64 && dt != LRA_F32 && dt != LRA_BF16) return LRA_EINVAL;
    if (r < 1 || k < r || l < r || k > kRMax || l > kRMax || iters < 1 || count > (int64_t)INT32_MAX)
        return LRA_EINVAL;
    std::vector<BlockDesc> desc((size_t)count);
    int64_t items = 1;
    for (int64_t b = 0; b < count; b++) {
        const lra_block &q = blocks[b];
        if (q.offset < 0 || q.m < 1 || q.n < 1 || q.lda < q.n || r > q.m || r > q.n) return LRA_EINVAL;
        desc[b] = BlockDesc{q.offset, q.m, q.n, q.lda};
        items = std::max(items, std::max(q.m, q.n));
    }
    if (count == 0) return LRA_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    lra_status st;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    DevInfo dinfo;
    if ((st = dev_info(ws->device, &dinfo)) != LRA_OK) return st;
    int occ = lra::dmm_occupancy(dt);
    if (occ < 1) occ = 1;
    const int64_t grid = std::min<int64_t>((int64_t)dinfo.cus * occ, count);
    void *scr = nullptr;
    if ((st = ws_work(ws, stream, sizeof(double) * 2 * (size_t)items * (size_t)grid, &scr)) != LRA_OK) return st;
    unsigned char *ddesc = nullptr;
    if ((st = stage_desc(ws, stream, desc.data(), sizeof(BlockDesc) * count, &ddesc)) != LRA_OK) return st;
    hipError_t e = lra::launch_dmm(dt, base, reinterpret_cast<const BlockDesc *>(ddesc), count, seed, r, k, l, iters,
                                   static_cast<double *>(scr), items, (int)grid, I_out, J_out, U_out, infos, stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

lra_status lra_cur_leverage(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r,
                            const int64_t *I0, const int64_t *J0, int32_t k, int32_t l, uint64_t seed,
                            int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream) {
    if (!W || !I0 || !J0 || !I_out || !J_out || !U_out) return LRA_EINVAL;
    if (dt != LRA_F64 && dt != LRA_F32 && dt != LRA_BF16) return LRA_EINVAL;
    if (m < 1 || n < 1 || lda < n || r < 1 || r > kRMax || r > m || r > n || k < r || l < r || k > kSMax ||
        l > kSMax)
        return LRA_EINVAL;
    // the crude LRA's sets are read back and checked before any kernel reads
    // the matrix through them
    int64_t hi[kRMax], hj[kRMax];
    if (hipMemcpyAsync(hi, I0, sizeof(int64_t) * r, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(hj, J0, sizeof(int64_t) * r, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    for (int a = 0; a < r; a++)
        if (hi[a] < 0 || hi[a] >= m || hj[a] < 0 || hj[a] >= n) return LRA_EINVAL;

    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    lra_status st;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    const size_t bytes = lra::leverage_scratch_bytes(m, n, r);
    void *scr = nullptr;
    if ((st = ws_work(ws, stream, bytes + 64, &scr)) != LRA_OK) return st;
    double *lw = static_cast<double *>(scr);
    int32_t *flags = reinterpret_cast<int32_t *>(static_cast<char *>(scr) + bytes);
    hipError_t e = lra::launch_leverage(dt, W, m, n, lda, r, I0, J0, k, l, seed, lw, flags, I_out, J_out, U_out,
                                        info, stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

lra_status lra_cur_batched(const void *base, lra_dtype dt, const lra_block *blocks, int64_t count, int32_t r,
                           int32_t sweeps, uint64_t seed, const lra_opts *opts, int64_t *I_out, int64_t *J_out,
                           double *U_out, lra_info *infos, hipStream_t stream) {
    if (!base || !blocks || count < 0 || !I_out || !J_out || !U_out) return LRA_EINVAL;
    if (dt != LRA_F64 && dt != LRA_F32 && dt != LRA_BF16) return LRA_EINVAL;
    if (r < 1 || r > kRMax || sweeps < 1 || count > (int64_t)INT32_MAX) return LRA_EINVAL;
    CAConfig cfg;
    lra_opts o;
    lra_status st = fill_config(opts, r, sweeps, &cfg, &o);
    if (st != LRA_OK) return st;
    if (o.preprocess != LRA_PRE_NONE || o.init_cols) return LRA_EINVAL;
    if (count == 0) return LRA_OK;
    std::vector<BlockDesc> desc((size_t)count);
    std::vector<int64_t> dims((size_t)2 * count);
    for (int64_t b = 0; b < count; b++) {
        const lra_block &k = blocks[b];
        if (k.offset < 0 || k.m < 1 || k.n < 1 || k.lda < k.n || r > k.m || r > k.n) return LRA_EINVAL;
        desc[b] = BlockDesc{k.offset, k.m, k.n, k.lda};
        dims[2 * b] = k.m;
        dims[2 * b + 1] = k.n;
    }
    return batched_run((int)dt, base, desc.data(), dims.data(), count, cfg, seed, I_out, J_out, U_out, infos, stream);
}

lra_status lra_cur_batched_points(const double *pts, int64_t npts, const lra_pts_block *blocks, int64_t count,
                                  int32_t r, int32_t sweeps, uint64_t seed, const lra_opts *opts, int64_t *I_out,
                                  int64_t *J_out, double *U_out, lra_info *infos, hipStream_t stream) {
    if (!pts || !blocks || count < 0 || npts < 1 || !I_out || !J_out || !U_out) return LRA_EINVAL;
    if (r < 1 || r > kRMax || sweeps < 1 || count > (int64_t)INT32_MAX) return LRA_EINVAL;
    if (npts >= ((int64_t)1 << 39)) return LRA_EINVAL;  // item ids travel in 40 bits
    CAConfig cfg;
    lra_opts o;
    lra_status st = fill_config(opts, r, sweeps, &cfg, &o);
    if (st != LRA_OK) return st;
    if (o.preprocess != LRA_PRE_NONE || o.init_cols) return LRA_EINVAL;
    if (count == 0) return LRA_OK;
    std::vector<PtsDesc> desc((size_t)count);
    std::vector<int64_t> dims((size_t)2 * count);
    for (int64_t b = 0; b < count; b++) {
        const lra_pts_block &k = blocks[b];
        if (k.x_off < 0 || k.y_off < 0 || k.m < 1 || k.n < 1 || r > k.m || r > k.n) return LRA_EINVAL;
        if (k.m > npts - k.x_off || k.n > npts - k.y_off) return LRA_EINVAL;
        desc[b] = PtsDesc{k.x_off, k.y_off, k.m, k.n};
        dims[2 * b] = k.m;
        dims[2 * b + 1] = k.n;
    }
    return batched_run(kSrcPoints, pts, desc.data(), dims.data(), count, cfg, seed, I_out, J_out, U_out, infos,
                       stream);
}

lra_status lra_batch_set_rules(const lra_batch_rule *rules, int32_t count) {
    if (count < 0 || count > kMaxRules || (count > 0 && !rules)) return LRA_EINVAL;
    std::vector<lra_batch_rule> v;
    if (count == 0) {
        v = default_rules();
    } else {
        for (int32_t i = 0; i < count; i++) {
            const lra_batch_rule &q = rules[i];
            if (q.max_dim < 1 || q.r < 1 || q.r > kRMax || q.waves < 0 || q.items_per_lane < 0) return LRA_EINVAL;
            if (q.items_per_lane > 0) {
                if (!lra::reg_variant_exists(q.r, q.items_per_lane)) return LRA_EUNSUPPORTED;
                if (q.waves < 1 || q.waves > 8 || (int64_t)64 * q.items_per_lane * q.waves < q.max_dim)
                    return LRA_EINVAL;
            }
            v.push_back(q);
        }
        std::stable_sort(v.begin(), v.end(),
                         [](const lra_batch_rule &a, const lra_batch_rule &b) { return a.max_dim < b.max_dim; });
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_rules = v;
    g_rules_set = true;
    return LRA_OK;
}

int32_t lra_batch_get_rules(lra_batch_rule *out, int32_t cap) {
    std::lock_guard<std::mutex> lk(g_mu);
    const std::vector<lra_batch_rule> &v = current_rules();
    const int32_t n = (int32_t)v.size();
    for (int32_t i = 0; i < n && i < cap && out; i++) out[i] = v[i];
    return n;
}

lra_status lra_residual(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r, const int64_t *I,
                        const int64_t *J, const double *U, int32_t q, int32_t s, uint64_t seed, int32_t prec,
                        double *moments, hipStream_t stream) {
    if (!W || !I || !J || !U || !moments) return LRA_EINVAL;
    if (dt != LRA_F64 && dt != LRA_F32 && dt != LRA_BF16) return LRA_EINVAL;
    if (prec != LRA_PREC_PLAIN && prec != LRA_PREC_MIXED) return LRA_EINVAL;
    if (m < 1 || n < 1 || lda < n || r < 1 || r > kRMax || r > m || r > n) return LRA_EINVAL;
    if (q < 0 || s < 0 || (q == 0) != (s == 0) || q > 256 || s > 256 || q > m || s > n) return LRA_EINVAL;
    if (m >= ((int64_t)1 << 39) || n >= ((int64_t)1 << 39)) return LRA_EINVAL;
    if ((q ? q : m) > (int64_t)128 * 65535) return LRA_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    lra_status st;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    void *scr = nullptr;
    if ((st = ws_work(ws, stream, lra::residual_scratch_bytes(m, n, r, q, s, prec), &scr)) != LRA_OK)
        return st;
    if (lra::launch_residual(dt, W, m, n, lda, r, I, J, U, q, s, seed, prec, moments, scr, stream) !=
        hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

lra_status lra_posterior_test(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r,
                              const int64_t *I, const int64_t *J, const double *U, int32_t q, int32_t s,
                              uint64_t seed, int32_t prec, double tau, double z, lra_posterior *out,
                              hipStream_t stream) {
    if (!W || !I || !J || !U || !out) return LRA_EINVAL;
    if (dt != LRA_F64 && dt != LRA_F32 && dt != LRA_BF16) return LRA_EINVAL;
    if (prec != LRA_PREC_PLAIN && prec != LRA_PREC_MIXED) return LRA_EINVAL;
    if (m < 1 || n < 1 || lda < n || r < 1 || r > kRMax || r > m || r > n) return LRA_EINVAL;
    if (q < 1 || s < 1 || q > 256 || s > 256 || q > m || s > n || (int64_t)q * s < 2) return LRA_EINVAL;
    if (!(tau > 0.0) || !std::isfinite(tau) || !std::isfinite(z)) return LRA_EINVAL;
    if (m >= ((int64_t)1 << 39) || n >= ((int64_t)1 << 39)) return LRA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    lra_status st;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    const size_t bytes = (lra::residual_scratch_bytes(m, n, r, q, s, prec) + 255) & ~size_t(255);
    void *scr = nullptr;
    if ((st = ws_work(ws, stream, bytes + 4 * sizeof(double), &scr)) != LRA_OK) return st;
    double *mom = reinterpret_cast<double *>(static_cast<char *>(scr) + bytes);
    if (lra::launch_residual(dt, W, m, n, lda, r, I, J, U, q, s, seed, prec, mom, scr, stream) != hipSuccess ||
        lra::launch_posterior(mom, (int64_t)q * s, tau, z, out, stream) != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

lra_status lra_cur_adjoint(int64_t count, int64_t m, int64_t n, int32_t r, const double *C, const double *R,
                           const double *G, int64_t nnz, const int32_t *om_row, const int32_t *om_col,
                           const int32_t *col_order, const double *a_om, double *loss, double *dC, double *dR,
                           double *dG, int32_t *status, hipStream_t stream) {
    if (count < 0 || m < 1 || n < 1 || r < 1 || r > kRMax || nnz < 0) return LRA_EINVAL;
    if (m > INT32_MAX || n > INT32_MAX || nnz > INT32_MAX) return LRA_EINVAL;
    if (count == 0) return LRA_OK;
    if (!C || !R || !G || !loss || !dC || !dR || !dG || !status) return LRA_EINVAL;
    if (nnz > 0 && (!om_row || !om_col || !col_order || !a_om)) return LRA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *ws = nullptr;
    lra_status st;
    if ((st = get_ws(stream, &ws)) != LRA_OK) return st;
    void *scr = nullptr;
    if ((st = ws_work(ws, stream, lra::adjoint_scratch_bytes(count, m, n, nnz, r), &scr)) != LRA_OK) return st;
    if (lra::launch_adjoint(count, m, n, r, C, R, G, nnz, om_row, om_col, col_order, a_om, loss, dC, dR, dG, scr,
                            status, stream) != hipSuccess) {
        (void)hipGetLastError();
        return LRA_EDEVICE;
    }
    return LRA_OK;
}

}  // extern "C"
