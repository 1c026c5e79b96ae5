// lra_ca.hip -- cross-approximation (C-A) CUR on gfx950.
//
// One LRA runs inside one persistent launch.  A "team" of workgroups
// cooperates on it: every panel (the m x r column panel W[:, J], the n x r
// transposed row panel W[I, :]^T, the items x l abridged-SRHT sketch) is
// split by items (rows or columns of W) across the team, each workgroup
// keeping its slice in LDS as FP64, column-major (slot-major, odd stride), each
// item handled by a small group of consecutive lanes.  Every pivot or
// swap decision is an argmax over the whole panel: each workgroup reduces its
// slice with wavefront shuffles, publishes (value, item, slot) and the
// candidate's row as tagged words in a small exchange buffer, reads the other
// workgroups' words (no grid barrier, see the team exchange below) and
// reduces the team's candidates redundantly, so all of them apply the same
// rank-one update to their own slice.  A team of one workgroup (small
// matrices, and every block of a batch) skips the exchange entirely.
//
// The arithmetic follows the paper's steps (Appendix D, Algorithms alggos
// and algdomin; Appendix B for the sketch; Algorithm alg1tor for the greedy
// QRP; Algorithm algcnnncl for the nucleus); this file is compiled without
// floating-point contraction and every per-item sum runs in a fixed order,
// so results do not depend on the team size.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lra_common.h"
#include "lra_device.h"
#include "lra_internal.h"

namespace lra {

constexpr int kNWave = kBlock / kWave;
static_assert(kNWave <= 8, "the workgroup reduction combines at most eight wavefront partials");
static_assert(2 * kAftCoefs <= kRMax * (kRMax - 1) / 2, "the Fourier coefficient table fits the LU scratch");
constexpr int kChunk = 8;  // entries staged in registers per LDS round trip

// ---------------------------------------------------------------- tracing
// Built with -DLRA_TRACE, workgroup 0 of a launch records phase timestamps
// (device wall clock) and the time spent inside team selections in a device
// buffer that lra_trace_read() copies out.  Off by default: no cost.
#ifdef LRA_TRACE
constexpr int kTraceMax = 4096;
__device__ uint64_t g_trace[kTraceMax * 2];
__device__ int g_trace_n;
__device__ __forceinline__ void trace(int ev, uint64_t val = 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int i = g_trace_n;
        if (i < kTraceMax) {
            g_trace[2 * i] = ((uint64_t)ev << 56) | (wall_clock64() & 0x00ffffffffffffffull);
            g_trace[2 * i + 1] = val;
            g_trace_n = i + 1;
        }
    }
}
#define LRA_TR(ev, val) trace(ev, val)
// per selection and workgroup: wall clock when its header was stored and
// when its poll of the team's headers completed (first kSelTrace selections)
constexpr int kSelTrace = 1024;
__device__ uint64_t g_sel_pub[kSelTrace * 256];
__device__ uint64_t g_sel_done[kSelTrace * 256];
#else
#define LRA_TR(ev, val) ((void)0)
#endif

// ---------------------------------------------------------------- LDS state
struct Smem {
    int64_t Iset[kRMax], Jset[kRMax], Iprev[kRMax], Jprev[kRMax];
    int64_t slot_item[kRMax];
    int64_t samples[kLMax];  // sketch samples; the cynical CUR keeps its sketch rows and columns here
    uint8_t sgn[kLMax];   // sketch: combined signs of a sampled column's 2^d <= 8 terms
    double L11[kRMax * (kRMax - 1) / 2];
    double wrow[kLMax];
    double wprev[2][kRMax];  // LU: the pivot rows of the last two steps
    int64_t loc_item;        // the workgroup's best item of the last selection (-1: none)
    Best red[kNWave];
    double red2[kNWave];     // each wavefront's runner-up value
    int32_t red_flag[kNWave];
    Best win;
    double win_v2;   // the team's runner-up value (in the winner's workgroup; NaN elsewhere)
    double mmin;     // smallest decision margin this workgroup has seen
    int32_t win_flag;
    int32_t status;
    int32_t rank_found;
    int32_t nucleus_rank;
    int32_t job;
    int32_t xfail;   // a team poll timed out
    double vtv;
    double alpha;
    double pivot;    // swap selection: the winner's entry B[i*][j*]
    double logdet;
#ifdef LRA_TRACE
    uint64_t t_select;    // total time inside team selections
    uint64_t t_part[5];   // block reduce, header polls, row fetch, final barrier, wave arrival spread
    uint64_t t_arr[8];    // arrival time of each wavefront at the current selection
    uint64_t n_select;
    uint64_t t_loop[5];   // LU item loop, LU tail, swap item loop, swap tail, B solve
#endif
};

struct Team {
    int rank, size;
    unsigned epoch;   // number of team selections so far (same in every workgroup)
    uint64_t *xw;     // exchange words: headers [2][size][kHdrStride], then rows [2][size][kRowWords]; zeroed per launch
    uint64_t spin_limit;  // wall-clock ticks a poll may wait
};

// Team exchange without barriers or cache-maintenance fences: every 64-bit
// word carries a tag (derived from the selection number) above its data bits
// and is written and read with single-copy-atomic device-scope accesses,
// which go to the device-coherent level instead of the per-XCD L2.  A reader
// polls a word until its tag matches, so a value can never be taken from an
// older selection, whatever the order in which the writer's stores land.
// Row words carry 32-bit tags (selection + 1) over 32 data bits.  Header
// words carry 4-bit tags ((selection + 1) mod 16) over 60 data bits: every
// header word of parity p is rewritten at every selection of that parity,
// and no workgroup can publish selection e + 2 before every other one has
// finished reading selection e, so a header word holds either selection e
// or e - 2 while it is awaited for e, and those two tags differ.  The buffer
// is cleared before each launch; a cleared word (tag 0) is awaited only for
// e < 2, whose tags are 1 and 2.
template <int TB>
__device__ __forceinline__ void xput(uint64_t *p, uint32_t tag, uint64_t data) {
    __hip_atomic_store(p, ((uint64_t)tag << (64 - TB)) | data, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t xld(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lo_hi(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }

// Read N exchange words with TB-bit tags that all carry `tag`: the N loads
// are issued together, and only the words still stale are polled again; a
// null pointer stands for no word (its output is 0).  out[i] receives the
// data bits.  Every wait is bounded in wall-clock time: past `limit` ticks
// the workgroup records a failure in *fail, stops polling for the rest of
// the launch (its reads return 0) and runs to the end, so no wave can wait
// forever; the LRA then reports LRA_EDEVICE.
template <int N, int TB>
__device__ __forceinline__ void xget(const uint64_t *const (&p)[N], uint32_t tag, uint64_t (&out)[N], int *fail,
                                     uint64_t limit) {
    constexpr int kSh = 64 - TB;
    uint64_t v[N];
#pragma unroll
    for (int i = 0; i < N; i++) v[i] = p[i] ? xld(p[i]) : (uint64_t)tag << kSh;  // null: no word to wait for
    bool ok = true;
#pragma unroll
    for (int i = 0; i < N; i++) ok = ok && ((uint32_t)(v[i] >> kSh) == tag);
    if (!ok && !*(volatile int *)fail) {
        const uint64_t t0 = wall_clock64();
        for (;;) {
            __builtin_amdgcn_s_sleep(1);
            ok = true;
#pragma unroll
            for (int i = 0; i < N; i++) {
                if ((uint32_t)(v[i] >> kSh) != tag) v[i] = xld(p[i]);
            }
#pragma unroll
            for (int i = 0; i < N; i++) ok = ok && ((uint32_t)(v[i] >> kSh) == tag);
            if (ok) break;
            if (wall_clock64() - t0 > limit) {
                *(volatile int *)fail = 1;
                break;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < N; i++) out[i] = ok ? (v[i] & ((1ull << kSh) - 1)) : 0ull;
}

// The header wait of team_select: the NQ header groups of a lane (NQ x
// kHdrWords words; past the end of the team a lane reads its own
// workgroup's header and ignores it, so every load is unconditional and the
// compiler can count them).  Two batches of loads stay in flight, the second
// issued a short sleep after the first and each reissued as soon as it has
// been checked, so a header that lands is seen up to about half a round trip
// sooner than by waiting for one batch at a time (headline LRA 3.83 -> 3.73
// ms; three or four batches were slower).  Words are checked as in xget and
// the wait is bounded the same way; out[i] receives the data bits of word i.
template <int NQ>
__device__ __forceinline__ void poll_headers(const uint64_t *hdrs, int size, int rank, int lane, uint32_t htag,
                                             uint64_t (&out)[4 * kHdrWords], int *fail, uint64_t limit) {
    constexpr int N = NQ * kHdrWords;
    const uint64_t *p[N];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        const int g0 = lane + q * kWave;
#pragma unroll
        for (int w = 0; w < kHdrWords; w++)
            p[q * kHdrWords + w] = hdrs + (size_t)(g0 < size ? g0 : rank) * kHdrStride + w;
    }
    uint64_t a[N], b[N], v[N];
    unsigned got = 0;  // bit i: word i seen with the selection's tag
#pragma unroll
    for (int i = 0; i < N; i++) a[i] = xld(p[i]);
    __builtin_amdgcn_s_sleep(4);
#pragma unroll
    for (int i = 0; i < N; i++) b[i] = xld(p[i]);
    const unsigned all = (1u << N) - 1;
    uint64_t t0 = 0;
    bool ok = false;
    for (int it = 0;; it++) {
#pragma unroll
        for (int i = 0; i < N; i++)
            if (!(got >> i & 1) && (uint32_t)(a[i] >> 60) == htag) {
                v[i] = a[i];
                got |= 1u << i;
            }
        if (__all(got == all)) {
            ok = true;
            break;
        }
#pragma unroll
        for (int i = 0; i < N; i++) a[i] = xld(p[i]);
#pragma unroll
        for (int i = 0; i < N; i++)
            if (!(got >> i & 1) && (uint32_t)(b[i] >> 60) == htag) {
                v[i] = b[i];
                got |= 1u << i;
            }
        if (__all(got == all)) {
            ok = true;
            break;
        }
#pragma unroll
        for (int i = 0; i < N; i++) b[i] = xld(p[i]);
        if (*(volatile int *)fail) break;
        if (it == 0) {
            t0 = wall_clock64();
        } else if (wall_clock64() - t0 > limit) {
            *(volatile int *)fail = 1;
            break;
        }
    }
#pragma unroll
    for (int i = 0; i < 4 * kHdrWords; i++) out[i] = 0;
#pragma unroll
    for (int i = 0; i < N; i++) out[i] = ok ? (v[i] & ((1ull << 60) - 1)) : 0ull;
}

// Header of a team candidate in two 60-bit payloads: |value| (sign bit 0)
// bits 62..3, then value bits 2..0, item (40 bits; all ones: no candidate),
// slot (8 bits; 0xff: none) and the flags (8 bits).
constexpr uint64_t kItemNone = (1ull << 40) - 1;
__device__ __forceinline__ void encode_hdr(const Best &b, int flags, uint64_t &w0, uint64_t &w1) {
    const bool have = b.v >= 0.0;
    const uint64_t vb = have ? (uint64_t)__double_as_longlong(b.v) : 0ull;
    const uint64_t it = have ? (uint64_t)b.item : kItemNone;
    w0 = vb >> 3;
    w1 = (vb & 7ull) | (it << 3) | ((uint64_t)(b.slot & 0xff) << 43) | ((uint64_t)(flags & 0xff) << 51);
}
__device__ __forceinline__ Best decode_hdr(uint64_t w0, uint64_t w1, int aux, int &flags) {
    const uint64_t it = (w1 >> 3) & kItemNone;
    const int sl = (int)((w1 >> 43) & 0xffu);
    flags = (int)((w1 >> 51) & 0xffu);
    if (it == kItemNone) return none();
    return Best{__longlong_as_double((long long)((w0 << 3) | (w1 & 7ull))), (int64_t)it, sl == 0xff ? 0x7fffffff : sl,
                aux};
}

struct Geo {   // item partition of one panel across the team
    int64_t items, base;
    int ipw, cnt;
    int st;   // slot stride of the slot-major panel: ipw rounded up to odd (spreads LDS banks)
};

__device__ __forceinline__ Geo geo(const Team &tm, int64_t items) {
    Geo g;
    g.items = items;
    g.ipw = (int)((items + tm.size - 1) / tm.size);
    g.base = (int64_t)tm.rank * g.ipw;
    int64_t c = items - g.base;
    g.cnt = (int)(c < 0 ? 0 : (c > g.ipw ? g.ipw : c));
    g.st = g.ipw | 1;
    return g;
}

// Lanes that share one item in the maxvol loops.  The `nw` wavefronts from
// wavefront w0 on hold floor(64 / sub) groups of `sub` consecutive lanes each
// (the last 64 mod sub lanes of a wavefront stay idle: grp is out of range);
// lane s of a group owns slots s, s + sub, s + 2 sub, ... of an item, and
// group grp takes items grp, grp + ngrp, ...  sub (1..16, at most r)
// minimises the busiest SIMD's share of the work (owned slots per item plus a
// fixed cost per item), wavefront w running on SIMD w mod 4: each lane evaluates one candidate and the wavefront
// takes the cheapest (the smallest sub among equals).
struct LaneMap {
    int sub, s, grp, ngrp;
};
__device__ __forceinline__ LaneMap lane_map(int cnt, int r, int w0, int nw) {
    const int lane = threadIdx.x & (kWave - 1);
    int key = INT_MAX;
    {
        const int sub = lane + 1;
        if (sub <= 16 && sub <= r) {
            const int ipw = kWave / sub;
            const int passes = (cnt + ipw - 1) / ipw;  // wavefront passes over the items, dealt in turn
            const int nq = (nw + 3) / 4;               // wavefronts on the busiest SIMD (the one of w0)
            const int load = nq * (passes / nw) + min(nq, (passes % nw + 3) / 4);
            key = (load * ((r + sub - 1) / sub + 2)) * 32 + sub;  // + 2: the per-item work of a pass
        }
    }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) key = min(key, __shfl_xor(key, o));
    LaneMap m;
    m.sub = key & 31;
    const int ipw = kWave / m.sub;
    m.ngrp = nw * ipw;
    const int t = (int)threadIdx.x - w0 * kWave;
    const int w = t / kWave, l = t % kWave;
    if (t < 0 || w >= nw || l >= ipw * m.sub) {
        m.s = 0;
        m.grp = INT_MAX / 2;
    } else {
        m.s = l % m.sub;
        m.grp = w * ipw + l / m.sub;
    }
    return m;
}

// Sketch QRP, per item (entries panel[c * ipw + li]) and in the oracle's
// order of operations: chunks of N entries from entry c, offset o, all loads
// of a chunk issued before its arithmetic.  dot: acc += w_c z_c; upd:
// z_c <- z_c - f w_c, then nrm += z_c^2; nrm: nrm += z_c^2.
template <int N>
__device__ __forceinline__ void qrp_dot(const double *panel, int &o, int ipw, const double *w, int &c, double &acc) {
    double z[N], y[N];
#pragma unroll
    for (int u = 0; u < N; u++) {
        z[u] = panel[o + u * ipw];
        y[u] = w[c + u];
    }
#pragma unroll
    for (int u = 0; u < N; u++) acc += y[u] * z[u];
    o += N * ipw;
    c += N;
}
template <int N>
__device__ __forceinline__ void qrp_upd(double *panel, int &o, int ipw, const double *w, int &c, double f, double &nrm) {
    double z[N], y[N];
#pragma unroll
    for (int u = 0; u < N; u++) {
        z[u] = panel[o + u * ipw];
        y[u] = w[c + u];
    }
#pragma unroll
    for (int u = 0; u < N; u++) {
        z[u] = z[u] - f * y[u];
        panel[o + u * ipw] = z[u];
    }
#pragma unroll
    for (int u = 0; u < N; u++) nrm += z[u] * z[u];
    o += N * ipw;
    c += N;
}
template <int N>
__device__ __forceinline__ void qrp_nrm(const double *panel, int &o, int ipw, int &c, double &nrm) {
    double z[N];
#pragma unroll
    for (int u = 0; u < N; u++) z[u] = panel[o + u * ipw];
#pragma unroll
    for (int u = 0; u < N; u++) nrm += z[u] * z[u];
    o += N * ipw;
    c += N;
}
// The entries c0 .. l-1 of an item in chunks of 16, then 8, 4, 2 and 1.
#define LRA_QRP_RUN(FN, n, ...)                        \
    do {                                               \
        int n_ = (n);                                  \
        for (; n_ >= 16; n_ -= 16) FN<16>(__VA_ARGS__); \
        if (n_ & 8) FN<8>(__VA_ARGS__);                \
        if (n_ & 4) FN<4>(__VA_ARGS__);                \
        if (n_ & 2) FN<2>(__VA_ARGS__);                \
        if (n_ & 1) FN<1>(__VA_ARGS__);                \
    } while (0)

// Default hooks of team_select: the published row is the candidate's panel
// column as stored, and there is no work to overlap with the exchange.
struct PanelRow {
    const double *panel;
    int st;
    int64_t base;
    __device__ __forceinline__ double operator()(int t, int64_t item) const {
        return panel[t * st + (int)(item - base)];
    }
};
struct NoOverlap {
    __device__ __forceinline__ void operator()(int64_t) const {}
};

enum SelMode { kSelPlain = 0, kSelHouseholder = 1, kSelSwap = 2 };

// Team-wide selection.  Every thread passes its best candidate; the winner
// of the whole team lands in sm.win and its row (`width` entries, rowf(t,
// item) for t < width) in sm.wrow; the workgroup's own best item lands in
// sm.loc_item.  Wave 0 alone runs the exchange, so the call costs two
// workgroup barriers; between them waves 1.. run overlap(local best item).
// With kSelHouseholder, lane 0 also turns sm.wrow into the Householder vector
// of step `hstep` (oracle order: alpha = -sign(x0) ||x||, v0 = x0 - alpha,
// vtv = sum of v_c^2 in index order).  With kSelSwap it keeps the winner's
// entry at its slot in sm.pivot and subtracts 1 there in sm.wrow, so that
// sm.wrow holds B[i*,:] - e_j*^T, the vector of the rank-one swap update.
template <bool M, class RowFn, class Overlap>
__device__ __forceinline__ void team_select(Team &tm, Smem &sm, Best b, int flag, const Geo &g, int width, int mode,
                                            int hstep, const RowFn &rowf, const Overlap &overlap,
                                            double pub_min = -1.0, double b2 = -1.0) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#ifdef LRA_TRACE
    const uint64_t t_in = wall_clock64();
#endif
#ifdef LRA_TRACE
    if (lane == 0) sm.t_arr[w] = t_in;
#endif
    double wv2 = -1.0;
    if constexpr (M) b = wave_reduce2(b, b2, wv2);
    else b = wave_reduce(b);
    flag = wave_or(flag);
    if (lane == 0) {
        sm.red[w] = b;
        if constexpr (M) sm.red2[w] = wv2;
        sm.red_flag[w] = flag;
    }
    __syncthreads();
#ifdef LRA_TRACE
    if (threadIdx.x == 0) {
        uint64_t last = sm.t_arr[0];
        for (int q = 1; q < kNWave; q++) last = sm.t_arr[q] > last ? sm.t_arr[q] : last;
        sm.t_part[4] += last - sm.t_arr[0];
    }
    const uint64_t t_a = wall_clock64();
    uint64_t t_b = t_a, t_c = t_a;
#endif
    // every wavefront forms the workgroup's best candidate (a uniform value)
    Best loc = lane < kNWave ? sm.red[lane] : none();
    int f = lane < kNWave ? sm.red_flag[lane] : 0;
    loc = reduce8(loc);
    f = wave_or(f);
    // (M) the workgroup's runner-up: the best two values of the wavefronts' pairs
    double lv2 = -1.0;
    if constexpr (M) {
        double lv1 = lane < kNWave ? sm.red[lane].v : -1.0;
        lv2 = lane < kNWave ? sm.red2[lane] : -1.0;
        top2_8(lv1, lv2);
    }
    if (w != 0) overlap(loc.v >= 0.0 ? loc.item : (int64_t)-1);
    if (w == 0) {
        if (lane == 0) sm.loc_item = loc.v >= 0.0 ? loc.item : (int64_t)-1;
        Best win;
        int wf;
        double v2 = lv2;
        if (tm.size == 1) {
            win = loc;
            wf = f;
            for (int t = lane; t < width; t += kWave) sm.wrow[t] = loc.v >= 0 ? rowf(t, loc.item) : 0.0;
        } else {
            const uint32_t tag = tm.epoch + 1u, htag = tag & 0xfu;
            const int par = tm.epoch & 1;
            // every header on a line of its own (each read with the others,
            // all loads in flight at once); rows live in a separate region
            uint64_t *hdrs = tm.xw + (size_t)par * tm.size * kHdrStride;
            uint64_t *rows = tm.xw + (size_t)2 * tm.size * kHdrStride + (size_t)par * tm.size * kRowWords;
            uint64_t *mine = hdrs + (size_t)tm.rank * kHdrStride;
            uint64_t *myrow = rows + (size_t)tm.rank * kRowWords;
            // the header goes out first: the team waits on headers, while a
            // row is read only after its header has won
            if (lane == 0) {
                uint64_t h0, h1;
                encode_hdr(loc, f, h0, h1);
                xput<4>(mine + 0, htag, h0);
                xput<4>(mine + 1, htag, h1);
#ifdef LRA_TRACE
                if (tm.epoch < kSelTrace && tm.rank < 256) g_sel_pub[tm.epoch * 256 + tm.rank] = wall_clock64();
#endif
            }
            // a candidate at or below pub_min cannot be acted on (a swap
            // needs |B_ij| > 1 + delta): its row is not needed, not published
            if (loc.v > pub_min) {
                for (int t = lane; t < width; t += kWave) {
                    const double x = rowf(t, loc.item);
                    const uint64_t u = (uint64_t)__double_as_longlong(x);
                    xput<32>(myrow + 2 * t, tag, (uint32_t)u);
                    xput<32>(myrow + 2 * t + 1, tag, (uint32_t)(u >> 32));
                }
            }
            // every lane polls up to kMaxTeam / 64 headers (poll_headers)
            Best c = none();
            int cf = 0;
            double hv[4];  // each polled workgroup's best value
            {
                uint64_t d[4 * kHdrWords];
                const int nq = (tm.size + kWave - 1) / kWave;
                if (nq <= 1) poll_headers<1>(hdrs, tm.size, tm.rank, lane, htag, d, &sm.xfail, tm.spin_limit);
                else if (nq == 2) poll_headers<2>(hdrs, tm.size, tm.rank, lane, htag, d, &sm.xfail, tm.spin_limit);
                else if (nq == 3) poll_headers<3>(hdrs, tm.size, tm.rank, lane, htag, d, &sm.xfail, tm.spin_limit);
                else poll_headers<4>(hdrs, tm.size, tm.rank, lane, htag, d, &sm.xfail, tm.spin_limit);
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    hv[q] = -1.0;
                    if (lane + q * kWave >= tm.size) continue;
                    int fl;
                    const Best o = decode_hdr(d[q * kHdrWords], d[q * kHdrWords + 1], lane + q * kWave, fl);
                    if constexpr (M) hv[q] = o.v;
                    if (better(o.v, o.item, o.slot, c.v, c.item, c.slot)) c = o;
                    cf |= fl;
                }
            }
            win = wave_reduce(c);
            wf = wave_or(cf);
            // (M) the team's runner-up, known in the winner's workgroup: its
            // own runner-up and the second best of the workgroups' bests
            if constexpr (M) {
                double h1 = -1.0, h2 = -1.0;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    h2 = fmax(h2, fmin(hv[q], h1));
                    h1 = fmax(h1, hv[q]);
                }
                top2_wave(h1, h2);
                v2 = win.aux == tm.rank ? fmax(lv2, h2) : __builtin_nan("");
            }
#ifdef LRA_TRACE
            t_b = wall_clock64();
            if (lane == 0 && tm.epoch < kSelTrace && tm.rank < 256) g_sel_done[tm.epoch * 256 + tm.rank] = t_b;
#endif
            // no candidate in the whole team (every item is in the basis):
            // there is no winner row to fetch
            const bool have = win.v > pub_min && win.aux >= 0 && win.aux < tm.size;
            for (int t = lane; t < width; t += kWave) {
                double x = 0.0;
                if (have) {
                    const uint64_t *row = rows + (size_t)win.aux * kRowWords + 2 * t;
                    const uint64_t *const ps[2] = {row, row + 1};
                    uint64_t d[2];
                    xget<2, 32>(ps, tag, d, &sm.xfail, tm.spin_limit);
                    x = __longlong_as_double((long long)lo_hi((uint32_t)d[0], (uint32_t)d[1]));
                }
                sm.wrow[t] = x;
            }
#ifdef LRA_TRACE
            t_c = wall_clock64();
#endif
            // after a timed-out poll nothing read in this launch can be
            // trusted: report "no candidate", which ends every caller loop
            if (__any(*(volatile int *)&sm.xfail)) {
                win = none();
                wf = 0;
            }
        }
        __builtin_amdgcn_wave_barrier();  // sm.wrow written by every lane above
        if (lane == 0) {
            sm.win = win;
            sm.win_v2 = v2;
            sm.win_flag = wf;
            if (mode == kSelHouseholder && win.v > 0.0) {
                const double nx = sqrt(win.v);
                const double x0 = sm.wrow[hstep];
                const double alpha = (x0 >= 0.0) ? -nx : nx;
                sm.wrow[hstep] = x0 - alpha;
                double vtv = 0.0;
                int o = hstep, c = hstep;
                LRA_QRP_RUN(qrp_nrm, width - hstep, sm.wrow, o, 1, c, vtv);
                sm.vtv = vtv;
                sm.alpha = alpha;
            }
            if (mode == kSelSwap && win.v >= 0.0 && win.slot >= 0 && win.slot < width) {
                const double x = sm.wrow[win.slot];
                sm.pivot = x;
                sm.wrow[win.slot] = x - 1.0;
            }
        }
    }
#ifdef LRA_TRACE
    const uint64_t t_d = wall_clock64();
#endif
    tm.epoch++;
    __syncthreads();
#ifdef LRA_TRACE
    if (threadIdx.x == 0) {
        const uint64_t t_e = wall_clock64();
        sm.t_select += t_e - t_in;
        sm.t_part[0] += t_a - t_in;
        sm.t_part[1] += t_b - t_a;
        sm.t_part[2] += t_c - t_b;
        sm.t_part[3] += t_e - t_d;
        sm.n_select += 1;
    }
#endif
}

// One step of the swap scan over N owned slots of an item, in ascending slot
// order: x <- x - f w (w = B[i*,:] - e_j*^T, skipped when f = 0), then the
// running largest magnitude, the lowest slot among equals.  `o` is the panel
// offset of the item's current slot j (stride pstep = sub * st per slot).
template <int N, bool M>
__device__ __forceinline__ void swap_chunk(double *panel, const double *wrow, int &o, int pstep, int &j, int sub,
                                           double f, double &vb, double &vb2, int &jb) {
    double x[N];
#pragma unroll
    for (int u = 0; u < N; u++) x[u] = panel[o + u * pstep];
    if (f != 0.0) {
        double w[N];  // every load before the first store: they are not reordered
#pragma unroll
        for (int u = 0; u < N; u++) w[u] = wrow[j + u * sub];
#pragma unroll
        for (int u = 0; u < N; u++) {
            x[u] -= f * w[u];
            panel[o + u * pstep] = x[u];
        }
    }
    int kb = -1;
#pragma unroll
    for (int u = 0; u < N; u++) {
        const bool up = fabs(x[u]) > vb;
        kb = up ? u : kb;
        if constexpr (M) vb2 = fmax(vb2, fmin(fabs(x[u]), vb));  // the runner-up among the slots seen
        vb = fmax(vb, fabs(x[u]));  // finite entries: the same value as up ? |x| : vb
    }
    if (kb >= 0) jb = j + kb * sub;
    o += N * pstep;
    j += N * sub;
}

// x <- x - f w on N slots of an item (panel offset o, stride pstep; w
// indexed by slot j, stride sub); all loads are issued before the stores.
template <int N>
__device__ __forceinline__ void axpy_chunk(double *panel, const double *w, int &o, int pstep, int &j, int sub,
                                           double f) {
    double x[N], y[N];
#pragma unroll
    for (int u = 0; u < N; u++) {
        x[u] = panel[o + u * pstep];
        y[u] = w[j + u * sub];
    }
#pragma unroll
    for (int u = 0; u < N; u++) panel[o + u * pstep] = x[u] - f * y[u];
    o += N * pstep;
    j += N * sub;
}

// The same on n slots starting at slot j: full chunks, then 4, 2 and 1.
__device__ __forceinline__ void axpy_slots(double *panel, const double *w, int o, int pstep, int j, int sub, int n,
                                           double f) {
    for (; n >= kChunk; n -= kChunk) axpy_chunk<kChunk>(panel, w, o, pstep, j, sub, f);
    if (n & 4) axpy_chunk<4>(panel, w, o, pstep, j, sub, f);
    if (n & 2) axpy_chunk<2>(panel, w, o, pstep, j, sub, f);
    if (n & 1) axpy_chunk<1>(panel, w, o, pstep, j, sub, f);
}

__device__ __forceinline__ void fail_status(Smem &sm, int st, int rank) {
    if (threadIdx.x == 0) {
        sm.status = st;
        if (st == LRA_ESINGULAR) sm.rank_found = rank;
    }
    __syncthreads();
}

template <bool M = false>
__device__ __forceinline__ void team_select(Team &tm, Smem &sm, Best b, int flag, const double *panel, const Geo &g,
                                            int width, int mode = kSelPlain, int hstep = 0, double pub_min = -1.0,
                                            double b2 = -1.0) {
    team_select<M>(tm, sm, b, flag, g, width, mode, hstep, PanelRow{panel, g.st, g.base}, NoOverlap{}, pub_min, b2);
}

// A decision's margin (decision_gap of the winner and the team's runner-up),
// folded into the workgroup's minimum by the winner's workgroup (the others
// see NaN for the runner-up).  Thread 0.
__device__ __forceinline__ void note_margin(Smem &sm) {
    if (threadIdx.x == 0 && !isnan(sm.win_v2)) sm.mmin = fmin(sm.mmin, decision_gap(sm.win.v, sm.win_v2));
}

// ---------------------------------------------------------------- maxvol
// Dominant r x r submatrix of the tall panel held in `panel` (slot-major,
// stride g.st): pivoted LU start (Algorithm alggos, stages 1-2), then the
// swaps of Algorithm algdomin with the rank-one update of B.  flags[li] is 0
// for a candidate item and slot+1 for a basis item.  Each item is handled by a
// group of `sub` consecutive lanes of one wavefront (lane_map: lane s owns
// slots s, s + sub, ...); all lanes of a group read an item's flag and shared entries
// before any lane of the group overwrites them (one instruction stream), and
// lane 0 of the group writes the flag.  Each elimination step or swap is
// applied lazily, fused with the scan for the next decision; the arithmetic of
// every entry is the oracle's, in the oracle's order.  On return sm.slot_item
// holds the basis in slot order.  `bad` flags a non-finite entry gathered.
template <bool M>
__device__ __forceinline__ void maxvol(Team &tm, Smem &sm, double *panel, uint8_t *flags, const Geo &g, int r,
                                       double delta, int max_swaps, int bad, int32_t &swaps_total, int32_t &converged) {
    const int tid = threadIdx.x;
    const int st = g.st;
    const LaneMap lm = lane_map(g.cnt, r, 0, kNWave);
    const int sub = lm.sub, s = lm.s, grp = lm.grp, ngrp = lm.ngrp;
    const int jlast = (s < r) ? s + ((r - 1 - s) / sub) * sub : -1;  // last owned slot
    const int nown = (s < r) ? (r - 1 - s) / sub + 1 : 0;               // owned slots
    const int pstep = sub * st;
    // ---- pivoted LU.  A team of several workgroups uses look-ahead: before
    // selection k only column k takes the elimination with pivot row k-1
    // (sm.wrow); the other columns take it inside selection k, on waves 1..
    // while wave 0 waits for the team, except for the workgroup's own best
    // item, whose row wave 0 publishes with the elimination applied on the fly
    // and which is brought up to date after the selection if another item won.
    // A single workgroup has no exchange to hide work behind and eliminates
    // every column before the scan.  Every entry receives the eliminations in
    // order with the oracle's arithmetic either way.
    const bool ahead = tm.size > 1;
    const LaneMap ld = lane_map(g.cnt, r, 1, kNWave - 1);  // overlap lanes (waves 1..)
    const int subd = ld.sub, sd = ld.s, grpd = ld.grp, ngrpd = ld.ngrp;
    double pk = 1.0;
    for (int k = 0; k < r; k++) {
#ifdef LRA_TRACE
        const uint64_t q0 = wall_clock64();
#endif
        Best b = none();
        double b2 = -1.0;
        for (int li = grp; li < g.cnt; li += ngrp) {
            if (flags[li]) continue;
            if (k > 0) {
                const double l = panel[(k - 1) * st + li] / pk;
                if (ahead) {
                    if (k % sub == s) {
                        const double x = panel[k * st + li] - l * sm.wrow[k];
                        panel[k * st + li] = x;
                        if constexpr (M) consider2(b, b2, fabs(x), g.base + li, 0);
                        else consider(b, fabs(x), g.base + li, 0);
                    }
                } else {
                    const int jf = (k <= s) ? s : s + ((k - s + sub - 1) / sub) * sub;  // first owned slot >= k
                    if (jf <= jlast) axpy_slots(panel, sm.wrow, jf * st + li, pstep, jf, sub, (jlast - jf) / sub + 1, l);
                    if (k % sub == s) {
                        if constexpr (M) consider2(b, b2, fabs(panel[k * st + li]), g.base + li, 0);
                        else consider(b, fabs(panel[k * st + li]), g.base + li, 0);
                    }
                }
                if ((k - 1) % sub == s) panel[(k - 1) * st + li] = l;
            } else if (k % sub == s) {
                if constexpr (M) consider2(b, b2, fabs(panel[k * st + li]), g.base + li, 0);
                else consider(b, fabs(panel[k * st + li]), g.base + li, 0);
            }
        }
        if (k > 0 && tid < k - 1) sm.L11[(k - 1) * (k - 2) / 2 + tid] = sm.wrow[tid];
#ifdef LRA_TRACE
        const uint64_t q1 = wall_clock64();
        if (tid == 0) sm.t_loop[0] += q1 - q0;
#endif
        const double *wp = sm.wprev[(k + 1) & 1];  // pivot row k-1 (k >= 1)
        // the row a workgroup publishes: columns past k still lack elimination k-1
        auto rowf = [&](int t, int64_t item) -> double {
            const int li = (int)(item - g.base);
            double x = panel[t * st + li];
            if (ahead && k > 0 && t > k) x -= panel[(k - 1) * st + li] * wp[t];
            return x;
        };
        // elimination k-1 on columns k+1.. of every other candidate item
        auto overlap = [&](int64_t lbest) {
            if (!ahead || k == 0 || k + 1 >= r) return;
            const int jf = (k + 1 <= sd) ? sd : sd + ((k + 1 - sd + subd - 1) / subd) * subd;
            if (jf >= r) return;
            const int n = (r - 1 - jf) / subd + 1;
            for (int li = grpd; li < g.cnt; li += ngrpd) {
                if (flags[li] || g.base + li == lbest) continue;
                axpy_slots(panel, wp, jf * st + li, subd * st, jf, subd, n, panel[(k - 1) * st + li]);
            }
        };
        team_select<M>(tm, sm, b, k == 0 ? bad : 0, g, r, kSelPlain, 0, rowf, overlap, -1.0, b2);
#ifdef LRA_TRACE
        const uint64_t q2 = wall_clock64();
#endif
        if (sm.win_flag) return fail_status(sm, LRA_EINVAL, 0);
        if (!(sm.win.v > 0.0)) return fail_status(sm, LRA_ESINGULAR, k);
        if constexpr (M) note_margin(sm);
        const int64_t wit = sm.win.item;
        if (tid == 0) sm.slot_item[k] = wit;
        if (wit >= g.base && wit < g.base + g.cnt) {
            const int lw = (int)(wit - g.base);
            if (lw % ngrp == grp && s == 0) flags[lw] = (uint8_t)(k + 1);
        }
        // the workgroup's best item, if it did not win, takes elimination k-1
        // on its columns past k (one thread per column), before the next scan
        // (spread over threads: done in the scan by the item's own lanes it
        // makes this workgroup the team's last to publish)
        const int64_t lb = sm.loc_item;
        if (ahead && k > 0 && lb != wit && lb >= g.base && lb < g.base + g.cnt && tid < r - 1 - k) {
            const int li = (int)(lb - g.base);
            const int j = k + 1 + tid;
            panel[j * st + li] -= panel[(k - 1) * st + li] * wp[j];
        }
        pk = sm.wrow[k];
        if (ahead) {
            // the look-ahead keeps the pivot row for the next overlap, and the
            // fix-up above must land before the next scan reads column k+1
            if (tid < r) sm.wprev[k & 1][tid] = sm.wrow[tid];
            __syncthreads();
        }
        // (eager: the next scan touches only entries its own lanes own, and
        // the next selection's first barrier orders everything shared)
#ifdef LRA_TRACE
        if (tid == 0) sm.t_loop[1] += wall_clock64() - q2;
#endif
    }
#ifdef LRA_TRACE
    const uint64_t qs = wall_clock64();
#endif
    // last multipliers (no trailing columns), last row of L11
    for (int li = grp; li < g.cnt; li += ngrp)
        if (!flags[li] && (r - 1) % sub == s) panel[(r - 1) * st + li] /= pk;
    if (tid < r - 1) sm.L11[(r - 1) * (r - 2) / 2 + tid] = sm.wrow[tid];
    __syncthreads();
    // ---- B = L21 L11^{-1}: each item solves x L11 = l_i by column-oriented
    // back substitution (for k = r-1 .. 1, x_k is final and every x_j, j < k,
    // takes x_j - x_k L11[k][j]); basis items get unit rows.  One thread per
    // item, slots in register blocks of 8 from the top: a block first takes
    // the terms of the finished slots above it, then its own, so every x_j
    // still receives its terms in decreasing k.
    for (int li = tid; li < g.cnt; li += kBlock) {
        const int fl = flags[li];
        if (fl) {
            for (int j = 0; j < r; j++) panel[j * st + li] = (j == fl - 1) ? 1.0 : 0.0;
            continue;
        }
        for (int j0 = ((r - 1) / 8) * 8; j0 >= 0; j0 -= 8) {
            const int nb = min(8, r - j0);
            double xr[8];
#pragma unroll
            for (int u = 0; u < 8; u++) xr[u] = u < nb ? panel[(j0 + u) * st + li] : 0.0;
#pragma unroll 4
            for (int k = r - 1; k >= j0 + 8; k--) {
                const double xk = panel[k * st + li];
                const double *Lk = sm.L11 + k * (k - 1) / 2 + j0;
#pragma unroll
                for (int u = 0; u < 8; u++) xr[u] -= xk * Lk[u];
            }
#pragma unroll
            for (int q = 7; q >= 1; q--) {
                if (q >= nb) continue;
                const double *Lq = sm.L11 + (j0 + q) * (j0 + q - 1) / 2 + j0;
#pragma unroll
                for (int u = 0; u < q; u++) xr[u] -= xr[q] * Lq[u];
            }
#pragma unroll
            for (int u = 0; u < 8; u++)
                if (u < nb) panel[(j0 + u) * st + li] = xr[u];
        }
    }
    __syncthreads();
#ifdef LRA_TRACE
    if (tid == 0) sm.t_loop[4] += wall_clock64() - qs;
#endif
    // ---- swaps; each update is fused with the next scan
    const double thr = 1.0 + delta;
    int swaps = 0;
    int js = -1;
    int64_t wit = -1;
    double pv = 1.0;
    for (;;) {
#ifdef LRA_TRACE
        const uint64_t q0 = wall_clock64();
#endif
        Best b = none();
        double b2 = -1.0;
        for (int li = grp; li < g.cnt; li += ngrp) {
            const int fl = flags[li];
            const int64_t it = g.base + li;
            double f = 0.0;
            if (js >= 0) {
                if (it == wit) {  // enters the basis in slot js
                    for (int j = s; j < r; j += sub) panel[j * st + li] = (j == js) ? 1.0 : 0.0;
                    if (s == 0) flags[li] = (uint8_t)(js + 1);
                    continue;
                }
                if (fl != 0 && fl != js + 1) continue;  // other basis rows: B[i][js] = 0
                f = panel[js * st + li] / pv;
                if (fl && s == 0) flags[li] = 0;  // the old basis item leaves the basis
            } else if (fl) {
                continue;
            }
            // B[i,:] -= f (B[i*,:] - e_js^T) on the owned slots, and the scan of
            // the owned slots (largest magnitude, lowest slot among equals):
            // full chunks, then the remainder in chunks of 4, 2 and 1
            double vb = -1.0, vb2 = -1.0;
            int jb = 0, j = s, k = nown, o = s * st + li;
            for (; k >= kChunk; k -= kChunk) swap_chunk<kChunk, M>(panel, sm.wrow, o, pstep, j, sub, f, vb, vb2, jb);
            if (k & 4) swap_chunk<4, M>(panel, sm.wrow, o, pstep, j, sub, f, vb, vb2, jb);
            if (k & 2) swap_chunk<2, M>(panel, sm.wrow, o, pstep, j, sub, f, vb, vb2, jb);
            if (k & 1) swap_chunk<1, M>(panel, sm.wrow, o, pstep, j, sub, f, vb, vb2, jb);
            if (jlast >= 0) {
                if constexpr (M) {
                    b2 = fmax(b2, vb2);
                    consider2(b, b2, vb, it, jb);
                } else {
                    consider(b, vb, it, jb);
                }
            }
        }
#ifdef LRA_TRACE
        const uint64_t q1 = wall_clock64();
        if (tid == 0) sm.t_loop[2] += q1 - q0;
#endif
        team_select<M>(tm, sm, b, 0, panel, g, r, kSelSwap, 0, thr, b2);
#ifdef LRA_TRACE
        const uint64_t q2 = wall_clock64();
#endif
        const double v = sm.win.v;
        // the stop test's margin (every workgroup sees the winner's value)
        if constexpr (M)
            if (v >= 0.0 && tid == 0) sm.mmin = fmin(sm.mmin, fabs(v - thr) / thr);
        if (v < 0.0 || v <= thr) break;  // no candidate left, or dominant
        if (swaps >= max_swaps) {
            converged = 0;
            break;
        }
        if constexpr (M) note_margin(sm);
        js = sm.win.slot;
        wit = sm.win.item;
        pv = sm.pivot;
        if (tid == 0) sm.slot_item[js] = wit;
        swaps++;
#ifdef LRA_TRACE
        if (tid == 0) sm.t_loop[3] += wall_clock64() - q2;
#endif
    }
    swaps_total += swaps;
}

// ---------------------------------------------------------------- entry sources
// The sketch W[K, L] of a dense matrix (cynical CUR): entry (i, j) is
// W[K[i]][L[j]].
template <typename T>
struct IndexedSrc {
    const T *A;
    int64_t lda;
    const int64_t *K, *L;
    __device__ __forceinline__ double operator()(int64_t i, int64_t j) const {
        return Elem<T>::load(A, K[i] * lda + L[j]);
    }
};

// Entries of the pre-processed matrix W' = W M (Section 13, Tests 2 with
// abridged randomized Hadamard pre-processing): M = D (H_{2^d} (x) I_s) of
// order N = 2^d s >= n, D the Rademacher signs of SplitMix64 stream 1 (those
// of the abridged SRHT), W zero-padded to N columns.  Entry (i, b s + e) is
// the sum over a = 0 .. 2^d - 1 of +-W[i][a s + e] (sign D[a s + e]
// (-1)^{popcount(a & b)}), in that order; nothing of W' is stored.
template <typename T>
struct HadamardSrc {
    const T *A;
    int64_t lda, n, s;
    int q2;
    uint64_t seed;
    __device__ __forceinline__ double operator()(int64_t i, int64_t j) const {
        const int64_t b = j / s, e = j - b * s;
        double acc = 0.0;
        for (int a = 0; a < q2; a++) {
            const int64_t c = a * s + e;
            if (c >= n) break;  // c grows with a
            const double w = Elem<T>::load(A, i * lda + c);
            const bool neg = ((sm64(seed, 1, (uint64_t)c) >> 63) != 0) != ((__popcll((uint64_t)(a & b)) & 1) != 0);
            acc += neg ? -w : w;
        }
        return acc;
    }
};

// Gather `cnt` items x r entries of W into the slot-major panel, eight// Gather `cnt` items x r entries of W into the slot-major panel, eight
// independent loads in flight per thread.  col = true: item it, slot j reads
// W[it][set[j]]; col = false: W[set[j]][it] (coalesced across items).
template <class Src>
__device__ __forceinline__ int gather_panel(double *panel, const Geo &g, const Src &src, int r, bool col,
                                            const int64_t *set) {
    int bad = 0;
    const int tot = g.cnt * r;
    for (int e0 = threadIdx.x; e0 < tot; e0 += kBlock * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int e = e0 + u * kBlock;
            if (e < tot) {
                const int li = e % g.cnt, j = e / g.cnt;
                const int64_t it = g.base + li;
                v[u] = col ? src(it, set[j]) : src(set[j], it);
            }
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int e = e0 + u * kBlock;
            if (e < tot) {
                const int li = e % g.cnt, j = e / g.cnt;
                if (!isfinite(v[u])) bad = 1;
                panel[j * g.st + li] = v[u];
            }
        }
    }
    return bad;
}

// One C-A step.  col = true: panel = W[:, set_in] (items = rows of W);
// col = false: panel = W[set_in, :]^T (items = columns).  set_out receives
// the new sorted set.
template <bool M, class Src>
__device__ __forceinline__ void ca_step(Team &tm, Smem &sm, double *panel, uint8_t *flags, const Src &src, int64_t m,
                                       int64_t n, int r, bool col, const int64_t *set_in, int64_t *set_out,
                                       const CAConfig &cfg, int32_t &swaps_total, int32_t &converged) {
    const Geo g = geo(tm, col ? m : n);
    LRA_TR(10 + (col ? 0 : 1), 0);
    const int bad = gather_panel(panel, g, src, r, col, set_in);
    for (int li = threadIdx.x; li < g.cnt; li += kBlock) flags[li] = 0;
    __syncthreads();
    LRA_TR(12, 0);
    maxvol<M>(tm, sm, panel, flags, g, r, cfg.delta, cfg.max_swaps, bad, swaps_total, converged);
#ifdef LRA_TRACE
    LRA_TR(13, sm.t_select);
#endif
    if (threadIdx.x < kWave && sm.status == LRA_OK) {
        if (threadIdx.x < r) set_out[threadIdx.x] = sm.slot_item[threadIdx.x];
        sort_set_wave(set_out, r);
    }
    __syncthreads();
}

// ---------------------------------------------------------------- bidiagonal multiplier
// Quasi-Gaussian multiplier G_q = B_1 P_1 ... B_q P_q (eq. (def11), section on
// pre-processing with quasi Gaussian matrices): B_i cyclic bidiagonal with
// ones on the diagonal and a random sign s_{i,j} at row j, column (j-1) mod N;
// P_i e_c = e_{pi_i(c)}.  pi_i: four Feistel rounds on [0, 2^b) (b the even
// bit count with 2^b >= N, at least 2), round function the low b/2 bits of
// SplitMix64 stream 6 at index (4 (i-1) + round) 2^32 + right half, walked
// back into [0, N) (Black and Rogaway's cycle walking); s_{i,j} = -1 when
// the top bit of stream 7 at index (i-1) N + j is set.
__device__ int64_t feistel_perm(uint64_t seed, int factor, int64_t N, int64_t x) {
    int b = 2;
    while (((int64_t)1 << b) < N) b += 2;
    const int half = b / 2;
    const uint64_t mask = ((uint64_t)1 << half) - 1;
    uint64_t y = (uint64_t)x;
    // a cycle of the network through x returns into [0, N) within 2^b steps
    for (int64_t guard = (int64_t)1 << b; guard > 0; guard--) {
        uint64_t L = y >> half, R = y & mask;
#pragma unroll
        for (int rd = 0; rd < 4; rd++) {
            const uint64_t f = sm64(seed, 6, ((uint64_t)(4 * (factor - 1) + rd) << 32) | R) & mask;
            const uint64_t nl = R;
            R = L ^ f;
            L = nl;
        }
        y = (L << half) | R;
        if ((int64_t)y < N) return (int64_t)y;
    }
    return x;
}

// Table of the l sampled columns (distinct draws, stream 2, in draw order):
// for column t its term count, then positions and integer coefficients in
// ascending position order (equal positions merged, zero terms dropped).
// One workgroup of 256 threads; each thread expands whole columns.
__global__ void __launch_bounds__(256) bidiag_table_kernel(uint64_t seed, int64_t N, int q, int l, int32_t *tab) {
    __shared__ int64_t samples[kLMax];
    if (threadIdx.x < kWave) draw_distinct_wave(seed, 2, N, l, samples);
    __syncthreads();
    int32_t *cnt = tab, *pos_out = tab + kLMax, *coef_out = tab + kLMax + (size_t)kLMax * kBdTerms;
    for (int t = threadIdx.x; t < l; t += blockDim.x) {
        int64_t pos[kBdTerms], np[kBdTerms];
        int32_t coef[kBdTerms], nc[kBdTerms];
        int k = 1;
        pos[0] = samples[t];
        coef[0] = 1;
        for (int i = q; i >= 1; i--) {
            int nk = 0;
            for (int u = 0; u < k; u++) {
                const int64_t p = feistel_perm(seed, i, N, pos[u]);
                const int64_t p1 = (p + 1) % N;
                const int32_t sg = (sm64(seed, 7, (uint64_t)((i - 1) * N + p1)) >> 63) ? -1 : 1;
                np[nk] = p;
                nc[nk++] = coef[u];
                np[nk] = p1;
                nc[nk++] = coef[u] * sg;
            }
            for (int a = 1; a < nk; a++) {  // ascending positions
                const int64_t kp = np[a];
                const int32_t kc = nc[a];
                int b2 = a - 1;
                while (b2 >= 0 && np[b2] > kp) {
                    np[b2 + 1] = np[b2];
                    nc[b2 + 1] = nc[b2];
                    b2--;
                }
                np[b2 + 1] = kp;
                nc[b2 + 1] = kc;
            }
            k = 0;
            for (int a = 0; a < nk; a++) {
                if (k > 0 && pos[k - 1] == np[a]) {
                    coef[k - 1] += nc[a];
                } else {
                    pos[k] = np[a];
                    coef[k] = nc[a];
                    k++;
                }
            }
            int z = 0;
            for (int a = 0; a < k; a++)
                if (coef[a] != 0) {
                    pos[z] = pos[a];
                    coef[z] = coef[a];
                    z++;
                }
            k = z;
        }
        cnt[t] = k;
        for (int a = 0; a < k; a++) {
            pos_out[(size_t)t * kBdTerms + a] = (int32_t)pos[a];
            coef_out[(size_t)t * kBdTerms + a] = coef[a];
        }
    }
}

// Greedy Householder QRP over the team's items (Algorithm alg1tor): `steps`
// choices over the first `width` coordinates of every item (coordinate c of
// item li at panel[c * g.st + li]); flags[li] != 0 keeps an item out of the
// running and is set for every chosen item.  Step gg takes the item whose
// coordinates gg.. have the largest 2-norm (ties to the lowest item) and
// reflects them onto a multiple of e_gg; each reflection is applied lazily,
// fused with the next step's norms, in the oracle's order of operations.
// flush: also apply the last step's reflection, and write every chosen
// item's own image (alpha at its step, zeros after), so that on return the
// panel holds H_{steps-1} ... H_0 of every item.  tup / tdiag (optional)
// receive the chosen items in that final basis, an upper triangular matrix:
// tup[gg (gg - 1) / 2 + c] = coordinate c < gg of the item chosen at step
// gg, tdiag[gg] = its alpha.  out[gg] = the item chosen at step gg.  A zero
// norm ends the loop with ESINGULAR (rank = the step), a flagged non-finite
// entry (`bad`) with EINVAL.  Same thread-to-item mapping as every other
// per-item loop here (li = tid, tid + kBlock, ...).
template <bool M = false>
__device__ __forceinline__ void team_qrp(Team &tm, Smem &sm, double *panel, uint8_t *flags, const Geo &g, int width,
                                         int steps, int bad, bool flush, int64_t *out, double *tup, double *tdiag) {
    const int tid = threadIdx.x;
    const int ipw = g.st;
    for (int gg = 0; gg < steps + (flush ? 1 : 0); gg++) {
        const bool last = gg == steps;
        Best b = none();
        double b2 = -1.0;
        const double vtv = sm.vtv;
        for (int li = tid; li < g.cnt; li += kBlock) {
            if (flags[li]) continue;
            double nrm = 0.0;
            if (gg > 0 && vtv > 0.0) {  // reflection of step gg-1 (vector in sm.wrow[gg-1 ..])
                double acc = 0.0;
                int o = (gg - 1) * ipw + li, c = gg - 1;
                LRA_QRP_RUN(qrp_dot, width - gg + 1, panel, o, ipw, sm.wrow, c, acc);
                const double f = 2.0 * acc / vtv;
                // the update, and the norm of the entries from gg on in the
                // same pass (its terms in increasing index order)
                o = (gg - 1) * ipw + li;
                c = gg - 1;
                double nrm0 = 0.0;  // entry gg-1 takes the update only
                qrp_upd<1>(panel, o, ipw, sm.wrow, c, f, nrm0);
                LRA_QRP_RUN(qrp_upd, width - gg, panel, o, ipw, sm.wrow, c, f, nrm);
            } else if (!last) {
                int o = gg * ipw + li, c = gg;
                LRA_QRP_RUN(qrp_nrm, width - gg, panel, o, ipw, c, nrm);
            }
            if constexpr (M) consider2(b, b2, nrm, g.base + li, 0);
            else consider(b, nrm, g.base + li, 0);
        }
        if (last) break;
        team_select<M>(tm, sm, b, gg == 0 ? bad : 0, panel, g, width, kSelHouseholder, gg, -1.0, b2);
        if (sm.win_flag) return fail_status(sm, LRA_EINVAL, 0);
        if (!(sm.win.v > 0.0)) return fail_status(sm, LRA_ESINGULAR, gg);
        if constexpr (M) note_margin(sm);
        const int64_t wit = sm.win.item;
        if (tid == 0) out[gg] = wit;
        if (tup && tid < gg) tup[gg * (gg - 1) / 2 + tid] = sm.wrow[tid];
        if (tdiag && tid == 0) tdiag[gg] = sm.alpha;
        if (wit >= g.base && wit < g.base + g.cnt && (int)((wit - g.base) % kBlock) == tid) {
            const int li = (int)(wit - g.base);
            flags[li] = 1;
            if (flush) {
                // the published row was read before this point, by every
                // workgroup, from sm.wrow of its own
                panel[gg * ipw + li] = sm.alpha;
                for (int c = gg + 1; c < width; c++) panel[c * ipw + li] = 0.0;
            }
        }
    }
}

// Abridged SRHT sketch of the team's items (Appendix B): for sampled column
// t = b s + e of D H_{N,d}, Y[item][q] = sqrt(s/l) sum_a W[item][a s + e]
// D[a s + e] (-1)^{popcount(a & b)} (post-multiplication; pre-multiplication
// swaps the roles of rows and columns).  Then greedy Householder QRP over the
// items picks r of them (Algorithm alg1tor); each reflection is applied
// lazily, fused with the next norm scan.  The chosen items land in out.
// With `bd` (a bidiagonal-multiplier column table) the sketch entries are the
// table's signed-integer combinations of W's entries instead.
// cos and sin of 2 pi m / N (0 <= m < N) in a fixed order of IEEE
// operations, the oracle's definition: octant o = floor(8 m / N) and
// remainder rem = 8 m - o N as integers; x = (pi/4) rem / N for even o, or
// (pi/4) (N - rem) / N from the far end for odd o; cos x and sin x by their
// Taylor series through x^20 and x^21 (Horner in x^2, coefficients from
// a_k = -a_{k-1} / ((2k - 1) 2k) and b_k = -b_{k-1} / (2k (2k + 1))); then
// the octant's symmetry.
__device__ __forceinline__ void unit_root(int64_t m, int64_t N, double &c_out, double &s_out) {
    const double pi4 = 0x1.921fb54442d18p-1;
    const int64_t u = 8 * m;
    const int64_t o = u / N;
    const int64_t rem = u - o * N;
    const bool odd = (o & 1) != 0;
    const double x = (pi4 * (double)(odd ? N - rem : rem)) / (double)N;
    double a = 1.0, b = 1.0;
    double ak[11], bk[11];
    ak[0] = a;
    bk[0] = b;
#pragma unroll
    for (int k = 1; k < 11; k++) {
        a = -a / (double)((2 * k - 1) * (2 * k));
        b = -b / (double)((2 * k) * (2 * k + 1));
        ak[k] = a;
        bk[k] = b;
    }
    const double x2 = x * x;
    double pc = ak[10], ps = bk[10];
#pragma unroll
    for (int k = 9; k >= 0; k--) {
        pc = pc * x2 + ak[k];
        ps = ps * x2 + bk[k];
    }
    const double c = pc, s = x * ps;
    if (!odd) {
        const int q = (int)(o / 2);
        c_out = q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
        s_out = q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
    } else {
        const int q = (int)((o + 1) / 2);
        c_out = q == 1 ? s : q == 2 ? -c : q == 3 ? -s : c;
        s_out = q == 1 ? c : q == 2 ? s : q == 3 ? -c : -s;
    }
}

template <bool kFourier, bool M, class Src>
__device__ __forceinline__ void sketch_qrp(Team &tm, Smem &sm, double *panel, uint8_t *flags, const Src &src, int64_t m,
                                          int64_t n, int r, int side, int d, int l, uint64_t seed, int64_t *out,
                                          const int32_t *bd) {
    const int tid = threadIdx.x;
    const int64_t dim = side ? m : n;
    const Geo g = geo(tm, side ? n : m);
    const int64_t q2 = (int64_t)1 << d;
    const int64_t s = (dim + q2 - 1) / q2;
    const int64_t N = q2 * s;
    int bad = 0;
    if constexpr (kFourier) {
        // abridged randomized Fourier multiplier: sampled column t = b s + e
        // has coefficient i^{t_j} omega_N^{b j} at rows j = a s + e (zero past
        // the end); the table (cos and sin parts, l 2^d <= kAftCoefs each) sits
        // in the LU scratch, which no sketch touches
        if (tid < kWave) draw_distinct_wave(seed, 2, N, l, sm.samples);
        __syncthreads();
        double *const cre = sm.L11, *const cim = sm.L11 + kAftCoefs;
        for (int e2 = tid; e2 < l * (int)q2; e2 += kBlock) {
            const int q = e2 / (int)q2, a = e2 % (int)q2;
            const int64_t t = sm.samples[q];
            const int64_t bb = t / s, ee = t % s;
            const int64_t j = a * s + ee;
            double cr = 0.0, ci = 0.0;
            if (j < dim) {
                const int64_t mexp = (int64_t)(((uint64_t)bb * (uint64_t)j) % (uint64_t)N);
                double c, sn;
                unit_root(mexp, N, c, sn);
                const int tq = (int)(sm64(seed, 1, (uint64_t)j) >> 62);
                cr = tq == 0 ? c : tq == 1 ? -sn : tq == 2 ? -c : sn;
                ci = tq == 0 ? sn : tq == 1 ? c : tq == 2 ? -sn : -c;
            }
            cre[e2] = cr;
            cim[e2] = ci;
        }
        __syncthreads();
        LRA_TR(2, 0);
        const double scale = sqrt((double)s / (double)l);
        const int tot = g.cnt * l;
        for (int e = tid; e < tot; e += kBlock) {
            const int li = e % g.cnt, q = e / g.cnt;
            const int64_t it = g.base + li;
            const int64_t ee = sm.samples[q] % s;
            double w[8];
#pragma unroll
            for (int a = 0; a < 8; a++) {
                const int64_t j = a * s + ee;
                w[a] = (a < q2 && j < dim) ? (side ? src(j, it) : src(it, j)) : 0.0;
            }
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int a = 0; a < 8; a++)
                if (a < q2 && a * s + ee < dim) {
                    re += w[a] * cre[q * (int)q2 + a];
                    im += w[a] * cim[q * (int)q2 + a];
                }
            const double yr = scale * re, yi = scale * im;
            if (!isfinite(yr) || !isfinite(yi)) bad = 1;
            panel[q * g.st + li] = yr;
            panel[(l + q) * g.st + li] = yi;
        }
    } else {
    if (bd) {
        // bidiagonal-product multiplier: y = sum over the sampled column's
        // terms, in ascending position order, of coef * w (no scale)
        const int32_t *cnt = bd, *bpos = bd + kLMax, *bcoef = bd + kLMax + (size_t)kLMax * kBdTerms;
        const int tot = g.cnt * l;
        for (int e = tid; e < tot; e += kBlock) {
            const int li = e % g.cnt, q = e / g.cnt;
            const int64_t it = g.base + li;
            const int c = cnt[q];
            const int32_t *P = bpos + (size_t)q * kBdTerms, *C = bcoef + (size_t)q * kBdTerms;
            double acc = 0.0;
            for (int k = 0; k < c; k++) {
                const double w = side ? src(P[k], it) : src(it, P[k]);
                acc += (double)C[k] * w;
            }
            if (!isfinite(acc)) bad = 1;
            panel[q * g.st + li] = acc;
        }
    } else {
    if (tid < kWave) draw_distinct_wave(seed, 2, N, l, sm.samples);
    __syncthreads();
    LRA_TR(2, 0);
    const double scale = sqrt((double)s / (double)l);
    if (q2 <= 8) {
        // per sampled column t = b s + e: the offset e and the signs
        // D[a s + e] (-1)^{popcount(a & b)} of its 2^d terms as a bit mask, so
        // the item loop has no division and no hashing (each term is +-w exactly)
        for (int q = tid; q < l; q += kBlock) {
            const int64_t t = sm.samples[q];
            const int64_t bb = t / s, ee = t % s;
            uint32_t mask = 0;
            for (int64_t a = 0; a < q2; a++) {
                const int64_t c = a * s + ee;
                const double h = (__popcll((uint64_t)(a & bb)) & 1) ? -1.0 : 1.0;
                if (c < dim && rademacher(seed, c) * h < 0.0) mask |= 1u << a;
            }
            sm.sgn[q] = (uint8_t)mask;
            sm.samples[q] = ee;
        }
        __syncthreads();
        if (g.cnt > 0) {
            // thread -> (item, sample) without division: step by kBlock
            // entries, four entries per round so that 32 loads are in flight;
            // loads past the end read a valid entry and are discarded
            constexpr int kNP = 4;
            int li = tid % g.cnt, q = tid / g.cnt;
            const int dli = kBlock % g.cnt, dq = kBlock / g.cnt;
            while (q < l) {
                int pli[kNP], pq[kNP];
#pragma unroll
                for (int p = 0; p < kNP; p++) {
                    pli[p] = li;
                    pq[p] = q;
                    li += dli;
                    q += dq;
                    if (li >= g.cnt) {
                        li -= g.cnt;
                        q++;
                    }
                }
                double w[kNP][8];
#pragma unroll
                for (int p = 0; p < kNP; p++) {
                    const bool on = pq[p] < l;
                    const int64_t it = g.base + pli[p];
                    const int64_t ee = sm.samples[on ? pq[p] : 0];
#pragma unroll
                    for (int a = 0; a < 8; a++) {
                        const int64_t c = a * s + ee;
                        const int64_t cc = (a < q2 && c < dim) ? c : ee;  // ee < dim always
                        w[p][a] = side ? src(cc, it) : src(it, cc);
                    }
                }
#pragma unroll
                for (int p = 0; p < kNP; p++) {
                    if (pq[p] >= l) continue;
                    const int64_t ee = sm.samples[pq[p]];
                    const uint32_t mask = sm.sgn[pq[p]];
                    double acc = 0.0;
#pragma unroll
                    for (int a = 0; a < 8; a++)
                        if (a < q2 && a * s + ee < dim) acc += ((mask >> a) & 1u) ? -w[p][a] : w[p][a];
                    const double y = scale * acc;
                    if (!isfinite(y)) bad = 1;
                    panel[pq[p] * g.st + pli[p]] = y;
                }
            }
        }
    } else {
        const int tot = g.cnt * l;
        for (int e = tid; e < tot; e += kBlock) {
            const int li = e % g.cnt, q = e / g.cnt;
            const int64_t it = g.base + li;
            const int64_t t = sm.samples[q];
            const int64_t bb = t / s, ee = t % s;
            double acc = 0.0;
            for (int64_t a = 0; a < q2; a++) {
                const int64_t c = a * s + ee;
                if (c >= dim) continue;
                const double h = (__popcll((uint64_t)(a & bb)) & 1) ? -1.0 : 1.0;
                const double w = side ? src(c, it) : src(it, c);
                acc += w * rademacher(seed, c) * h;
            }
            const double y = scale * acc;
            if (!isfinite(y)) bad = 1;
            panel[q * g.st + li] = y;
        }
    }
    }  // sketch forms
    }  // the Fourier form is a separate instantiation
    for (int li = tid; li < g.cnt; li += kBlock) flags[li] = 0;
    __syncthreads();
    LRA_TR(3, 0);
    team_qrp<M>(tm, sm, panel, flags, g, kFourier ? 2 * l : l, r, bad, false, out, nullptr, nullptr);
    if (sm.status != LRA_OK) return;
    __syncthreads();
#ifdef LRA_TRACE
    LRA_TR(4, sm.t_select);
#endif
}

// ---------------------------------------------------------------- r-projective volume
// One orthogonaliser pass over every item of the slice: z <- z - f (w . z) w,
// f = f0 (w . z), w = sm.wrow[0 .. r-1] (the picked item's z), the dot
// product and the new |z|^2 in index order.  Returns the best candidate
// (flag 0) by |z|^2 when want_members is false, else the best member (flag
// nonzero) by max(0, 1 - |z|^2) (the factor by which dropping it scales
// v_2^2 in an orthonormal-row set, eq. (eqa)).
__device__ __forceinline__ Best orth_pass(Smem &sm, double *panel, const uint8_t *flags, const Geo &g, int r,
                                          double f0, bool want_members) {
    const int ipw = g.st;
    Best b = none();
    for (int li = threadIdx.x; li < g.cnt; li += kBlock) {
        double acc = 0.0;
        int o = li, c = 0;
        LRA_QRP_RUN(qrp_dot, r, panel, o, ipw, sm.wrow, c, acc);
        double nrm = 0.0;
        o = li;
        c = 0;
        LRA_QRP_RUN(qrp_upd, r, panel, o, ipw, sm.wrow, c, f0 * acc, nrm);
        if (want_members) {
            if (flags[li]) consider(b, fmax(0.0, 1.0 - nrm), g.base + li, 0);
        } else if (!flags[li]) {
            consider(b, nrm, g.base + li, 0);
        }
    }
    return b;
}

// k items whose vectors span a submatrix of large r-projective volume
// (Algorithm algprjvlm, transposed; Algorithms alg1tor and algrup and the
// expansion-contraction recipe after them as its black box).  The panel
// holds one w-vector per item (a row of W[:, J] in a column step, a column
// of W[I, :] in a row step).
//  1. r QRP steps over all w coordinates, flushed: the first r coordinates
//     of every item are then R' = Q_r^T (item), Q_r spanning the r pivots.
//  2. Algorithm alg1tor on R' (r QRP steps over the first r coordinates,
//     every item a candidate again); its chosen vectors, in the final basis,
//     form the upper triangular T (sm.L11 packed by columns, sm.wprev[0] the
//     diagonal).
//  3. Algorithm algrup: every item y becomes z = T^{-1} y, so that the
//     chosen set has orthonormal rows (its members become e_g exactly) and a
//     candidate's expansion factor of eq. (eqb) is 1 + |z|^2.  Each step
//     takes the largest |z|^2 (ties to the lowest item); with b its z and
//     beta = |b|^2, the orthogonaliser of the grown set, I + gamma b b^T /
//     beta with gamma = 1 / sqrt(1 + beta) - 1, is applied to every item as
//     z <- z - (b . z) b / (q (1 + q)), q = sqrt(1 + beta).
//  4. Exchanges: expand by the best candidate b (factor 1 + beta), then the
//     member s (not b) of least leverage |z_s|^2 in the grown set would
//     leave (factor 1 - |z_s|^2); while the product exceeds 1 + delta (at
//     most max_swaps times) s leaves, and the orthogonaliser of the shrunk
//     set, z <- z + (s . z) s / (q (1 + q)) with q = sqrt(1 - |z_s|^2), is
//     applied to every item.
// out[0..k-1] = the items (an exchange puts b in s's place); ESINGULAR
// (rank = the step) when stage 1 or 2 meets a zero norm.  swaps and
// converged accumulate over calls.
__device__ __forceinline__ void projvol_select(Team &tm, Smem &sm, double *panel, uint8_t *flags, const Geo &g, int w,
                                               int r, int k, int bad, int64_t *out, double delta, int max_swaps,
                                               int32_t &swaps, int32_t &converged) {
    const int tid = threadIdx.x;
    const int ipw = g.st;
    double *const tup = sm.L11, *const tdiag = sm.wprev[0];
    team_qrp(tm, sm, panel, flags, g, w, r, bad, true, out, nullptr, nullptr);
    if (sm.status != LRA_OK) return;
    for (int li = tid; li < g.cnt; li += kBlock) flags[li] = 0;
    team_qrp(tm, sm, panel, flags, g, r, r, 0, true, out, tup, tdiag);
    if (sm.status != LRA_OK) return;
    __syncthreads();  // T complete in every workgroup
    Best b = none();
    for (int li = tid; li < g.cnt; li += kBlock) {
        for (int c = r - 1; c >= 0; c--) {
            double x = panel[c * ipw + li];
            for (int j = c + 1; j < r; j++) x -= tup[j * (j - 1) / 2 + c] * panel[j * ipw + li];
            x /= tdiag[c];
            panel[c * ipw + li] = x;
        }
        if (flags[li]) continue;
        double s = 0.0;
        for (int c = 0; c < r; c++) s += panel[c * ipw + li] * panel[c * ipw + li];
        consider(b, s, g.base + li, 0);
    }
    auto owner = [&](int64_t it) {
        return it >= g.base && it < g.base + g.cnt && (int)((it - g.base) % kBlock) == tid;
    };
    for (int gg = r; gg < k; gg++) {
        team_select(tm, sm, b, 0, panel, g, r);
        if (!(sm.win.v >= 0.0)) return fail_status(sm, LRA_ESINGULAR, gg);
        const int64_t wit = sm.win.item;
        if (tid == 0) out[gg] = wit;
        if (owner(wit)) flags[wit - g.base] = 1;
        const double q = sqrt(1.0 + sm.win.v);
        b = orth_pass(sm, panel, flags, g, r, 1.0 / (q * (1.0 + q)), false);
    }
    int32_t sw = 0;
    while ((int64_t)k < g.items) {
        team_select(tm, sm, b, 0, panel, g, r);
        if (!(sm.win.v >= 0.0)) break;
        const int64_t bi = sm.win.item;
        const double grow = 1.0 + sm.win.v;
        const double q = sqrt(grow);
        Best m = orth_pass(sm, panel, flags, g, r, 1.0 / (q * (1.0 + q)), true);
        team_select(tm, sm, m, 0, panel, g, r);
        if (!(sm.win.v >= 0.0)) break;
        const int64_t si = sm.win.item;
        const double shrink = sm.win.v;
        if (!(grow * shrink > 1.0 + delta)) break;
        if (sw >= max_swaps) {
            converged = 0;
            break;
        }
        if (owner(bi)) flags[bi - g.base] = 1;
        if (owner(si)) flags[si - g.base] = 0;
        if (tid == 0)
            for (int j = 0; j < k; j++)
                if (out[j] == si) {
                    out[j] = bi;
                    break;
                }
        sw++;
        const double q2 = sqrt(shrink);
        b = orth_pass(sm, panel, flags, g, r, -1.0 / (q2 * (1.0 + q2)), false);
    }
    swaps += sw;
    __syncthreads();
}

// The whole C-A path for one matrix, executed by every workgroup of a team.
// imap / jmap (optional) translate the returned row and column ids (a solve
// on a sketch); swaps_base and team_report fold in an earlier phase.
// kFourier: the instantiation that seeds from the abridged Fourier sketch
// (a separate kernel, so that the other starts carry none of its code).
template <bool kFourier, bool M, class Src>
__device__ __forceinline__ void ca_solve(Team &tm, Smem &sm, double *dyn, uint8_t *flags, const Src &src, int64_t m,
                                        int64_t n, uint64_t seed, const CAConfig &cfg, int64_t *I_out, int64_t *J_out,
                                        double *U_out, lra_info *info, const int64_t *imap = nullptr,
                                        const int64_t *jmap = nullptr, int32_t swaps_base = 0,
                                        int32_t team_report = 0) {
    const int tid = threadIdx.x;
    const int r = cfg.r;
    int32_t swaps_total = 0, converged = 1, sweeps_run = 0;
    int seed_step = 0;
    if (tid == 0) {
        sm.status = LRA_OK;
        sm.rank_found = r;
        sm.nucleus_rank = r;
        sm.xfail = 0;
        sm.mmin = 1.0;
#ifdef LRA_TRACE
        sm.t_select = 0;
        sm.t_part[0] = sm.t_part[1] = sm.t_part[2] = sm.t_part[3] = sm.t_part[4] = 0;
        sm.n_select = 0;
        sm.t_loop[0] = sm.t_loop[1] = sm.t_loop[2] = sm.t_loop[3] = sm.t_loop[4] = 0;
#endif
    }
    LRA_TR(1, 0);
    __syncthreads();
    // ---- start set
    if (cfg.pre == LRA_PRE_ASRHT || cfg.pre == LRA_PRE_BIDIAG || cfg.pre == LRA_PRE_ASRFT) {
        // pre-multiplication for m >= n (either form is allowed when m = n;
        // this one reads whole rows of W and yields the start columns directly)
        const int side = (m >= n) ? 1 : 0;
        const int32_t *bd = cfg.pre == LRA_PRE_BIDIAG ? cfg.bd_table : nullptr;
        // the items x l sketch slice lives in LDS when it fits, else in a
        // per-workgroup slice of global memory (touched by this workgroup only)
        // (two call sites so that each copy knows its panel's address space)
        if (cfg.sketch_ws) {
            const int64_t st_s = (((side ? n : m) + tm.size - 1) / tm.size) | 1;
            const int wsk = kFourier ? 2 * cfg.ah_samples : cfg.ah_samples;
            sketch_qrp<kFourier, M>(tm, sm, cfg.sketch_ws + (size_t)tm.rank * st_s * wsk, flags, src, m, n, r, side,
                                 cfg.ah_depth, cfg.ah_samples, seed, side ? sm.Jset : sm.Iset, bd);
        } else {
            sketch_qrp<kFourier, M>(tm, sm, dyn, flags, src, m, n, r, side, cfg.ah_depth, cfg.ah_samples, seed,
                                 side ? sm.Jset : sm.Iset, bd);
        }
        if (sm.status != LRA_OK) goto finish;
        if (tid < kWave) sort_set_wave(side ? sm.Jset : sm.Iset, r);
        __syncthreads();
        seed_step = side ? 0 : 1;  // a row start set needs one row step first
    } else if (cfg.init_cols) {
        if (tid < r) sm.Jset[tid] = cfg.init_cols[tid];
        __syncthreads();
        if (tid < kWave) sort_set_wave(sm.Jset, r);
        __syncthreads();
    } else {
        if (tid < kWave) {
            draw_distinct_wave(seed, 0, n, r, sm.Jset);
            __builtin_amdgcn_wave_barrier();
            sort_set_wave(sm.Jset, r);
        }
        __syncthreads();
    }
    // ---- steps: the optional seed row step, then a column step and a row
    // step per sweep (one call site: the step is inlined once)
    for (int st = 0; st < seed_step + 2 * cfg.sweeps; st++) {
        const bool col = st >= seed_step && ((st - seed_step) & 1) == 0;
        ca_step<M>(tm, sm, dyn, flags, src, m, n, r, col, col ? sm.Jset : sm.Iset, col ? sm.Iset : sm.Jset, cfg,
                swaps_total, converged);
        if (sm.status != LRA_OK) goto finish;
        if (st < seed_step || col) continue;
        const int sw = (st - seed_step) / 2;  // sweep sw is complete
        sweeps_run = sw + 1;
        bool same = sw > 0;
        for (int j = 0; j < r && same; j++)
            same = (sm.Iset[j] == sm.Iprev[j]) && (sm.Jset[j] == sm.Jprev[j]);
        __syncthreads();
        if (same) break;
        if (tid < r) {
            sm.Iprev[tid] = sm.Iset[tid];
            sm.Jprev[tid] = sm.Jset[tid];
        }
        __syncthreads();
    }
    LRA_TR(20, 0);
#ifdef LRA_TRACE
    LRA_TR(30, sm.t_part[0]);
    LRA_TR(31, sm.t_part[1]);
    LRA_TR(32, sm.t_part[2]);
    LRA_TR(33, sm.t_part[3]);
    LRA_TR(34, sm.n_select);
    LRA_TR(40, sm.t_part[4]);
    LRA_TR(35, sm.t_loop[0]);
    LRA_TR(36, sm.t_loop[1]);
    LRA_TR(37, sm.t_loop[2]);
    LRA_TR(38, sm.t_loop[3]);
    LRA_TR(39, sm.t_loop[4]);
#endif
    if (tm.rank == 0) nucleus(sm, dyn, src, r, cfg.refine_steps, kBlock, U_out);
    LRA_TR(21, 0);
finish:
    __syncthreads();
    // the run's smallest decision margin: a team folds every workgroup's own
    // into the info record's margin word (zeroed before the launch) as the
    // complement of its bits, so that the largest word holds the smallest
    // margin, and counts arrivals in its spare word; workgroup 0 waits for all
    double mm = __builtin_nan("");
    if constexpr (M) {
        if (tm.size == 1) {
            mm = sm.mmin;
        } else if (info && tid == 0) {
            unsigned long long *mw = reinterpret_cast<unsigned long long *>(&info->min_margin);
            unsigned *cnt = reinterpret_cast<unsigned *>(&info->reserved);
            atomicMax(mw, ~(unsigned long long)__double_as_longlong(sm.mmin));
            __threadfence();
            atomicAdd(cnt, 1u);
            if (tm.rank == 0) {
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)tm.size) {
                    if (wall_clock64() - t0 > tm.spin_limit) {
                        sm.xfail = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __threadfence();
                mm = __longlong_as_double(
                    (long long)~__hip_atomic_load(mw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            }
        }
    }
    if (tm.rank != 0) return;
    __syncthreads();
    const int st = sm.xfail ? LRA_EDEVICE : sm.status;
    if (tid < r) {
        I_out[tid] = st == LRA_OK ? (imap ? imap[sm.Iset[tid]] : sm.Iset[tid]) : -1;
        J_out[tid] = st == LRA_OK ? (jmap ? jmap[sm.Jset[tid]] : sm.Jset[tid]) : -1;
    }
    if (st != LRA_OK)
        for (int e = tid; e < r * r; e += kBlock) U_out[e] = __builtin_nan("");
    if (tid == 0 && info) {
        lra_info inf;
        inf.status = st;
        inf.sweeps_run = sweeps_run;
        inf.swaps_total = swaps_base + swaps_total;
        inf.converged = (st == LRA_OK) ? converged : 0;
        inf.rank_found = sm.rank_found;
        inf.team_size = team_report ? team_report : tm.size;
        inf.nucleus_rank = st == LRA_OK ? sm.nucleus_rank : 0;
        inf.reserved = 0;
        inf.det_log_abs = st == LRA_OK ? sm.logdet : 0.0;
        inf.min_margin = mm;
        *info = inf;
    }
}

// ---------------------------------------------------------------- kernels
template <typename T, bool kFourier, bool M>
__global__ void __launch_bounds__(kBlock) ca_team_kernel(const T *A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                                                         CAConfig cfg, TeamWs ws, int64_t *I_out, int64_t *J_out,
                                                         double *U_out, lra_info *info) {
    __shared__ Smem sm;
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    double *dyn = reinterpret_cast<double *>(lds_dyn);
    uint8_t *flags = lds_dyn + cfg.panel_bytes;
    Team tm;
    tm.rank = blockIdx.x;
    tm.size = gridDim.x;
    tm.epoch = 0;
    tm.xw = ws.xw;
    tm.spin_limit = ws.spin_limit;
    ca_solve<kFourier, M>(tm, sm, dyn, flags, DenseSrc<T>{A, lda}, m, n, seed, cfg, I_out, J_out, U_out, info);
}

// C-A CUR of the pre-processed matrix W' = W M (HadamardSrc), m x N.
template <typename T, bool M>
__global__ void __launch_bounds__(kBlock) ca_hadamard_kernel(const T *A, int64_t m, int64_t n, int64_t lda, int d,
                                                             uint64_t seed, CAConfig cfg, TeamWs ws, int64_t *I_out,
                                                             int64_t *J_out, double *U_out, lra_info *info) {
    __shared__ Smem sm;
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    double *dyn = reinterpret_cast<double *>(lds_dyn);
    uint8_t *flags = lds_dyn + cfg.panel_bytes;
    Team tm;
    tm.rank = blockIdx.x;
    tm.size = gridDim.x;
    tm.epoch = 0;
    tm.xw = ws.xw;
    tm.spin_limit = ws.spin_limit;
    const int q2 = 1 << d;
    const int64_t s = (n + q2 - 1) / q2;
    ca_solve<false, M>(tm, sm, dyn, flags, HadamardSrc<T>{A, lda, n, s, q2, seed}, m, (int64_t)q2 * s, seed, cfg, I_out, J_out,
             U_out, info);
}

// Cynical CUR (Section 1.3, Fig. 3; Tests 3 and 4 of Section 13): k random
// columns L (and, with no loops, k random rows K, stream 5), `loops` C-A loops
// at rank k over the whole team (cfg_k), then workgroup 0 alone runs C-A at
// rank r on the k x k sketch W[K, L] (cfg_r, seed + 1) and maps its sets back.
template <typename T>
__global__ void __launch_bounds__(kBlock) ca_cynical_kernel(const T *A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                                                            int32_t loops, CAConfig cfg_k, CAConfig cfg_r, TeamWs ws,
                                                            int64_t *I_out, int64_t *J_out, double *U_out,
                                                            lra_info *info) {
    __shared__ Smem sm;
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    double *dyn = reinterpret_cast<double *>(lds_dyn);
    uint8_t *flags = lds_dyn + cfg_k.panel_bytes;
    Team tm;
    tm.rank = blockIdx.x;
    tm.size = gridDim.x;
    tm.epoch = 0;
    tm.xw = ws.xw;
    tm.spin_limit = ws.spin_limit;
    const int tid = threadIdx.x;
    const int k = cfg_k.r, r = cfg_r.r;
    const DenseSrc<T> src{A, lda};
    if (tid == 0) {
        sm.status = LRA_OK;
        sm.rank_found = k;
        sm.xfail = 0;
    }
    if (tid < kWave) {
        draw_distinct_wave(seed, 0, n, k, sm.Jset);
        __builtin_amdgcn_wave_barrier();
        sort_set_wave(sm.Jset, k);
        if (loops == 0) {
            __builtin_amdgcn_wave_barrier();
            draw_distinct_wave(seed, 5, m, k, sm.Iset);
            __builtin_amdgcn_wave_barrier();
            sort_set_wave(sm.Iset, k);
        }
    }
    __syncthreads();
    int32_t swaps = 0, converged = 1;
    for (int s = 0; s < loops; s++) {
        ca_step<false>(tm, sm, dyn, flags, src, m, n, k, true, sm.Jset, sm.Iset, cfg_k, swaps, converged);
        if (sm.status != LRA_OK) break;
        ca_step<false>(tm, sm, dyn, flags, src, m, n, k, false, sm.Iset, sm.Jset, cfg_k, swaps, converged);
        if (sm.status != LRA_OK) break;
        bool same = s > 0;
        for (int j = 0; j < k && same; j++) same = (sm.Iset[j] == sm.Iprev[j]) && (sm.Jset[j] == sm.Jprev[j]);
        __syncthreads();
        if (same) break;
        if (tid < k) {
            sm.Iprev[tid] = sm.Iset[tid];
            sm.Jprev[tid] = sm.Jset[tid];
        }
        __syncthreads();
    }
    __syncthreads();
    if (tm.rank != 0) return;
    const int team = tm.size;
    if (sm.status != LRA_OK || sm.xfail) {
        const int st = sm.xfail ? LRA_EDEVICE : sm.status;
        if (tid < r) {
            I_out[tid] = -1;
            J_out[tid] = -1;
        }
        for (int e = tid; e < r * r; e += kBlock) U_out[e] = __builtin_nan("");
        if (tid == 0 && info) {
            lra_info inf;
            inf.status = st;
            inf.sweeps_run = 0;
            inf.swaps_total = swaps;
            inf.converged = 0;
            inf.rank_found = sm.rank_found;
            inf.team_size = team;
            inf.nucleus_rank = 0;
            inf.reserved = 0;
            inf.det_log_abs = 0.0;
            inf.min_margin = __builtin_nan("");
            *info = inf;
        }
        return;
    }
    // the sketch's rows and columns (the inner solve draws no samples)
    static_assert(kLMax >= 2 * kRMax, "the sketch sets fit in the sample buffer");
    int64_t *const Kset = sm.samples, *const Lset = sm.samples + kRMax;
    if (tid < k) {
        Kset[tid] = sm.Iset[tid];
        Lset[tid] = sm.Jset[tid];
    }
    __syncthreads();
    Team solo;
    solo.rank = 0;
    solo.size = 1;
    solo.epoch = 0;
    solo.xw = nullptr;
    solo.spin_limit = 0;
    ca_solve<false, false>(solo, sm, dyn, flags, IndexedSrc<T>{A, lda, Kset, Lset}, k, k, seed + 1, cfg_r, I_out, J_out, U_out,
             info, Kset, Lset, swaps, team);
}

// C-A with k x l generators of large r-projective volume: l random start
// columns (stream 0), then sweeps of a column step (k rows of W[:, J] by
// projvol_select) and a row step (l columns of W[I, :]), stopping at a fixed
// point; nucleus W[I, J]_r^+ in workgroup 0.  cfg.r = r; cfg.delta and
// cfg.max_swaps govern each step's exchanges.
template <typename T>
__global__ void __launch_bounds__(kBlock) ca_projective_kernel(const T *A, int64_t m, int64_t n, int64_t lda,
                                                               uint64_t seed, int32_t k, int32_t l, CAConfig cfg,
                                                               TeamWs ws, int64_t *I_out, int64_t *J_out,
                                                               double *U_out, lra_info *info) {
    __shared__ Smem sm;
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    double *dyn = reinterpret_cast<double *>(lds_dyn);
    uint8_t *flags = lds_dyn + cfg.panel_bytes;
    Team tm;
    tm.rank = blockIdx.x;
    tm.size = gridDim.x;
    tm.epoch = 0;
    tm.xw = ws.xw;
    tm.spin_limit = ws.spin_limit;
    const int tid = threadIdx.x;
    const int r = cfg.r;
    const DenseSrc<T> src{A, lda};
    if (tid == 0) {
        sm.status = LRA_OK;
        sm.rank_found = r;
        sm.nucleus_rank = r;
        sm.xfail = 0;
        sm.vtv = 0.0;
        sm.logdet = 0.0;
    }
    if (tid < kWave) {
        draw_distinct_wave(seed, 0, n, l, sm.Jset);
        __builtin_amdgcn_wave_barrier();
        sort_set_wave(sm.Jset, l);
    }
    __syncthreads();
    int32_t sweeps_run = 0, swaps = 0, converged = 1;
    for (int s = 0; s < cfg.sweeps; s++) {
        {
            const Geo g = geo(tm, m);
            const int bad = gather_panel(dyn, g, src, l, true, sm.Jset);
            for (int li = tid; li < g.cnt; li += kBlock) flags[li] = 0;
            __syncthreads();
            projvol_select(tm, sm, dyn, flags, g, l, r, k, bad, sm.Iset, cfg.delta, cfg.max_swaps, swaps, converged);
            if (sm.status != LRA_OK) break;
            if (tid < kWave) sort_set_wave(sm.Iset, k);
            __syncthreads();
        }
        {
            const Geo g = geo(tm, n);
            const int bad = gather_panel(dyn, g, src, k, false, sm.Iset);
            for (int li = tid; li < g.cnt; li += kBlock) flags[li] = 0;
            __syncthreads();
            projvol_select(tm, sm, dyn, flags, g, k, r, l, bad, sm.Jset, cfg.delta, cfg.max_swaps, swaps, converged);
            if (sm.status != LRA_OK) break;
            if (tid < kWave) sort_set_wave(sm.Jset, l);
            __syncthreads();
        }
        sweeps_run = s + 1;
        bool same = s > 0;
        for (int j = 0; j < k && same; j++) same = sm.Iset[j] == sm.Iprev[j];
        for (int j = 0; j < l && same; j++) same = sm.Jset[j] == sm.Jprev[j];
        __syncthreads();
        if (same) break;
        if (tid < k) sm.Iprev[tid] = sm.Iset[tid];
        if (tid < l) sm.Jprev[tid] = sm.Jset[tid];
        __syncthreads();
    }
    __syncthreads();
    if (tm.rank != 0) return;
    const int st = sm.xfail ? LRA_EDEVICE : sm.status;
    if (st == LRA_OK) nucleus_trunc(sm, dyn, src, k, l, r, U_out);
    if (tid < k) I_out[tid] = st == LRA_OK ? sm.Iset[tid] : -1;
    if (tid < l) J_out[tid] = st == LRA_OK ? sm.Jset[tid] : -1;
    if (st != LRA_OK)
        for (int e = tid; e < l * k; e += kBlock) U_out[e] = __builtin_nan("");
    if (tid == 0 && info) {
        lra_info inf;
        inf.status = st;
        inf.sweeps_run = sweeps_run;
        inf.swaps_total = swaps;
        inf.converged = st == LRA_OK ? converged : 0;
        inf.rank_found = sm.rank_found;
        inf.team_size = tm.size;
        inf.nucleus_rank = st == LRA_OK ? sm.nucleus_rank : 0;
        inf.reserved = 0;
        inf.det_log_abs = st == LRA_OK ? sm.logdet : 0.0;
        inf.min_margin = __builtin_nan("");
        *info = inf;
    }
}

// The few LDS fields the uniform-score CUR needs (sets, nucleus results):
// a small static footprint lets two workgroups share a CU at k = l = 64.
struct UniSmem {
    int64_t Iset[kRMax], Jset[kRMax];
    int32_t nucleus_rank;
    double logdet;
};

// CUR with uniform leverage scores (Algorithm algcurlevsc with p_j = 1/n,
// pbar_i = 1/m) for many blocks, one workgroup per block in turn: l column
// draws (stream 8) and k row draws (stream 9) with replacement, sorted;
// M = Dbar W[I, J] D with Dbar = sqrt(m / k), D = sqrt(n / l); U = D M_r^+
// Dbar by nucleus_trunc.  Only the k l generator entries are read.  Block b
// uses seed + b; every block costs the same, so blocks are dealt round-robin.
template <typename T>
__global__ void __launch_bounds__(kBlock) ca_uniform_kernel(const T *base, const BlockDesc *blocks, int64_t count,
                                                            uint64_t seed, int32_t r, int32_t k, int32_t l,
                                                            int64_t *I_out, int64_t *J_out, double *U_out,
                                                            lra_info *infos) {
    __shared__ UniSmem sm;
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    double *dyn = reinterpret_cast<double *>(lds_dyn);
    const int tid = threadIdx.x;
    for (int64_t b = blockIdx.x; b < count; b += gridDim.x) {
        const BlockDesc d = blocks[b];
        const DenseSrc<T> src{base + d.offset, d.lda};
        const uint64_t sd = seed + (uint64_t)b;
        if (tid < kWave) {
            draw_uniform_wave(sd, 8, d.n, l, sm.Jset);
            draw_uniform_wave(sd, 9, d.m, k, sm.Iset);
            __builtin_amdgcn_wave_barrier();
            sort_set_wave(sm.Jset, l);
            sort_set_wave(sm.Iset, k);
        }
        __syncthreads();
        int bad = 0;
        for (int e = tid; e < k * l; e += kBlock) bad |= !isfinite(src(sm.Iset[e / l], sm.Jset[e % l]));
        bad = __syncthreads_or(bad);
        double *const U = U_out + b * (int64_t)l * k;
        if (!bad) {
            const double dm = sqrt((double)d.m / (double)k), dn = sqrt((double)d.n / (double)l);
            nucleus_trunc(sm, dyn, src, k, l, r, U, dm, dn);
        } else {
            for (int e = tid; e < l * k; e += kBlock) U[e] = __builtin_nan("");
        }
        if (tid < k) I_out[b * k + tid] = bad ? -1 : sm.Iset[tid];
        if (tid < l) J_out[b * l + tid] = bad ? -1 : sm.Jset[tid];
        if (tid == 0 && infos) {
            lra_info inf;
            inf.status = bad ? LRA_EINVAL : LRA_OK;
            inf.sweeps_run = 0;
            inf.swaps_total = 0;
            inf.converged = bad ? 0 : 1;
            inf.rank_found = r;
            inf.team_size = 1;
            inf.nucleus_rank = bad ? 0 : sm.nucleus_rank;
            inf.reserved = 0;
            inf.det_log_abs = bad ? 0.0 : sm.logdet;
            inf.min_margin = __builtin_nan("");
            infos[b] = inf;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- leverage scores
// Refinement of a CUR LRA by its leverage scores (section on refining an LRA
// with leverage scores; Algorithm algcurlevsc with the crude LRA's scores,
// Algorithm algsmplex for the draws): six launches on one stream.
//  1. lev_gather_kernel (grid-stride): the items' r-vectors in FP64, one row
//     per a of P (r x (n + m)): columns j of R = W[I0, :] at 0 .. n-1, rows i
//     of C = W[:, J0] at n .. n+m-1, so that every later pass reads them
//     coalesced; flags a non-finite entry.
//  2. lev_gram_kernel (a thread per lower-triangle entry of R R^T and C^T C):
//     each entry summed over the items in increasing order (the oracle's
//     order), two batches of loads in flight ahead of the dependent sum.
//  3. lev_chol_kernel (a workgroup per side): the lower Cholesky factors in
//     LDS, entry formulas and orders of the oracle.
//  4. lev_score_kernel (a thread per item): q_i = |L^{-1} x_i|^2 by the
//     row-oriented forward solve.
//  5. lev_cdf_kernel (a workgroup per side): running sums of the scores in
//     item order, chunks staged through LDS, one lane adding.
//  6. lev_pick_kernel (one workgroup): k + l draws u_t = (x >> 11) 2^-53 from
//     SplitMix64 streams 8 / 9 (first item whose running sum exceeds u_t S),
//     sorted; D = 1 / sqrt(l q_j / S), Dbar likewise; U = D M_r^+ Dbar by
//     nucleus_trunc.
// ws layout (doubles): L_R, L_C, G_R, G_C [64 x 64 each], q (n + m), cdf
// (n + m), P (r x (n + m)); flags: [0] non-finite entry, [1] Gram not
// positive definite.
struct LevSmem {
    int64_t Iset[kSMax], Jset[kSMax];
    int64_t tmp[2 * kSMax];
    double dk[kSMax], dl[kSMax];
    int32_t nucleus_rank;
    double logdet;
};

__device__ __forceinline__ double *lev_scores(double *ws) { return ws + 4 * kRMax * kRMax; }
// Jacobi work space of the nucleus beyond 64 rows or columns: after the
// scores, running sums and the FP64 factors (2 kSMax^2 doubles).
__device__ __forceinline__ double *lev_jacobi_ws(double *ws, int64_t m, int64_t n, int r) {
    return lev_scores(ws) + (size_t)(2 + r) * (size_t)(n + m);
}

template <typename T>
__global__ void __launch_bounds__(256) lev_gather_kernel(const T *A, int64_t m, int64_t n, int64_t lda, int r,
                                                         const int64_t *I0, const int64_t *J0, double *ws,
                                                         int32_t *flags) {
    const DenseSrc<T> src{A, lda};
    const int64_t items = n + m, total = items * r;
    double *P = lev_scores(ws) + 2 * items;
    int bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(e / items);
        const int64_t it = e - (int64_t)a * items;
        const double v = it < n ? src(I0[a], it) : src(it - n, J0[a]);
        if (!isfinite(v)) bad = 1;
        P[e] = v;
    }
    if (bad) flags[0] = 1;
}

// A thread per lower-triangle entry (a, b), b <= a, of one side's Gram
// matrix, summing x_a x_b over the items in increasing order.  The items go
// by in batches of 12 held in three register sets, so that two batches'
// loads are in flight while one is added (the sum itself is a dependent
// chain and cannot be split without changing the order).
__global__ void __launch_bounds__(64) lev_gram_kernel(int64_t m, int64_t n, int r, double *ws) {
    constexpr int kB = 12;
    const int tri = r * (r + 1) / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * tri) return;
    const int side = e / tri, t = e - side * tri;
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= t) a++;
    const int b = t - a * (a + 1) / 2;
    const int64_t items = n + m, cnt = side == 0 ? n : m;
    const double *P = lev_scores(ws) + 2 * items + (side == 0 ? 0 : n);
    const double *xa = P + (int64_t)a * items, *xb = P + (int64_t)b * items;
    double s = 0.0;
    double a0[kB], b0[kB], a1[kB], b1[kB], a2[kB], b2[kB];
    auto load = [&](double(&pa)[kB], double(&pb)[kB], int64_t j) {
#pragma unroll
        for (int u = 0; u < kB; u++) {
            pa[u] = xa[j * kB + u];
            pb[u] = xb[j * kB + u];
        }
    };
    auto add = [&](const double(&pa)[kB], const double(&pb)[kB]) {
#pragma unroll
        for (int u = 0; u < kB; u++) s += pa[u] * pb[u];
    };
    const int64_t nb = cnt / kB;  // full batches
    int64_t j = 0;
    if (nb > 0) load(a0, b0, 0);
    if (nb > 1) load(a1, b1, 1);
    // on entry: set 0 holds batch j, set 1 batch j + 1 (when they exist)
    for (; j + 3 <= nb; j += 3) {
        load(a2, b2, j + 2);
        add(a0, b0);
        if (j + 3 < nb) load(a0, b0, j + 3);
        add(a1, b1);
        if (j + 4 < nb) load(a1, b1, j + 4);
        add(a2, b2);
    }
    if (j < nb) add(a0, b0);
    if (j + 1 < nb) add(a1, b1);
    for (int64_t i = nb * kB; i < cnt; i++) s += xa[i] * xb[i];
    ws[(size_t)(2 + side) * kRMax * kRMax + a * r + b] = s;
}

__global__ void __launch_bounds__(kBlock) lev_chol_kernel(int r, double *ws, int32_t *flags) {
    __shared__ double s_g[kRMax * kRMax];
    __shared__ double L[kRMax * kRMax];
    __shared__ int s_sing;
    const int tid = threadIdx.x, side = blockIdx.x;
    const double *G = ws + (size_t)(2 + side) * kRMax * kRMax;
    for (int e = tid; e < r * r; e += kBlock) {
        const int a = e / r, b = e % r;
        s_g[e] = b <= a ? G[e] : 0.0;
    }
    for (int e = tid; e < kRMax * kRMax; e += kBlock) L[e] = 0.0;
    if (tid == 0) s_sing = 0;
    __syncthreads();
    // column b at a time: the diagonal, then the column below it
    for (int b = 0; b < r; b++) {
        if (tid == 0) {
            double sd = s_g[b * r + b];
            for (int c = 0; c < b; c++) sd -= L[b * kRMax + c] * L[b * kRMax + c];
            if (!(sd > 0.0)) s_sing = 1;
            L[b * kRMax + b] = sqrt(sd);
        }
        __syncthreads();
        if (s_sing) break;
        const int a = b + 1 + tid;
        if (a < r) {
            double sa = s_g[a * r + b];
            for (int c = 0; c < b; c++) sa -= L[a * kRMax + c] * L[b * kRMax + c];
            L[a * kRMax + b] = sa / L[b * kRMax + b];
        }
        __syncthreads();
    }
    if (tid == 0 && s_sing) flags[1] = 1;
    for (int e = tid; e < r * kRMax; e += kBlock) ws[(size_t)side * kRMax * kRMax + e] = L[e];
}

__global__ void __launch_bounds__(256) lev_score_kernel(int64_t m, int64_t n, int r, double *ws) {
    const int64_t items = n + m;
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= items) return;
    const int side = it < n ? 0 : 1;
    const double *L = ws + (size_t)side * kRMax * kRMax;
    const double *P = lev_scores(ws) + 2 * items + it;
    // fully unrolled over the largest rank so that z stays in registers
    double z[kRMax];
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < kRMax; a++) {
        if (a < r) {
            double x = P[(int64_t)a * items];
#pragma unroll
            for (int c = 0; c < a; c++) x -= L[a * kRMax + c] * z[c];
            z[a] = x / L[a * kRMax + a];
            s += z[a] * z[a];
        }
    }
    lev_scores(ws)[it] = s;
}

// running sums of the scores in item order: workgroup 0 the columns (n),
// workgroup 1 the rows (m); each chunk is staged in LDS by the workgroup and
// summed by lane 0, eight values loaded ahead of the dependent adds
__global__ void __launch_bounds__(256) lev_cdf_kernel(int64_t m, int64_t n, double *ws) {
    constexpr int kChunk = 2048;
    __shared__ double s_q[kChunk], s_c[kChunk];
    const int tid = threadIdx.x, side = blockIdx.x;
    double *q = lev_scores(ws), *cdf = q + n + m;
    const int64_t off = side == 0 ? 0 : n, cnt = side == 0 ? n : m;
    double acc = 0.0;
    for (int64_t i0 = 0; i0 < cnt; i0 += kChunk) {
        const int len = (int)min<int64_t>(kChunk, cnt - i0);
        for (int t = tid; t < len; t += 256) s_q[t] = q[off + i0 + t];
        __syncthreads();
        if (tid == 0) {
            // the next 16 values are read while the current 16 are added
            constexpr int kB = 16;
            int t = 0;
            double cur[kB];
            if (len >= kB) {
#pragma unroll
                for (int u = 0; u < kB; u++) cur[u] = s_q[u];
                for (; t + 2 * kB <= len; t += kB) {
                    double nxt[kB];
#pragma unroll
                    for (int u = 0; u < kB; u++) nxt[u] = s_q[t + kB + u];
#pragma unroll
                    for (int u = 0; u < kB; u++) {
                        acc += cur[u];
                        s_c[t + u] = acc;
                    }
#pragma unroll
                    for (int u = 0; u < kB; u++) cur[u] = nxt[u];
                }
#pragma unroll
                for (int u = 0; u < kB; u++) {
                    acc += cur[u];
                    s_c[t + u] = acc;
                }
                t += kB;
            }
            for (; t < len; t++) {
                acc += s_q[t];
                s_c[t] = acc;
            }
        }
        __syncthreads();
        for (int t = tid; t < len; t += 256) cdf[off + i0 + t] = s_c[t];
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) lev_pick_kernel(const T *A, int64_t m, int64_t n, int64_t lda, int r,
                                                          int k, int l, uint64_t seed, double *ws,
                                                          const int32_t *flags, int64_t *I_out, int64_t *J_out,
                                                          double *U_out, lra_info *info) {
    __shared__ LevSmem sm;
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    double *dyn = reinterpret_cast<double *>(lds_dyn);
    const int tid = threadIdx.x;
    const DenseSrc<T> src{A, lda};
    const double *q = lev_scores(ws);
    const double *cdf = q + n + m;
    int st = flags[0] ? LRA_EINVAL : flags[1] ? LRA_ESINGULAR : LRA_OK;
    if (st == LRA_OK) {
        // draws: threads 0 .. l-1 columns, l .. l+k-1 rows
        if (tid < k + l) {
            const bool col = tid < l;
            const int t = col ? tid : tid - l;
            const int64_t off = col ? 0 : n, cnt = col ? n : m;
            const double S = cdf[off + cnt - 1];
            const double u = (double)(sm64(seed, col ? 8 : 9, (uint64_t)t) >> 11) * 0x1p-53;
            const double target = u * S;
            int64_t lo = 0, hi = cnt - 1;
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (cdf[off + mid] > target) hi = mid;
                else lo = mid + 1;
            }
            if (col) sm.Jset[t] = lo;
            else sm.Iset[t] = lo;
        }
        __syncthreads();
        sort_two_sets(sm.Jset, l, sm.Iset, k, sm.tmp);
        if (tid < l) sm.dl[tid] = 1.0 / sqrt(((double)l * q[sm.Jset[tid]]) / cdf[n - 1]);
        if (tid >= kSMax && tid < kSMax + k)
            sm.dk[tid - kSMax] = 1.0 / sqrt(((double)k * q[n + sm.Iset[tid - kSMax]]) / cdf[n + m - 1]);
        __syncthreads();
        int bad = 0;
        for (int e = tid; e < k * l; e += kBlock) bad |= !isfinite(src(sm.Iset[e / l], sm.Jset[e % l]));
        if (__syncthreads_or(bad)) st = LRA_EINVAL;
    }
    if (st == LRA_OK) {
        // up to 64 rows or columns the rotations run in LDS, beyond in the
        // global workspace (one workgroup: L2-resident)
        const int nr = k > l ? k : l;
        if (nr <= kRMax)
            nucleus_trunc<kRMax / 16>(sm, dyn, src, k, l, r, U_out, 1.0, 1.0, sm.dk, sm.dl);
        else if (nr <= 128)
            nucleus_trunc<8>(sm, lev_jacobi_ws(ws, m, n, r), src, k, l, r, U_out, 1.0, 1.0, sm.dk, sm.dl);
        else
            nucleus_trunc<16>(sm, lev_jacobi_ws(ws, m, n, r), src, k, l, r, U_out, 1.0, 1.0, sm.dk, sm.dl);
    }
    if (tid < k) I_out[tid] = st == LRA_OK ? sm.Iset[tid] : -1;
    if (tid < l) J_out[tid] = st == LRA_OK ? sm.Jset[tid] : -1;
    if (st != LRA_OK)
        for (int e = tid; e < l * k; e += kBlock) U_out[e] = __builtin_nan("");
    if (tid == 0 && info) {
        lra_info inf;
        inf.status = st;
        inf.sweeps_run = 0;
        inf.swaps_total = 0;
        inf.converged = st == LRA_OK ? 1 : 0;
        inf.rank_found = st == LRA_ESINGULAR ? 0 : r;
        inf.team_size = 1;
        inf.nucleus_rank = st == LRA_OK ? sm.nucleus_rank : 0;
        inf.reserved = 0;
        inf.det_log_abs = st == LRA_OK ? sm.logdet : 0.0;
        inf.min_margin = __builtin_nan("");
        *info = inf;
    }
}

template <typename T, bool M>
__global__ void __launch_bounds__(kBlock) ca_batched_kernel(const T *base, const BlockDesc *blocks, const int32_t *order,
                                                            int64_t count, uint64_t seed, CAConfig cfg, unsigned *queue,
                                                            int64_t *I_out, int64_t *J_out, double *U_out,
                                                            lra_info *infos) {
    __shared__ Smem sm;
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    double *dyn = reinterpret_cast<double *>(lds_dyn);
    uint8_t *flags = lds_dyn + cfg.panel_bytes;
    Team tm;
    tm.rank = 0;
    tm.size = 1;
    tm.epoch = 0;
    tm.xw = nullptr;
    tm.spin_limit = 0;
    const int r = cfg.r;
    for (;;) {
        if (threadIdx.x == 0) sm.job = (int32_t)atomicAdd(queue, 1u);
        __syncthreads();
        const int64_t job = sm.job;
        __syncthreads();
        if (job >= count) break;
        const int32_t b = order[job];
        const BlockDesc d = blocks[b];
        ca_solve<false, M>(tm, sm, dyn, flags, DenseSrc<T>{base + d.offset, d.lda}, d.m, d.n, seed + (uint64_t)b, cfg,
                 I_out + (int64_t)b * r, J_out + (int64_t)b * r, U_out + (int64_t)b * r * r,
                 infos ? infos + b : nullptr);
        __syncthreads();
    }
}

// Far-field blocks evaluated from their point sets: the batched loop with
// entries computed on the fly.
template <bool M>
__global__ void __launch_bounds__(kBlock) ca_points_kernel(const double *pts, const PtsDesc *blocks,
                                                           const int32_t *order, int64_t count, uint64_t seed,
                                                           CAConfig cfg, unsigned *queue, int64_t *I_out,
                                                           int64_t *J_out, double *U_out, lra_info *infos) {
    __shared__ Smem sm;
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    double *dyn = reinterpret_cast<double *>(lds_dyn);
    uint8_t *flags = lds_dyn + cfg.panel_bytes;
    Team tm;
    tm.rank = 0;
    tm.size = 1;
    tm.epoch = 0;
    tm.xw = nullptr;
    tm.spin_limit = 0;
    const int r = cfg.r;
    for (;;) {
        if (threadIdx.x == 0) sm.job = (int32_t)atomicAdd(queue, 1u);
        __syncthreads();
        const int64_t job = sm.job;
        __syncthreads();
        if (job >= count) break;
        const int32_t b = order[job];
        const PtsDesc d = blocks[b];
        ca_solve<false, M>(tm, sm, dyn, flags, PointSrc{pts + 2 * d.x_off, pts + 2 * d.y_off}, d.m, d.n, seed + (uint64_t)b, cfg,
                 I_out + (int64_t)b * r, J_out + (int64_t)b * r, U_out + (int64_t)b * r * r,
                 infos ? infos + b : nullptr);
        __syncthreads();
    }
}

__global__ void zero_u32_kernel(unsigned *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

__global__ void zero_u64_kernel(uint64_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// The exchange words, and (info non-null) the info record's margin word and
// arrival counter, which a team's workgroups fold their margins into.
__global__ void zero_team_kernel(uint64_t *p, int64_t n, lra_info *info) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
    if (info && blockIdx.x == 0 && threadIdx.x == 0) {
        info->reserved = 0;
        *reinterpret_cast<unsigned long long *>(&info->min_margin) = 0ull;
    }
}

// ---------------------------------------------------------------- launchers
template <typename T>
static hipError_t launch_team_t(const void *A, int64_t m, int64_t n, int64_t lda, uint64_t seed, const CAConfig &cfg,
                                const TeamWs &ws, int team, size_t dyn_bytes, int64_t *I_out, int64_t *J_out,
                                double *U_out, lra_info *info, hipStream_t stream) {
    // margins (cfg.margins) select the instantiation that tracks them
    auto kern = cfg.margins ? (cfg.pre == LRA_PRE_ASRFT ? ca_team_kernel<T, true, true> : ca_team_kernel<T, false, true>)
                            : (cfg.pre == LRA_PRE_ASRFT ? ca_team_kernel<T, true, false>
                                                        : ca_team_kernel<T, false, false>);
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes);
    (void)e;
    if (team > 1) {
        const int64_t words = (int64_t)2 * team * kSlotWords;
        hipLaunchKernelGGL(zero_team_kernel, dim3((unsigned)std::min<int64_t>(256, (words + 255) / 256)), dim3(256), 0,
                           stream, ws.xw, words, cfg.margins ? info : nullptr);
    }
    const T *Ap = static_cast<const T *>(A);
    CAConfig c = cfg;
    TeamWs w = ws;
    void *args[] = {(void *)&Ap, (void *)&m, (void *)&n, (void *)&lda, (void *)&seed, (void *)&c,
                    (void *)&w, (void *)&I_out, (void *)&J_out, (void *)&U_out, (void *)&info};
    return hipLaunchCooperativeKernel((const void *)kern, dim3(team), dim3(kBlock), args, (unsigned)dyn_bytes, stream);
}

hipError_t launch_team(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, uint64_t seed, const CAConfig &cfg,
                       const TeamWs &ws, int team, size_t dyn_bytes, int64_t *I_out, int64_t *J_out, double *U_out,
                       lra_info *info, hipStream_t stream) {
    switch (dtype) {
    case LRA_F64:
        return launch_team_t<double>(A, m, n, lda, seed, cfg, ws, team, dyn_bytes, I_out, J_out, U_out, info, stream);
    case LRA_F32:
        return launch_team_t<float>(A, m, n, lda, seed, cfg, ws, team, dyn_bytes, I_out, J_out, U_out, info, stream);
    default:
        return launch_team_t<uint16_t>(A, m, n, lda, seed, cfg, ws, team, dyn_bytes, I_out, J_out, U_out, info,
                                       stream);
    }
}

template <typename T>
static hipError_t launch_hadamard_t(const void *A, int64_t m, int64_t n, int64_t lda, int d, uint64_t seed,
                                    const CAConfig &cfg, const TeamWs &ws, int team, size_t dyn_bytes, int64_t *I_out,
                                    int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream) {
    auto kern = cfg.margins ? ca_hadamard_kernel<T, true> : ca_hadamard_kernel<T, false>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes);
    (void)e;
    if (team > 1) {
        const int64_t words = (int64_t)2 * team * kSlotWords;
        hipLaunchKernelGGL(zero_team_kernel, dim3((unsigned)std::min<int64_t>(256, (words + 255) / 256)), dim3(256), 0,
                           stream, ws.xw, words, cfg.margins ? info : nullptr);
    }
    const T *Ap = static_cast<const T *>(A);
    CAConfig c = cfg;
    TeamWs w = ws;
    void *args[] = {(void *)&Ap,   (void *)&m,     (void *)&n,     (void *)&lda,  (void *)&d,   (void *)&seed,
                    (void *)&c,    (void *)&w,     (void *)&I_out, (void *)&J_out, (void *)&U_out, (void *)&info};
    return hipLaunchCooperativeKernel((const void *)kern, dim3(team), dim3(kBlock), args, (unsigned)dyn_bytes, stream);
}

hipError_t launch_hadamard(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, int d, uint64_t seed,
                           const CAConfig &cfg, const TeamWs &ws, int team, size_t dyn_bytes, int64_t *I_out,
                           int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream) {
    switch (dtype) {
    case LRA_F64:
        return launch_hadamard_t<double>(A, m, n, lda, d, seed, cfg, ws, team, dyn_bytes, I_out, J_out, U_out, info,
                                         stream);
    case LRA_F32:
        return launch_hadamard_t<float>(A, m, n, lda, d, seed, cfg, ws, team, dyn_bytes, I_out, J_out, U_out, info,
                                        stream);
    default:
        return launch_hadamard_t<uint16_t>(A, m, n, lda, d, seed, cfg, ws, team, dyn_bytes, I_out, J_out, U_out,
                                           info, stream);
    }
}

hipError_t launch_bidiag_table(uint64_t seed, int64_t N, int q, int l, int32_t *table, hipStream_t stream) {
    hipLaunchKernelGGL(bidiag_table_kernel, dim3(1), dim3(256), 0, stream, seed, N, q, l, table);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_cynical_t(const void *A, int64_t m, int64_t n, int64_t lda, uint64_t seed, int32_t loops,
                                   const CAConfig &cfg_k, const CAConfig &cfg_r, const TeamWs &ws, int team,
                                   size_t dyn_bytes, int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info,
                                   hipStream_t stream) {
    auto kern = ca_cynical_kernel<T>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes);
    (void)e;
    if (team > 1) {
        const int64_t words = (int64_t)2 * team * kSlotWords;
        hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)std::min<int64_t>(256, (words + 255) / 256)), dim3(256), 0,
                           stream, ws.xw, words);
    }
    const T *Ap = static_cast<const T *>(A);
    CAConfig ck = cfg_k, cr = cfg_r;
    TeamWs w = ws;
    void *args[] = {(void *)&Ap, (void *)&m,  (void *)&n,     (void *)&lda,   (void *)&seed, (void *)&loops,
                    (void *)&ck, (void *)&cr, (void *)&w,     (void *)&I_out, (void *)&J_out, (void *)&U_out,
                    (void *)&info};
    return hipLaunchCooperativeKernel((const void *)kern, dim3(team), dim3(kBlock), args, (unsigned)dyn_bytes, stream);
}

hipError_t launch_cynical(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, uint64_t seed, int32_t loops,
                          const CAConfig &cfg_k, const CAConfig &cfg_r, const TeamWs &ws, int team, size_t dyn_bytes,
                          int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream) {
    switch (dtype) {
    case LRA_F64:
        return launch_cynical_t<double>(A, m, n, lda, seed, loops, cfg_k, cfg_r, ws, team, dyn_bytes, I_out, J_out,
                                        U_out, info, stream);
    case LRA_F32:
        return launch_cynical_t<float>(A, m, n, lda, seed, loops, cfg_k, cfg_r, ws, team, dyn_bytes, I_out, J_out,
                                       U_out, info, stream);
    default:
        return launch_cynical_t<uint16_t>(A, m, n, lda, seed, loops, cfg_k, cfg_r, ws, team, dyn_bytes, I_out, J_out,
                                          U_out, info, stream);
    }
}

template <typename T>
static hipError_t launch_projective_t(const void *A, int64_t m, int64_t n, int64_t lda, uint64_t seed, int32_t k,
                                      int32_t l, const CAConfig &cfg, const TeamWs &ws, int team, size_t dyn_bytes,
                                      int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info,
                                      hipStream_t stream) {
    auto kern = ca_projective_kernel<T>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes);
    (void)e;
    if (team > 1) {
        const int64_t words = (int64_t)2 * team * kSlotWords;
        hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)std::min<int64_t>(256, (words + 255) / 256)), dim3(256), 0,
                           stream, ws.xw, words);
    }
    const T *Ap = static_cast<const T *>(A);
    CAConfig c = cfg;
    TeamWs w = ws;
    void *args[] = {(void *)&Ap, (void *)&m, (void *)&n,     (void *)&lda,   (void *)&seed,  (void *)&k,
                    (void *)&l,  (void *)&c, (void *)&w,     (void *)&I_out, (void *)&J_out, (void *)&U_out,
                    (void *)&info};
    return hipLaunchCooperativeKernel((const void *)kern, dim3(team), dim3(kBlock), args, (unsigned)dyn_bytes, stream);
}

hipError_t launch_projective(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, uint64_t seed, int32_t k,
                             int32_t l, const CAConfig &cfg, const TeamWs &ws, int team, size_t dyn_bytes,
                             int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream) {
    switch (dtype) {
    case LRA_F64:
        return launch_projective_t<double>(A, m, n, lda, seed, k, l, cfg, ws, team, dyn_bytes, I_out, J_out, U_out,
                                           info, stream);
    case LRA_F32:
        return launch_projective_t<float>(A, m, n, lda, seed, k, l, cfg, ws, team, dyn_bytes, I_out, J_out, U_out,
                                          info, stream);
    default:
        return launch_projective_t<uint16_t>(A, m, n, lda, seed, k, l, cfg, ws, team, dyn_bytes, I_out, J_out, U_out,
                                             info, stream);
    }
}

template <typename T>
static hipError_t launch_uniform_t(const void *base, const BlockDesc *blocks, int64_t count, uint64_t seed, int32_t r,
                                   int32_t k, int32_t l, int grid, size_t dyn_bytes, int64_t *I_out, int64_t *J_out,
                                   double *U_out, lra_info *infos, hipStream_t stream) {
    auto kern = ca_uniform_kernel<T>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes);
    (void)e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), dyn_bytes, stream, static_cast<const T *>(base), blocks, count,
                       seed, r, k, l, I_out, J_out, U_out, infos);
    return hipGetLastError();
}

hipError_t launch_uniform(int dtype, const void *base, const BlockDesc *blocks, int64_t count, uint64_t seed,
                          int32_t r, int32_t k, int32_t l, int grid, size_t dyn_bytes, int64_t *I_out, int64_t *J_out,
                          double *U_out, lra_info *infos, hipStream_t stream) {
    switch (dtype) {
    case LRA_F64:
        return launch_uniform_t<double>(base, blocks, count, seed, r, k, l, grid, dyn_bytes, I_out, J_out, U_out,
                                        infos, stream);
    case LRA_F32:
        return launch_uniform_t<float>(base, blocks, count, seed, r, k, l, grid, dyn_bytes, I_out, J_out, U_out, infos,
                                       stream);
    default:
        return launch_uniform_t<uint16_t>(base, blocks, count, seed, r, k, l, grid, dyn_bytes, I_out, J_out, U_out,
                                          infos, stream);
    }
}

int uniform_occupancy(int dtype, size_t dyn_bytes) {
    int blocks = 0;
    hipError_t e;
    if (dtype == LRA_F64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_uniform_kernel<double>, kBlock, dyn_bytes);
    else if (dtype == LRA_F32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_uniform_kernel<float>, kBlock, dyn_bytes);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_uniform_kernel<uint16_t>, kBlock, dyn_bytes);
    if (e != hipSuccess) return 0;
    return blocks;
}

template <typename T>
static hipError_t launch_leverage_t(const void *A, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I0,
                                   const int64_t *J0, int k, int l, uint64_t seed, double *ws, int32_t *flags,
                                   int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream) {
    const T *Ap = static_cast<const T *>(A);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, stream, reinterpret_cast<unsigned *>(flags), 2);
    const int64_t items = n + m;
    const int64_t gather_blocks = std::min<int64_t>((items * r + 255) / 256, 4096);
    hipLaunchKernelGGL(lev_gather_kernel<T>, dim3((unsigned)gather_blocks), dim3(256), 0, stream, Ap, m, n, lda, r,
                       I0, J0, ws, flags);
    const int entries = r * (r + 1);
    hipLaunchKernelGGL(lev_gram_kernel, dim3((unsigned)((entries + 63) / 64)), dim3(64), 0, stream, m, n, r, ws);
    hipLaunchKernelGGL(lev_chol_kernel, dim3(2), dim3(kBlock), 0, stream, r, ws, flags);
    hipLaunchKernelGGL(lev_score_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, stream, m, n, r, ws);
    hipLaunchKernelGGL(lev_cdf_kernel, dim3(2), dim3(256), 0, stream, m, n, ws);
    const size_t dyn = std::max(k, l) <= kRMax ? sizeof(double) * (size_t)std::min(k, l) * (size_t)(k + l) : 0;
    auto kern = lev_pick_kernel<T>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    (void)e;
    hipLaunchKernelGGL(kern, dim3(1), dim3(kBlock), dyn, stream, Ap, m, n, lda, r, k, l, seed, ws,
                       static_cast<const int32_t *>(flags), I_out, J_out, U_out, info);
    return hipGetLastError();
}

hipError_t launch_leverage(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I0,
                           const int64_t *J0, int k, int l, uint64_t seed, double *ws, int32_t *flags,
                           int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream) {
    switch (dtype) {
    case LRA_F64:
        return launch_leverage_t<double>(A, m, n, lda, r, I0, J0, k, l, seed, ws, flags, I_out, J_out, U_out, info,
                                         stream);
    case LRA_F32:
        return launch_leverage_t<float>(A, m, n, lda, r, I0, J0, k, l, seed, ws, flags, I_out, J_out, U_out, info,
                                        stream);
    default:
        return launch_leverage_t<uint16_t>(A, m, n, lda, r, I0, J0, k, l, seed, ws, flags, I_out, J_out, U_out, info,
                                           stream);
    }
}

size_t leverage_scratch_bytes(int64_t m, int64_t n, int r) {
    return sizeof(double) * ((size_t)4 * kRMax * kRMax + (size_t)(2 + r) * (size_t)(n + m) + 2 * (size_t)kSMax * kSMax);
}

template <typename T>
static hipError_t launch_batched_t(const void *base, const BlockDesc *blocks, const int32_t *order, int64_t count,
                                   uint64_t seed, const CAConfig &cfg, unsigned *queue, int grid, size_t dyn_bytes,
                                   int64_t *I_out, int64_t *J_out, double *U_out, lra_info *infos,
                                   hipStream_t stream) {
    auto kern = cfg.margins ? ca_batched_kernel<T, true> : ca_batched_kernel<T, false>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes);
    (void)e;
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, stream, queue, 1);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), dyn_bytes, stream, static_cast<const T *>(base), blocks, order,
                       count, seed, cfg, queue, I_out, J_out, U_out, infos);
    return hipGetLastError();
}

hipError_t launch_batched(int dtype, const void *base, const BlockDesc *blocks, const int32_t *order, int64_t count,
                          uint64_t seed, const CAConfig &cfg, unsigned *queue, int grid, size_t dyn_bytes,
                          int64_t *I_out, int64_t *J_out, double *U_out, lra_info *infos, hipStream_t stream) {
    switch (dtype) {
    case LRA_F64:
        return launch_batched_t<double>(base, blocks, order, count, seed, cfg, queue, grid, dyn_bytes, I_out, J_out,
                                        U_out, infos, stream);
    case LRA_F32:
        return launch_batched_t<float>(base, blocks, order, count, seed, cfg, queue, grid, dyn_bytes, I_out, J_out,
                                       U_out, infos, stream);
    default:
        return launch_batched_t<uint16_t>(base, blocks, order, count, seed, cfg, queue, grid, dyn_bytes, I_out, J_out,
                                          U_out, infos, stream);
    }
}

hipError_t launch_points(const double *pts, const PtsDesc *blocks, const int32_t *order, int64_t count,
                         uint64_t seed, const CAConfig &cfg, unsigned *queue, int grid, size_t dyn_bytes,
                         int64_t *I_out, int64_t *J_out, double *U_out, lra_info *infos, hipStream_t stream) {
    auto kern = cfg.margins ? ca_points_kernel<true> : ca_points_kernel<false>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes);
    (void)e;
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, stream, queue, 1);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), dyn_bytes, stream, pts, blocks, order, count, seed, cfg, queue,
                       I_out, J_out, U_out, infos);
    return hipGetLastError();
}

int points_occupancy(size_t dyn_bytes) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_points_kernel<true>, kBlock, dyn_bytes) != hipSuccess)
        return 0;
    return blocks;
}

int batched_occupancy(int dtype, size_t dyn_bytes) {
    int blocks = 0;
    hipError_t e;
    if (dtype == LRA_F64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_batched_kernel<double, true>, kBlock, dyn_bytes);
    else if (dtype == LRA_F32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_batched_kernel<float, true>, kBlock, dyn_bytes);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_batched_kernel<uint16_t, true>, kBlock, dyn_bytes);
    if (e != hipSuccess) return 0;
    return blocks;
}

// Static LDS of the C-A kernels as compiled (the Smem block plus the
// function-level shared variables of the nucleus and inverse), the largest
// over the element types and entry sources; queried once.
size_t static_lds_bytes() {
    static size_t bytes = 0;
    if (bytes == 0) {
        const void *fns[] = {(const void *)ca_team_kernel<double, false, false>,
                             (const void *)ca_team_kernel<float, false, false>,
                             (const void *)ca_team_kernel<uint16_t, false, false>,
                             (const void *)ca_team_kernel<double, false, true>,
                             (const void *)ca_team_kernel<float, false, true>,
                             (const void *)ca_team_kernel<uint16_t, false, true>,
                             (const void *)ca_team_kernel<double, true, false>,
                             (const void *)ca_team_kernel<float, true, false>,
                             (const void *)ca_team_kernel<uint16_t, true, false>,
                             (const void *)ca_team_kernel<double, true, true>,
                             (const void *)ca_team_kernel<float, true, true>,
                             (const void *)ca_team_kernel<uint16_t, true, true>,
                             (const void *)ca_batched_kernel<double, false>,
                             (const void *)ca_batched_kernel<float, false>,
                             (const void *)ca_batched_kernel<uint16_t, false>,
                             (const void *)ca_batched_kernel<double, true>,
                             (const void *)ca_batched_kernel<float, true>,
                             (const void *)ca_batched_kernel<uint16_t, true>,
                             (const void *)ca_points_kernel<false>,
                             (const void *)ca_points_kernel<true>,
                             (const void *)ca_cynical_kernel<double>,
                             (const void *)ca_cynical_kernel<float>,
                             (const void *)ca_cynical_kernel<uint16_t>,
                             (const void *)ca_hadamard_kernel<double, false>,
                             (const void *)ca_hadamard_kernel<float, false>,
                             (const void *)ca_hadamard_kernel<uint16_t, false>,
                             (const void *)ca_hadamard_kernel<double, true>,
                             (const void *)ca_hadamard_kernel<float, true>,
                             (const void *)ca_hadamard_kernel<uint16_t, true>,
                             (const void *)ca_projective_kernel<double>,
                             (const void *)ca_projective_kernel<float>,
                             (const void *)ca_projective_kernel<uint16_t>,
                             (const void *)ca_uniform_kernel<double>,
                             (const void *)ca_uniform_kernel<float>,
                             (const void *)ca_uniform_kernel<uint16_t>};
        size_t mx = sizeof(Smem) + sizeof(int) * kRMax;
        for (const void *f : fns) {
            hipFuncAttributes attr;
            if (hipFuncGetAttributes(&attr, f) == hipSuccess && attr.sharedSizeBytes > mx) mx = attr.sharedSizeBytes;
        }
        bytes = mx;
    }
    return bytes;
}

}  // namespace lra

#ifdef LRA_TRACE
// Copy the per-selection publish / poll-done clocks ([kSelTrace][256] each).
extern "C" int lra_trace_sel(uint64_t *pub, uint64_t *done) {
    if (hipMemcpyFromSymbol(pub, HIP_SYMBOL(lra::g_sel_pub), sizeof(uint64_t) * lra::kSelTrace * 256) != hipSuccess)
        return -1;
    if (hipMemcpyFromSymbol(done, HIP_SYMBOL(lra::g_sel_done), sizeof(uint64_t) * lra::kSelTrace * 256) != hipSuccess)
        return -1;
    return lra::kSelTrace;
}

// Copy the trace of the last traced launches out and reset it (tracing builds only).
extern "C" int lra_trace_read(uint64_t *host, int max_events) {
    int n = 0;
    if (hipMemcpyFromSymbol(&n, HIP_SYMBOL(lra::g_trace_n), sizeof(int)) != hipSuccess) return -1;
    if (n > max_events) n = max_events;
    if (n > 0 && hipMemcpyFromSymbol(host, HIP_SYMBOL(lra::g_trace), sizeof(uint64_t) * 2 * n) != hipSuccess) return -1;
    int z = 0;
    if (hipMemcpyToSymbol(HIP_SYMBOL(lra::g_trace_n), &z, sizeof(int)) != hipSuccess) return -1;
    return n;
}
#endif
