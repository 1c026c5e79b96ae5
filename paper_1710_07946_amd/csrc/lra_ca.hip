// lra_ca.hip -- cross-approximation (C-A) CUR on gfx950.
//
// One LRA runs inside one persistent launch.  A "team" of workgroups
// cooperates on it: every panel (the m x r column panel W[:, J], the n x r
// transposed row panel W[I, :]^T, the items x l abridged-SRHT sketch) is
// split by items (rows or columns of W) across the team, each workgroup
// keeping its slice in LDS as FP64, column-major (slot-major), so that one
// thread owns one item and LDS accesses are conflict-free.  Every pivot or
// swap decision is an argmax over the whole panel: each workgroup reduces its
// slice with wavefront shuffles, publishes (value, item, slot) and the
// candidate's row to a small exchange buffer, and after one grid barrier every
// workgroup reduces the team's candidates redundantly, so all of them apply
// the same rank-one update to their own slice.  A team of one workgroup
// (small matrices, and every block of a batch) skips the barrier entirely.
//
// The arithmetic follows the paper's steps (Appendix D, Algorithms alggos
// and algdomin; Appendix B for the sketch; Algorithm alg1tor for the greedy
// QRP; Algorithm algcnnncl for the nucleus); this file is compiled without
// floating-point contraction and every per-item sum runs in a fixed order,
// so results do not depend on the team size.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lra_internal.h"

namespace lra {

constexpr int kWave = 64;
constexpr int kNWave = kBlock / kWave;

// ---------------------------------------------------------------- elements
template <typename T> struct Elem;
template <> struct Elem<double> {
    static __device__ __forceinline__ double load(const double *p, int64_t o) { return p[o]; }
};
template <> struct Elem<float> {
    static __device__ __forceinline__ double load(const float *p, int64_t o) { return (double)p[o]; }
};
template <> struct Elem<uint16_t> {
    static __device__ __forceinline__ double load(const uint16_t *p, int64_t o) {
        return (double)__uint_as_float(((uint32_t)p[o]) << 16);
    }
};

// ---------------------------------------------------------------- SplitMix64
// Counter form of SplitMix64 (Steele, Lea, Flood 2014): output i of the
// sequence whose state starts at `seed` is mix(seed + (i+1) gamma); stream s
// offsets the counter by s * 2^40.
__device__ __forceinline__ uint64_t sm64(uint64_t seed, uint64_t stream, uint64_t i) {
    uint64_t z = seed + 0x9e3779b97f4a7c15ULL * ((stream << 40) + i + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double rademacher(uint64_t seed, int64_t c) {
    return (sm64(seed, 1, (uint64_t)c) >> 63) ? -1.0 : 1.0;
}

// k <= 256 distinct draws from [0, n) in draw order (rejection of the top
// 2^64 mod n words, duplicates skipped).  Run by all 64 lanes of one wave:
// 64 counters are hashed at once, then accepted in counter order.
__device__ void draw_distinct_wave(uint64_t seed, uint64_t stream, int64_t n, int k, int64_t *out) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t un = (uint64_t)n;
    const uint64_t rem = (0 - un) % un;
    const uint64_t lim = 0 - rem;
    // list entry q lives in lane q % 64, register q / 64
    int64_t m0 = -1, m1 = -1, m2 = -1, m3 = -1;
    int got = 0;
    uint64_t ctr = 0;
    while (got < k) {
        uint64_t u = sm64(seed, stream, ctr + (uint64_t)lane);
        int ok = !(rem != 0 && u >= lim);
        int64_t v = (int64_t)(u % un);
        for (int t = 0; t < kWave && got < k; t++) {
            int okt = __shfl(ok, t);
            int64_t vt = __shfl(v, t);
            if (!okt) continue;
            bool dup = (lane < got && m0 == vt) || (lane + 64 < got && m1 == vt) ||
                       (lane + 128 < got && m2 == vt) || (lane + 192 < got && m3 == vt);
            if (__any(dup)) continue;
            if (lane == (got & (kWave - 1))) {
                const int q = got >> 6;
                m0 = q == 0 ? vt : m0;
                m1 = q == 1 ? vt : m1;
                m2 = q == 2 ? vt : m2;
                m3 = q == 3 ? vt : m3;
            }
            got++;
        }
        ctr += kWave;
    }
    if (lane < k) out[lane] = m0;
    if (lane + 64 < k) out[lane + 64] = m1;
    if (lane + 128 < k) out[lane + 128] = m2;
    if (lane + 192 < k) out[lane + 192] = m3;
}

// ---------------------------------------------------------------- argmax
struct Best {
    double v;      // |value| compared; -1 when there is no candidate
    int64_t item;  // global item id (row or column of W)
    int32_t slot;  // basis slot (swap search) or 0
    int32_t aux;   // owner workgroup (team reduction) or local item index
};

__device__ __forceinline__ bool better(double v1, int64_t i1, int s1, double v2, int64_t i2, int s2) {
    return v1 > v2 || (v1 == v2 && (i1 < i2 || (i1 == i2 && s1 < s2)));
}

__device__ __forceinline__ Best none() { return Best{-1.0, INT64_MAX, 0x7fffffff, -1}; }

__device__ __forceinline__ void consider(Best &b, double v, int64_t item, int slot, int aux) {
    if (better(v, item, slot, b.v, b.item, b.slot)) b = Best{v, item, slot, aux};
}

__device__ __forceinline__ Best wave_reduce(Best b) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        Best o;
        o.v = __shfl_xor(b.v, off);
        o.item = __shfl_xor(b.item, off);
        o.slot = __shfl_xor(b.slot, off);
        o.aux = __shfl_xor(b.aux, off);
        if (better(o.v, o.item, o.slot, b.v, b.item, b.slot)) b = o;
    }
    return b;
}

// ---------------------------------------------------------------- LDS state
struct Smem {
    int64_t Iset[kRMax], Jset[kRMax], Iprev[kRMax], Jprev[kRMax];
    int64_t slot_item[kRMax];
    int64_t samples[kLMax];
    double L11[kRMax * (kRMax - 1) / 2];
    double wrow[kLMax];
    Best red[kNWave];
    int32_t red_flag[kNWave];
    Best win;
    int32_t win_flag;
    int32_t status;
    int32_t rank_found;
    int32_t job;
    double vtv;
    double logdet;
};

struct Team {
    int rank, size;
    unsigned epoch;
    unsigned *bar;
    XchHeader *hdr;
    double *rows;  // [2][size][kLMax]
};

// Grid-wide barrier for a cooperative team: every workgroup adds one to a
// counter and waits until it reaches (epoch + 1) * size.  The release fence
// publishes this workgroup's global writes (exchange buffer) before the
// arrival; the acquire fence after the wait makes the others' writes visible.
__device__ void team_barrier(Team &tm) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned target = (tm.epoch + 1u) * (unsigned)tm.size;
        __hip_atomic_fetch_add(tm.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (__hip_atomic_load(tm.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target)
            __builtin_amdgcn_s_sleep(1);
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    tm.epoch++;
}

// Workgroup reduction of per-thread candidates; the result lands in sm.win
// (for a team of one) or is the workgroup's team candidate.
__device__ Best block_reduce(Best b, int flag, Smem &sm, int32_t *flag_out) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    b = wave_reduce(b);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) flag |= __shfl_xor(flag, off);
    __syncthreads();
    if (lane == 0) {
        sm.red[w] = b;
        sm.red_flag[w] = flag;
    }
    __syncthreads();
    Best r = sm.red[0];
    int f = sm.red_flag[0];
#pragma unroll
    for (int q = 1; q < kNWave; q++) {
        Best o = sm.red[q];
        if (better(o.v, o.item, o.slot, r.v, r.item, r.slot)) r = o;
        f |= sm.red_flag[q];
    }
    *flag_out = f;
    return r;
}

// Team-wide selection: reduce the per-thread candidates to the team's winner
// and copy the winner's row (width values of its panel column) to sm.wrow.
// b.aux holds the local item index of the candidate.  All threads must call.
__device__ void team_select(Team &tm, Smem &sm, Best b, int flag, const double *panel, int ipw, int width) {
    int32_t f;
    Best local = block_reduce(b, flag, sm, &f);
    if (tm.size == 1) {
        if (threadIdx.x < width) sm.wrow[threadIdx.x] = local.v >= 0 ? panel[threadIdx.x * ipw + local.aux] : 0.0;
        if (threadIdx.x == 0) {
            sm.win = local;
            sm.win.aux = 0;
            sm.win_flag = f;
        }
        __syncthreads();
        return;
    }
    const int par = tm.epoch & 1;
    XchHeader *H = tm.hdr + (size_t)par * tm.size;
    double *Rw = tm.rows + (size_t)par * tm.size * kLMax;
    if (threadIdx.x == 0) {
        XchHeader h;
        h.val = local.v;
        h.item = local.item;
        h.slot = local.slot;
        h.flags = f;
        H[tm.rank] = h;
    }
    if (threadIdx.x < width)
        Rw[(size_t)tm.rank * kLMax + threadIdx.x] = local.v >= 0 ? panel[threadIdx.x * ipw + local.aux] : 0.0;
    team_barrier(tm);
    Best c = none();
    int cf = 0;
    for (int g = threadIdx.x; g < tm.size; g += kBlock) {
        XchHeader h = H[g];
        consider(c, h.val, h.item, h.slot, g);
        cf |= h.flags;
    }
    Best w = block_reduce(c, cf, sm, &f);
    if (threadIdx.x < width) sm.wrow[threadIdx.x] = Rw[(size_t)w.aux * kLMax + threadIdx.x];
    if (threadIdx.x == 0) {
        sm.win = w;
        sm.win_flag = f;
    }
    __syncthreads();
}

__device__ void sort_small(int64_t *a, int r) {
    for (int i = 1; i < r; i++) {
        int64_t x = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > x) {
            a[j + 1] = a[j];
            j--;
        }
        a[j + 1] = x;
    }
}

struct Geo {   // item partition of one panel across the team
    int64_t items, base;
    int ipw, cnt;
};

__device__ __forceinline__ Geo geo(const Team &tm, int64_t items) {
    Geo g;
    g.items = items;
    g.ipw = (int)((items + tm.size - 1) / tm.size);
    g.base = (int64_t)tm.rank * g.ipw;
    int64_t c = items - g.base;
    g.cnt = (int)(c < 0 ? 0 : (c > g.ipw ? g.ipw : c));
    return g;
}

// ---------------------------------------------------------------- maxvol
// Dominant r x r submatrix of the tall panel held in `panel` (slot-major,
// stride g.ipw): pivoted LU start (Algorithm alggos, stages 1-2), then the
// swaps of Algorithm algdomin with the rank-one update of B.  flags[li] is 0
// for a candidate item, slot+1 for a basis item.  On return sm.slot_item
// holds the basis in slot order.  `bad` flags a non-finite entry read.
__device__ void maxvol(Team &tm, Smem &sm, double *panel, uint8_t *flags, const Geo &g, int r, double delta,
                       int max_swaps, int bad, int32_t &swaps_total, int32_t &converged) {
    const int tid = threadIdx.x;
    const int ipw = g.ipw;
    // ---- pivoted LU: r steps
    for (int k = 0; k < r; k++) {
        Best b = none();
        for (int li = tid; li < g.cnt; li += kBlock)
            if (!flags[li]) consider(b, fabs(panel[k * ipw + li]), g.base + li, 0, li);
        team_select(tm, sm, b, k == 0 ? bad : 0, panel, ipw, r);
        if (sm.win_flag) {
            if (tid == 0) sm.status = LRA_EINVAL;
            __syncthreads();
            return;
        }
        if (!(sm.win.v > 0.0)) {
            if (tid == 0) {
                sm.status = LRA_ESINGULAR;
                sm.rank_found = k;
            }
            __syncthreads();
            return;
        }
        const int64_t wit = sm.win.item;
        if (tid == 0) {
            sm.slot_item[k] = wit;
            if (wit >= g.base && wit < g.base + g.cnt) flags[wit - g.base] = (uint8_t)(k + 1);
        }
        if (tid < k) sm.L11[k * (k - 1) / 2 + tid] = sm.wrow[tid];
        __syncthreads();
        const double pk = sm.wrow[k];
        for (int li = tid; li < g.cnt; li += kBlock) {
            if (flags[li]) continue;
            double l = panel[k * ipw + li] / pk;
            panel[k * ipw + li] = l;
            for (int j = k + 1; j < r; j++) panel[j * ipw + li] -= l * sm.wrow[j];
        }
        __syncthreads();
    }
    // ---- B = L21 L11^{-1} for candidates, unit rows for the basis
    for (int li = tid; li < g.cnt; li += kBlock) {
        const int fl = flags[li];
        if (fl) {
            for (int j = 0; j < r; j++) panel[j * ipw + li] = (j == fl - 1) ? 1.0 : 0.0;
            continue;
        }
        for (int j = r - 1; j >= 0; j--) {
            double s = panel[j * ipw + li];
            for (int kk = j + 1; kk < r; kk++) s -= panel[kk * ipw + li] * sm.L11[kk * (kk - 1) / 2 + j];
            panel[j * ipw + li] = s;
        }
    }
    __syncthreads();
    // ---- swaps
    const double thr = 1.0 + delta;
    int swaps = 0;
    for (;;) {
        Best b = none();
        for (int li = tid; li < g.cnt; li += kBlock) {
            if (flags[li]) continue;
            const int64_t it = g.base + li;
            for (int j = 0; j < r; j++) consider(b, fabs(panel[j * ipw + li]), it, j, li);
        }
        team_select(tm, sm, b, 0, panel, ipw, r);
        const double v = sm.win.v;
        if (v < 0.0 || v <= thr) break;         // no candidate left, or dominant
        if (swaps >= max_swaps) {
            converged = 0;
            break;
        }
        const int js = sm.win.slot;
        const int64_t wit = sm.win.item;
        const int64_t old = sm.slot_item[js];
        const double pv = sm.wrow[js];
        __syncthreads();
        if (tid == 0) sm.wrow[js] -= 1.0;  // B[i,:] - e_j^T
        __syncthreads();
        for (int li = tid; li < g.cnt; li += kBlock) {
            const int fl = flags[li];
            if (g.base + li == wit) continue;
            if (fl != 0 && fl != js + 1) continue;  // other basis rows: B[i][js] = 0
            const double f = panel[js * ipw + li] / pv;
            if (f == 0.0) continue;
            for (int j = 0; j < r; j++) panel[j * ipw + li] -= f * sm.wrow[j];
        }
        __syncthreads();
        if (wit >= g.base && wit < g.base + g.cnt) {
            const int lw = (int)(wit - g.base);
            if (tid < r) panel[tid * ipw + lw] = (tid == js) ? 1.0 : 0.0;
            if (tid == 0) flags[lw] = (uint8_t)(js + 1);
        }
        if (tid == 0) {
            if (old >= g.base && old < g.base + g.cnt) flags[old - g.base] = 0;
            sm.slot_item[js] = wit;
        }
        swaps++;
        __syncthreads();
    }
    swaps_total += swaps;
}

// One C-A step.  col = true: panel = W[:, set_in] (items = rows of W);
// col = false: panel = W[set_in, :]^T (items = columns).  set_out receives
// the new sorted set.
template <typename T>
__device__ void ca_step(Team &tm, Smem &sm, double *panel, uint8_t *flags, const T *A, int64_t m, int64_t n,
                        int64_t lda, int r, bool col, const int64_t *set_in, int64_t *set_out, const CAConfig &cfg,
                        int32_t &swaps_total, int32_t &converged) {
    const Geo g = geo(tm, col ? m : n);
    int bad = 0;
    const int tot = g.cnt * r;
    for (int e = threadIdx.x; e < tot; e += kBlock) {
        const int li = e % g.cnt, j = e / g.cnt;
        const int64_t it = g.base + li;
        const int64_t off = col ? it * lda + set_in[j] : set_in[j] * lda + it;
        const double v = Elem<T>::load(A, off);
        if (!isfinite(v)) bad = 1;
        panel[j * g.ipw + li] = v;
    }
    for (int li = threadIdx.x; li < g.cnt; li += kBlock) flags[li] = 0;
    __syncthreads();
    maxvol(tm, sm, panel, flags, g, r, cfg.delta, cfg.max_swaps, bad, swaps_total, converged);
    if (threadIdx.x == 0 && sm.status == LRA_OK) {
        for (int j = 0; j < r; j++) set_out[j] = sm.slot_item[j];
        sort_small(set_out, r);
    }
    __syncthreads();
}

// Abridged SRHT sketch of the team's items (Appendix B): for sampled column
// t = b s + e of D H_{N,d}, Y[item][q] = sqrt(s/l) sum_a W[item][a s + e]
// D[a s + e] (-1)^{popcount(a & b)} (post-multiplication; pre-multiplication
// swaps the roles of rows and columns).  Then greedy Householder QRP over the
// items picks r of them (Algorithm alg1tor).  The chosen items land in out.
template <typename T>
__device__ void sketch_qrp(Team &tm, Smem &sm, double *panel, uint8_t *flags, const T *A, int64_t m, int64_t n,
                           int64_t lda, int r, int side, int d, int l, uint64_t seed, int64_t *out) {
    const int tid = threadIdx.x;
    const int64_t dim = side ? m : n;
    const Geo g = geo(tm, side ? n : m);
    const int64_t q2 = (int64_t)1 << d;
    const int64_t s = (dim + q2 - 1) / q2;
    const int64_t N = q2 * s;
    if (tid < kWave) draw_distinct_wave(seed, 2, N, l, sm.samples);
    __syncthreads();
    const double scale = sqrt((double)s / (double)l);
    int bad = 0;
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
            const double w = side ? Elem<T>::load(A, c * lda + it) : Elem<T>::load(A, it * lda + c);
            acc += w * rademacher(seed, c) * h;
        }
        const double y = scale * acc;
        if (!isfinite(y)) bad = 1;
        panel[q * g.ipw + li] = y;
    }
    for (int li = tid; li < g.cnt; li += kBlock) flags[li] = 0;
    __syncthreads();
    const int ipw = g.ipw;
    for (int gg = 0; gg < r; gg++) {
        Best b = none();
        for (int li = tid; li < g.cnt; li += kBlock) {
            if (flags[li]) continue;
            double acc = 0.0;
            for (int c = gg; c < l; c++) {
                const double z = panel[c * ipw + li];
                acc += z * z;
            }
            consider(b, acc, g.base + li, 0, li);
        }
        team_select(tm, sm, b, gg == 0 ? bad : 0, panel, ipw, l);
        if (sm.win_flag) {
            if (tid == 0) sm.status = LRA_EINVAL;
            __syncthreads();
            return;
        }
        if (!(sm.win.v > 0.0)) {
            if (tid == 0) {
                sm.status = LRA_ESINGULAR;
                sm.rank_found = gg;
            }
            __syncthreads();
            return;
        }
        const int64_t wit = sm.win.item;
        if (tid == 0) {
            out[gg] = wit;
            if (wit >= g.base && wit < g.base + g.cnt) flags[wit - g.base] = 1;
            const double nx = sqrt(sm.win.v);
            const double x0 = sm.wrow[gg];
            const double alpha = (x0 >= 0.0) ? -nx : nx;
            sm.wrow[gg] = x0 - alpha;
            double vtv = 0.0;
            for (int c = gg; c < l; c++) vtv += sm.wrow[c] * sm.wrow[c];
            sm.vtv = vtv;
        }
        __syncthreads();
        const double vtv = sm.vtv;
        if (vtv > 0.0) {
            for (int li = tid; li < g.cnt; li += kBlock) {
                if (flags[li]) continue;
                double acc = 0.0;
                for (int c = gg; c < l; c++) acc += sm.wrow[c] * panel[c * ipw + li];
                const double f = 2.0 * acc / vtv;
                for (int c = gg; c < l; c++) panel[c * ipw + li] -= f * sm.wrow[c];
            }
        }
        __syncthreads();
    }
}

// Nucleus U = G^{-1}, G = W[I, J] (I, J sorted), by LU with partial pivoting
// (ties to the lowest row) and r column solves, then `refine` steps of
// X <- X + X (I - G X) (Algorithm algcnnncl with k = l = r).  One workgroup;
// `ws` holds 4 r^2 doubles.  Writes U (row-major, J-order x I-order).
template <typename T>
__device__ void nucleus(Smem &sm, double *ws, const T *A, int64_t lda, int r, int refine, double *U_out) {
    const int tid = threadIdx.x;
    double *G = ws, *LU = ws + r * r, *X = ws + 2 * r * r, *X2 = ws + 3 * r * r;
    __shared__ int p[kRMax];
    for (int e = tid; e < r * r; e += kBlock) {
        const int a = e / r, b = e % r;
        const double v = Elem<T>::load(A, sm.Iset[a] * lda + sm.Jset[b]);
        G[e] = v;
        LU[e] = v;
    }
    if (tid < r) p[tid] = tid;
    if (tid == 0) sm.logdet = 0.0;
    __syncthreads();
    for (int k = 0; k < r; k++) {
        if (tid == 0) {
            int best = k;
            double bv = fabs(LU[p[k] * r + k]);
            for (int i = k + 1; i < r; i++) {
                const double a = fabs(LU[p[i] * r + k]);
                if (a > bv || (a == bv && p[i] < p[best])) {
                    bv = a;
                    best = i;
                }
            }
            if (bv == 0.0) {
                sm.status = LRA_ESINGULAR;
                sm.rank_found = r - 1;
            } else {
                const int t = p[k];
                p[k] = p[best];
                p[best] = t;
                sm.logdet += log(bv);
            }
        }
        __syncthreads();
        if (sm.status != LRA_OK) return;
        const int pk = p[k];
        const double piv = LU[pk * r + k];
        for (int i = k + 1 + tid; i < r; i += kBlock) {
            const int pi = p[i];
            const double l = LU[pi * r + k] / piv;
            LU[pi * r + k] = l;
            for (int j = k + 1; j < r; j++) LU[pi * r + j] -= l * LU[pk * r + j];
        }
        __syncthreads();
    }
    // column c of G^{-1}: L y = P e_c, U x = y (stored in column c of X)
    for (int c = tid; c < r; c += kBlock) {
        for (int i = 0; i < r; i++) {
            const int pi = p[i];
            double s = (pi == c) ? 1.0 : 0.0;
            for (int j = 0; j < i; j++) s -= LU[pi * r + j] * X[j * r + c];
            X[i * r + c] = s;
        }
        for (int i = r - 1; i >= 0; i--) {
            const int pi = p[i];
            double s = X[i * r + c];
            for (int j = i + 1; j < r; j++) s -= LU[pi * r + j] * X[j * r + c];
            X[i * r + c] = s / LU[pi * r + i];
        }
    }
    __syncthreads();
    for (int it = 0; it < refine; it++) {
        double *Tm = LU;  // T = I - G X
        for (int e = tid; e < r * r; e += kBlock) {
            const int i = e / r, j = e % r;
            double s = (i == j) ? 1.0 : 0.0;
            for (int q = 0; q < r; q++) s -= G[i * r + q] * X[q * r + j];
            Tm[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < r * r; e += kBlock) {
            const int i = e / r, j = e % r;
            double s = X[e];
            for (int q = 0; q < r; q++) s += X[i * r + q] * Tm[q * r + j];
            X2[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < r * r; e += kBlock) X[e] = X2[e];
        __syncthreads();
    }
    for (int e = tid; e < r * r; e += kBlock) U_out[e] = X[e];
}

// The whole C-A path for one matrix, executed by every workgroup of a team.
template <typename T>
__device__ void ca_solve(Team &tm, Smem &sm, double *dyn, uint8_t *flags, const T *A, int64_t m, int64_t n,
                         int64_t lda, uint64_t seed, const CAConfig &cfg, int64_t *I_out, int64_t *J_out,
                         double *U_out, lra_info *info) {
    const int tid = threadIdx.x;
    const int r = cfg.r;
    int32_t swaps_total = 0, converged = 1, sweeps_run = 0;
    if (tid == 0) {
        sm.status = LRA_OK;
        sm.rank_found = r;
    }
    __syncthreads();
    // ---- start set
    if (cfg.pre == LRA_PRE_ASRHT) {
        const int side = (m > n) ? 1 : 0;
        sketch_qrp<T>(tm, sm, dyn, flags, A, m, n, lda, r, side, cfg.ah_depth, cfg.ah_samples, seed,
                      side ? sm.Jset : sm.Iset);
        if (sm.status != LRA_OK) goto finish;
        if (tid == 0) sort_small(side ? sm.Jset : sm.Iset, r);
        __syncthreads();
        if (!side) {
            ca_step<T>(tm, sm, dyn, flags, A, m, n, lda, r, false, sm.Iset, sm.Jset, cfg, swaps_total, converged);
            if (sm.status != LRA_OK) goto finish;
        }
    } else if (cfg.init_cols) {
        if (tid < r) sm.Jset[tid] = cfg.init_cols[tid];
        __syncthreads();
        if (tid == 0) sort_small(sm.Jset, r);
        __syncthreads();
    } else {
        if (tid < kWave) draw_distinct_wave(seed, 0, n, r, sm.Jset);
        __syncthreads();
        if (tid == 0) sort_small(sm.Jset, r);
        __syncthreads();
    }
    // ---- sweeps
    for (int s = 0; s < cfg.sweeps; s++) {
        ca_step<T>(tm, sm, dyn, flags, A, m, n, lda, r, true, sm.Jset, sm.Iset, cfg, swaps_total, converged);
        if (sm.status != LRA_OK) goto finish;
        ca_step<T>(tm, sm, dyn, flags, A, m, n, lda, r, false, sm.Iset, sm.Jset, cfg, swaps_total, converged);
        if (sm.status != LRA_OK) goto finish;
        sweeps_run = s + 1;
        bool same = s > 0;
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
    if (tm.rank == 0) nucleus<T>(sm, dyn, A, lda, r, cfg.refine_steps, U_out);
finish:
    __syncthreads();
    if (tm.rank != 0) return;
    const int st = sm.status;
    if (tid < r) {
        I_out[tid] = st == LRA_OK ? sm.Iset[tid] : -1;
        J_out[tid] = st == LRA_OK ? sm.Jset[tid] : -1;
    }
    if (st != LRA_OK)
        for (int e = tid; e < r * r; e += kBlock) U_out[e] = __builtin_nan("");
    if (tid == 0 && info) {
        lra_info inf;
        inf.status = st;
        inf.sweeps_run = sweeps_run;
        inf.swaps_total = swaps_total;
        inf.converged = (st == LRA_OK) ? converged : 0;
        inf.rank_found = sm.rank_found;
        inf.team_size = tm.size;
        inf.det_log_abs = st == LRA_OK ? sm.logdet : 0.0;
        *info = inf;
    }
}

// ---------------------------------------------------------------- kernels
template <typename T>
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
    tm.bar = ws.bar;
    tm.hdr = ws.hdr;
    tm.rows = ws.rows;
    ca_solve<T>(tm, sm, dyn, flags, A, m, n, lda, seed, cfg, I_out, J_out, U_out, info);
}

template <typename T>
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
    tm.bar = nullptr;
    tm.hdr = nullptr;
    tm.rows = nullptr;
    const int r = cfg.r;
    for (;;) {
        if (threadIdx.x == 0) sm.job = (int32_t)atomicAdd(queue, 1u);
        __syncthreads();
        const int64_t job = sm.job;
        __syncthreads();
        if (job >= count) break;
        const int32_t b = order[job];
        const BlockDesc d = blocks[b];
        ca_solve<T>(tm, sm, dyn, flags, base + d.offset, d.m, d.n, d.lda, seed + (uint64_t)b, cfg,
                    I_out + (int64_t)b * r, J_out + (int64_t)b * r, U_out + (int64_t)b * r * r,
                    infos ? infos + b : nullptr);
        __syncthreads();
    }
}

__global__ void zero_u32_kernel(unsigned *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------- launchers
template <typename T>
static hipError_t launch_team_t(const void *A, int64_t m, int64_t n, int64_t lda, uint64_t seed, const CAConfig &cfg,
                                const TeamWs &ws, int team, size_t dyn_bytes, int64_t *I_out, int64_t *J_out,
                                double *U_out, lra_info *info, hipStream_t stream) {
    auto kern = ca_team_kernel<T>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes);
    (void)e;
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, stream, ws.bar, 1);
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
static hipError_t launch_batched_t(const void *base, const BlockDesc *blocks, const int32_t *order, int64_t count,
                                   uint64_t seed, const CAConfig &cfg, unsigned *queue, int grid, size_t dyn_bytes,
                                   int64_t *I_out, int64_t *J_out, double *U_out, lra_info *infos,
                                   hipStream_t stream) {
    auto kern = ca_batched_kernel<T>;
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

int batched_occupancy(int dtype, size_t dyn_bytes) {
    int blocks = 0;
    hipError_t e;
    if (dtype == LRA_F64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_batched_kernel<double>, kBlock, dyn_bytes);
    else if (dtype == LRA_F32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_batched_kernel<float>, kBlock, dyn_bytes);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_batched_kernel<uint16_t>, kBlock, dyn_bytes);
    if (e != hipSuccess) return 0;
    return blocks;
}

size_t static_lds_bytes() { return sizeof(Smem) + sizeof(int) * kRMax; }

}  // namespace lra
