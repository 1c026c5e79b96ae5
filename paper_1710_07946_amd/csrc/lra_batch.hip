// lra_batch.hip -- batched C-A CUR with the panels held in registers.
//
// A batch is many independent blocks, each solved by the C-A loop of lra_cur
// (random start columns, alternating column and row steps, each a pivoted LU
// start and the swaps of Algorithm algdomin on the gathered panel, the
// fixed-point exit, the nucleus of Algorithm algcnnncl) on one workgroup of
// W wavefronts.  Here the panel of a step never leaves the VGPRs: lane l of
// wavefront w holds items ((p W + w) 64 + l) for p < P, each with all R of
// its slots, so every scan, elimination and rank-one update is register
// arithmetic and a decision costs one wavefront reduction plus, for W > 1,
// one exchange of W partials through LDS.  A small LDS footprint (the sets,
// the L11 factor, the r x r nucleus) lets several workgroups share a CU.
//
// Blocks are binned by their larger dimension; each bin runs as one
// persistent launch of the variant (P, W) chosen for it, blocks taken from a
// device counter, largest first.  The arithmetic, the tie rules and the order
// of every per-entry operation are those of the LDS kernel of lra_ca.hip and
// of the oracle (no floating-point contraction), so both kernels return
// identical index sets and nuclei.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lra_common.h"
#include "lra_device.h"
#include "lra_internal.h"

namespace lra {
namespace {

constexpr int kRegMaxWaves = 8;

// Built with -DLRA_TRACE, workgroup 0 of each launch adds the wall-clock
// ticks of its phases (gathers, LU, B solve, swaps, nucleus) and its counts
// of decisions and blocks to g_regtr, which lra_trace_reg() copies out.
#ifdef LRA_TRACE
__device__ uint64_t g_regtr[16];
#define REG_TIC(v) const uint64_t v = (blockIdx.x == 0 && threadIdx.x == 0) ? wall_clock64() : 0
#define REG_TOC(slot, v) \
    do { if (blockIdx.x == 0 && threadIdx.x == 0) g_regtr[slot] += wall_clock64() - v; } while (0)
#define REG_CNT(slot, n) \
    do { if (blockIdx.x == 0 && threadIdx.x == 0) g_regtr[slot] += (n); } while (0)
#else
#define REG_TIC(v) ((void)0)
#define REG_TOC(slot, v) ((void)0)
#define REG_CNT(slot, n) ((void)0)
#endif

template <int R>
struct RegSmem {
    int64_t Iset[R], Jset[R], Iprev[R], Jprev[R];
    int64_t slot_item[R];
    double L11[R * (R - 1) / 2];
    double wrow[R];
    double nuc[4 * R * R];
    Best red[kRegMaxWaves];
    double red2[kRegMaxWaves];
    int32_t red_flag[kRegMaxWaves];
    double mmin;   // smallest decision margin of the block so far
    int32_t job;
    int32_t status;
    int32_t rank_found;
    int32_t nucleus_rank;
    double logdet;
};

// Item of slot p of this lane: ((p W + w) 64 + lane).
__device__ __forceinline__ int64_t reg_item(int p, int nw) {
    return ((int64_t)(p * nw + (int)(threadIdx.x >> 6)) << 6) + (threadIdx.x & 63);
}

// Every index into a lane's register arrays is a compile-time constant (a
// run-time index would send the arrays to scratch memory): the LU steps are
// unrolled by template recursion, the winner's row reaches LDS from the one
// lane that holds it, and an entry at a run-time slot j is the one-hot sum
// sum_t x_t [t == j], which equals x_j exactly for finite entries (x 1 = x,
// x 0 = 0 and adding zeros leaves x unchanged).
template <int R>
__device__ __forceinline__ double onehot(const double (&x)[R], int j) {
    static_assert((R & (R - 1)) == 0, "a power-of-two width");
    // a binary tree of selects on the bits of j: R - 1 selects
    double v[R];
#pragma unroll
    for (int t = 0; t < R; t++) v[t] = x[t];
#pragma unroll
    for (int h = 1; h < R; h <<= 1) {
        const bool hi = (j & h) != 0;
#pragma unroll
        for (int t = 0; t < R; t += 2 * h) v[t] = hi ? v[t + h] : v[t];
    }
    return v[0];
}

// One decision of the workgroup: the wavefront reductions, then (W > 1) the
// W partials through LDS, so every wavefront holds the same winner, flag and
// runner-up value (v2: the largest candidate value other than the winner's,
// b2 being each thread's own runner-up);
// the winner's panel row (its R entries) lands in sm.wrow.  The row is read
// from LDS where it is used (a uniform value: no registers held for it).
// The order is total (value, then lowest item, then lowest slot), so the
// result does not depend on how the candidates were split.
template <int R, int P, bool M>
__device__ __forceinline__ void reg_select(RegSmem<R> &sm, int nw, Best b, double b2, int flag,
                                           const double (&x)[P][R], Best &win, int &wflag, double &v2) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v2 = -1.0;
    if constexpr (M) b = wave_reduce2(b, b2, v2);
    else b = wave_reduce(b);
    flag = wave_or(flag);
    if (nw > 1) {
        if (lane == 0) {
            sm.red[wv] = b;
            if constexpr (M) sm.red2[wv] = v2;
            sm.red_flag[wv] = flag;
        }
        __syncthreads();
        const Best c = lane < nw ? sm.red[lane] : none();
        const int f = lane < nw ? sm.red_flag[lane] : 0;
        b = reduce8(c);
        if constexpr (M) {
            double t1 = c.v, t2 = lane < nw ? sm.red2[lane] : -1.0;
            top2_8(t1, t2);
            v2 = t2;
        }
        flag = wave_or(f);
    }
    win = b;
    wflag = flag;
    if (!(win.v >= 0.0)) return;  // no candidate: no row
    // the lane holding the winner writes its row (LDS accesses of one
    // wavefront complete in order; W > 1 needs the barrier)
#pragma unroll
    for (int p = 0; p < P; p++)
        if (reg_item(p, nw) == win.item) {
#pragma unroll
            for (int t = 0; t < R; t++) sm.wrow[t] = x[p][t];
        }
    if (nw > 1) __syncthreads();
}

// Step K of the pivoted LU (Algorithm alggos, stages 1-2) on the register
// panel, then the following steps: elimination K-1 is applied to every
// candidate item's slots from K on (fused with the scan), the item with the
// largest |x_K| (lowest item among equals) becomes basis slot K, its row
// gives pivot row K.  Returns false (status set) on a non-finite entry or a
// zero pivot.
template <int R, int P, int K, bool M>
__device__ __forceinline__ bool reg_lu(RegSmem<R> &sm, int nw, double (&x)[P][R], int (&fl)[P], int bad,
                                       double pk) {
    const int tid = threadIdx.x;
    __builtin_amdgcn_sched_barrier(0);  // no step's work moves into another's
    Best b = none();
    double b2 = -1.0;
#pragma unroll
    for (int p = 0; p < P; p++) {
        if (fl[p] != 0) continue;
        if (K > 0) {
            const double l = x[p][K > 0 ? K - 1 : 0] / pk;
#pragma unroll
            for (int t = K; t < R; t++) x[p][t] -= l * sm.wrow[t];
            x[p][K > 0 ? K - 1 : 0] = l;
        }
        if constexpr (M) consider2(b, b2, fabs(x[p][K]), reg_item(p, nw), 0);
        else consider(b, fabs(x[p][K]), reg_item(p, nw), 0);
    }
    Best win;
    int wf;
    double v2;
    reg_select<R, P, M>(sm, nw, b, b2, K == 0 ? bad : 0, x, win, wf, v2);
    if (wf || !(win.v > 0.0)) {
        if (tid == 0) {
            sm.status = wf ? LRA_EINVAL : LRA_ESINGULAR;
            if (!wf) sm.rank_found = K;
        }
        __syncthreads();
        return false;
    }
    if (tid == 0) {
        if constexpr (M) sm.mmin = fmin(sm.mmin, decision_gap(win.v, v2));
        sm.slot_item[K] = win.item;
#pragma unroll
        for (int j = 0; j < K; j++) sm.L11[K * (K - 1) / 2 + j] = sm.wrow[j];
    }
#pragma unroll
    for (int p = 0; p < P; p++)
        if (reg_item(p, nw) == win.item) fl[p] = K + 1;
    if constexpr (K + 1 < R) {
        return reg_lu<R, P, K + 1, M>(sm, nw, x, fl, 0, sm.wrow[K]);
    } else {
        // last multipliers (no trailing columns)
        const double pl = sm.wrow[R - 1];
#pragma unroll
        for (int p = 0; p < P; p++)
            if (fl[p] == 0) x[p][R - 1] /= pl;
        return true;
    }
}

// One C-A step on the register panel.  col = true: items are the rows of the
// m x n block and the panel is W[:, set_in]; col = false: items are the
// columns and the panel is W[set_in, :]^T.  Pivoted LU (elimination applied
// one step late, fused with the next scan), B = L21 L11^{-1} by
// column-oriented back substitution, then the swaps of Algorithm algdomin
// with the rank-one update of B, each fused with the next scan.  Returns
// false (status set) on a non-finite entry or a rank-deficient panel; else
// set_out holds the new sorted set.
template <int R, int P, bool M, class Src>
__device__ __forceinline__ bool reg_step(RegSmem<R> &sm, int nw, const Src &src, int64_t items, bool col,
                                         const int64_t *set_in, int64_t *set_out, double delta, int max_swaps,
                                         int32_t &swaps_total, int32_t &converged) {
    const int tid = threadIdx.x;
    double x[P][R];
    int fl[P];  // 0: candidate item, s + 1: basis item of slot s, -1: no item
    int bad = 0;
    REG_TIC(t_g);
    {
        int64_t sv[R];
#pragma unroll
        for (int t = 0; t < R; t++) sv[t] = set_in[t];
        // every lane loads (a lane past the last item reads item 0 and keeps
        // zeros), so the loads of an item slot issue back to back; one item
        // slot at a time keeps their addresses within the register budget
#pragma unroll
        for (int p = 0; p < P; p++) {
            const int64_t it = reg_item(p, nw);
            const bool ok = it < items;
            const int64_t ic = ok ? it : 0;
            fl[p] = ok ? 0 : -1;
            double v[R];
            if (col) {
#pragma unroll
                for (int t = 0; t < R; t++) v[t] = src(ic, sv[t]);
            } else {
#pragma unroll
                for (int t = 0; t < R; t++) v[t] = src(sv[t], ic);
            }
#pragma unroll
            for (int t = 0; t < R; t++) x[p][t] = ok ? v[t] : 0.0;
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int p = 0; p < P; p++)
#pragma unroll
            for (int t = 0; t < R; t++) bad |= (fl[p] == 0) & !isfinite(x[p][t]);
    }
#ifdef LRA_TRACE
    if (tid == 0 && blockIdx.x == 0) {
        // the gather's loads have landed once their values are used
        double s0 = 0.0;
#pragma unroll
        for (int p = 0; p < P; p++) s0 += x[p][0];
        if (s0 == 1.2345e300) g_regtr[15] = 1;
    }
#endif
    REG_TOC(0, t_g);
    REG_TIC(t_lu);
    if (!reg_lu<R, P, 0, M>(sm, nw, x, fl, bad, 1.0)) return false;
    __syncthreads();  // L11 written by thread 0
    REG_TOC(1, t_lu);
    REG_CNT(6, R);
    REG_TIC(t_b);
    // ---- B = L21 L11^{-1}: for k = R-1 .. 1, x_k is final and every x_j,
    // j < k, takes x_j - x_k L11[k][j]; basis items get unit rows
#pragma unroll
    for (int p = 0; p < P; p++)
        if (fl[p] > 0) {
#pragma unroll
            for (int t = 0; t < R; t++) x[p][t] = (t == fl[p] - 1) ? 1.0 : 0.0;
        }
#pragma unroll
    for (int k = R - 1; k >= 1; k--) {
#pragma unroll
        for (int j = 0; j < R - 1; j++) {
            if (j >= k) continue;
            const double c = sm.L11[k * (k - 1) / 2 + j];
#pragma unroll
            for (int p = 0; p < P; p++)
                if (fl[p] == 0) x[p][j] -= x[p][k] * c;
        }
        __builtin_amdgcn_sched_barrier(0);  // one row of L11 in registers at a time
    }
    REG_TOC(2, t_b);
    REG_TIC(t_sw);
    // ---- swaps, each update fused with the next scan
    const double thr = 1.0 + delta;
    int swaps = 0, js = -1;
    int64_t wit = -1;
    double pv = 1.0;
    for (;;) {
        Best b = none();
        double b2 = -1.0;
#pragma unroll
        for (int p = 0; p < P; p++) {
            if (fl[p] < 0) continue;
            const int64_t it = reg_item(p, nw);
            double f = 0.0;
            if (js >= 0) {
                if (it == wit) {  // enters the basis in slot js
#pragma unroll
                    for (int t = 0; t < R; t++) x[p][t] = (t == js) ? 1.0 : 0.0;
                    fl[p] = js + 1;
                    continue;
                }
                if (fl[p] != 0 && fl[p] != js + 1) continue;  // other basis rows: B[i][js] = 0
                f = onehot(x[p], js) / pv;
                if (fl[p]) fl[p] = 0;  // the old basis item leaves the basis
            } else if (fl[p]) {
                continue;
            }
            if (f != 0.0) {
                // w = B[i*,:] - e_js^T, formed from the row in LDS
#pragma unroll
                for (int t = 0; t < R; t++) x[p][t] -= f * (sm.wrow[t] - (double)(t == js));
            }
            double vb = -1.0, vb2 = -1.0;
            int jb = 0;
#pragma unroll
            for (int t = 0; t < R; t++) {
                const bool up = fabs(x[p][t]) > vb;
                jb = up ? t : jb;
                if constexpr (M) vb2 = fmax(vb2, fmin(fabs(x[p][t]), vb));
                vb = fmax(vb, fabs(x[p][t]));  // finite entries: the same value as up ? |x| : vb
            }
            if constexpr (M) {
                b2 = fmax(b2, vb2);
                consider2(b, b2, vb, it, jb);
            } else {
                consider(b, vb, it, jb);
            }
        }
        Best win;
        int wf;
        double v2;
        reg_select<R, P, M>(sm, nw, b, b2, 0, x, win, wf, v2);
        const double v = win.v;
        // margins: the stop test's, then (a swap) the search's
        if constexpr (M)
            if (v >= 0.0 && tid == 0) sm.mmin = fmin(sm.mmin, fabs(v - thr) / thr);
        if (v < 0.0 || v <= thr) break;  // no candidate left, or dominant
        if (swaps >= max_swaps) {
            converged = 0;
            break;
        }
        if constexpr (M)
            if (tid == 0) sm.mmin = fmin(sm.mmin, decision_gap(v, v2));
        // the next scan applies B <- B - B[:,js] (B[i*,:] - e_js^T) / B[i*,js]
        js = win.slot;
        wit = win.item;
        pv = sm.wrow[js];
        if (tid == 0) sm.slot_item[js] = wit;
        swaps++;
    }
    swaps_total += swaps;
    REG_TOC(3, t_sw);
    REG_CNT(7, swaps + 1);
    __syncthreads();  // slot_item written by thread 0 (wavefront 0 sorts it)
    if (tid < 64) {
        if (tid < R) set_out[tid] = sm.slot_item[tid];
        sort_set_wave(set_out, R);
    }
    __syncthreads();
    return true;
}

// The whole LRA of one block (the C-A loop of lra_cur with a random start).
template <int R, int P, bool M, class Src>
__device__ __forceinline__ void reg_solve(RegSmem<R> &sm, int nw, const Src &src, int64_t m, int64_t n, uint64_t seed,
                                          int sweeps, double delta, int max_swaps, int refine, int64_t *I_out,
                                          int64_t *J_out, double *U_out, lra_info *info) {
    const int tid = threadIdx.x;
    int32_t swaps_total = 0, converged = 1, sweeps_run = 0;
    if (tid == 0) {
        sm.status = LRA_OK;
        sm.rank_found = R;
        sm.nucleus_rank = R;
        sm.logdet = 0.0;
        sm.mmin = 1.0;
    }
    if (tid < 64) {
        draw_distinct_wave(seed, 0, n, R, sm.Jset);
        __builtin_amdgcn_wave_barrier();
        sort_set_wave(sm.Jset, R);
    }
    __syncthreads();
    bool ok = true;
    // a column step and a row step per sweep (one call site: the step is
    // inlined once)
    for (int st = 0; st < 2 * sweeps; st++) {
        const bool col = (st & 1) == 0;
        ok = reg_step<R, P, M>(sm, nw, src, col ? m : n, col, col ? sm.Jset : sm.Iset, col ? sm.Iset : sm.Jset, delta,
                            max_swaps, swaps_total, converged);
        if (!ok) break;
        if (col) continue;
        const int sw = st / 2;
        sweeps_run = sw + 1;
        bool same = sw > 0;
        for (int j = 0; j < R && same; j++) same = (sm.Iset[j] == sm.Iprev[j]) && (sm.Jset[j] == sm.Jprev[j]);
        __syncthreads();
        if (same) break;
        if (tid < R) {
            sm.Iprev[tid] = sm.Iset[tid];
            sm.Jprev[tid] = sm.Jset[tid];
        }
        __syncthreads();
    }
    REG_TIC(t_n);
    if (ok) nucleus(sm, sm.nuc, src, R, refine, 64 * nw, U_out);
    REG_TOC(4, t_n);
    REG_CNT(8, 1);
    __syncthreads();
    const int st = sm.status;
    if (tid < R) {
        I_out[tid] = st == LRA_OK ? sm.Iset[tid] : -1;
        J_out[tid] = st == LRA_OK ? sm.Jset[tid] : -1;
    }
    if (st != LRA_OK)
        for (int e = tid; e < R * R; e += 64 * nw) U_out[e] = __builtin_nan("");
    if (tid == 0 && info) {
        lra_info inf;
        inf.status = st;
        inf.sweeps_run = sweeps_run;
        inf.swaps_total = swaps_total;
        inf.converged = (st == LRA_OK) ? converged : 0;
        inf.rank_found = sm.rank_found;
        inf.team_size = 1;
        inf.nucleus_rank = st == LRA_OK ? sm.nucleus_rank : 0;
        inf.reserved = 0;
        inf.det_log_abs = st == LRA_OK ? sm.logdet : 0.0;
        inf.min_margin = M ? sm.mmin : __builtin_nan("");
        *info = inf;
    }
}

// Persistent loop over the blocks order[0 .. count) of one bin, taken from
// *queue; workgroups of 64 nw threads.
template <int R, int P, bool M, class Desc, class MakeSrc>
__device__ __forceinline__ void reg_loop(const Desc *blocks, const int32_t *order, int64_t count, uint64_t seed,
                                         int sweeps, double delta, int max_swaps, int refine, unsigned *queue,
                                         int64_t *I_out, int64_t *J_out, double *U_out, lra_info *infos,
                                         const MakeSrc &make) {
    __shared__ RegSmem<R> sm;
    const int nw = (int)(blockDim.x >> 6);
    for (;;) {
        if (threadIdx.x == 0) sm.job = (int32_t)atomicAdd(queue, 1u);
        __syncthreads();
        const int64_t job = sm.job;
        __syncthreads();
        if (job >= count) break;
        const int32_t b = order[job];
        const Desc d = blocks[b];
        REG_TIC(t_blk);
        reg_solve<R, P, M>(sm, nw, make(d), d.m, d.n, seed + (uint64_t)b, sweeps, delta, max_swaps, refine,
                        I_out + (int64_t)b * R, J_out + (int64_t)b * R, U_out + (int64_t)b * R * R,
                        infos ? infos + b : nullptr);
        REG_TOC(5, t_blk);
        __syncthreads();
    }
}

template <typename T>
struct MakeDense {
    const T *base;
    __device__ __forceinline__ DenseSrc<T> operator()(const BlockDesc &d) const {
        return DenseSrc<T>{base + d.offset, d.lda};
    }
};
struct MakePoints {
    const double *pts;
    __device__ __forceinline__ PointSrc operator()(const PtsDesc &d) const {
        return PointSrc{pts + 2 * d.x_off, pts + 2 * d.y_off};
    }
};

template <int R, int P, typename T, bool M>
__global__ void __launch_bounds__(64 * kRegMaxWaves) ca_reg_kernel(const T *base, const BlockDesc *blocks,
                                                                   const int32_t *order, int64_t count, uint64_t seed,
                                                                   int sweeps, double delta, int max_swaps, int refine,
                                                                   unsigned *queue, int64_t *I_out, int64_t *J_out,
                                                                   double *U_out, lra_info *infos) {
    reg_loop<R, P, M>(blocks, order, count, seed, sweeps, delta, max_swaps, refine, queue, I_out, J_out, U_out, infos,
                      MakeDense<T>{base});
}

template <int R, int P, bool M>
__global__ void __launch_bounds__(64 * kRegMaxWaves) ca_reg_points_kernel(const double *pts, const PtsDesc *blocks,
                                                                          const int32_t *order, int64_t count,
                                                                          uint64_t seed, int sweeps, double delta,
                                                                          int max_swaps, int refine, unsigned *queue,
                                                                          int64_t *I_out, int64_t *J_out,
                                                                          double *U_out, lra_info *infos) {
    reg_loop<R, P, M>(blocks, order, count, seed, sweeps, delta, max_swaps, refine, queue, I_out, J_out, U_out, infos,
                      MakePoints{pts});
}

// Kernel of a register variant for a source (a dtype code; any other value:
// point sets).
template <int R, int P, bool M>
const void *reg_kernel_fn(int src) {
    switch (src) {
    case LRA_F64: return (const void *)ca_reg_kernel<R, P, double, M>;
    case LRA_F32: return (const void *)ca_reg_kernel<R, P, float, M>;
    case LRA_BF16: return (const void *)ca_reg_kernel<R, P, uint16_t, M>;
    default: return (const void *)ca_reg_points_kernel<R, P, M>;
    }
}

// (margins: the instantiation that tracks the decisions' margins)
const void *reg_kernel(int R, int P, int src, bool margins = true) {
    if (R == 16 && P == 2) return margins ? reg_kernel_fn<16, 2, true>(src) : reg_kernel_fn<16, 2, false>(src);
    return nullptr;
}

}  // namespace

bool reg_variant_exists(int r, int P) { return reg_kernel(r, P, LRA_F64) != nullptr; }

int reg_occupancy(int r, int P, int waves, int src) {
    const void *f = reg_kernel(r, P, src);
    if (!f) return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, 64 * waves, 0) != hipSuccess) return 0;
    return blocks;
}

hipError_t launch_reg(int src, int r, int P, int waves, const void *base, const void *blocks, const int32_t *order,
                      int64_t count, uint64_t seed, const CAConfig &cfg, unsigned *queue, int grid, int64_t *I_out,
                      int64_t *J_out, double *U_out, lra_info *infos, hipStream_t stream) {
    const void *f = reg_kernel(r, P, src, cfg.margins != 0);
    if (!f || waves < 1 || waves > kRegMaxWaves || grid < 1) return hipErrorInvalidValue;
    int sweeps = cfg.sweeps, max_swaps = cfg.max_swaps, refine = cfg.refine_steps;
    double delta = cfg.delta;
    void *args[] = {(void *)&base,   (void *)&blocks, (void *)&order,     (void *)&count,  (void *)&seed,
                    (void *)&sweeps, (void *)&delta,  (void *)&max_swaps, (void *)&refine, (void *)&queue,
                    (void *)&I_out,  (void *)&J_out,  (void *)&U_out,     (void *)&infos};
    return hipLaunchKernel(f, dim3(grid), dim3(64 * waves), args, 0, stream);
}

}  // namespace lra

#ifdef LRA_TRACE
// Copy and clear the register kernel's phase ticks (tracing builds only):
// gathers, LU, B solve, swaps, nucleus, whole blocks; LU decisions, swap
// decisions, blocks.
extern "C" int lra_trace_reg(uint64_t *host) {
    if (hipMemcpyFromSymbol(host, HIP_SYMBOL(lra::g_regtr), sizeof(uint64_t) * 16) != hipSuccess) return -1;
    uint64_t z[16] = {0};
    if (hipMemcpyToSymbol(HIP_SYMBOL(lra::g_regtr), z, sizeof(z)) != hipSuccess) return -1;
    return 16;
}
#endif
