// lra_dmm.hip -- C-A whose step subalgorithm is the leverage-score sampling
// of DMM08 applied to every vertical and horizontal sketch (Section "Testing
// C-A acceleration of the algorithms of DMM08", Tables 7 and 8; the sampling
// of Algorithm algcurlevsc by Algorithm algsmplex, the scores of eq. eqlevsc
// with beta = 1 taken of the sketch).  One workgroup per block, blocks dealt
// round-robin over a persistent grid.
//
// A half-step on a sketch P (items x w, w <= 64; entries formed from W and
// the current rescaling when read, never stored):
//   1. Gram matrix G = P^T P (w x w) in LDS, P staged through LDS 64 items
//      at a time, each entry summed over the items in increasing order;
//   2. one-sided Jacobi sweeps on G (the truncated nucleus's rotation loop,
//      without the rotations among directions far below the kept ones):
//      G V = V Lambda, so the eigenvalues of G, the squared singular values
//      of P, are the column norms and V its right singular vectors;
//   3. kept: the r largest eigenvalues above 1e-13 times the largest (ties
//      to the lower index); score q_i = sum over the kept, largest first, of
//      (P_i . v_a)^2 / lambda_a, i.e. |row i of P's dominant left singular
//      factor|^2; running sums in item order (a wavefront scan per 512
//      items, the wavefront totals added in order);
//   4. cnt draws u_t = (x >> 11) 2^-53 from SplitMix64 output t of the
//      step's stream, each the first item whose running sum exceeds u_t S
//      (binary search), rescaled by 1 / sqrt(cnt q_i / S), sorted by item.
// The Gram route reads P twice and squares its condition: the kept values
// are far above the squared rounding level for the inputs the method is
// meant for, and the threshold leaves out a direction only at rounding
// level.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lra_common.h"

namespace lra {

// Built with -DLRA_TRACE, workgroup 0 adds the wall-clock ticks of each phase
// (and the Jacobi sweeps and half-steps) to g_dmmtr; lra_trace_dmm() copies
// them out and clears them.
#ifdef LRA_TRACE
__device__ uint64_t g_dmmtr[8];
#define DMM_TIC(v) const uint64_t v = (blockIdx.x == 0 && threadIdx.x == 0) ? wall_clock64() : 0
#define DMM_TOC(slot, v) \
    do { if (blockIdx.x == 0 && threadIdx.x == 0) g_dmmtr[slot] += wall_clock64() - v; } while (0)
#define DMM_CNT(slot, n) \
    do { if (blockIdx.x == 0 && threadIdx.x == 0) g_dmmtr[slot] += (n); } while (0)
#else
#define DMM_TIC(v) ((void)0)
#define DMM_TOC(slot, v) ((void)0)
#define DMM_CNT(slot, n) ((void)0)
#endif

namespace {

constexpr int kDmmChunk = 64;             // sketch rows staged in LDS at a time
constexpr int kDmmPs = kRMax + 1;         // their LDS row stride (doubles)
typedef double v4d __attribute__((ext_vector_type(4)));
// Pairs of Gram columns whose squared norms are both below 1e-20 of the
// largest, or both below 1e-4 of the r-th largest (eigenvalues below 1e-10
// lambda_max, or below 1e-2 lambda_r), are not rotated against each other:
// they can mix only directions far below the kept ones, while every pair
// with a column above the floor is still rotated until orthogonal.
constexpr double kDmmPairFloor = 1e-20;
constexpr double kDmmGapFloor = 1e-4;

// FP64 MFMA 16x16x4: A operand of lane l is A[l % 16][l / 16], B operand
// B[l / 16][l % 16], output v is D[l / 16 + 4 v][l % 16].
__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct DmmSmem {
    int64_t Iset[kRMax], Jset[kRMax];
    double dk[kRMax], dl[kRMax];
    double lam[kRMax];
    int keep[kRMax];
    int nkeep;
    double wtot[kBlock / kWave];
    double carry;
    int status;
    int32_t nucleus_rank;
    double logdet;
    double mmin;   // smallest distance of a draw from its item's boundaries, relative to S
};

// Entry (item, c) of the row-step sketch W[:, J] D (ROWS) or of the
// column-step sketch Dbar W[I, :] (items are columns of W).
template <bool ROWS, typename T>
__device__ __forceinline__ double sketch_entry(const DmmSmem &sm, const DenseSrc<T> &src, int64_t item, int c) {
    return ROWS ? src(item, sm.Jset[c]) * sm.dl[c] : sm.dk[c] * src(sm.Iset[c], item);
}

// Stage items i0 .. i0 + 63 of the sketch into Pc (row-major, stride
// kDmmPs), zero beyond the last item (up to a multiple of 4) and in columns
// w .. wp - 1; returns whether a staged entry is not finite.
template <bool ROWS, typename T>
__device__ __forceinline__ int stage_chunk(const DmmSmem &sm, const DenseSrc<T> &src, double *Pc, int64_t i0,
                                           int64_t items, int w, int wp) {
    const int nb = items - i0 < kDmmChunk ? (int)(items - i0) : kDmmChunk, nb4 = (nb + 3) & ~3;
    int bad = 0;
    for (int e = threadIdx.x; e < nb4 * wp; e += kBlock) {
        // row step: a row's entries side by side; column step: a selected
        // row's run of consecutive columns side by side
        const int it = ROWS ? e / wp : e % nb4, c = ROWS ? e % wp : e / nb4;
        double x = 0.0;
        if (it < nb && c < w) {
            x = sketch_entry<ROWS>(sm, src, i0 + it, c);
            bad |= !isfinite(x);
        }
        Pc[it * kDmmPs + c] = x;
    }
    return bad;
}

// One-sided Jacobi sweeps on the w x w Gram matrix A (column-major, in
// LDS), rotations accumulated in V (set to the identity by the caller): the
// rotation loop of the truncated nucleus (round-robin pairs, a pair rotated
// unless |a_p . a_q| <= w eps sqrt(|a_p|^2 |a_q|^2), eps = 2^-52, or a
// column is negligible, or the sine is zero; at most 60 sweeps, each pair on
// the 16 lanes of a DPP row), with the pair floor above recomputed at every
// sweep's start from the squared column norms.  Returns the sweeps run.
__device__ __forceinline__ int dmm_sweeps(double *A, double *V, int w, int r) {
    constexpr int RL = kRMax / 16;
    const int tid = threadIdx.x;
    __shared__ int s_rot;
    __shared__ double s_nrm[kRMax];
    __shared__ double s_small, s_negl;
    const int lp = w + (w & 1);
    const int grp = tid / 16, j = tid % 16, ngrp = kBlock / 16;
    const double tol = (double)w * 0x1p-52;
    int sweep = 0;
    for (; sweep < 60 && w > 1; sweep++) {
        for (int c = grp; c < w; c += ngrp) {
            double s2 = 0.0;
#pragma unroll
            for (int u = 0; u < RL; u++) {
                const int i = j + 16 * u;
                const double x = i < w ? A[c * w + i] : 0.0;
                s2 += x * x;
            }
            s2 = row_sum16(s2);
            if (j == 0) s_nrm[c] = s2;
        }
        if (tid == 0) s_rot = 0;
        __syncthreads();
        if (tid < kWave) {
            // the largest and the r-th largest squared norm (one wavefront,
            // w <= 64; with r >= w no pair can fall below the r-th largest)
            const double x = tid < w ? s_nrm[tid] : -1.0;
            int gt = 0, ge = 0;
            if (r < w) {
                for (int c = 0; c < w; c++) {
                    gt += s_nrm[c] > x ? 1 : 0;
                    ge += s_nrm[c] >= x ? 1 : 0;
                }
            }
            const double big = wave_max(x);
            const unsigned long long at = __ballot(r < w && tid < w && gt < r && r <= ge);
            const double rth = at ? __shfl(x, __ffsll((long long)at) - 1) : 0.0;
            if (tid == 0) {
                s_negl = tol * tol * big;
                s_small = fmax(kDmmPairFloor * big, kDmmGapFloor * rth);
            }
        }
        __syncthreads();
        const double negl = s_negl, small = s_small;
        for (int t = 0; t < lp - 1; t++) {
            for (int pr = grp; pr < lp / 2; pr += ngrp) {
                int pc, qc;
                jacobi_pair(t, pr, lp, pc, qc);
                if (qc >= w) continue;
                const double *ap = A + pc * w, *aq = A + qc * w;
                double x[RL], y[RL];
#pragma unroll
                for (int u = 0; u < RL; u++) {
                    const int i = j + 16 * u;
                    x[u] = i < w ? ap[i] : 0.0;
                    y[u] = i < w ? aq[i] : 0.0;
                }
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int u = 0; u < RL; u++) {
                    al += x[u] * x[u];
                    be += y[u] * y[u];
                    ga += x[u] * y[u];
                }
                al = row_sum16(al);
                be = row_sum16(be);
                ga = row_sum16(ga);
                if (ga == 0.0 || fabs(ga) <= tol * sqrt(al * be)) continue;
                if (al <= negl || be <= negl) continue;
                if (al <= small && be <= small) continue;
                const double ze = (be - al) / (2.0 * ga);
                const double tt = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
                const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
                if (sn == 0.0) continue;
#pragma unroll
                for (int u = 0; u < RL; u++) {
                    const int i = j + 16 * u;
                    if (i < w) {
                        A[pc * w + i] = cs * x[u] - sn * y[u];
                        A[qc * w + i] = sn * x[u] + cs * y[u];
                    }
                }
                double vx[RL], vy[RL];
#pragma unroll
                for (int u = 0; u < RL; u++) {
                    const int i = j + 16 * u;
                    vx[u] = i < w ? V[pc * w + i] : 0.0;
                    vy[u] = i < w ? V[qc * w + i] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < RL; u++) {
                    const int i = j + 16 * u;
                    if (i < w) {
                        V[pc * w + i] = cs * vx[u] - sn * vy[u];
                        V[qc * w + i] = sn * vx[u] + cs * vy[u];
                    }
                }
                if (j == 0) s_rot = 1;
            }
            __syncthreads();
        }
        const int rot = *(volatile int *)&s_rot;
        __syncthreads();
        if (!rot) break;
    }
    return w > 1 ? (sweep < 60 ? sweep + 1 : 60) : 0;
}

// One half-step (see the file comment).  ROWS: items = rows of W, w = l,
// draws k rows into sm.Iset / sm.dk; else items = columns, w = k, draws l
// columns into sm.Jset / sm.dl.  q, cdf: `items` doubles of this
// workgroup's global scratch.  Returns the status in sm.status.
template <bool ROWS, typename T>
__device__ __forceinline__ void dmm_half(DmmSmem &sm, double *lds, const DenseSrc<T> &src, int64_t items, int w, int r,
                                         int cnt, uint64_t seed, uint64_t stream, double *q, double *cdf) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    double *A = lds, *V = lds + kRMax * kRMax, *Pc = lds + 2 * kRMax * kRMax;
    double *Ps = Pc + kDmmChunk * kDmmPs;  // per-tile score partials, 4 x kDmmChunk
    // 1. Gram matrix on the FP64 matrix cores: 16 x 16 tiles (ta, tb) of G,
    // tile t = wave + 8 u, each product over 4 staged items
    DMM_TIC(t0);
    const int nt = (w + 15) / 16, wp = 16 * nt;
    v4d acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    int bad = 0;
    for (int64_t i0 = 0; i0 < items; i0 += kDmmChunk) {
        bad |= stage_chunk<ROWS>(sm, src, Pc, i0, items, w, wp);
        __syncthreads();
        const int nb4 = ((items - i0 < kDmmChunk ? (int)(items - i0) : kDmmChunk) + 3) & ~3;
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int t = wv + 8 * u;
            if (t < nt * nt) {
                const double *pa = Pc + (lane >> 4) * kDmmPs + 16 * (t % nt) + (lane & 15);
                const double *pb = Pc + (lane >> 4) * kDmmPs + 16 * (t / nt) + (lane & 15);
                v4d c = acc[u];
                for (int it = 0; it < nb4; it += 4) c = mfma4(pa[it * kDmmPs], pb[it * kDmmPs], c);
                acc[u] = c;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 2; u++) {
        const int t = wv + 8 * u;
        if (t < nt * nt) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int a = 16 * (t % nt) + (lane >> 4) + 4 * v, bcol = 16 * (t / nt) + (lane & 15);
                if (a < w && bcol < w) A[bcol * w + a] = acc[u][v];  // column bcol, row a
            }
        }
    }
    for (int e = tid; e < w * w; e += kBlock) V[e] = (e / w == e % w) ? 1.0 : 0.0;
    bad = __syncthreads_or(bad);
    if (bad) {
        if (tid == 0) sm.status = LRA_EINVAL;
        __syncthreads();
        return;
    }
    DMM_TOC(0, t0);
    // 2. eigenvectors of G
    DMM_TIC(t1);
    const int nsw = dmm_sweeps(A, V, w, r);
    DMM_TOC(1, t1);
    DMM_CNT(6, nsw);
    DMM_CNT(7, 1);
    (void)nsw;
    DMM_TIC(t2);
    // 3. the kept directions, largest first
    for (int c = tid; c < w; c += kBlock) {
        double s2 = 0.0;
        for (int i = 0; i < w; i++) s2 += A[c * w + i] * A[c * w + i];
        sm.lam[c] = sqrt(s2);
    }
    __syncthreads();
    if (tid < kWave) {
        const double lc = tid < w ? sm.lam[tid] : -1.0;
        double lmax = 0.0;
        int above = 0;
        for (int c = 0; c < w; c++) {
            const double x = sm.lam[c];
            lmax = x > lmax ? x : lmax;
            above += (x > lc || (x == lc && c < tid)) ? 1 : 0;
        }
        const bool kept = tid < w && above < r && lc > 1e-13 * lmax;
        if (kept) sm.keep[above] = tid;
        const int nk = __popcll(__ballot(kept));
        if (tid == 0) {
            sm.nkeep = nk;
            sm.carry = 0.0;
            if (nk == 0) sm.status = LRA_ESINGULAR;
        }
    }
    __syncthreads();
    const int nk = sm.nkeep;
    if (nk == 0) return;
    // scores of kDmmChunk staged items at a time on the matrix cores: the
    // projections P_i . v_a of 16 items x 16 kept directions per tile, squared, divided by
    // lambda_a and summed over the tile's directions (the 16 lanes of a DPP
    // row), then over the direction tiles in order; tile t: items
    // 16 (t % 4), directions 16 (t / 4), waves taking tiles in turn
    const int ndt = (nk + 15) / 16;
    for (int64_t i0 = 0; i0 < items; i0 += kDmmChunk) {
        stage_chunk<ROWS>(sm, src, Pc, i0, items, w, wp);
        __syncthreads();
        for (int t = wv; t < 4 * ndt; t += kBlock / kWave) {
            const int it0 = 16 * (t % 4), d0 = 16 * (t / 4);
            const int dj = d0 + (lane & 15);
            const int vcol = dj < nk ? sm.keep[dj] : 0;
            const double *pa = Pc + (it0 + (lane & 15)) * kDmmPs + (lane >> 4);
            const double *pv = V + vcol * w + (lane >> 4);
            v4d c = {0.0, 0.0, 0.0, 0.0};
            for (int c0 = 0; c0 < wp; c0 += 4) {
                const bool in = c0 + (lane >> 4) < w && dj < nk;
                c = mfma4(pa[c0], in ? pv[c0] : 0.0, c);
            }
            const double il = dj < nk ? 1.0 / sm.lam[vcol] : 0.0;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const double y = row_sum16(c[v] * c[v] * il);
                if ((lane & 15) == 0) Ps[(t / 4) * kDmmChunk + it0 + (lane >> 4) + 4 * v] = y;
            }
        }
        __syncthreads();
        if (tid < kDmmChunk && i0 + tid < items) {
            double sc = 0.0;
            for (int dt = 0; dt < ndt; dt++) sc += Ps[dt * kDmmChunk + tid];
            q[i0 + tid] = sc;
        }
        __syncthreads();
    }
    __threadfence_block();
    __syncthreads();
    // running sums in item order: a wavefront scan per kBlock items, the
    // wavefront totals added in order
    for (int64_t i0 = 0; i0 < items; i0 += kBlock) {
        const int64_t i = i0 + tid;
        const double s = i < items ? q[i] : 0.0;
        double incl = s;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const double y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        if (lane == kWave - 1) sm.wtot[wv] = incl;
        __syncthreads();
        double base = sm.carry;
        for (int v = 0; v < wv; v++) base += sm.wtot[v];
        if (i < items) cdf[i] = base + incl;
        __syncthreads();
        if (tid == kBlock - 1) {
            double c = sm.carry;
            for (int v = 0; v < kBlock / kWave; v++) c += sm.wtot[v];
            sm.carry = c;
        }
        __threadfence_block();
        __syncthreads();
    }
    DMM_TOC(2, t2);
    // 4. draws, rescaling and sort (one wavefront)
    DMM_TIC(t3);
    if (tid < kWave) {
        const double S = sm.carry;
        int64_t idx = INT64_MAX;
        double sc = 0.0, gap = 1.0;
        if (tid < cnt) {
            const double u = (double)(sm64(seed, stream, (uint64_t)tid) >> 11) * 0x1p-53;
            const double target = u * S;
            int64_t lo = 0, hi = items - 1;
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (cdf[mid] > target) hi = mid;
                else lo = mid + 1;
            }
            idx = lo;
            sc = 1.0 / sqrt(((double)cnt * q[lo]) / S);
            gap = fmin((cdf[lo] - target) / S, (target - (lo > 0 ? cdf[lo - 1] : 0.0)) / S);
        }
        gap = -wave_max(-gap);
        if (tid == 0) sm.mmin = fmin(sm.mmin, gap);
        int rank = 0;
        for (int j = 0; j < cnt; j++) {
            const int64_t y = __shfl(idx, j);
            rank += (y < idx) || (y == idx && j < tid);
        }
        if (tid < cnt) {
            if (ROWS) {
                sm.Iset[rank] = idx;
                sm.dk[rank] = sc;
            } else {
                sm.Jset[rank] = idx;
                sm.dl[rank] = sc;
            }
        }
    }
    __syncthreads();
    DMM_TOC(3, t3);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) ca_dmm_kernel(const T *base, const BlockDesc *blocks, int64_t count,
                                                        uint64_t seed, int32_t r, int32_t k, int32_t l, int32_t iters,
                                                        double *scratch, int64_t scratch_items, int64_t *I_out,
                                                        int64_t *J_out, double *U_out, lra_info *infos) {
    __shared__ DmmSmem sm;
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    double *lds = reinterpret_cast<double *>(lds_dyn);
    const int tid = threadIdx.x;
    double *q = scratch + (size_t)blockIdx.x * 2 * (size_t)scratch_items;
    double *cdf = q + scratch_items;
    for (int64_t b = blockIdx.x; b < count; b += gridDim.x) {
        const BlockDesc d = blocks[b];
        const DenseSrc<T> src{base + d.offset, d.lda};
        const uint64_t sd = seed + (uint64_t)b;
        if (tid < kWave) {
            draw_uniform_wave(sd, 8, d.n, l, sm.Jset);
            __builtin_amdgcn_wave_barrier();
            sort_set_wave(sm.Jset, l);
            if (tid < l) sm.dl[tid] = sqrt((double)d.n / (double)l);
            if (tid == 0) {
                sm.status = LRA_OK;
                sm.mmin = 1.0;
            }
        }
        __syncthreads();
        int t = 0;
        for (; t < iters; t++) {
            dmm_half<true>(sm, lds, src, d.m, l, r, k, sd, 16 + 2 * (uint64_t)t, q, cdf);
            if (sm.status != LRA_OK) break;
            dmm_half<false>(sm, lds, src, d.n, k, r, l, sd, 17 + 2 * (uint64_t)t, q, cdf);
            if (sm.status != LRA_OK) break;
        }
        const int st = sm.status;
        double *const U = U_out + b * (int64_t)l * k;
        if (st == LRA_OK) {
            DMM_TIC(t4);
            nucleus_trunc(sm, lds, src, k, l, r, U, 1.0, 1.0, sm.dk, sm.dl);
            DMM_TOC(4, t4);
            DMM_CNT(5, 1);
        } else {
            for (int e = tid; e < l * k; e += kBlock) U[e] = __builtin_nan("");
        }
        if (tid < k) I_out[b * k + tid] = st == LRA_OK ? sm.Iset[tid] : -1;
        if (tid < l) J_out[b * l + tid] = st == LRA_OK ? sm.Jset[tid] : -1;
        if (tid == 0 && infos) {
            lra_info inf;
            inf.status = st;
            inf.sweeps_run = st == LRA_OK ? iters : t + 1;
            inf.swaps_total = 0;
            inf.converged = st == LRA_OK ? 1 : 0;
            inf.rank_found = st == LRA_ESINGULAR ? 0 : r;
            inf.team_size = 1;
            inf.nucleus_rank = st == LRA_OK ? sm.nucleus_rank : 0;
            inf.reserved = 0;
            inf.det_log_abs = st == LRA_OK ? sm.logdet : 0.0;
            inf.min_margin = sm.mmin;
            infos[b] = inf;
        }
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_dmm_t(const void *base, const BlockDesc *blocks, int64_t count, uint64_t seed, int r, int k, int l,
                        int iters, double *scratch, int64_t scratch_items, int grid, int64_t *I_out, int64_t *J_out,
                        double *U_out, lra_info *infos, hipStream_t stream) {
    auto kern = ca_dmm_kernel<T>;
    const size_t dyn = dmm_lds_bytes();
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), dyn, stream, static_cast<const T *>(base), blocks, count, seed,
                       r, k, l, iters, scratch, scratch_items, I_out, J_out, U_out, infos);
    return hipGetLastError();
}

}  // namespace

size_t dmm_lds_bytes() {
    return sizeof(double) * (2 * (size_t)kRMax * kRMax + (size_t)kDmmChunk * kDmmPs + 4 * (size_t)kDmmChunk);
}

int dmm_occupancy(int dtype) {
    int blocks = 0;
    hipError_t e;
    const size_t dyn = dmm_lds_bytes();
    if (dtype == LRA_F64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_dmm_kernel<double>, kBlock, dyn);
    else if (dtype == LRA_F32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_dmm_kernel<float>, kBlock, dyn);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ca_dmm_kernel<uint16_t>, kBlock, dyn);
    return e == hipSuccess ? blocks : 0;
}

hipError_t launch_dmm(int dtype, const void *base, const BlockDesc *blocks, int64_t count, uint64_t seed, int r, int k,
                      int l, int iters, double *scratch, int64_t scratch_items, int grid, int64_t *I_out,
                      int64_t *J_out, double *U_out, lra_info *infos, hipStream_t stream) {
    switch (dtype) {
    case LRA_F64:
        return launch_dmm_t<double>(base, blocks, count, seed, r, k, l, iters, scratch, scratch_items, grid, I_out,
                                    J_out, U_out, infos, stream);
    case LRA_F32:
        return launch_dmm_t<float>(base, blocks, count, seed, r, k, l, iters, scratch, scratch_items, grid, I_out,
                                   J_out, U_out, infos, stream);
    default:
        return launch_dmm_t<uint16_t>(base, blocks, count, seed, r, k, l, iters, scratch, scratch_items, grid, I_out,
                                      J_out, U_out, infos, stream);
    }
}

}  // namespace lra

#ifdef LRA_TRACE
extern "C" int lra_trace_dmm(uint64_t *host) {
    if (hipMemcpyFromSymbol(host, HIP_SYMBOL(lra::g_dmmtr), sizeof(uint64_t) * 8) != hipSuccess) return -1;
    uint64_t z[8] = {0};
    if (hipMemcpyToSymbol(HIP_SYMBOL(lra::g_dmmtr), z, sizeof(z)) != hipSuccess) return -1;
    return 8;
}
#endif
