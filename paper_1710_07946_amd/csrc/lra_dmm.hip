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
//   2. one-sided Jacobi sweeps on G (the truncated nucleus's rotation loop):
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
namespace {

constexpr int kDmmChunk = 64;             // sketch rows staged per Gram pass
constexpr int kDmmPs = kRMax + 1;         // their LDS row stride (doubles)
constexpr int kDmmProj = 16;              // kept directions projected per pass over an item
constexpr int kDmmGram = kRMax * kRMax / kBlock;  // Gram entries per thread

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
};

// Entry (item, c) of the row-step sketch W[:, J] D (ROWS) or of the
// column-step sketch Dbar W[I, :] (items are columns of W).
template <bool ROWS, typename T>
__device__ __forceinline__ double sketch_entry(const DmmSmem &sm, const DenseSrc<T> &src, int64_t item, int c) {
    return ROWS ? src(item, sm.Jset[c]) * sm.dl[c] : sm.dk[c] * src(sm.Iset[c], item);
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
    // 1. Gram matrix
    double acc[kDmmGram];
#pragma unroll
    for (int u = 0; u < kDmmGram; u++) acc[u] = 0.0;
    int bad = 0;
    for (int64_t i0 = 0; i0 < items; i0 += kDmmChunk) {
        const int nb = items - i0 < kDmmChunk ? (int)(items - i0) : kDmmChunk;
        for (int e = tid; e < nb * w; e += kBlock) {
            // row step: a row's w entries side by side; column step: a
            // selected row's run of consecutive columns side by side
            const int it = ROWS ? e / w : e % nb, c = ROWS ? e % w : e / nb;
            const double x = sketch_entry<ROWS>(sm, src, i0 + it, c);
            bad |= !isfinite(x);
            Pc[it * kDmmPs + c] = x;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kDmmGram; u++) {
            const int e = tid + u * kBlock;
            if (e < w * w) {
                const int a = e % w, b = e / w;
                double s = acc[u];
                for (int it = 0; it < nb; it++) s += Pc[it * kDmmPs + a] * Pc[it * kDmmPs + b];
                acc[u] = s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kDmmGram; u++) {
        const int e = tid + u * kBlock;
        if (e < w * w) {
            A[e] = acc[u];  // column b, row a (G is symmetric)
            V[e] = (e / w == e % w) ? 1.0 : 0.0;
        }
    }
    bad = __syncthreads_or(bad);
    if (bad) {
        if (tid == 0) sm.status = LRA_EINVAL;
        __syncthreads();
        return;
    }
    // 2. eigenvectors of G
    jacobi_sweeps(A, V, w, w);
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
    // scores and their running sums, kBlock items at a time
    for (int64_t i0 = 0; i0 < items; i0 += kBlock) {
        const int64_t i = i0 + tid;
        double s = 0.0;
        if (i < items) {
            for (int t0 = 0; t0 < nk; t0 += kDmmProj) {
                double pr[kDmmProj];
#pragma unroll
                for (int t = 0; t < kDmmProj; t++) pr[t] = 0.0;
                for (int c = 0; c < w; c++) {
                    const double x = sketch_entry<ROWS>(sm, src, i, c);
#pragma unroll
                    for (int t = 0; t < kDmmProj; t++)
                        if (t0 + t < nk) pr[t] += x * V[sm.keep[t0 + t] * w + c];
                }
#pragma unroll
                for (int t = 0; t < kDmmProj; t++)
                    if (t0 + t < nk) s += pr[t] * pr[t] / sm.lam[sm.keep[t0 + t]];
            }
        }
        // inclusive scan: within the wavefront, then the wavefront totals in order
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
        if (i < items) {
            q[i] = s;
            cdf[i] = base + incl;
        }
        __syncthreads();
        if (tid == kBlock - 1) {
            double c = sm.carry;
            for (int v = 0; v < kBlock / kWave; v++) c += sm.wtot[v];
            sm.carry = c;
        }
        __threadfence_block();
        __syncthreads();
    }
    // 4. draws, rescaling and sort (one wavefront)
    if (tid < kWave) {
        const double S = sm.carry;
        int64_t idx = INT64_MAX;
        double sc = 0.0;
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
        }
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
            if (tid == 0) sm.status = LRA_OK;
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
            nucleus_trunc(sm, lds, src, k, l, r, U, 1.0, 1.0, sm.dk, sm.dl);
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

size_t dmm_lds_bytes() { return sizeof(double) * (2 * (size_t)kRMax * kRMax + (size_t)kDmmChunk * kDmmPs); }

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
