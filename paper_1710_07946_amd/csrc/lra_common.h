// lra_common.h -- pieces shared by the C-A kernels: the wavefront argmax with
// the oracle's tie rule, set sorting, the entry sources through which the
// kernels read W, and the r x r nucleus.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lra_device.h"
#include "lra_internal.h"

namespace lra {

// ---------------------------------------------------------------- argmax
// Candidates are ordered by value, then lowest item, then lowest slot: the
// tie rule of the oracle's sequential scans.
struct Best {
    double v;      // |value| compared; -1 when there is no candidate
    int64_t item;  // global item id (row or column of W)
    int32_t slot;  // basis slot (swap search) or 0
    int32_t aux;   // owner workgroup (team reduction only)
};

// (bitwise on the comparisons: no branches in the wavefront reductions)
__device__ __forceinline__ bool better(double v1, int64_t i1, int s1, double v2, int64_t i2, int s2) {
    return (v1 > v2) | ((v1 == v2) & ((i1 < i2) | ((i1 == i2) & (s1 < s2))));
}

__device__ __forceinline__ Best none() { return Best{-1.0, INT64_MAX, 0x7fffffff, -1}; }

__device__ __forceinline__ void consider(Best &b, double v, int64_t item, int slot, int aux = -1) {
    if (better(v, item, slot, b.v, b.item, b.slot)) b = Best{v, item, slot, aux};
}

// Wavefront argmax without LDS traffic: four DPP butterflies (quad swaps,
// half-row and row mirrors) leave every lane of a 16-lane row with the row's
// best, then two row broadcasts (row 0 into row 1 and row 2 into row 3, then
// row 1 into rows 2 and 3) leave the wavefront's best in lane 63.  Lanes a
// step does not write keep their own value.  The order is total, so the
// result does not depend on the tree's shape.  All 64 lanes must be active.
template <int CTRL, int RM = 0xf>
__device__ __forceinline__ int dpp32(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, RM, 0xf, false);
}
template <int CTRL, int RM = 0xf>
__device__ __forceinline__ int64_t dpp64(int64_t v) {
    const int lo = dpp32<CTRL, RM>((int)(uint32_t)v), hi = dpp32<CTRL, RM>((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int64_t rdl64(int64_t v, int lane) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int CTRL, int RM = 0xf>
__device__ __forceinline__ void dpp_step(Best &b) {
    const double ov = __longlong_as_double(dpp64<CTRL, RM>(__double_as_longlong(b.v)));
    const int64_t oi = dpp64<CTRL, RM>(b.item);
    const int os = dpp32<CTRL, RM>(b.slot), oa = dpp32<CTRL, RM>(b.aux);
    const bool up = better(ov, oi, os, b.v, b.item, b.slot);
    b.v = up ? ov : b.v;
    b.item = up ? oi : b.item;
    b.slot = up ? os : b.slot;
    b.aux = up ? oa : b.aux;
}
__device__ __forceinline__ Best rdl_best(const Best &b, int lane) {
    return Best{__longlong_as_double(rdl64(__double_as_longlong(b.v), lane)), rdl64(b.item, lane),
                __builtin_amdgcn_readlane(b.slot, lane), __builtin_amdgcn_readlane(b.aux, lane)};
}
constexpr int kDppQuadSwap1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;
constexpr int kDppRowBcast15 = 0x142;  // lane 15 of a row to the whole next row
constexpr int kDppRowBcast31 = 0x143;  // lane 31 to rows 2 and 3

__device__ __forceinline__ Best wave_reduce_full(Best b) {
    dpp_step<kDppQuadSwap1>(b);
    dpp_step<kDppQuadSwap2>(b);
    dpp_step<kDppHalfMirror>(b);
    dpp_step<kDppMirror>(b);
    dpp_step<kDppRowBcast15, 0xa>(b);
    dpp_step<kDppRowBcast31, 0xc>(b);
    return rdl_best(b, 63);
}

template <int CTRL, int RM = 0xf>
__device__ __forceinline__ double dpp_max(double v) {
    return fmax(v, __longlong_as_double(dpp64<CTRL, RM>(__double_as_longlong(v))));
}

// The same result, cheaper in the usual case: the largest value alone goes
// through the butterflies (candidate values are finite, or -1 for none); if
// exactly one lane holds it, that lane's candidate wins, and ties go through
// the full (value, item, slot) reduction.
__device__ __forceinline__ Best wave_reduce(Best b) {
    double m = dpp_max<kDppQuadSwap1>(b.v);
    m = dpp_max<kDppQuadSwap2>(m);
    m = dpp_max<kDppHalfMirror>(m);
    m = dpp_max<kDppMirror>(m);
    m = dpp_max<kDppRowBcast15, 0xa>(m);
    m = dpp_max<kDppRowBcast31, 0xc>(m);
    const double top = __longlong_as_double(rdl64(__double_as_longlong(m), 63));
    const unsigned long long hold = __ballot(b.v == top);
    if (__popcll(hold) == 1) return rdl_best(b, __ffsll((long long)hold) - 1);
    return wave_reduce_full(b);
}

// Largest value over the wavefront, in every lane.
__device__ __forceinline__ double wave_max(double v) {
    v = dpp_max<kDppQuadSwap1>(v);
    v = dpp_max<kDppQuadSwap2>(v);
    v = dpp_max<kDppHalfMirror>(v);
    v = dpp_max<kDppMirror>(v);
    v = dpp_max<kDppRowBcast15, 0xa>(v);
    v = dpp_max<kDppRowBcast31, 0xc>(v);
    return __longlong_as_double(rdl64(__double_as_longlong(v), 63));
}

// Largest value over lanes 0..7, in every lane.
__device__ __forceinline__ double max8(double v) {
    v = dpp_max<kDppQuadSwap1>(v);
    v = dpp_max<kDppQuadSwap2>(v);
    v = dpp_max<kDppHalfMirror>(v);
    return __longlong_as_double(rdl64(__double_as_longlong(v), 0));
}

// The best two values of two disjoint candidate sets, merged: the lane's
// (m, m2) with those of the lane the DPP control names; a lane the row mask
// leaves unwritten merges with the empty set (-1, -1).
template <int CTRL, int RM = 0xf>
__device__ __forceinline__ void pair_step(double &m, double &m2) {
    constexpr int kNegOneHi = (int)0xBFF00000;  // high word of -1.0 (low word 0)
    const uint64_t a = (uint64_t)__double_as_longlong(m), a2 = (uint64_t)__double_as_longlong(m2);
    const int olo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)a, CTRL, RM, 0xf, false);
    const int ohi = __builtin_amdgcn_update_dpp(kNegOneHi, (int)(uint32_t)(a >> 32), CTRL, RM, 0xf, false);
    const int plo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)a2, CTRL, RM, 0xf, false);
    const int phi = __builtin_amdgcn_update_dpp(kNegOneHi, (int)(uint32_t)(a2 >> 32), CTRL, RM, 0xf, false);
    const double o = __longlong_as_double((long long)(((uint64_t)(uint32_t)ohi << 32) | (uint32_t)olo));
    const double o2 = __longlong_as_double((long long)(((uint64_t)(uint32_t)phi << 32) | (uint32_t)plo));
    m2 = fmax(fmax(m2, o2), fmin(m, o));
    m = fmax(m, o);
}

// wave_reduce, and the runner-up value of the wavefront (all lanes): the
// largest value among the lanes' candidates other than the winner, b2 being
// each lane's own runner-up (-1 for none).  Equal values count, so a tie
// leaves the runner-up equal to the winner's value.  The best two values
// travel through the butterflies together (the pair merge of disjoint sets
// is exact and order-free).
__device__ __forceinline__ Best wave_reduce2(Best b, double b2, double &v2) {
    double m = b.v, m2 = b2;
    pair_step<kDppQuadSwap1>(m, m2);
    pair_step<kDppQuadSwap2>(m, m2);
    pair_step<kDppHalfMirror>(m, m2);
    pair_step<kDppMirror>(m, m2);
    pair_step<kDppRowBcast15, 0xa>(m, m2);
    pair_step<kDppRowBcast31, 0xc>(m, m2);
    const double top = __longlong_as_double(rdl64(__double_as_longlong(m), 63));
    v2 = __longlong_as_double(rdl64(__double_as_longlong(m2), 63));
    const unsigned long long hold = __ballot(b.v == top);
    if (__popcll(hold) == 1) return rdl_best(b, __ffsll((long long)hold) - 1);
    return wave_reduce_full(b);
}

// The best two values over lanes 0..7 (others ignored), in every lane.
__device__ __forceinline__ void top2_8(double &m, double &m2) {
    pair_step<kDppQuadSwap1>(m, m2);
    pair_step<kDppQuadSwap2>(m, m2);
    pair_step<kDppHalfMirror>(m, m2);
    m = __longlong_as_double(rdl64(__double_as_longlong(m), 0));
    m2 = __longlong_as_double(rdl64(__double_as_longlong(m2), 0));
}

// The best two values over the wavefront, in every lane.
__device__ __forceinline__ void top2_wave(double &m, double &m2) {
    pair_step<kDppQuadSwap1>(m, m2);
    pair_step<kDppQuadSwap2>(m, m2);
    pair_step<kDppHalfMirror>(m, m2);
    pair_step<kDppMirror>(m, m2);
    pair_step<kDppRowBcast15, 0xa>(m, m2);
    pair_step<kDppRowBcast31, 0xc>(m, m2);
    m = __longlong_as_double(rdl64(__double_as_longlong(m), 63));
    m2 = __longlong_as_double(rdl64(__double_as_longlong(m2), 63));
}

// A candidate's value v, tracked with the runner-up b2 of the candidates seen
// so far (the largest value other than the best one; -1 for none).
__device__ __forceinline__ void consider2(Best &b, double &b2, double v, int64_t item, int slot) {
    b2 = fmax(b2, fmin(v, b.v));
    consider(b, v, item, slot);
}

// The relative gap (v1 - v2) / v1 between a decision's winner and runner-up
// (1 without a runner-up, 0 for a zero winner).
__device__ __forceinline__ double decision_gap(double v1, double v2) {
    if (v2 < 0.0) return 1.0;
    return v1 > 0.0 ? (v1 - v2) / v1 : 0.0;
}

// The same over lanes 0..7 only (the other lanes' values are ignored): the
// two quad swaps and the half-row mirror combine the first eight lanes.
__device__ __forceinline__ Best reduce8(Best b) {
    dpp_step<kDppQuadSwap1>(b);
    dpp_step<kDppQuadSwap2>(b);
    dpp_step<kDppHalfMirror>(b);
    return rdl_best(b, 0);
}

__device__ __forceinline__ int wave_or(int f) {
    f |= dpp32<kDppQuadSwap1>(f);
    f |= dpp32<kDppQuadSwap2>(f);
    f |= dpp32<kDppHalfMirror>(f);
    f |= dpp32<kDppMirror>(f);
    f |= dpp32<kDppRowBcast15, 0xa>(f);
    f |= dpp32<kDppRowBcast31, 0xc>(f);
    return __builtin_amdgcn_readlane(f, 63);
}

// Sort r <= 64 distinct indices in LDS ascending: every lane of one wave
// takes one entry, counts the entries below it with shuffles and stores it at
// its rank.
__device__ __forceinline__ void sort_set_wave(int64_t *a, int r) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t x = lane < r ? a[lane] : INT64_MAX;
    int rank = 0;
    for (int j = 0; j < r; j++) {
        const int64_t y = __shfl(x, j);
        rank += (y < x) || (y == x && j < lane);
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < r) a[rank] = x;
    __builtin_amdgcn_wave_barrier();
}

// Sort two sets of at most kBlock / 2 indices ascending at once (threads
// 0 .. kBlock/2 - 1 rank the first, the others the second; each entry goes
// to its rank, ties kept in order), staged through tmp (na + nb entries).
// Every thread of the workgroup calls.
__device__ __forceinline__ void sort_two_sets(int64_t *a, int na, int64_t *b, int nb, int64_t *tmp) {
    const int tid = threadIdx.x, half = kBlock / 2;
    const bool first = tid < half;
    const int t = first ? tid : tid - half, cnt = first ? na : nb;
    int64_t *set = first ? a : b;
    int64_t *out = first ? tmp : tmp + na;
    int64_t x = 0;
    int rank = 0;
    if (t < cnt) {
        x = set[t];
        for (int j = 0; j < cnt; j++) {
            const int64_t y = set[j];
            rank += (y < x) || (y == x && j < t);
        }
    }
    __syncthreads();
    if (t < cnt) out[rank] = x;
    __syncthreads();
    if (t < cnt) set[t] = out[t];
    __syncthreads();
}

// ---------------------------------------------------------------- entry sources
// Where the entries W[i][j] of one matrix come from: a dense row-major array
// (FP64, FP32 or BF16 as stored, converted to FP64), or, for far-field
// interaction blocks, evaluated on the fly from the two point sets as
// K_ij = 1 / |x_i - y_j| in FP64 (dx dx + dy dy, then a correctly rounded
// square root and division), so that no entry is ever stored.
template <typename T>
struct DenseSrc {
    const T *A;
    int64_t lda;
    __device__ __forceinline__ double operator()(int64_t i, int64_t j) const { return Elem<T>::load(A, i * lda + j); }
};
struct PointSrc {
    const double *x;  // row points, (x0, x1) pairs
    const double *y;  // column points
    __device__ __forceinline__ double operator()(int64_t i, int64_t j) const {
        const double dx = x[2 * i] - y[2 * j], dy = x[2 * i + 1] - y[2 * j + 1];
        return 1.0 / sqrt(dx * dx + dy * dy);
    }
};

// ---------------------------------------------------------------- nucleus
// U = G^{-1} for the generator G = W[I, J] of the sorted sets in sm.Iset and
// sm.Jset (Algorithm algcnnncl with k = l = r: the canonical nucleus is the
// inverse): LU with partial pivoting and column solves in the oracle's
// arithmetic, then `refine` steps X <- X + X (I - G X).  An exactly zero pivot,
// or pivot magnitudes spread by more than 1e14, selects the pseudo-inverse of
// G truncated at 1e-14 of its largest singular value (one-sided Jacobi).
// ws holds 4 r^2 doubles of LDS; every one of the workgroup's `nthreads`
// threads calls.
template <class SM, class Src>
__device__ __forceinline__ void nucleus(SM &sm, double *ws, const Src &src, int r, int refine, int nthreads,
                                        double *U_out) {
    const int tid = threadIdx.x;
    double *G = ws, *LU = ws + r * r, *X = ws + 2 * r * r, *X2 = ws + 3 * r * r;
    __shared__ int p[kRMax];
    for (int e = tid; e < r * r; e += nthreads) {
        const int a = e / r, b = e % r;
        const double v = src(sm.Iset[a], sm.Jset[b]);
        G[e] = v;
        LU[e] = v;
    }
    __syncthreads();
    __shared__ int sing;
    __shared__ double ld;
    // one wavefront for small r (no barriers); the whole workgroup for
    // larger r, where the single wavefront's solves are latency-bound (both
    // compute every entry with the same operations)
    if (r <= 24)
        inverse_wave(LU, X, p, r, &sing, &ld);
    else
        inverse_lds(LU, X, p, r, nthreads, &sing, &ld);
    // an exactly zero pivot, or pivot magnitudes spread by more than 1e14 (a
    // condition estimate from the same factors): truncated pseudo-inverse
    __shared__ int fallback;
    if (tid == 0) {
        int fb = sing;
        if (!sing) {
            double pmax = 0.0, pmin = INFINITY;
            for (int k = 0; k < r; k++) {
                const double a = fabs(LU[p[k] * r + k]);
                pmax = a > pmax ? a : pmax;
                pmin = a < pmin ? a : pmin;
            }
            fb = pmax > 1e14 * pmin;
        }
        fallback = fb;
    }
    __syncthreads();
    if (fallback) {
        __shared__ int rank;
        pinv_jacobi_lds(G, LU, X2, X, r, 1e-14, nthreads, &rank);
        if (tid == 0) {
            sm.nucleus_rank = rank;
            sm.logdet = (rank == r && !sing) ? ld : -INFINITY;
        }
        for (int e = tid; e < r * r; e += nthreads) U_out[e] = X[e];
        return;
    }
    if (tid == 0) sm.logdet = ld;
    for (int it = 0; it < refine; it++) {
        double *Tm = LU;  // T = I - G X
        for (int e = tid; e < r * r; e += nthreads) {
            const int i = e / r, j = e % r;
            double s = (i == j) ? 1.0 : 0.0;
#pragma unroll 4
            for (int q = 0; q < r; q++) s -= G[i * r + q] * X[q * r + j];
            Tm[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < r * r; e += nthreads) {
            const int i = e / r, j = e % r;
            double s = X[e];
#pragma unroll 4
            for (int q = 0; q < r; q++) s += X[i * r + q] * Tm[q * r + j];
            X2[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < r * r; e += nthreads) X[e] = X2[e];
        __syncthreads();
    }
    for (int e = tid; e < r * r; e += nthreads) U_out[e] = X[e];
}

// ---------------------------------------------------------------- truncated nucleus
// Sum over the 16 lanes of a DPP row, every lane receiving the same value:
// quad swaps, then the half-row and row mirrors pair equal partial sums, so
// each step adds the same two numbers (in either order) in every lane.
__device__ __forceinline__ double row_sum16(double v) {
    v += __longlong_as_double(dpp64<kDppQuadSwap1>(__double_as_longlong(v)));
    v += __longlong_as_double(dpp64<kDppQuadSwap2>(__double_as_longlong(v)));
    v += __longlong_as_double(dpp64<kDppHalfMirror>(__double_as_longlong(v)));
    v += __longlong_as_double(dpp64<kDppMirror>(__double_as_longlong(v)));
    return v;
}

// One-sided Jacobi (Hestenes) sweeps on the nc <= nr columns (length
// nr <= 16 RL, RL entries per lane) of A, column-major in LDS or global
// memory, accumulating the rotations in V (nc x nc, column-major, set to the
// identity by the caller): the oracle's round-robin
// pair order (a dummy position for odd nc), a pair rotated unless
// |a_p . a_q| <= nr eps sqrt(|a_p|^2 |a_q|^2), eps = 2^-52, or a column is
// negligible (|a|^2 <= (nr eps)^2 times the largest squared column norm at
// the sweep's start), or the sine is zero; sweeps until none rotates, at most
// 60.  Each pair runs on the 16 lanes of a DPP row.  On return the columns of
// A = A_in V are orthogonal; returns the number of sweeps run.  pair_floor >
// 0 also leaves alone a pair whose two squared norms are both at most
// pair_floor times that largest one (for callers that need only the dominant
// columns).  One workgroup of kBlock threads, every thread calls.
template <int RL = kRMax / 16>
__device__ __forceinline__ int jacobi_sweeps(double *A, double *V, int nr, int nc, double pair_floor = 0.0) {
    const int tid = threadIdx.x;
    __shared__ int s_rot;
    __shared__ double s_nrm[16 * RL];
    __shared__ double s_big;
    const int lp = nc + (nc & 1);
    const int grp = tid / 16, j = tid % 16, ngrp = kBlock / 16;
    const double tol = (double)nr * 0x1p-52;
    int sweep = 0;
    for (; sweep < 60 && nc > 1; sweep++) {
        // squared column norms, then their maximum
        for (int c = grp; c < nc; c += ngrp) {
            double s2 = 0.0;
#pragma unroll
            for (int u = 0; u < RL; u++) {
                const int i = j + 16 * u;
                const double x = i < nr ? A[c * nr + i] : 0.0;
                s2 += x * x;
            }
            s2 = row_sum16(s2);
            if (j == 0) s_nrm[c] = s2;
        }
        if (tid == 0) s_rot = 0;
        __syncthreads();
        if (tid == 0) {
            double bg = 0.0;
            for (int c = 0; c < nc; c++) bg = s_nrm[c] > bg ? s_nrm[c] : bg;
            s_big = bg;
        }
        __syncthreads();
        const double negl = tol * tol * s_big, small = pair_floor * s_big;
        for (int t = 0; t < lp - 1; t++) {
            for (int pr = grp; pr < lp / 2; pr += ngrp) {
                int pc, qc;
                jacobi_pair(t, pr, lp, pc, qc);
                if (qc >= nc) continue;
                const double *ap = A + pc * nr, *aq = A + qc * nr;
                double x[RL], y[RL];
#pragma unroll
                for (int u = 0; u < RL; u++) {
                    const int i = j + 16 * u;
                    x[u] = i < nr ? ap[i] : 0.0;
                    y[u] = i < nr ? aq[i] : 0.0;
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
                    if (i < nr) {
                        A[pc * nr + i] = cs * x[u] - sn * y[u];
                        A[qc * nr + i] = sn * x[u] + cs * y[u];
                    }
                }
                double vx[RL], vy[RL];
#pragma unroll
                for (int u = 0; u < RL; u++) {
                    const int i = j + 16 * u;
                    vx[u] = i < nc ? V[pc * nc + i] : 0.0;
                    vy[u] = i < nc ? V[qc * nc + i] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < RL; u++) {
                    const int i = j + 16 * u;
                    if (i < nc) {
                        V[pc * nc + i] = cs * vx[u] - sn * vy[u];
                        V[qc * nc + i] = sn * vx[u] + cs * vy[u];
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
    return nc > 1 ? (sweep < 60 ? sweep + 1 : 60) : 0;
}

// Nucleus of a k x l generator (Algorithm algcnnncl): U = G_r^+, the
// pseudo-inverse of G's rank-r SVD truncation, G = src(I[a], J[b]).
// One-sided Jacobi on the nc = min(k, l) columns (length nr = max(k, l)) of
// G, or of G^T when G is wide, in the oracle's round-robin order (a dummy
// position for odd nc; a pair rotated unless |a_p . a_q| <= nr eps
// sqrt(|a_p|^2 |a_q|^2), eps = 2^-52, or a column is negligible, |a|^2 <=
// (nr eps)^2 times the largest squared column norm at the sweep's start, or
// the sine is zero; sweeps until none rotates, at most 60), each pair on
// the 16 lanes of a DPP row; then the r largest sigma_j
// above max(1e-14, nr eps) max sigma (ties to the lower j) are kept.  With B = A V
// rotated: U = sum over kept j of v_j b_j^T / sigma_j^2 (G tall) or
// b_j v_j^T / sigma_j^2 (G wide), l x k row-major.  ws: nr nc + nc^2
// doubles, column-major, so that a pair's lanes read consecutive entries.
// sm.nucleus_rank = the number kept, sm.logdet = the sum of their logs.
// dl, dr: the generator is taken as (dl G) dr entrywise and U returned as
// (dr U) dl, the scalar rescalings Dbar, D of a CUR by sampling; dla / dra
// (optional) give one factor per row of G and per column instead.  RL: rows
// per lane of the rotations, max(k, l) <= 16 RL; ws may lie in LDS or in
// global memory.  One workgroup, every thread calls.
template <int RL = kRMax / 16, class SM, class Src>
__device__ __forceinline__ void nucleus_trunc(SM &sm, double *ws, const Src &src, int k, int l, int r,
                                              double *U_out, double dl = 1.0, double dr = 1.0,
                                              const double *dla = nullptr, const double *dra = nullptr) {
    const int tid = threadIdx.x;
    const bool wide = k < l;
    const int nr = wide ? l : k, nc = wide ? k : l;
    double *A = ws, *V = ws + nr * nc;
    __shared__ double s_sig[16 * RL];
    __shared__ int s_keep[16 * RL];
    for (int e = tid; e < nr * nc; e += kBlock) {
        const int i = e % nr, c = e / nr;
        const int ia = wide ? c : i, jb = wide ? i : c;  // row (I) and column (J) of the entry
        A[e] = ((dla ? dla[ia] : dl) * src(sm.Iset[ia], sm.Jset[jb])) * (dra ? dra[jb] : dr);
    }
    for (int e = tid; e < nc * nc; e += kBlock) V[e] = (e / nc == e % nc) ? 1.0 : 0.0;
    __syncthreads();
    jacobi_sweeps<RL>(A, V, nr, nc);
    for (int c = tid; c < nc; c += kBlock) {
        double s2 = 0.0;
        for (int i = 0; i < nr; i++) s2 += A[c * nr + i] * A[c * nr + i];
        s_sig[c] = sqrt(s2);
    }
    __syncthreads();
    if (tid < nc) {
        double smax = 0.0;
        int above = 0;
        for (int c = 0; c < nc; c++) {
            smax = s_sig[c] > smax ? s_sig[c] : smax;
            above += (s_sig[c] > s_sig[tid] || (s_sig[c] == s_sig[tid] && c < tid)) ? 1 : 0;
        }
        // rank tolerance max(1e-14, max(k, l) eps): never below the level at
        // which the rotation test leaves a column as negligible
        const double thr = fmax(1e-14, (double)nr * 0x1p-52);
        s_keep[tid] = (above < r && s_sig[tid] > thr * smax) ? 1 : 0;
    }
    __syncthreads();
    if (tid == 0) {
        int kept = 0;
        double lv = 0.0;
        for (int c = 0; c < nc; c++)
            if (s_keep[c]) {
                kept++;
                lv += log(s_sig[c]);
            }
        sm.nucleus_rank = kept;
        sm.logdet = lv;
    }
    for (int e = tid; e < l * k; e += kBlock) {
        const int a = e / k, bb = e % k;
        double acc = 0.0;
        for (int c = 0; c < nc; c++)
            if (s_keep[c])
                acc += (wide ? A[c * nr + a] * V[c * nc + bb] : V[c * nc + a] * A[c * nr + bb]) /
                       (s_sig[c] * s_sig[c]);
        U_out[e] = ((dra ? dra[a] : dr) * acc) * (dla ? dla[bb] : dl);
    }
    __syncthreads();
}

}  // namespace lra
