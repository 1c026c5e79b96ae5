// lra_device.h -- device helpers shared by the library's kernels: exact
// element upcast, the SplitMix64 counter generator and the wave-level
// distinct draw.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lra {

constexpr int kWave = 64;
constexpr int kInvChunk = 8;

// ---------------------------------------------------------------- elements
// load(): the entry at offset o as FP64; conv(): the same upcast of a raw
// value already in a register (BF16 is carried as its 16-bit pattern).
template <typename T> struct Elem;
template <> struct Elem<double> {
    static __device__ __forceinline__ double conv(double v) { return v; }
    static __device__ __forceinline__ double load(const double *p, int64_t o) { return p[o]; }
};
template <> struct Elem<float> {
    static __device__ __forceinline__ double conv(float v) { return (double)v; }
    static __device__ __forceinline__ double load(const float *p, int64_t o) { return (double)p[o]; }
};
template <> struct Elem<uint16_t> {
    static __device__ __forceinline__ double conv(uint16_t v) { return (double)__uint_as_float(((uint32_t)v) << 16); }
    static __device__ __forceinline__ double load(const uint16_t *p, int64_t o) { return conv(p[o]); }
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
__device__ __forceinline__ void draw_distinct_wave(uint64_t seed, uint64_t stream, int64_t n, int k, int64_t *out) {
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
            // candidate t of this round, read out of its lane (t is uniform)
            const int okt = __builtin_amdgcn_readlane(ok, t);
            const int64_t vt = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)((uint64_t)v >> 32), t)
                                          << 32) |
                                         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, t));
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



// ---------------------------------------------------------------- DPP argmax
// Argmax over a wavefront of (value, key) pairs: largest value, then lowest
// key; also returns the winning lane.  Four DPP butterflies (quad swaps,
// half-row and row mirrors) leave each 16-lane row with its best, then the
// four rows are combined from uniform read-outs.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int64_t b = __double_as_longlong(v);
    const int lo = dpp_i32<CTRL>((int)(uint32_t)b), hi = dpp_i32<CTRL>((int)(uint32_t)((uint64_t)b >> 32));
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double rdl_f64(double v, int lane) {
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)b >> 32), lane);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
struct KeyMax {
    double v;
    int key, who;
};
__device__ __forceinline__ bool key_better(double v1, int k1, double v2, int k2) {
    return v1 > v2 || (v1 == v2 && k1 < k2);
}
template <int CTRL>
__device__ __forceinline__ void keymax_step(KeyMax &b) {
    const double ov = dpp_f64<CTRL>(b.v);
    const int ok = dpp_i32<CTRL>(b.key), ow = dpp_i32<CTRL>(b.who);
    if (key_better(ov, ok, b.v, b.key)) b = KeyMax{ov, ok, ow};
}
__device__ __forceinline__ KeyMax wave_keymax(KeyMax b) {
    keymax_step<0xB1>(b);    // quad_perm [1,0,3,2]
    keymax_step<0x4E>(b);    // quad_perm [2,3,0,1]
    keymax_step<0x141>(b);   // row half mirror
    keymax_step<0x140>(b);   // row mirror
    KeyMax r{rdl_f64(b.v, 0), __builtin_amdgcn_readlane(b.key, 0), __builtin_amdgcn_readlane(b.who, 0)};
#pragma unroll
    for (int row = 1; row < 4; row++) {
        const KeyMax o{rdl_f64(b.v, 16 * row), __builtin_amdgcn_readlane(b.key, 16 * row),
                       __builtin_amdgcn_readlane(b.who, 16 * row)};
        if (key_better(o.v, o.key, r.v, r.key)) r = o;
    }
    return r;
}

// Inverse of an r x r matrix (r <= 64) held in LDS, with the arithmetic of
// the oracle's routine entry for entry: LU with partial pivoting (largest
// magnitude, ties to the lowest original row), then for each column c of the
// inverse L y = P e_c and U x = y.
//  * pivot search: wave 0, one lane per permutation position (DPP argmax);
//  * elimination of step k: 8 consecutive lanes per trailing row (one
//    wavefront reads the row's entry k before its first lane stores the
//    multiplier there);
//  * forward solve, column-oriented: after y_j is final every later row
//    subtracts L_ij y_j, so each row still subtracts its terms in increasing j;
//  * backward solve: one thread per column, the oracle's row order.
// LU holds G on entry and the factors on exit (rows in original order, p the
// permutation), X receives G^{-1}.  *sing_out = 1 if a pivot is exactly zero
// (X is then not written); *logdet = log |det G|.  Every thread of the block
// (nthreads, a multiple of 64) must call.
__device__ __forceinline__ void inverse_lds(double *LU, double *X, int *p, int r, int nthreads, int *sing_out,
                                            double *logdet) {
    const int tid = threadIdx.x;
    __shared__ double s_pk;
    if (tid < r) p[tid] = tid;
    if (tid == 0) {
        *sing_out = 0;
        *logdet = 0.0;
    }
    __syncthreads();
    for (int k = 0; k < r; k++) {
        if (tid < kWave) {
            const int lane = tid;
            const bool cand = lane >= k && lane < r;
            const int pl = lane < r ? p[lane] : 0x7fffffff;
            KeyMax c{cand ? fabs(LU[pl * r + k]) : -1.0, cand ? pl : 0x7fffffff, lane};
            c = wave_keymax(c);
            if (lane == 0) {
                if (c.v == 0.0) {
                    *sing_out = 1;
                } else {
                    const int pk_row = p[c.who];
                    p[c.who] = p[k];
                    p[k] = pk_row;
                    s_pk = LU[pk_row * r + k];
                    *logdet += log(fabs(s_pk));
                }
            }
        }
        __syncthreads();
        if (*(volatile int *)sing_out) return;
        const double pk = s_pk;
        const int pr = p[k];
        for (int q = tid; q < (r - k - 1) * 8; q += nthreads) {
            const int i = k + 1 + q / 8, t = q % 8;
            const int pi = p[i];
            const double l = LU[pi * r + k] / pk;
            for (int j = k + 1 + t; j < r; j += 8) LU[pi * r + j] -= l * LU[pr * r + j];
            if (t == 0) LU[pi * r + k] = l;
        }
        __syncthreads();
    }
    // forward: X[i][c] = (p_i == c) - sum_{j < i} L[p_i][j] X[j][c], column-oriented
    const int c = tid % kWave, rg = tid / kWave, ng = nthreads / kWave;
    if (c < r)
        for (int i = rg; i < r; i += ng) X[i * r + c] = (p[i] == c) ? 1.0 : 0.0;
    __syncthreads();
    for (int j = 0; j < r - 1; j++) {
        if (c < r) {
            const double xj = X[j * r + c];
            for (int i = j + 1 + rg; i < r; i += ng) X[i * r + c] -= LU[p[i] * r + j] * xj;
        }
        __syncthreads();
    }
    // backward: x_i = (y_i - sum_{j > i} U[p_i][j] x_j) / U[p_i][i], j increasing
    for (int cc = tid; cc < r; cc += nthreads) {
        for (int ii = r - 1; ii >= 0; ii--) {
            const int pi = p[ii];
            double sum = X[ii * r + cc];
            for (int j0 = ii + 1; j0 < r; j0 += kInvChunk) {
                double a[kInvChunk], x[kInvChunk];
#pragma unroll
                for (int u = 0; u < kInvChunk; u++) {
                    const int j = min(j0 + u, r - 1);
                    a[u] = LU[pi * r + j];
                    x[u] = X[j * r + cc];
                }
#pragma unroll
                for (int u = 0; u < kInvChunk; u++) sum -= (j0 + u < r) ? a[u] * x[u] : 0.0;
            }
            X[ii * r + cc] = sum / LU[pi * r + ii];
        }
    }
    __syncthreads();
}

// The inverse of inverse_lds, every entry computed by the same operations in
// the same order, run by wavefront 0 alone (lockstep, so no barriers; the
// other wavefronts return at once and the caller synchronizes): lane i holds
// permutation position i, the pivot search is a DPP argmax over the lanes,
// lane i eliminates row p_i, and lane c solves column c of the inverse
// (forward: X[i][c] takes its terms in increasing j; backward: x_i =
// (y_i - sum_{j > i} U[p_i][j] x_j) / U[p_i][i] with j increasing).  LDS
// accesses of one wavefront complete in program order.  r <= 64.
__device__ __forceinline__ void inverse_wave(double *LU, double *X, int *p, int r, int *sing_out, double *logdet) {
    if (threadIdx.x >= kWave) return;
    const int lane = threadIdx.x;
    int pi = lane;  // row at permutation position `lane`
    double ld = 0.0;
    int sing = 0;
    for (int k = 0; k < r; k++) {
        const bool cand = lane >= k && lane < r;
        KeyMax c{cand ? fabs(LU[pi * r + k]) : -1.0, cand ? pi : 0x7fffffff, lane};
        c = wave_keymax(c);
        if (c.v == 0.0) {
            sing = 1;
            break;
        }
        const int pw = __builtin_amdgcn_readlane(pi, c.who), pkr = __builtin_amdgcn_readlane(pi, k);
        pi = (lane == k) ? pw : (lane == c.who ? pkr : pi);
        const double pk = LU[pw * r + k];
        ld += log(fabs(pk));
        __builtin_amdgcn_wave_barrier();
        if (lane > k && lane < r) {
            const double l = LU[pi * r + k] / pk;
            for (int j = k + 1; j < r; j++) LU[pi * r + j] -= l * LU[pw * r + j];
            LU[pi * r + k] = l;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (lane < r) p[lane] = pi;
    if (lane == 0) {
        *sing_out = sing;
        *logdet = ld;
    }
    if (sing) return;
    __builtin_amdgcn_wave_barrier();
    // forward, column c by lane c: X[i][c] = (p_i == c) - sum_{j < i} L[p_i][j] X[j][c]
    if (lane < r) {
        const int c = lane;
        for (int i = 0; i < r; i++) X[i * r + c] = (p[i] == c) ? 1.0 : 0.0;
        for (int j = 0; j < r - 1; j++) {
            const double xj = X[j * r + c];
            for (int i = j + 1; i < r; i++) X[i * r + c] -= LU[p[i] * r + j] * xj;
        }
        // backward: x_i = (y_i - sum_{j > i} U[p_i][j] x_j) / U[p_i][i], j increasing
        for (int ii = r - 1; ii >= 0; ii--) {
            const int q = p[ii];
            double sum = X[ii * r + c];
            for (int j = ii + 1; j < r; j++) sum -= LU[q * r + j] * X[j * r + c];
            X[ii * r + c] = sum / LU[q * r + ii];
        }
    }
}

// k i.i.d. draws from [0, n) with replacement, in draw order: the accepted
// outputs of the stream (the top 2^64 mod n words rejected), reduced mod n.
// Run by all 64 lanes of one wave: 64 counters are hashed at once and the
// accepted ones placed by their rank among the round's accepted lanes.
__device__ __forceinline__ void draw_uniform_wave(uint64_t seed, uint64_t stream, int64_t n, int k, int64_t *out) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t un = (uint64_t)n;
    const uint64_t rem = (0 - un) % un;
    const uint64_t lim = 0 - rem;
    int got = 0;
    uint64_t ctr = 0;
    while (got < k) {
        const uint64_t u = sm64(seed, stream, ctr + (uint64_t)lane);
        const bool ok = !(rem != 0 && u >= lim);
        const uint64_t acc = __ballot(ok);
        const int pos = got + __popcll(acc & ((1ull << lane) - 1ull));
        if (ok && pos < k) out[pos] = (int64_t)(u % un);
        got += __popcll(acc);
        ctr += kWave;
    }
}

// Truncated pseudo-inverse by one-sided Jacobi SVD, the rule of the
// oracle's routine: columns of A = G rotated in round-robin pair order
// (position 0 fixed, the others rotating, a dummy position for odd r), a pair
// rotated unless |a_p . a_q| <= 1e-15 sqrt(|a_p|^2 |a_q|^2), sweeps until one
// applies no rotation (at most 60); then X = sum over sigma_j > rtol max sigma
// of v_j a_j^T / sigma_j^2.  Each pair is handled by 16 lanes (its three dot
// products summed as a butterfly, so rounding differs from the oracle's
// sequential sums).  G, A, V, X: r x r in LDS (A and V are work space).
// Every thread of the block (nthreads, a multiple of 64) must call; r <= 64.
__device__ __forceinline__ void jacobi_pair(int t, int k, int rp, int &p, int &q) {
    const int a = (k == 0) ? 0 : ((k - 1 + t) % (rp - 1)) + 1;
    const int kk = rp - 1 - k;
    const int b = ((kk - 1 + t) % (rp - 1)) + 1;
    p = a < b ? a : b;
    q = a < b ? b : a;
}

__device__ __forceinline__ double sum16(double v) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ void pinv_jacobi_lds(const double *G, double *A, double *V, double *X, int r, double rtol,
                                                int nthreads, int *rank_out) {
    const int tid = threadIdx.x;
    __shared__ int s_rot;
    __shared__ double s_sig[64];
    for (int e = tid; e < r * r; e += nthreads) {
        A[e] = G[e];
        V[e] = (e / r == e % r) ? 1.0 : 0.0;
    }
    const int rp = r + (r & 1);
    const int grp = tid / 16, j = tid % 16, ngrp = nthreads / 16;
    for (int sweep = 0; sweep < 60 && r > 1; sweep++) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int t = 0; t < rp - 1; t++) {
            for (int k = grp; k < rp / 2; k += ngrp) {
                int pc, qc;
                jacobi_pair(t, k, rp, pc, qc);
                if (qc >= r) continue;  // paired with the padding position
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = j; i < r; i += 16) {
                    const double x = A[i * r + pc], y = A[i * r + qc];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                al = sum16(al);
                be = sum16(be);
                ga = sum16(ga);
                if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
                const double ze = (be - al) / (2.0 * ga);
                const double tt = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
                const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
                for (int i = j; i < r; i += 16) {
                    double x = A[i * r + pc], y = A[i * r + qc];
                    A[i * r + pc] = c * x - sn * y;
                    A[i * r + qc] = sn * x + c * y;
                    x = V[i * r + pc];
                    y = V[i * r + qc];
                    V[i * r + pc] = c * x - sn * y;
                    V[i * r + qc] = sn * x + c * y;
                }
                if (j == 0) s_rot = 1;
            }
            __syncthreads();
        }
        const int rot = *(volatile int *)&s_rot;
        __syncthreads();
        if (!rot) break;
    }
    for (int c = tid; c < r; c += nthreads) {
        double s2 = 0.0;
        for (int i = 0; i < r; i++) s2 += A[i * r + c] * A[i * r + c];
        s_sig[c] = sqrt(s2);
    }
    __syncthreads();
    double smax = 0.0;
    int rank = 0;
    for (int c = 0; c < r; c++) smax = s_sig[c] > smax ? s_sig[c] : smax;
    for (int c = 0; c < r; c++) rank += s_sig[c] > rtol * smax ? 1 : 0;
    for (int e = tid; e < r * r; e += nthreads) {
        const int a = e / r, b = e % r;
        double acc = 0.0;
        for (int c = 0; c < r; c++)
            if (s_sig[c] > rtol * smax) acc += V[a * r + c] * A[b * r + c] / (s_sig[c] * s_sig[c]);
        X[e] = acc;
    }
    if (tid == 0) *rank_out = rank;
    __syncthreads();
}

}  // namespace lra
