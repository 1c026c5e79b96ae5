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



// Inverse of an r x r matrix (r <= 64) held in LDS: LU with partial pivoting
// (largest magnitude, ties to the lowest row) in wave 0, then one column
// solve per thread, in the order of the oracle's routine.  LU holds G on entry
// and the factors on exit, X receives G^{-1}, p (LDS, r ints) the row order.
// *sing_out = 1 if a pivot is exactly zero (X is then not written);
// *logdet = log |det G|.  Every thread of the block must call.
__device__ __forceinline__ void inverse_lds(double *LU, double *X, int *p, int r, int nthreads, int *sing_out,
                                            double *logdet) {
    const int tid = threadIdx.x;
    __syncthreads();
    // LU with partial pivoting in wave 0: lane i works on the row at position
    // i of the permutation (its original index held in register pi).
    if (tid < kWave) {
        const int lane = tid;
        int pi = lane;
        double ld = 0.0;
        int sing = 0;
        for (int k = 0; k < r; k++) {
            const bool cand = lane >= k && lane < r;
            double a = cand ? fabs(LU[pi * r + k]) : -1.0;
            int key = cand ? pi : 0x7fffffff, who = lane;
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) {
                const double oa = __shfl_xor(a, off);
                const int ok = __shfl_xor(key, off), ow = __shfl_xor(who, off);
                if (oa > a || (oa == a && ok < key)) {
                    a = oa;
                    key = ok;
                    who = ow;
                }
            }
            if (a == 0.0) {  // largest magnitude ties go to the lowest row
                sing = 1;
                break;
            }
            const int p_k = __shfl(pi, k), p_w = __shfl(pi, who);
            if (lane == k) pi = p_w;
            else if (lane == who) pi = p_k;
            ld += log(a);
            const int prow = p_w;
            const double piv = LU[prow * r + k];
            __builtin_amdgcn_wave_barrier();
            if (lane > k && lane < r) {
                const double l = LU[pi * r + k] / piv;
                LU[pi * r + k] = l;
                for (int j0 = k + 1; j0 < r; j0 += kInvChunk) {
                    double av[kInvChunk], uv[kInvChunk];
#pragma unroll
                    for (int u = 0; u < kInvChunk; u++) {
                        const int j = min(j0 + u, r - 1);  // past the end: repeat entry r-1
                        av[u] = LU[pi * r + j];
                        uv[u] = LU[prow * r + j];
                    }
#pragma unroll
                    for (int u = 0; u < kInvChunk; u++) LU[pi * r + min(j0 + u, r - 1)] = av[u] - l * uv[u];
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (lane < r) p[lane] = pi;
        if (lane == 0) {
            *sing_out = sing;
            *logdet = ld;
        }
    }
    __syncthreads();
    if (*(volatile int *)sing_out) return;
    // column c of G^{-1}: L y = P e_c, U x = y (stored in column c of X)
    for (int c = tid; c < r; c += nthreads) {
        for (int i = 0; i < r; i++) {
            const int pi = p[i];
            double s = (pi == c) ? 1.0 : 0.0;
            for (int j0 = 0; j0 < i; j0 += kInvChunk) {
                double a[kInvChunk], x[kInvChunk];
#pragma unroll
                for (int u = 0; u < kInvChunk; u++) {
                    const int j = min(j0 + u, i - 1);
                    a[u] = LU[pi * r + j];
                    x[u] = X[j * r + c];
                }
#pragma unroll
                for (int u = 0; u < kInvChunk; u++) s -= (j0 + u < i) ? a[u] * x[u] : 0.0;
            }
            X[i * r + c] = s;
        }
        for (int i = r - 1; i >= 0; i--) {
            const int pi = p[i];
            double s = X[i * r + c];
            for (int j0 = i + 1; j0 < r; j0 += kInvChunk) {
                double a[kInvChunk], x[kInvChunk];
#pragma unroll
                for (int u = 0; u < kInvChunk; u++) {
                    const int j = min(j0 + u, r - 1);
                    a[u] = LU[pi * r + j];
                    x[u] = X[j * r + c];
                }
#pragma unroll
                for (int u = 0; u < kInvChunk; u++) s -= (j0 + u < r) ? a[u] * x[u] : 0.0;
            }
            X[i * r + c] = s / LU[pi * r + i];
        }
    }
    __syncthreads();
}

}  // namespace lra
