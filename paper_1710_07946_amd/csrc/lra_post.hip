// lra_post.hip -- kernels that use a computed CUR: the residual moments of
// E = W - C U R (full, or a random q x s sample for the a-posteriori
// estimate), and the adjoint of the CUR reconstruction at fixed index sets.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lra_device.h"
#include "lra_internal.h"

namespace lra {


// ------------------------------------------------------------------ residual
// E = W[rows, cols] - Cg Z with Cg = W[rows, J] (nq x r) and Z = U W[I, cols]
// (r x ns), zero-padded along the rank to rp.  The product runs on the
// matrix cores: FP64 MFMA for the plain path, three BF16 MFMAs of a hi/lo
// split with FP32 accumulation for the mixed path.  A workgroup of 8 waves
// owns 128 rows (16 per wave, whose Cg part stays in registers) and a range
// of columns, walked in chunks of CH columns, two 16-column tiles at a time
// (two independent accumulator chains per wave).  The loop is
// software-pipelined: while chunk c is multiplied out of one LDS buffer, the
// W entries and the Z slice of chunk c + 1 are already in flight into
// registers, and the Z slice goes to the other LDS buffer afterwards.  Every
// lane keeps FP64 partial sums of e, e^2, |e| and w^2.
constexpr int kResThreads = 512;
constexpr int kResWaves = kResThreads / 64;
constexpr int kResRows = 16 * kResWaves;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Sample rows (stream 3) and columns (stream 4) of E, q, s <= 256.
__global__ void resid_sample_kernel(uint64_t seed, int64_t m, int64_t n, int q, int s, int64_t *rows,
                                    int64_t *cols) {
    if (threadIdx.x < kWave) draw_distinct_wave(seed, 3, m, q, rows);
    else if (threadIdx.x < 2 * kWave) draw_distinct_wave(seed, 4, n, s, cols);
}

// Split an FP64 value into BF16 hi + lo (x ~ hi + lo to about 2^-17 relative),
// returned as their 16-bit patterns.
__device__ __forceinline__ void split_bf16(double x, uint16_t &hi, uint16_t &lo) {
    const __bf16 h = (__bf16)(float)x;
    const __bf16 l = (__bf16)(float)(x - (double)(float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
}

// Z[a][c] = sum_b U[a][b] W[I[b]][col c] for a < r (b in increasing order),
// zero for r <= a < rp; 64 columns per workgroup, the W[I, cols] slice and U
// staged in LDS.  An index of I outside [0, m) makes its column NaN.  Plain:
// Z is FP64 [rp][ns].  Mixed: Z is split into BF16 hi and lo patterns stored
// column-major [ns][rp] (a column's rank entries contiguous).
template <typename T>
__global__ void __launch_bounds__(256) resid_z_kernel(const T *A, int64_t m, int64_t lda, int r, int rp,
                                                      const int64_t *I, const double *U, const int64_t *cols,
                                                      int64_t ns, int mixed, double *Z, uint16_t *Zhi,
                                                      uint16_t *Zlo) {
    __shared__ double us[kRMax * kRMax];
    __shared__ double wg[kRMax * 64];
    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    for (int e = tid; e < r * r; e += 256) us[e] = U[e];
    for (int e = tid; e < r * 64; e += 256) {
        const int b = e >> 6;
        const int64_t c = c0 + (e & 63);
        const int64_t i = I[b];
        double v = 0.0;
        if (c < ns) v = (i >= 0 && i < m) ? Elem<T>::load(A, i * lda + (cols ? cols[c] : c)) : __builtin_nan("");
        wg[e] = v;
    }
    __syncthreads();
    const int c = tid & 63;
    const int64_t col = c0 + c;
    if (col >= ns) return;
    for (int a = tid >> 6; a < rp; a += 4) {
        double acc = 0.0;
        if (a < r)
            for (int b = 0; b < r; b++) acc += us[a * r + b] * wg[b * 64 + c];
        if (mixed) split_bf16(acc, Zhi[col * rp + a], Zlo[col * rp + a]);
        else Z[(int64_t)a * ns + col] = acc;
    }
}

// Cg[i][a] = W[rows[i]][J[a]] for a < r, zero for r <= a < rp (nq x rp).
template <typename T>
__global__ void resid_c_kernel(const T *A, int64_t n, int64_t lda, int r, int rp, const int64_t *J,
                               const int64_t *rows, int64_t nq, double *Cg) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nq * rp) return;
    const int64_t i = e / rp;
    const int a = (int)(e % rp);
    double v = 0.0;
    if (a < r) {
        const int64_t j = J[a];
        v = (j >= 0 && j < n) ? Elem<T>::load(A, (rows ? rows[i] : i) * lda + j) : __builtin_nan("");
    }
    Cg[e] = v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// The product is formed transposed, E^T tile = Z^T Cg^T, so that the four
// outputs of a lane are four consecutive columns of one row (one vector load
// of W per tile).  Output v of lane l in a 16 x 16 tile: row l % 16,
// column 4 (l / 16) + v.

// Plain core: FP64 MFMA 16x16x4 (A operand of lane l: A[l % 16][l / 16], B
// operand: B[l / 16][l % 16], output v: D[l / 16 + 4 v][l % 16]).  B = the
// lane's Cg row, held in registers: Cg[row0 + l % 16][4 s + l / 16].  A = Z^T
// with its 16 rows permuted so that output row l / 16 + 4 v is column
// 4 (l / 16) + v: lane l reads Z[4 s + l / 16][4 (l % 4) + (l % 16) / 4].
// KMAX = upper bound of rp / 4.
template <int KMAX, int CH>
struct F64Core {
    typedef double Acc;                                     // arithmetic of the epilogue
    static constexpr int kStride = CH + 16;                 // doubles per staged Z row
    static constexpr int kLdsBytes = 4 * KMAX * kStride * 8;
    static constexpr int kZU = (4 * KMAX * CH + kResThreads - 1) / kResThreads;
    double bf[KMAX];
    double zr[kZU];
    int ks;
    __device__ __forceinline__ void load_cg(const double *Cg, int rp, int64_t row0, int64_t nq, int lane) {
        ks = rp / 4;
        const int64_t row = row0 + (lane & 15);
#pragma unroll
        for (int s = 0; s < KMAX; s++) bf[s] = (s < ks && row < nq) ? Cg[row * rp + 4 * s + (lane >> 4)] : 0.0;
    }
    __device__ __forceinline__ void fetch_z(const double *Zg, const uint16_t *, const uint16_t *, int64_t ns, int rp,
                                            int64_t c0, int64_t cend, int tid) {
#pragma unroll
        for (int u = 0; u < kZU; u++) {
            const int e = tid + u * kResThreads;
            const int k = e / CH, c = e % CH;
            zr[u] = (k < rp && c0 + c < cend) ? Zg[(int64_t)k * ns + c0 + c] : 0.0;
        }
    }
    __device__ __forceinline__ void store_z(char *lds, int tid) {
        double *z = reinterpret_cast<double *>(lds);
#pragma unroll
        for (int u = 0; u < kZU; u++) {
            const int e = tid + u * kResThreads;
            if (e < 4 * KMAX * CH) z[(e / CH) * kStride + e % CH] = zr[u];
        }
    }
    // tiles t and t + 1 of the chunk
    __device__ __forceinline__ void tile2(const char *lds, int t, int lane, Acc (&x)[2][4]) const {
        const double *z = reinterpret_cast<const double *>(lds) + (lane >> 4) * kStride + 16 * t +
                          4 * (lane & 3) + ((lane & 15) >> 2);
        v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KMAX; s++) {
            if (s < ks) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(z[4 * s * kStride], bf[s], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(z[4 * s * kStride + 16], bf[s], acc1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; v++) {
            x[0][v] = acc0[v];
            x[1][v] = acc1[v];
        }
    }
};

// Mixed core: BF16 MFMA 16x16x32 with FP32 accumulation on a hi/lo split of
// both factors (lo*hi + hi*lo + hi*hi; lo*lo is dropped).  A operand of lane
// l: A[l % 16][8 (l / 16) + e], e = 0..7; B operand: B[8 (l / 16) + e][l % 16];
// output v: D[4 (l / 16) + v][l % 16].  A = Z^T read from the staged slice,
// which is column-major (hi, then lo) so that a lane's eight rank entries are
// one 16-byte read; B = the lane's Cg row in registers.
template <int KS, int CH>
struct Bf16x3Core {
    typedef float Acc;                                       // arithmetic of the epilogue
    static constexpr int kCol = 32 * KS + 8;                 // bf16 per staged column (16-byte pad)
    static constexpr int kHalf = CH * kCol;                  // bf16 per half (hi or lo)
    static constexpr int kLdsBytes = 2 * kHalf * 2;
    static constexpr int kVec = CH * 32 * KS / 8;            // 16-byte vectors per half
    static constexpr int kZU = (2 * kVec + kResThreads - 1) / kResThreads;
    v8bf bhi[KS], blo[KS];
    v4u zr[kZU];
    __device__ __forceinline__ void load_cg(const double *Cg, int rp, int64_t row0, int64_t nq, int lane) {
        const int64_t row = row0 + (lane & 15);
#pragma unroll
        for (int s = 0; s < KS; s++)
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int k = 32 * s + 8 * (lane >> 4) + e;
                uint16_t h, l;
                split_bf16((row < nq && k < rp) ? Cg[row * rp + k] : 0.0, h, l);
                bhi[s][e] = __builtin_bit_cast(__bf16, h);
                blo[s][e] = __builtin_bit_cast(__bf16, l);
            }
    }
    // vector index e: half = e / kVec, column c = (e % kVec) / (4 KS), rank
    // group g = e % (4 KS) (8 entries each); rp = 32 KS here
    __device__ __forceinline__ void fetch_z(const double *, const uint16_t *Zhi, const uint16_t *Zlo, int64_t,
                                            int rp, int64_t c0, int64_t cend, int tid) {
#pragma unroll
        for (int u = 0; u < kZU; u++) {
            const int e = tid + u * kResThreads;
            const int h = e / kVec, c = (e % kVec) / (4 * KS), g = e % (4 * KS);
            v4u v = {0u, 0u, 0u, 0u};
            if (e < 2 * kVec && c0 + c < cend)
                v = *reinterpret_cast<const v4u *>((h ? Zlo : Zhi) + (c0 + c) * rp + 8 * g);
            zr[u] = v;
        }
    }
    __device__ __forceinline__ void store_z(char *lds, int tid) {
        uint16_t *z = reinterpret_cast<uint16_t *>(lds);
#pragma unroll
        for (int u = 0; u < kZU; u++) {
            const int e = tid + u * kResThreads;
            const int h = e / kVec, c = (e % kVec) / (4 * KS), g = e % (4 * KS);
            if (e < 2 * kVec) *reinterpret_cast<v4u *>(z + h * kHalf + c * kCol + 8 * g) = zr[u];
        }
    }
    __device__ __forceinline__ void tile2(const char *lds, int t, int lane, Acc (&x)[2][4]) const {
        const uint16_t *z = reinterpret_cast<const uint16_t *>(lds) + (16 * t + (lane & 15)) * kCol + 8 * (lane >> 4);
        v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; s++) {
            const v8bf zh0 = *reinterpret_cast<const v8bf *>(z + 32 * s);
            const v8bf zl0 = *reinterpret_cast<const v8bf *>(z + kHalf + 32 * s);
            const v8bf zh1 = *reinterpret_cast<const v8bf *>(z + 16 * kCol + 32 * s);
            const v8bf zl1 = *reinterpret_cast<const v8bf *>(z + kHalf + 16 * kCol + 32 * s);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh0, blo[s], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh1, blo[s], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zl0, bhi[s], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zl1, bhi[s], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh0, bhi[s], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh1, bhi[s], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; v++) {
            x[0][v] = acc0[v];
            x[1][v] = acc1[v];
        }
    }
};

// Four consecutive entries of W (one vector load when `vec`, else one by one
// with the column bound).
template <typename T> struct Quad;
template <> struct Quad<float> {
    typedef float V __attribute__((ext_vector_type(4)));
};
template <> struct Quad<double> {
    typedef double V __attribute__((ext_vector_type(4)));
};
template <> struct Quad<uint16_t> {
    typedef uint16_t V __attribute__((ext_vector_type(4)));
};

// The residual kernel proper, generic over the core.  Workgroup (x, y) takes
// rows [128 y, 128 y + 128) and columns [split x, split x + split).  `vec`:
// rows start 4-entry aligned and the columns are contiguous, so a lane's
// four columns are one aligned vector.
template <typename T, class Core, int CH>
__global__ void __launch_bounds__(kResThreads) resid_kernel(const T *A, int64_t lda, const int64_t *rows,
                                                            const int64_t *cols, int64_t nq, int64_t ns, int rp,
                                                            int64_t split, int vec, const double *Cg,
                                                            const double *Zg, const uint16_t *Zhi,
                                                            const uint16_t *Zlo, double *partials) {
    constexpr int NT = CH / 16;   // 16-column tiles per chunk (even)
    typedef typename Quad<T>::V V;
    __shared__ __align__(16) char lds[2][Core::kLdsBytes];
    __shared__ double red[kResWaves][4];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t row0 = (int64_t)blockIdx.y * kResRows + wave * 16;
    const int64_t cbeg = (int64_t)blockIdx.x * split;
    const int64_t cend = std::min<int64_t>(ns, cbeg + split);
    Core core;
    core.load_cg(Cg, rp, row0, nq, lane);
    const int64_t myrow = row0 + (lane & 15);
    const bool rok = myrow < nq;
    const T *wrow = A + (rok ? (rows ? rows[myrow] : myrow) * lda : 0);
    const int cq = 4 * (lane >> 4);   // first of the lane's four columns in a tile
    V wa[NT], wb[NT];
    double se = 0.0, se2 = 0.0, sabs = 0.0, sw2 = 0.0;

    auto fetch_w = [&](V (&w)[NT], int64_t c0) {
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int64_t cj = c0 + 16 * t + cq;
            V v = {T(0), T(0), T(0), T(0)};
            if (rok) {
                if (vec && cj + 3 < cend) {
                    v = *reinterpret_cast<const V *>(wrow + cj);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        if (cj + e < cend) v[e] = wrow[cols ? cols[cj + e] : cj + e];
                }
            }
            w[t] = v;
        }
    };
    // the chunk's sums are formed in the core's epilogue arithmetic (FP32 on
    // the mixed path) and added to the FP64 totals once per chunk
    auto compute = [&](const char *buf, V (&w)[NT], int64_t c0) {
        typedef typename Core::Acc Acc;
        Acc ce = 0, ce2 = 0, cabs = 0, cw2 = 0;
#pragma unroll
        for (int t = 0; t < NT; t += 2) {
            if (c0 + 16 * t >= cend) break;
            Acc x[2][4];
            core.tile2(buf, t, lane, x);
            if (rok) {
#pragma unroll
                for (int h = 0; h < 2; h++)
#pragma unroll
                    for (int v = 0; v < 4; v++)
                        if (c0 + 16 * (t + h) + cq + v < cend) {
                            const Acc wv = (Acc)Elem<T>::conv(w[t + h][v]);
                            const Acc e = wv - x[h][v];
                            ce += e;
                            ce2 += e * e;
                            cabs += fabs(e);
                            cw2 += wv * wv;
                        }
            }
        }
        se += (double)ce;
        se2 += (double)ce2;
        sabs += (double)cabs;
        sw2 += (double)cw2;
    };

    if (cbeg < cend) {
        fetch_w(wa, cbeg);
        core.fetch_z(Zg, Zhi, Zlo, ns, rp, cbeg, cend, tid);
        core.store_z(lds[0], tid);
        __syncthreads();
        for (int64_t c0 = cbeg; c0 < cend; c0 += 2 * CH) {
            const bool more1 = c0 + CH < cend;
            if (more1) {
                fetch_w(wb, c0 + CH);
                core.fetch_z(Zg, Zhi, Zlo, ns, rp, c0 + CH, cend, tid);
            }
            compute(lds[0], wa, c0);
            if (more1) core.store_z(lds[1], tid);
            __syncthreads();
            if (!more1) break;
            const bool more2 = c0 + 2 * CH < cend;
            if (more2) {
                fetch_w(wa, c0 + 2 * CH);
                core.fetch_z(Zg, Zhi, Zlo, ns, rp, c0 + 2 * CH, cend, tid);
            }
            compute(lds[1], wb, c0 + CH);
            if (more2) core.store_z(lds[0], tid);
            __syncthreads();
        }
    }
    // fixed-order reduction: butterfly within each wave, then the waves in order
    const double v0 = wave_sum(se), v1 = wave_sum(se2), v2 = wave_sum(sabs), v3 = wave_sum(sw2);
    if (lane == 0) {
        red[wave][0] = v0;
        red[wave][1] = v1;
        red[wave][2] = v2;
        red[wave][3] = v3;
    }
    __syncthreads();
    if (tid < 4) {
        double acc = 0.0;
        for (int w = 0; w < kResWaves; w++) acc += red[w][tid];
        partials[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 4 + tid] = acc;
    }
}

// Sum the per-workgroup partials in a fixed order.
__global__ void resid_sum_kernel(const double *partials, int64_t nblocks, double *out) {
    __shared__ double red[4][256];
    const int tid = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t b = tid; b < nblocks; b += 256)
        for (int k = 0; k < 4; k++) acc[k] += partials[b * 4 + k];
    for (int k = 0; k < 4; k++) red[k][tid] = acc[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
            for (int k = 0; k < 4; k++) red[k][tid] += red[k][tid + h];
        __syncthreads();
    }
    if (tid < 4) out[tid] = red[tid][0];
}

static int resid_rp(int r, int prec) { return prec == LRA_PREC_MIXED ? (r + 31) / 32 * 32 : (r + 3) / 4 * 4; }

// Column range per workgroup: about 2048 workgroups in all (several waves of
// workgroups per CU, so the last one is short), in whole 64-column chunks.
static int64_t resid_split(int64_t nq, int64_t ns) {
    const int64_t ry = (nq + kResRows - 1) / kResRows;
    const int64_t gx = std::max<int64_t>(1, (2048 + ry - 1) / ry);
    const int64_t split = ((ns + gx - 1) / gx + 63) / 64 * 64;
    return std::max<int64_t>(64, split);
}

static dim3 resid_grid(int64_t nq, int64_t ns) {
    const int64_t split = resid_split(nq, ns);
    return dim3((unsigned)((ns + split - 1) / split), (unsigned)((nq + kResRows - 1) / kResRows));
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t residual_scratch_bytes(int64_t m, int64_t n, int r, int q, int s, int prec) {
    const int64_t nq = q ? q : m, ns = s ? s : n;
    const int rp = resid_rp(r, prec);
    const dim3 g = resid_grid(nq, ns);
    return align256(512 * sizeof(int64_t)) + align256(sizeof(double) * (size_t)rp * ns) +
           align256(sizeof(double) * (size_t)nq * rp) + align256(sizeof(double) * 4 * (size_t)g.x * g.y);
}

template <typename T, class Core, int CH>
static void launch_resid_core(dim3 grid, int64_t split, int vec, hipStream_t stream, const T *A, int64_t lda,
                              const int64_t *rows, const int64_t *cols, int64_t nq, int64_t ns, int rp,
                              const double *Cg, const double *Z, const uint16_t *Zhi, const uint16_t *Zlo,
                              double *partials) {
    hipLaunchKernelGGL((resid_kernel<T, Core, CH>), grid, dim3(kResThreads), 0, stream, A, lda, rows, cols, nq, ns, rp,
                       split, vec, Cg, Z, Zhi, Zlo, partials);
}

template <typename T>
static hipError_t residual_t(const void *Av, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I,
                             const int64_t *J, const double *U, int q, int s, uint64_t seed, int prec, double *out,
                             char *scratch, hipStream_t stream) {
    // 64-column chunks, 32 for FP64 inputs (the prefetched W takes twice the registers)
    constexpr int CH = sizeof(T) == 8 ? 32 : 64;
    const T *A = static_cast<const T *>(Av);
    const int64_t nq = q ? q : m, ns = s ? s : n;
    const int rp = resid_rp(r, prec);
    const bool mixed = prec == LRA_PREC_MIXED;
    char *p = scratch;
    int64_t *rows = nullptr, *cols = nullptr;
    if (q) {
        rows = reinterpret_cast<int64_t *>(p);
        cols = rows + 256;
        hipLaunchKernelGGL(resid_sample_kernel, dim3(1), dim3(2 * kWave), 0, stream, seed, m, n, q, s, rows, cols);
    }
    p += align256(512 * sizeof(int64_t));
    double *Z = reinterpret_cast<double *>(p);   // FP64 [rp][ns], or the BF16 hi and lo halves [ns][rp]
    uint16_t *Zhi = reinterpret_cast<uint16_t *>(p);
    uint16_t *Zlo = Zhi + (size_t)rp * ns;
    p += align256(sizeof(double) * (size_t)rp * ns);
    double *Cg = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * (size_t)nq * rp);
    double *partials = reinterpret_cast<double *>(p);
    hipLaunchKernelGGL(resid_z_kernel<T>, dim3((unsigned)((ns + 63) / 64)), dim3(256), 0, stream, A, m, lda, r, rp, I,
                       U, cols, ns, mixed ? 1 : 0, Z, Zhi, Zlo);
    hipLaunchKernelGGL(resid_c_kernel<T>, dim3((unsigned)((nq * rp + 255) / 256)), dim3(256), 0, stream, A, n, lda, r,
                       rp, J, rows, nq, Cg);
    const dim3 grid = resid_grid(nq, ns);
    const int64_t split = resid_split(nq, ns);
    // the rank-64 FP64 core works on 32-column chunks (its fragments take many registers)
    using CoreM1 = Bf16x3Core<1, CH>;
    using CoreM2 = Bf16x3Core<2, CH>;
    using CoreP4 = F64Core<4, CH>;
    using CoreP8 = F64Core<8, CH>;
    using CoreP16 = F64Core<16, 32>;
    const int vec = (!cols && lda % 4 == 0 && reinterpret_cast<uintptr_t>(A) % (4 * sizeof(T)) == 0) ? 1 : 0;
#define LRA_RES(CORE, C) \
    launch_resid_core<T, CORE, C>(grid, split, vec, stream, A, lda, rows, cols, nq, ns, rp, Cg, Z, Zhi, Zlo, partials)
    if (mixed) {
        if (rp <= 32) LRA_RES(CoreM1, CH);
        else LRA_RES(CoreM2, CH);
    } else {
        if (rp <= 16) LRA_RES(CoreP4, CH);
        else if (rp <= 32) LRA_RES(CoreP8, CH);
        else LRA_RES(CoreP16, 32);
    }
#undef LRA_RES
    hipLaunchKernelGGL(resid_sum_kernel, dim3(1), dim3(256), 0, stream, partials, (int64_t)grid.x * grid.y, out);
    return hipGetLastError();
}

// The a-posteriori variance test on the moments of a q x s residual sample
// (Section 4: the sampled error entries as observed values of one Gaussian
// variable): mean, mean of |g|, variance sum e^2 / K - mean^2 (clamped at
// 0), and the one-sided test K var <= tau^2 ((K - 1) - z sqrt(2 (K - 1))).
__global__ void posterior_kernel(const double *mom, int64_t K, double tau, double z, lra_posterior *out) {
    if (threadIdx.x != 0) return;
    const double k = (double)K;
    const double mean = mom[0] / k;
    const double var = fmax(mom[1] / k - mean * mean, 0.0);
    const double dof = (double)(K - 1);
    const double thr = tau * tau * (dof - z * sqrt(2.0 * dof)) / k;
    lra_posterior p;
    p.K = K;
    p.mean = mean;
    p.mean_abs = mom[2] / k;
    p.var = var;
    p.threshold = thr;
    p.accept = var <= thr ? 1 : 0;
    p.reserved = 0;
    *out = p;
}

hipError_t launch_posterior(const double *moments, int64_t K, double tau, double z, lra_posterior *out,
                            hipStream_t stream) {
    hipLaunchKernelGGL(posterior_kernel, dim3(1), dim3(64), 0, stream, moments, K, tau, z, out);
    return hipGetLastError();
}

hipError_t launch_residual(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I,
                           const int64_t *J, const double *U, int q, int s, uint64_t seed, int prec, double *out,
                           void *scratch, hipStream_t stream) {
    char *sc = static_cast<char *>(scratch);
    if (dtype == LRA_F64) return residual_t<double>(A, m, n, lda, r, I, J, U, q, s, seed, prec, out, sc, stream);
    if (dtype == LRA_F32) return residual_t<float>(A, m, n, lda, r, I, J, U, q, s, seed, prec, out, sc, stream);
    return residual_t<uint16_t>(A, m, n, lda, r, I, J, U, q, s, seed, prec, out, sc, stream);
}

// ------------------------------------------------------------------ adjoint
// L = sum over Omega of (a_ij - (C Z)_ij)^2 with Z = G^{-1} R, for a batch of
// equal-shape blocks:
//   index   one thread per Omega entry: checks the indices, the row order and
//           the column order (col_order), fills the row pointers, the column
//           pointers and the column-ordered copies of the row indices and
//           values; any violation sets the block's flag;
//   inverse one workgroup per block: G^{-1} by LU with partial pivoting in
//           LDS, or the block's error status;
//   stage   Z^T (n x rp, rank padded to rp = 8 G) and, when r < rp, a padded
//           copy of C;
//   rows    G lanes per row of C, 8 rank entries each: x = C_i . Z_j per
//           entry of the row, loss, dC_i = sum ebar Z_j;
//   cols    G lanes per column: dZ_j = sum ebar C_i, dR_j = G^{-T} dZ_j, and
//           this workgroup's share of T = dZ Z^T;
//   final   one workgroup per block: loss and T summed over the workgroups in
//           a fixed order, dG = -G^{-T} T.
// The row and column launches put all workgroups of a block on one XCD (the
// hardware deals workgroup w to XCD w mod 8), so a block's Z^T and C stay in
// that XCD's L2.  Every sum runs in a fixed order: results are deterministic.
constexpr int kAdjThreads = 512;
constexpr int kXcds = 8;

struct AdjLayout {   // per-block scratch, byte offsets from the block's base
    int64_t stride, gi, zt, cp, rowptr, colptr, crow, cval, lossp, tp, flag;
};

__device__ __forceinline__ char *adj_base(char *ws, const AdjLayout &L, int64_t b) { return ws + b * L.stride; }

__global__ void adj_clear_kernel(int64_t count, AdjLayout L, char *ws) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < count) *reinterpret_cast<int32_t *>(adj_base(ws, L, b) + L.flag) = 0;
}

// Thread q in [0, nnz] of block blockIdx.y.  Pointer entries are written only
// from a pair of consecutive entries whose indices were checked, so every
// store stays inside the block's arrays whatever the input.
__global__ void __launch_bounds__(256) adj_index_kernel(int64_t m, int64_t n, int64_t nnz, const int32_t *orow_b,
                                                        const int32_t *ocol_b, const int32_t *corder_b,
                                                        const double *aval_b, AdjLayout L, char *ws) {
    const int64_t b = blockIdx.y;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q > nnz) return;
    const int32_t *orow = orow_b + b * nnz, *ocol = ocol_b + b * nnz, *corder = corder_b + b * nnz;
    char *base = adj_base(ws, L, b);
    int32_t *rowptr = reinterpret_cast<int32_t *>(base + L.rowptr);
    int32_t *colptr = reinterpret_cast<int32_t *>(base + L.colptr);
    bool bad = false;
    // rows: entry q and its predecessor
    const int64_t cur = q < nnz ? orow[q] : m;
    const int64_t prev = q > 0 ? orow[q - 1] : -1;
    const bool rok = cur >= 0 && cur <= m && prev >= -1 && prev < m && prev <= cur &&
                     (q == nnz || (cur < m && ocol[q] >= 0 && ocol[q] < n));
    if (rok) {
        for (int64_t i = prev + 1; i <= cur; i++) rowptr[i] = (int32_t)q;
    } else {
        bad = true;
    }
    // columns: position q of the column order and its predecessor
    bool cok = true;
    int64_t tq = -1, cc = n, pc = -1;
    if (q < nnz) {
        tq = corder[q];
        if (tq >= 0 && tq < nnz) cc = ocol[tq];
        else cok = false;
    }
    if (q > 0) {
        const int64_t tp = corder[q - 1];
        if (tp >= 0 && tp < nnz) pc = ocol[tp];
        else cok = false;
    }
    cok = cok && cc >= 0 && cc <= n && pc >= -1 && pc < n && pc <= cc && (q == nnz || cc < n);
    if (cok) {
        for (int64_t j = pc + 1; j <= cc; j++) colptr[j] = (int32_t)q;
    } else {
        bad = true;
    }
    if (tq >= 0 && tq < nnz) {
        reinterpret_cast<int32_t *>(base + L.crow)[q] = orow[tq];
        reinterpret_cast<double *>(base + L.cval)[q] = aval_b[b * nnz + tq];
    }
    if (bad) atomicOr(reinterpret_cast<int32_t *>(base + L.flag), 1);
}

__global__ void __launch_bounds__(kAdjThreads) adj_inverse_kernel(int r, const double *Gb, AdjLayout L, char *ws,
                                                                  double *loss, int32_t *status) {
    extern __shared__ __align__(16) double lds[];
    double *LU = lds, *Gi = lds + r * r;
    __shared__ int p[kRMax];
    __shared__ int sing;
    __shared__ double ld;
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    char *base = adj_base(ws, L, b);
    if (*reinterpret_cast<const int32_t *>(base + L.flag)) {
        if (tid == 0) {
            status[b] = LRA_EINVAL;
            loss[b] = __builtin_nan("");
        }
        return;
    }
    for (int e = tid; e < r * r; e += kAdjThreads) LU[e] = Gb[b * r * r + e];
    __syncthreads();
    inverse_lds(LU, Gi, p, r, kAdjThreads, &sing, &ld);
    if (sing) {
        if (tid == 0) {
            status[b] = LRA_ESINGULAR;
            loss[b] = __builtin_nan("");
        }
        return;
    }
    double *gi = reinterpret_cast<double *>(base + L.gi);
    for (int e = tid; e < r * r; e += kAdjThreads) gi[e] = Gi[e];
    if (tid == 0) status[b] = LRA_OK;
}

// Z^T[j][a] = sum_q Gi[a][q] R[q][j] (q increasing; a < r, zero up to RP):
// one column per thread, its RP sums in registers, G^{-1} transposed in LDS
// (read as broadcasts).  Grid (chunks of 256 columns, blocks).
template <int RP>
__global__ void __launch_bounds__(256) adj_z_kernel(int64_t n, int r, const double *Rb, AdjLayout L, char *ws,
                                                    const int32_t *status) {
    __shared__ __align__(16) double gt[kRMax * RP];
    const int64_t b = blockIdx.y;
    if (status[b] != LRA_OK) return;
    const int tid = threadIdx.x;
    char *base = adj_base(ws, L, b);
    const double *gi = reinterpret_cast<const double *>(base + L.gi);
    for (int e = tid; e < r * RP; e += 256) {
        const int q = e / RP, a = e % RP;
        gt[e] = a < r ? gi[a * r + q] : 0.0;
    }
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * 256 + tid;
    if (j >= n) return;
    const double *R = Rb + b * r * n + j;
    double acc[RP];
#pragma unroll
    for (int a = 0; a < RP; a++) acc[a] = 0.0;
    for (int q = 0; q < r; q++) {
        const double rq = R[(int64_t)q * n];
#pragma unroll
        for (int a = 0; a < RP; a++) acc[a] += gt[q * RP + a] * rq;
    }
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 *zt = reinterpret_cast<d2 *>(reinterpret_cast<double *>(base + L.zt) + j * RP);
#pragma unroll
    for (int a = 0; a < RP; a += 2) zt[a / 2] = d2{acc[a], acc[a + 1]};
}

// Cp[i][a] = C[i][a] (zero for r <= a < rp), only when r < rp.  Grid (chunks
// of 256 entries, blocks).
__global__ void adj_c_kernel(int64_t m, int r, int rp, const double *Cb, AdjLayout L, char *ws,
                             const int32_t *status) {
    const int64_t b = blockIdx.y;
    if (status[b] != LRA_OK) return;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= m * rp) return;
    const int64_t i = e / rp;
    const int a = (int)(e % rp);
    reinterpret_cast<double *>(adj_base(ws, L, b) + L.cp)[e] = a < r ? Cb[b * m * r + i * r + a] : 0.0;
}

// Work index of workgroup w when `total` work items are dealt so that each
// XCD gets a contiguous range (w mod 8 = XCD).  Returns -1 past the end.
__device__ __forceinline__ int64_t xcd_work(int64_t w, int64_t total) {
    const int64_t per = (total + kXcds - 1) / kXcds;
    const int64_t l = (w % kXcds) * per + w / kXcds;
    return l < total ? l : -1;
}

__device__ __forceinline__ void load8(const double *p, double (&v)[8]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        const d2 t = *reinterpret_cast<const d2 *>(p + k);
        v[k] = t[0];
        v[k + 1] = t[1];
    }
}

// Sum over the G lanes of an item group (consecutive lanes), butterfly order.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// One pass over the entries of an item (a row for the row pass, a column for
// the column pass): `fixed` holds the item's own 8 rank entries, `other` is
// the matrix gathered per entry (Z^T or C, stride rp), idx/val the entries'
// other index and value.  The next entry's index, value and gather are
// issued before the current one is used.  Returns in `acc` the sum of
// ebar * other over the entries and adds e^2 to *lsum.
template <int G>
__device__ __forceinline__ void adj_item_pass(const double (&fixed)[8], const double *other, int rp, int g,
                                              const int32_t *idx, const double *val, int32_t q0, int32_t q1,
                                              double (&acc)[8], double *lsum) {
#pragma unroll
    for (int k = 0; k < 8; k++) acc[k] = 0.0;
    if (q0 >= q1) return;
    double o[8];
    load8(other + (int64_t)idx[q0] * rp + 8 * g, o);
    double av = val[q0];
    for (int32_t q = q0; q < q1; q++) {
        double on[8];
        double avn = 0.0;
        if (q + 1 < q1) {
            load8(other + (int64_t)idx[q + 1] * rp + 8 * g, on);
            avn = val[q + 1];
        }
        double x = 0.0;
#pragma unroll
        for (int k = 0; k < 8; k++) x += fixed[k] * o[k];
        x = group_sum<G>(x);
        const double e = av - x;
        *lsum += e * e;
        const double eb = -2.0 * e;
#pragma unroll
        for (int k = 0; k < 8; k++) acc[k] += eb * o[k];
        if (q + 1 < q1) {
#pragma unroll
            for (int k = 0; k < 8; k++) o[k] = on[k];
            av = avn;
        }
    }
}

// Row pass.  Items = rows of C; G lanes per row, lane g holds rank entries
// 8 g .. 8 g + 7.  Per entry (i, j) of the row: x = sum_a C_ia Z_aj,
// e = a_ij - x, loss += e^2, dC_i += -2 e Z_j.
template <int G>
__global__ void __launch_bounds__(kAdjThreads) adj_row_kernel(int64_t count, int64_t m, int r, int64_t nnz,
                                                              const double *Cb, const int32_t *ocol_b,
                                                              const double *aval_b, int64_t chunks, AdjLayout L,
                                                              char *ws, double *dCb, const int32_t *status) {
    constexpr int kItems = kAdjThreads / G, RP = 8 * G;
    __shared__ double red[kAdjThreads / kWave];
    const int64_t wk = xcd_work(blockIdx.x, count * chunks);
    if (wk < 0) return;
    const int64_t b = wk / chunks, chunk = wk % chunks;
    if (status[b] != LRA_OK) return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), g = tid % G;
    char *base = adj_base(ws, L, b);
    const int32_t *rowptr = reinterpret_cast<const int32_t *>(base + L.rowptr);
    const double *zt = reinterpret_cast<const double *>(base + L.zt);
    const double *cm = r == RP ? Cb + b * m * r : reinterpret_cast<const double *>(base + L.cp);
    const int64_t i = chunk * kItems + tid / G;
    double lsum = 0.0;
    if (i < m) {
        double c[8], dc[8];
        load8(cm + i * RP + 8 * g, c);
        adj_item_pass<G>(c, zt, RP, g, ocol_b + b * nnz, aval_b + b * nnz, rowptr[i], rowptr[i + 1], dc, &lsum);
        double *dC = dCb + b * m * r + i * r;
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (8 * g + k < r) dC[8 * g + k] = dc[k];
    }
    if (g != 0) lsum = 0.0;   // every lane of a group computed the same e
    const double wsum = wave_sum(lsum);
    if (lane == 0) red[tid / kWave] = wsum;
    __syncthreads();
    if (tid == 0) {
        double acc = 0.0;
        for (int w = 0; w < kAdjThreads / kWave; w++) acc += red[w];
        reinterpret_cast<double *>(base + L.lossp)[chunk] = acc;
    }
}

// Column pass.  Items = columns; G lanes per column.  Per entry (i, j):
// ebar = -2 (a_ij - C_i . Z_j), dZ_j += ebar C_i; then dR_j = G^{-T} dZ_j and
// this workgroup's part of T = sum_j dZ_j Z_j^T.
template <int G>
__global__ void __launch_bounds__(kAdjThreads) adj_col_kernel(int64_t count, int64_t m, int64_t n, int r,
                                                              const double *Cb, int64_t chunks, AdjLayout L,
                                                              char *ws, double *dRb, const int32_t *status) {
    constexpr int kItems = kAdjThreads / G, RP = 8 * G;
    extern __shared__ __align__(16) double lds[];
    double *dzs = lds;                       // [kItems][RP]
    double *zs = lds + kItems * RP;          // [kItems][RP]
    double *gs = lds + 2 * kItems * RP;      // Gi, r x r
    const int64_t wk = xcd_work(blockIdx.x, count * chunks);
    if (wk < 0) return;
    const int64_t b = wk / chunks, chunk = wk % chunks;
    if (status[b] != LRA_OK) return;
    const int tid = threadIdx.x, g = tid % G, li = tid / G;
    char *base = adj_base(ws, L, b);
    const double *gi = reinterpret_cast<const double *>(base + L.gi);
    for (int e = tid; e < r * r; e += kAdjThreads) gs[e] = gi[e];
    const int32_t *colptr = reinterpret_cast<const int32_t *>(base + L.colptr);
    const double *zt = reinterpret_cast<const double *>(base + L.zt);
    const double *cm = r == RP ? Cb + b * m * r : reinterpret_cast<const double *>(base + L.cp);
    const int64_t j = chunk * kItems + li;
    double z[8], dz[8];
#pragma unroll
    for (int k = 0; k < 8; k++) z[k] = dz[k] = 0.0;
    if (j < n) {
        double unused = 0.0;
        load8(zt + j * RP + 8 * g, z);
        adj_item_pass<G>(z, cm, RP, g, reinterpret_cast<const int32_t *>(base + L.crow),
                         reinterpret_cast<const double *>(base + L.cval), colptr[j], colptr[j + 1], dz, &unused);
    }
#pragma unroll
    for (int k = 0; k < 8; k++) {
        dzs[li * RP + 8 * g + k] = dz[k];
        zs[li * RP + 8 * g + k] = z[k];
    }
    __syncthreads();
    if (j < n) {
        // dR[a][j] = sum_q Gi[q][a] dZ[q][j], q increasing
        double *dR = dRb + b * r * n;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int a = 8 * g + k;
            if (a < r) {
                double acc = 0.0;
                for (int q = 0; q < r; q++) acc += gs[q * r + a] * dzs[li * RP + q];
                dR[(int64_t)a * n + j] = acc;
            }
        }
    }
    // T part: Tp[a][c] = sum over this workgroup's columns (in order) of dZ[a] Z[c]
    const int nit = (int)std::min<int64_t>(kItems, n - chunk * kItems);
    double *tp = reinterpret_cast<double *>(base + L.tp) + chunk * r * r;
    for (int e = tid; e < r * r; e += kAdjThreads) {
        const int a = e / r, c = e % r;
        double acc = 0.0;
        for (int it = 0; it < nit; it++) acc += dzs[it * RP + a] * zs[it * RP + c];
        tp[e] = acc;
    }
}

// Loss = sum of the row workgroups' partials, T = sum of the column
// workgroups' parts (both in workgroup order), dG = -G^{-T} T.
__global__ void __launch_bounds__(256) adj_final_kernel(int r, int64_t rchunks, int64_t cchunks, AdjLayout L,
                                                        char *ws, double *loss, double *dGb, const int32_t *status) {
    __shared__ double ts[kRMax * kRMax];
    const int64_t b = blockIdx.x;
    if (status[b] != LRA_OK) return;
    char *base = adj_base(ws, L, b);
    const double *gi = reinterpret_cast<const double *>(base + L.gi);
    const double *tp = reinterpret_cast<const double *>(base + L.tp);
    for (int e = threadIdx.x; e < r * r; e += 256) {
        double acc = 0.0;
        for (int64_t c = 0; c < cchunks; c++) acc += tp[c * r * r + e];
        ts[e] = acc;
    }
    __syncthreads();
    double *dG = dGb + b * r * r;
    for (int e = threadIdx.x; e < r * r; e += 256) {
        const int a = e / r, c = e % r;
        double acc = 0.0;
        for (int q = 0; q < r; q++) acc += gi[q * r + a] * ts[q * r + c];
        dG[e] = -acc;
    }
    if (threadIdx.x == 0) {
        const double *lp = reinterpret_cast<const double *>(base + L.lossp);
        double acc = 0.0;
        for (int64_t c = 0; c < rchunks; c++) acc += lp[c];
        loss[b] = acc;
    }
}

static int adj_lanes(int r) { return r <= 8 ? 1 : r <= 16 ? 2 : r <= 32 ? 4 : 8; }

static AdjLayout adj_layout(int64_t m, int64_t n, int64_t nnz, int r) {
    const int G = adj_lanes(r), rp = 8 * G, items = kAdjThreads / G;
    const int64_t rch = (m + items - 1) / items, cch = (n + items - 1) / items;
    AdjLayout L;
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o += (bytes + 255) / 256 * 256;
        return at;
    };
    L.gi = take(8 * (int64_t)r * r);
    L.zt = take(8 * n * rp);
    L.cp = take(r == rp ? 0 : 8 * m * rp);
    L.rowptr = take(4 * (m + 1));
    L.colptr = take(4 * (n + 1));
    L.crow = take(4 * nnz);
    L.cval = take(8 * nnz);
    L.lossp = take(8 * rch);
    L.tp = take(8 * cch * r * r);
    L.flag = take(4);
    L.stride = o;
    return L;
}

size_t adjoint_scratch_bytes(int64_t count, int64_t m, int64_t n, int64_t nnz, int r) {
    return (size_t)(adj_layout(m, n, nnz, r).stride * count);
}

template <int G>
static void launch_adj_passes(int64_t count, int64_t m, int64_t n, int r, int64_t nnz, const double *C,
                              const double *R, const int32_t *ocol, const double *aval, const AdjLayout &L, char *ws,
                              double *dC, double *dR, const int32_t *status, hipStream_t stream) {
    constexpr int items = kAdjThreads / G, RP = 8 * G;
    const int64_t rch = (m + items - 1) / items, cch = (n + items - 1) / items;
    hipLaunchKernelGGL(adj_z_kernel<RP>, dim3((unsigned)((n + 255) / 256), (unsigned)count), dim3(256), 0, stream, n,
                       r, R, L, ws, status);
    if (r < RP)
        hipLaunchKernelGGL(adj_c_kernel, dim3((unsigned)((m * RP + 255) / 256), (unsigned)count), dim3(256), 0, stream,
                           m, r, RP, C, L, ws, status);
    // one workgroup per (block, chunk), rounded up to whole rounds of the XCDs
    auto wgs = [&](int64_t chunks) { return (unsigned)(kXcds * ((count * chunks + kXcds - 1) / kXcds)); };
    hipLaunchKernelGGL(adj_row_kernel<G>, dim3(wgs(rch)), dim3(kAdjThreads), 0, stream, count, m, r, nnz, C, ocol,
                       aval, rch, L, ws, dC, status);
    const size_t lds = sizeof(double) * (2 * (size_t)items * RP + (size_t)r * r);
    hipLaunchKernelGGL(adj_col_kernel<G>, dim3(wgs(cch)), dim3(kAdjThreads), lds, stream, count, m, n, r, C, cch, L,
                       ws, dR, status);
}

hipError_t launch_adjoint(int64_t count, int64_t m, int64_t n, int r, const double *C, const double *R,
                          const double *G, int64_t nnz, const int32_t *orow, const int32_t *ocol,
                          const int32_t *corder, const double *aval, double *loss, double *dC, double *dR,
                          double *dG, void *scratch, int32_t *status, hipStream_t stream) {
    char *ws = static_cast<char *>(scratch);
    const AdjLayout L = adj_layout(m, n, nnz, r);
    const int Gl = adj_lanes(r), items = kAdjThreads / Gl;
    const int64_t rch = (m + items - 1) / items, cch = (n + items - 1) / items;
    hipLaunchKernelGGL(adj_clear_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, count, L, ws);
    hipLaunchKernelGGL(adj_index_kernel, dim3((unsigned)((nnz + 1 + 255) / 256), (unsigned)count), dim3(256), 0, stream,
                       m, n, nnz, orow, ocol, corder, aval, L, ws);
    hipLaunchKernelGGL(adj_inverse_kernel, dim3((unsigned)count), dim3(kAdjThreads), sizeof(double) * 2 * r * r, stream,
                       r, G, L, ws, loss, status);
    switch (Gl) {
    case 1: launch_adj_passes<1>(count, m, n, r, nnz, C, R, ocol, aval, L, ws, dC, dR, status, stream); break;
    case 2: launch_adj_passes<2>(count, m, n, r, nnz, C, R, ocol, aval, L, ws, dC, dR, status, stream); break;
    case 4: launch_adj_passes<4>(count, m, n, r, nnz, C, R, ocol, aval, L, ws, dC, dR, status, stream); break;
    default: launch_adj_passes<8>(count, m, n, r, nnz, C, R, ocol, aval, L, ws, dC, dR, status, stream); break;
    }
    hipLaunchKernelGGL(adj_final_kernel, dim3((unsigned)count), dim3(256), 0, stream, r, rch, cch, L, ws, loss, dG,
                       status);
    return hipGetLastError();
}

}  // namespace lra
