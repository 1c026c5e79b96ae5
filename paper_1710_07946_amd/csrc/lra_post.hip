// lra_post.hip -- kernels that use a computed CUR: the residual moments of
// E = W - C U R (full, or a random q x s sample for the a-posteriori
// estimate), and the adjoint of the CUR reconstruction at fixed index sets.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lra_device.h"
#include "lra_internal.h"

namespace lra {

constexpr int kResTileRows = 64;   // rows of E per residual workgroup
constexpr int kResThreads = 256;   // one column of E per thread
constexpr int kAdjThreads = 512;

// ------------------------------------------------------------------ residual
// Sample rows (stream 3) and columns (stream 4) of E, q, s <= 256.
__global__ void resid_sample_kernel(uint64_t seed, int64_t m, int64_t n, int q, int s, int64_t *rows,
                                    int64_t *cols) {
    if (threadIdx.x < kWave) draw_distinct_wave(seed, 3, m, q, rows);
    else if (threadIdx.x < 2 * kWave) draw_distinct_wave(seed, 4, n, s, cols);
}

// Z = U W[I, cols] (r x ns, FP64), one column per thread; the sum over b runs
// in increasing order.
template <typename T, int RM>
__global__ void __launch_bounds__(kResThreads) resid_z_kernel(const T *A, int64_t m, int64_t lda, int r, const int64_t *I,
                                                              const double *U, const int64_t *cols, int64_t ns,
                                                              double *Z) {
    const int64_t c = (int64_t)blockIdx.x * kResThreads + threadIdx.x;
    if (c >= ns) return;
    const int64_t col = cols ? cols[c] : c;
    double rc[RM];
#pragma unroll
    for (int b = 0; b < RM; b++) {
        const int64_t i = b < r ? I[b] : 0;
        // an index outside [0, m) is not read: it turns the moments into NaN
        rc[b] = b >= r ? 0.0 : (i >= 0 && i < m) ? Elem<T>::load(A, i * lda + col) : __builtin_nan("");
    }
    for (int a = 0; a < r; a++) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < RM; b++)
            if (b < r) acc += U[a * r + b] * rc[b];
        Z[(int64_t)a * ns + c] = acc;
    }
}

// Cg = W[rows, J] (nq x r, FP64).
template <typename T>
__global__ void resid_c_kernel(const T *A, int64_t n, int64_t lda, int r, const int64_t *J, const int64_t *rows,
                               int64_t nq, double *Cg) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nq * r) return;
    const int64_t i = e / r;
    const int64_t j = J[e % r];
    Cg[e] = (j >= 0 && j < n) ? Elem<T>::load(A, (rows ? rows[i] : i) * lda + j) : __builtin_nan("");
}

// Moments of E over a 64-row x 256-column tile: each thread owns one column
// (its r entries of Z in registers) and walks the tile's rows; the tile's
// rows of C are staged in LDS.  x = sum_a C[i][a] Z[a][c] in increasing a.
// Per-workgroup partial sums (sum e, e^2, |e|, w^2) go to `partials`.
template <typename T, int RM>
__global__ void __launch_bounds__(kResThreads) resid_kernel(const T *A, int64_t lda, int r, const int64_t *rows,
                                                            const int64_t *cols, int64_t nq, int64_t ns,
                                                            const double *Z, const double *Cg, double *partials) {
    __shared__ double cs[kResTileRows * RM];
    __shared__ double red[4][kResThreads];
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.y * kResTileRows;
    const int64_t c = (int64_t)blockIdx.x * kResThreads + tid;
    const int nrows = (int)std::min<int64_t>(kResTileRows, nq - row0);
    for (int e = tid; e < nrows * r; e += kResThreads) cs[e] = Cg[row0 * r + e];
    __syncthreads();
    double se = 0.0, se2 = 0.0, sabs = 0.0, sw2 = 0.0;
    if (c < ns) {
        double z[RM];
#pragma unroll
        for (int a = 0; a < RM; a++) z[a] = a < r ? Z[(int64_t)a * ns + c] : 0.0;
        const int64_t col = cols ? cols[c] : c;
        for (int i = 0; i < nrows; i++) {
            const int64_t row = rows ? rows[row0 + i] : row0 + i;
            const double w = Elem<T>::load(A, row * lda + col);
            double x = 0.0;
#pragma unroll
            for (int a = 0; a < RM; a++)
                if (a < r) x += cs[i * r + a] * z[a];
            const double e = w - x;
            se += e;
            se2 += e * e;
            sabs += fabs(e);
            sw2 += w * w;
        }
    }
    red[0][tid] = se;
    red[1][tid] = se2;
    red[2][tid] = sabs;
    red[3][tid] = sw2;
    __syncthreads();
    for (int h = kResThreads / 2; h > 0; h >>= 1) {  // fixed pairwise tree
        if (tid < h)
            for (int k = 0; k < 4; k++) red[k][tid] += red[k][tid + h];
        __syncthreads();
    }
    if (tid < 4) partials[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 4 + tid] = red[tid][0];
}

// Sum the per-workgroup partials in a fixed order.
__global__ void resid_sum_kernel(const double *partials, int64_t nblocks, double *out) {
    __shared__ double red[4][kResThreads];
    const int tid = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t b = tid; b < nblocks; b += kResThreads)
        for (int k = 0; k < 4; k++) acc[k] += partials[b * 4 + k];
    for (int k = 0; k < 4; k++) red[k][tid] = acc[k];
    __syncthreads();
    for (int h = kResThreads / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int k = 0; k < 4; k++) red[k][tid] += red[k][tid + h];
        __syncthreads();
    }
    if (tid < 4) out[tid] = red[tid][0];
}

template <typename T, int RM>
static hipError_t residual_t(const void *Av, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I,
                             const int64_t *J, const double *U, int q, int s, uint64_t seed, double *out,
                             char *scratch, hipStream_t stream) {
    const T *A = static_cast<const T *>(Av);
    const int64_t nq = q ? q : m, ns = s ? s : n;
    int64_t *rows = nullptr, *cols = nullptr;
    char *p = scratch;
    if (q) {
        rows = reinterpret_cast<int64_t *>(p);
        p += 256 * sizeof(int64_t);
        cols = reinterpret_cast<int64_t *>(p);
        p += 256 * sizeof(int64_t);
        hipLaunchKernelGGL(resid_sample_kernel, dim3(1), dim3(2 * kWave), 0, stream, seed, m, n, q, s, rows, cols);
    }
    double *Z = reinterpret_cast<double *>(p);
    p += sizeof(double) * (size_t)r * ns;
    double *Cg = reinterpret_cast<double *>(p);
    p += sizeof(double) * (size_t)nq * r;
    double *partials = reinterpret_cast<double *>(p);
    hipLaunchKernelGGL((resid_z_kernel<T, RM>), dim3((unsigned)((ns + kResThreads - 1) / kResThreads)), dim3(kResThreads),
                       0, stream, A, m, lda, r, I, U, cols, ns, Z);
    hipLaunchKernelGGL(resid_c_kernel<T>, dim3((unsigned)((nq * r + 255) / 256)), dim3(256), 0, stream, A, n, lda, r,
                       J, rows, nq, Cg);
    const dim3 grid((unsigned)((ns + kResThreads - 1) / kResThreads), (unsigned)((nq + kResTileRows - 1) / kResTileRows));
    hipLaunchKernelGGL((resid_kernel<T, RM>), grid, dim3(kResThreads), 0, stream, A, lda, r, rows, cols, nq, ns, Z, Cg,
                       partials);
    hipLaunchKernelGGL(resid_sum_kernel, dim3(1), dim3(kResThreads), 0, stream, partials,
                       (int64_t)grid.x * grid.y, out);
    return hipGetLastError();
}

size_t residual_scratch_bytes(int64_t m, int64_t n, int r, int q, int s) {
    const int64_t nq = q ? q : m, ns = s ? s : n;
    const int64_t nblocks = ((ns + kResThreads - 1) / kResThreads) * ((nq + kResTileRows - 1) / kResTileRows);
    return 512 * sizeof(int64_t) + sizeof(double) * ((size_t)r * ns + (size_t)nq * r + 4 * (size_t)nblocks);
}

hipError_t launch_residual(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I,
                           const int64_t *J, const double *U, int q, int s, uint64_t seed, double *out, void *scratch,
                           hipStream_t stream) {
    char *sc = static_cast<char *>(scratch);
#define LRA_RES(TT, RR) return residual_t<TT, RR>(A, m, n, lda, r, I, J, U, q, s, seed, out, sc, stream)
#define LRA_RES_R(TT)      \
    if (r <= 16) LRA_RES(TT, 16); \
    if (r <= 32) LRA_RES(TT, 32); \
    LRA_RES(TT, 64)
    if (dtype == LRA_F64) { LRA_RES_R(double); }
    if (dtype == LRA_F32) { LRA_RES_R(float); }
    LRA_RES_R(uint16_t);
#undef LRA_RES_R
#undef LRA_RES
}

// ------------------------------------------------------------------ adjoint
// One workgroup per block b of the batch.  With Z = G^{-1} R, the loss
// L = sum over Omega of (a_ij - (C Z)_ij)^2 and Ebar = -2 (a - C Z) on Omega:
//   dC = Ebar Z^T (row pass over Omega in row order),
//   dZ = C^T Ebar (column pass in column order), dR = G^{-T} dZ,
//   dG = -G^{-T} dZ Z^T.
// Omega is given sorted by row (then column) with `corder`, the stable
// permutation that sorts it by column, so both passes are plain gathers and
// every sum runs in the order of the oracle's scan.  Z and dZ go to the
// block's slice of `ws` (2 r n doubles).  The r x r inverse uses LDS.
__device__ __forceinline__ int64_t lower_bound_i32(const int32_t *a, int64_t n, int32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int64_t lower_bound_perm(const int32_t *a, const int32_t *perm, int64_t n, int32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[perm[mid]] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int RM>
__global__ void __launch_bounds__(kAdjThreads) adjoint_kernel(int64_t m, int64_t n, int r, const double *Cb,
                                                              const double *Rb, const double *Gb, int64_t nnz,
                                                              const int32_t *orow_b, const int32_t *ocol_b,
                                                              const int32_t *corder_b, const double *aval_b,
                                                              double *loss, double *dCb, double *dRb, double *dGb,
                                                              double *ws, int32_t *status) {
    extern __shared__ __align__(16) double lds[];
    double *LU = lds, *Gi = lds + r * r, *Tm = lds + 2 * r * r;
    __shared__ int p[RM];
    __shared__ int sing;
    __shared__ double ld;
    __shared__ double red[kAdjThreads];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const double *C = Cb + b * m * r, *R = Rb + b * r * n, *G = Gb + b * r * r;
    const int32_t *orow = orow_b + b * nnz, *ocol = ocol_b + b * nnz, *corder = corder_b + b * nnz;
    const double *aval = aval_b + b * nnz;
    double *dC = dCb + b * m * r, *dR = dRb + b * r * n, *dG = dGb + b * r * r;
    double *Z = ws + b * 2 * r * n, *dZ = Z + (int64_t)r * n;

    // Omega indices outside the block (or a col_order entry outside [0, nnz))
    // are reported as LRA_EINVAL before anything is read through them
    int bad = 0;
    for (int64_t q = tid; q < nnz; q += kAdjThreads) {
        const int32_t i = orow[q], j = ocol[q], t = corder[q];
        bad |= (i < 0 || i >= m || j < 0 || j >= n || t < 0 || t >= nnz) ? 1 : 0;
    }
    if (__syncthreads_or(bad)) {
        if (tid == 0) {
            status[b] = LRA_EINVAL;
            loss[b] = __builtin_nan("");
        }
        return;
    }
    for (int e = tid; e < r * r; e += kAdjThreads) LU[e] = G[e];
    __syncthreads();
    inverse_lds(LU, Gi, p, r, kAdjThreads, &sing, &ld);
    if (sing) {
        if (tid == 0) {
            status[b] = LRA_ESINGULAR;
            loss[b] = __builtin_nan("");
        }
        return;
    }
    // Z = G^{-1} R, one column per thread
    for (int64_t j = tid; j < n; j += kAdjThreads) {
        double rc[RM];
#pragma unroll
        for (int q = 0; q < RM; q++) rc[q] = q < r ? R[(int64_t)q * n + j] : 0.0;
        for (int a = 0; a < r; a++) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < RM; q++)
                if (q < r) acc += Gi[a * r + q] * rc[q];
            Z[(int64_t)a * n + j] = acc;
        }
    }
    __threadfence();
    __syncthreads();
    // row pass: loss and dC, one row per thread
    double lsum = 0.0;
    for (int64_t i = tid; i < m; i += kAdjThreads) {
        const int64_t q0 = lower_bound_i32(orow, nnz, (int32_t)i), q1 = lower_bound_i32(orow, nnz, (int32_t)(i + 1));
        double ci[RM], dc[RM];
#pragma unroll
        for (int a = 0; a < RM; a++) {
            ci[a] = a < r ? C[i * r + a] : 0.0;
            dc[a] = 0.0;
        }
        for (int64_t q = q0; q < q1; q++) {
            const int64_t j = ocol[q];
            double zj[RM];
#pragma unroll
            for (int a = 0; a < RM; a++) zj[a] = a < r ? Z[(int64_t)a * n + j] : 0.0;
            double x = 0.0;
#pragma unroll
            for (int a = 0; a < RM; a++)
                if (a < r) x += ci[a] * zj[a];
            const double e = aval[q] - x;
            lsum += e * e;
            const double eb = -2.0 * e;
#pragma unroll
            for (int a = 0; a < RM; a++)
                if (a < r) dc[a] += eb * zj[a];
        }
        for (int a = 0; a < r; a++) dC[i * r + a] = dc[a];
    }
    // column pass: dZ and dR, one column per thread
    for (int64_t j = tid; j < n; j += kAdjThreads) {
        const int64_t t0 = lower_bound_perm(ocol, corder, nnz, (int32_t)j);
        const int64_t t1 = lower_bound_perm(ocol, corder, nnz, (int32_t)(j + 1));
        double zj[RM], dz[RM];
#pragma unroll
        for (int a = 0; a < RM; a++) {
            zj[a] = a < r ? Z[(int64_t)a * n + j] : 0.0;
            dz[a] = 0.0;
        }
        for (int64_t t = t0; t < t1; t++) {
            const int64_t q = corder[t];
            const int64_t i = orow[q];
            double ci[RM];
#pragma unroll
            for (int a = 0; a < RM; a++) ci[a] = a < r ? C[i * r + a] : 0.0;
            double x = 0.0;
#pragma unroll
            for (int a = 0; a < RM; a++)
                if (a < r) x += ci[a] * zj[a];
            const double eb = -2.0 * (aval[q] - x);
#pragma unroll
            for (int a = 0; a < RM; a++)
                if (a < r) dz[a] += eb * ci[a];
        }
        for (int a = 0; a < r; a++) {
            dZ[(int64_t)a * n + j] = dz[a];
            double acc = 0.0;  // (G^{-T} dZ)[a][j] = sum_q Gi[q][a] dZ[q][j]
#pragma unroll
            for (int q = 0; q < RM; q++)
                if (q < r) acc += Gi[q * r + a] * dz[q];
            dR[(int64_t)a * n + j] = acc;
        }
    }
    __threadfence();
    __syncthreads();
    // T = dZ Z^T, then dG = -G^{-T} T
    for (int e = tid; e < r * r; e += kAdjThreads) {
        const int a = e / r, c2 = e % r;
        double acc = 0.0;
        for (int64_t j = 0; j < n; j++) acc += dZ[(int64_t)a * n + j] * Z[(int64_t)c2 * n + j];
        Tm[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < r * r; e += kAdjThreads) {
        const int a = e / r, c2 = e % r;
        double acc = 0.0;
        for (int q = 0; q < r; q++) acc += Gi[q * r + a] * Tm[q * r + c2];
        dG[e] = -acc;
    }
    red[tid] = lsum;
    __syncthreads();
    for (int h = kAdjThreads / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) {
        loss[b] = red[0];
        status[b] = LRA_OK;
    }
}

hipError_t launch_adjoint(int64_t count, int64_t m, int64_t n, int r, const double *C, const double *R,
                          const double *G, int64_t nnz, const int32_t *orow, const int32_t *ocol,
                          const int32_t *corder, const double *aval, double *loss, double *dC, double *dR,
                          double *dG, double *ws, int32_t *status, hipStream_t stream) {
    const size_t lds = sizeof(double) * 3 * (size_t)r * r;
#define LRA_ADJ(RR)                                                                                              \
    hipLaunchKernelGGL(adjoint_kernel<RR>, dim3((unsigned)count), dim3(kAdjThreads), lds, stream, m, n, r, C, R, G, \
                       nnz, orow, ocol, corder, aval, loss, dC, dR, dG, ws, status)
    if (r <= 16) LRA_ADJ(16);
    else if (r <= 32) LRA_ADJ(32);
    else LRA_ADJ(64);
#undef LRA_ADJ
    return hipGetLastError();
}

}  // namespace lra
