// lra_internal.h -- private declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lra_cur.h"

namespace lra {

constexpr int kBlock = 512;  // threads per workgroup (8 wavefronts, two per SIMD)
constexpr int kRMax = 64;    // largest supported rank
constexpr int kLMax = 256;   // largest number of sampled SRHT columns
constexpr int kSMax = 256;   // largest number of rows or columns drawn by the leverage-score refinement

// Team exchange (64-bit tagged words): per workgroup and parity 2 header
// words (value, item, slot and flags in two 60-bit payloads), each
// workgroup's header on a 128-byte line of its own (headers sharing a line
// serialise the stores of different workgroups to it), and 2 words per row
// entry.
constexpr int kHdrWords = 2;
constexpr int kHdrStride = 16;
constexpr int kMaxTeam = 256;
constexpr int kRowWords = 2 * kLMax;
constexpr int kSlotWords = kHdrStride + kRowWords;  // exchange words per workgroup and parity

struct CAConfig {
    int32_t r, sweeps;
    double delta;
    int32_t max_swaps;
    int32_t pre, ah_depth, ah_samples, refine_steps;
    int32_t panel_bytes;      // offset of the flag bytes inside dynamic LDS
    const int64_t *init_cols; // device copy of the warm-start columns, or null
    double *sketch_ws;        // global sketch panels [team][ipw * l] when they do not fit LDS, else null
    const int32_t *bd_table;  // bidiagonal start: per sampled column its term count, positions, coefficients
    int32_t margins;          // 1: report the decisions' smallest margin in lra_info.min_margin (else NaN)
};

// Complex coefficients of the abridged Fourier sketch (l 2^d <= kAftCoefs,
// cos and sin each): they fit the LU scratch of Smem (kRMax (kRMax - 1) / 2
// doubles).
constexpr int kAftCoefs = 1008;

// Terms of one sampled column of the bidiagonal-product multiplier (2^q, q <= 6).
constexpr int kBdTerms = 64;
// Table layout: cnt[kLMax], then pos[kLMax][kBdTerms], then coef[kLMax][kBdTerms].
constexpr size_t kBdTableInts = (size_t)kLMax * (1 + 2 * kBdTerms);

struct TeamWs {
    uint64_t *xw;         // exchange words [2][team][kSlotWords]
    uint64_t spin_limit;  // wall-clock ticks one exchange poll may wait before the launch gives up
};

struct BlockDesc {
    int64_t offset, m, n, lda;
};
// Point-set block: rows x_off .. x_off + m - 1, columns y_off .. y_off + n - 1
// of the point buffer (same size as BlockDesc, so both share one buffer).
struct PtsDesc {
    int64_t x_off, y_off, m, n;
};
static_assert(sizeof(PtsDesc) == sizeof(BlockDesc), "block descriptors share one device buffer");


hipError_t launch_team(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, uint64_t seed, const CAConfig &cfg,
                       const TeamWs &ws, int team, size_t dyn_bytes, int64_t *I_out, int64_t *J_out, double *U_out,
                       lra_info *info, hipStream_t stream);

hipError_t launch_batched(int dtype, const void *base, const BlockDesc *blocks, const int32_t *order, int64_t count,
                          uint64_t seed, const CAConfig &cfg, unsigned *queue, int grid, size_t dyn_bytes,
                          int64_t *I_out, int64_t *J_out, double *U_out, lra_info *infos, hipStream_t stream);

int batched_occupancy(int dtype, size_t dyn_bytes);
hipError_t launch_points(const double *pts, const PtsDesc *blocks, const int32_t *order, int64_t count,
                         uint64_t seed, const CAConfig &cfg, unsigned *queue, int grid, size_t dyn_bytes,
                         int64_t *I_out, int64_t *J_out, double *U_out, lra_info *infos, hipStream_t stream);
int points_occupancy(size_t dyn_bytes);
hipError_t launch_hadamard(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, int d, uint64_t seed,
                           const CAConfig &cfg, const TeamWs &ws, int team, size_t dyn_bytes, int64_t *I_out,
                           int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream);
hipError_t launch_bidiag_table(uint64_t seed, int64_t N, int q, int l, int32_t *table, hipStream_t stream);
hipError_t launch_cynical(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, uint64_t seed, int32_t loops,
                          const CAConfig &cfg_k, const CAConfig &cfg_r, const TeamWs &ws, int team, size_t dyn_bytes,
                          int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream);
hipError_t launch_projective(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, uint64_t seed, int32_t k,
                             int32_t l, const CAConfig &cfg, const TeamWs &ws, int team, size_t dyn_bytes,
                             int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream);
hipError_t launch_uniform(int dtype, const void *base, const BlockDesc *blocks, int64_t count, uint64_t seed,
                          int32_t r, int32_t k, int32_t l, int grid, size_t dyn_bytes, int64_t *I_out, int64_t *J_out,
                          double *U_out, lra_info *infos, hipStream_t stream);
int uniform_occupancy(int dtype, size_t dyn_bytes);
hipError_t launch_leverage(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I0,
                           const int64_t *J0, int k, int l, uint64_t seed, double *ws, int32_t *flags,
                           int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream);
size_t leverage_scratch_bytes(int64_t m, int64_t n, int r);

size_t residual_scratch_bytes(int64_t m, int64_t n, int r, int q, int s, int prec);
hipError_t launch_residual(int dtype, const void *A, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I,
                           const int64_t *J, const double *U, int q, int s, uint64_t seed, int prec, double *out,
                           void *scratch, hipStream_t stream);
hipError_t launch_posterior(const double *moments, int64_t K, double tau, double z, lra_posterior *out,
                            hipStream_t stream);
size_t adjoint_scratch_bytes(int64_t count, int64_t m, int64_t n, int64_t nnz, int r);
hipError_t launch_adjoint(int64_t count, int64_t m, int64_t n, int r, const double *C, const double *R,
                          const double *G, int64_t nnz, const int32_t *orow, const int32_t *ocol,
                          const int32_t *corder, const double *aval, double *loss, double *dC, double *dR,
                          double *dG, void *scratch, int32_t *status, hipStream_t stream);
hipError_t launch_xlat(uint64_t *buf, int rounds, uint64_t limit, hipStream_t stream);
// C-A with DMM08 sampling of every sketch (lra_dmm.hip): one workgroup per
// block; scratch holds 2 scratch_items doubles per workgroup of the grid.
size_t dmm_lds_bytes();
int dmm_occupancy(int dtype);
hipError_t launch_dmm(int dtype, const void *base, const BlockDesc *blocks, int64_t count, uint64_t seed, int r, int k,
                      int l, int iters, double *scratch, int64_t scratch_items, int grid, int64_t *I_out,
                      int64_t *J_out, double *U_out, lra_info *infos, hipStream_t stream);
size_t static_lds_bytes();
__global__ void zero_u32_kernel(unsigned *p, int n);
__global__ void zero_team_kernel(uint64_t *p, int64_t n, lra_info *info);

// Batched C-A with register-resident panels (lra_batch.hip): variants exist
// for rank r and P items per lane; `src` is the dtype code, or 3 for point sets.
bool reg_variant_exists(int r, int P);
int reg_occupancy(int r, int P, int waves, int src);
hipError_t launch_reg(int src, int r, int P, int waves, const void *base, const void *blocks, const int32_t *order,
                      int64_t count, uint64_t seed, const CAConfig &cfg, unsigned *queue, int grid, int64_t *I_out,
                      int64_t *J_out, double *U_out, lra_info *infos, hipStream_t stream);

}  // namespace lra
