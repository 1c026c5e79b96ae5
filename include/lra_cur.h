/*
 * lra_cur.h -- C ABI of the MI355X (gfx950) cross-approximation CUR library.
 *
 * The library computes CUR low-rank approximations W' = C U R of an m x n
 * matrix W, with C = W[:, J] (r columns), R = W[I, :] (r rows) and the r x r
 * nucleus U = W[I, J]^{-1} (or, for a numerically singular generator, the
 * pseudo-inverse of its truncation), by cross-approximation (C-A) iterations:
 * alternating maxvol searches on the gathered m x r column panel and the
 * r x n row panel (Pan, Luan, Svadlenka, Zhao, "Superfast Accurate Low Rank
 * Approximation": CUR definition eq. (eqcur0), C-A loops in Section 1.3 and
 * Fig. 4, Tests 2 and eq. (eqtsts1) in Section 13, the dominant-submatrix
 * search of Algorithms alggos and algdomin in Appendix D, the canonical
 * nucleus of Algorithm algcnnncl in Section 3, and the abridged randomized
 * Hadamard pre-processing of Section 11 and Appendix B).
 *
 * Conventions shared by every entry point
 *   - W is dense, row-major, element (i, j) at W[i * lda + j], lda >= n, and
 *     resides in device memory of the current HIP device.
 *   - Index sets are 0-based int64 and are returned sorted ascending.
 *   - U is returned row-major r x r with rows ordered like J and columns
 *     ordered like I, so that W' = W[:, J] * U * W[I, :].
 *   - All device pointers are owned by the caller.  The library keeps a small
 *     cached workspace per (device, stream); lra_release() frees it.
 *   - Calls are asynchronous on `stream`.  The return value reports argument
 *     and launch errors only.  Failures found while computing (a rank
 *     deficient panel, a non-finite entry read) are written to the `status`
 *     field of the optional device-resident lra_info.
 *   - Results are deterministic for a given input, seed, options and device.
 *   - Calls that share a (device, stream) workspace are ordered by the stream;
 *     calls on different streams use different workspaces.
 */
#ifndef LRA_CUR_H
#define LRA_CUR_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LRA_OK = 0,
    LRA_EINVAL = 1,       /* bad argument, or a non-finite entry in a panel read */
    LRA_ESINGULAR = 2,    /* a gathered panel (or the sketch) has rank < r */
    LRA_EDEVICE = 3,      /* HIP runtime error */
    LRA_ENOMEM = 4,       /* workspace allocation failed */
    LRA_EUNSUPPORTED = 5  /* shape does not fit the on-chip panel layout */
} lra_status;

typedef enum { LRA_F64 = 0, LRA_F32 = 1, LRA_BF16 = 2 } lra_dtype;

typedef enum {
    LRA_PREC_PLAIN = 0,  /* FP64 arithmetic (FP64 matrix cores for dense products) */
    LRA_PREC_MIXED = 1   /* dense products as three BF16 matrix-core products of a
                            hi/lo split, FP32 accumulation; sums stay FP64 */
} lra_prec;

typedef enum {
    LRA_PRE_NONE = 0,  /* random initial column set (seeded) */
    LRA_PRE_ASRHT = 1, /* start set from greedy QRP on an abridged SRHT sketch: columns
                          of M^T W (m >= n, the start column set itself) or rows of
                          W M (m < n, followed by one row step) */
    LRA_PRE_BIDIAG = 2, /* the same with the quasi-Gaussian multiplier of random
                          bidiagonal factors G_q = B_1 P_1 ... B_q P_q (eq. (def11),
                          section on pre-processing with quasi Gaussian matrices),
                          q = ah_depth <= 6 factors, l = ah_samples sampled columns;
                          the multiplied dimension must stay below 2^31 */
    LRA_PRE_ASRFT = 3  /* the same with the abridged randomized Fourier multiplier
                          D Omega_{N,d} (App. B, eq. (eqfd) stopped after d <= 3
                          stages: column b s + e holds omega_N^{b j} at rows
                          j = a s + e, omega_N = exp(2 pi i / N)), D_j = i^{t_j}
                          with t_j the top two bits of SplitMix64 stream 1, l =
                          ah_samples complex columns (r <= 2l, l 2^d <= 1008,
                          l <= 128); the seed QRP runs on the real form of the
                          sketch, Re y_q and Im y_q as coordinates q and l + q */
} lra_pre;

typedef struct {
    double delta;          /* maxvol stops when every |B_ij| <= 1 + delta; default 0.01 */
    int32_t max_swaps;     /* swap cap per maxvol search; < 0 selects 16 r (default) */
    int32_t preprocess;    /* lra_pre; default LRA_PRE_NONE */
    int32_t ah_depth;      /* abridged Hadamard recursion depth d, or bidiagonal factor count q; default 3 */
    int32_t ah_samples;    /* sampled multiplier columns l (r <= l <= 256); <= 0 selects 2 r */
    int32_t refine_steps;  /* iterative refinement steps of the nucleus inverse; default 0 */
    int32_t team_size;     /* workgroups cooperating on one LRA; <= 0 chooses automatically */
    int32_t track_margin;  /* 1: report lra_info.min_margin (C-A entry points; costs time), 0 (default): NaN */
    const int64_t *init_cols; /* optional HOST array of r distinct start columns (warm start) */
} lra_opts;

typedef struct {
    int32_t status;        /* lra_status of the device computation */
    int32_t sweeps_run;    /* sweeps executed (stops early at a fixed point) */
    int32_t swaps_total;   /* maxvol swaps over all steps */
    int32_t converged;     /* 1 if every maxvol search met the 1 + delta rule */
    int32_t rank_found;    /* r, or the rank of the first rank-deficient panel */
    int32_t team_size;     /* workgroups used */
    int32_t nucleus_rank;  /* r, or the rank kept by the truncated pseudo-inverse nucleus */
    int32_t reserved;
    double det_log_abs;    /* log |det W[I, J]| of the final generator (-inf if singular) */
    double min_margin;     /* the smallest relative margin of the run's decisions (below); NaN where not tracked */
} lra_info;
/* min_margin: with opts.track_margin = 1, lra_cur, lra_cur_noalloc,
 * lra_cur_hadamard and the batched C-A entry points take, at every
 * decision, the gap between the winner and the runner-up relative to the
 * winner, (v1 - v2) / v1, over all candidates (pivot |C_ik| of the panel LU,
 * |B_ij| of a swap search, squared norm of the sketch QRP; 1 without a
 * runner-up, 0 for a tie), and at every stop test of a swap search
 * |v1 - (1 + delta)| / (1 + delta); the minimum over the run, 1 when nothing
 * was decided.  A decision whose margin is near rounding level could go the
 * other way under a perturbation of that size.  Tracking carries the best two
 * values through every reduction (a separate kernel instantiation; about
 * 8% slower for one team LRA, 15% for a batch).  lra_cur_dmm_batched reports
 * the smallest distance of a draw's target u_t S from the running sums that
 * bound the item it picked, relative to S.  The other entry points report
 * NaN. */

/* Fill *o with the defaults listed above. */
void lra_default_opts(lra_opts *o);

/* C-A CUR of one matrix.
 *   W       device, dtype `dt`, m x n with leading dimension lda.
 *   r       target rank, 1 <= r <= min(m, n, 64).
 *   sweeps  number of C-A loops (column step, then row step), >= 1.
 *   seed    seeds the SplitMix64 draws (initial columns, SRHT signs and samples).
 *   opts    NULL for defaults.
 *   I_out, J_out   device int64[r]; U_out device double[r * r];
 *   info    device lra_info or NULL.
 * Panels live in on-chip memory: every cooperating workgroup holds
 * ceil(max(m, n) / team) items of max(r, l) doubles; shapes that do not fit
 * return LRA_EUNSUPPORTED. */
lra_status lra_cur(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r,
                   int32_t sweeps, uint64_t seed, const lra_opts *opts, int64_t *I_out, int64_t *J_out,
                   double *U_out, lra_info *info, hipStream_t stream);

/* Bytes of device scratch that lra_cur_noalloc keeps on each GPU it runs on. */
#define LRA_NOALLOC_SCRATCH_BYTES 10683392

/* lra_cur for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * computation, results and arguments as lra_cur, but every work buffer of
 * the launch (the team exchange words, the bidiagonal column table, the
 * global sketch panel) lives in one fixed device array of
 * LRA_NOALLOC_SCRATCH_BYTES per GPU, set up on the first call on that GPU and
 * held until the process ends.  The call allocates nothing: no hipMalloc,
 * no hipFree, no host allocation.  The caller still owns W and the outputs.
 *   - All calls on one GPU share its array, which keeps the last call's
 *     contents: calls that overlap in time on one GPU (on different streams
 *     or from different threads) race, and the caller must order them.  The
 *     exchange words are cleared by a kernel at the start of every
 *     multi-workgroup launch; nothing else has to start at zero.
 *   - opts->init_cols must be NULL (LRA_EINVAL): a host start set would need
 *     a staging copy.
 *   - When the sketch slices do not fit on chip the launch needs
 *     team x ceil(items / team) x l doubles of global sketch panel (items =
 *     the dimension the multiplier acts on); above 8 MiB the call returns
 *     LRA_EUNSUPPORTED and launches nothing.
 * Errors and asynchrony otherwise as for lra_cur. */
lra_status lra_cur_noalloc(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r,
                           int32_t sweeps, uint64_t seed, const lra_opts *opts, int64_t *I_out, int64_t *J_out,
                           double *U_out, lra_info *info, hipStream_t stream);

/* C-A CUR of the pre-processed matrix W' = W M (Section 13: Tests 2 on inputs
 * multiplied by an abridged randomized Hadamard matrix; Appendix B for the
 * multiplier).  M = D (H_{2^d} (x) I_s) has order N = 2^d s, s = ceil(n / 2^d)
 * (W is zero-padded to N columns), D = diag of the Rademacher signs of
 * SplitMix64 stream 1 of `seed` (the signs of LRA_PRE_ASRHT), H_{2^d} the
 * Sylvester-Hadamard matrix, no scale: entry (i, b s + e) of W' is the sum
 * over a = 0 .. 2^d - 1 (in that order, a s + e < n) of
 * W[i][a s + e] D[a s + e] (-1)^{popcount(a & b)}.  The entries are formed on
 * the fly; W' is never stored.  Returns I (rows of W' = rows of W), J
 * (columns of W', in [0, N)) and U for W' ~ W'[:, J] U W'[I, :]; since
 * M M^T = 2^d I, the LRA of W is W ~ W'[:, J] U W'[I, :] M^T / 2^d.
 *   0 <= d <= 6; 1 <= r <= min(m, n, 64); opts->preprocess and
 *   opts->init_cols are not supported (LRA_EINVAL).  Start set, sweeps,
 *   outputs and errors otherwise as lra_cur on an m x N matrix. */
lra_status lra_cur_hadamard(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r,
                            int32_t sweeps, uint64_t seed, int32_t d, const lra_opts *opts, int64_t *I_out,
                            int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream);

/* Cynical CUR (Section 1.3 and Fig. 3: an r x r generator of locally maximal
 * volume inside a random k x k sketch; Section 13, Tests 3 with loops = 0 and
 * Tests 4 with loops = 1, k = l = 4r in the paper).
 *   L   k distinct random columns (stream 0 of `seed`);
 *   loops = 0: K k distinct random rows (stream 5);
 *   loops >= 1: that many C-A loops at rank k from L (column step, row step),
 *               stopping early at a fixed point, give K and L;
 *   then C-A at rank r on the k x k matrix W[K, L] (seed + 1, `sweeps` loops)
 *   and U = W[I, J]^{-1} with the same nucleus rules as lra_cur.
 * 1 <= r <= k <= min(m, n, 64); opts->preprocess and opts->init_cols are not
 * supported (LRA_EINVAL); opts->max_swaps applies to both ranks (default 16
 * times the rank).  info describes the rank-r C-A on the sketch, with
 * swaps_total counting both phases and team_size the team of the rank-k
 * loops (1 when loops = 0).  Arguments, layout and errors otherwise as for
 * lra_cur. */
lra_status lra_cur_cynical(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r, int32_t k,
                           int32_t loops, int32_t sweeps, uint64_t seed, const lra_opts *opts, int64_t *I_out,
                           int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream);

/* C-A with k x l CUR generators of large r-projective volume (section
 * "Extension of the maximization of the r-projective volume", Algorithm
 * algprjvlm transposed as its Remark reprvtov allows, with the greedy
 * Algorithms alg1tor and algrup of the Appendix and the expansion-
 * contraction exchanges that follow them as its black box) and the
 * canonical nucleus U = W[I, J]_r^+ of Algorithm algcnnncl; Theorem th3
 * bounds the error of such a CUR by a factor that shrinks as k, l grow past r.
 *   J starts as l distinct random columns (stream 0 of `seed`).  A sweep is a
 *   column step, I = k rows chosen in W[:, J], and a row step, J = l columns
 *   chosen in W[I, :], each by: r steps of greedy Householder QRP of the
 *   panel's items truncated at r (R' = Q_r^T panel^T), greedy QRP on R'
 *   (r items), then greedy expansion to k (or l) items, each time the item
 *   y maximising y^T (S S^T)^{-1} y, S the chosen columns of R' (ties to the
 *   lowest item); then exchanges: add the best candidate b, drop the member
 *   s != b of least y_s^T (S' S'^T)^{-1} y_s in the grown set S', while the
 *   product of the two volume factors exceeds 1 + opts->delta, at most
 *   opts->max_swaps times per step (defaults 0.01 and 16 r).  The loop stops
 *   early when a sweep repeats the sets.
 *   U = pseudo-inverse of the rank-r SVD truncation of W[I, J] (one-sided
 *   Jacobi; the r largest singular values above max(1e-14, max(k, l) 2^-52) times the
 *   largest).
 * Outputs (device): I_out int64[k], J_out int64[l], both ascending; U_out
 * double[l * k], row-major, J-order x I-order, so W ~ W[:, J] U W[I, :].
 * info (device, may be NULL): nucleus_rank = singular values kept,
 * det_log_abs = log of their product (the r-projective volume of W[I, J]),
 * swaps_total = exchanges over all steps, converged = 0 when a cap stopped
 * a profitable exchange.
 * 1 <= r <= min(k, l); k <= min(m, 64); l <= min(n, 64); sweeps >= 1.
 * opts->delta, opts->max_swaps and opts->team_size are used;
 * opts->preprocess and opts->init_cols must be unset (LRA_EINVAL).  ESINGULAR: a panel of rank below r (rank_found = the
 * step).  Errors and asynchrony otherwise as for lra_cur. */
lra_status lra_cur_projective(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r, int32_t k,
                              int32_t l, int32_t sweeps, uint64_t seed, const lra_opts *opts, int64_t *I_out,
                              int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream);

/* One block of a batch: the block starts `offset` elements after `base`. */
typedef struct {
    int64_t offset, m, n, lda;
} lra_block;

/* C-A CUR of many independent blocks (one workgroup per block, blocks taken
 * from device work queues largest first).  Block b uses seed + b and gets
 * exactly the sets and nucleus that lra_cur returns for it alone with seed
 * + b.  Blocks are binned by max(m, n) with the rule table below; each bin is
 * one persistent launch on `stream`, of the register-panel kernel variant
 * its rule names, or of the LDS-panel kernel when no rule covers the block.
 * `blocks` is a HOST array of `count` descriptors, copied through a pinned
 * staging buffer (the call does not wait for the device; a call whose
 * descriptors equal the previous call's on this stream copies nothing).
 * Outputs are packed: I_out/J_out int64[count * r], U_out double[count * r *
 * r], infos lra_info[count] (device, may be NULL).  opts->preprocess and
 * opts->init_cols are not supported here (LRA_EINVAL). */
lra_status lra_cur_batched(const void *base, lra_dtype dt, const lra_block *blocks, int64_t count, int32_t r,
                           int32_t sweeps, uint64_t seed, const lra_opts *opts, int64_t *I_out, int64_t *J_out,
                           double *U_out, lra_info *infos, hipStream_t stream);

/* One rule of the batched launch's bin table: blocks of rank r whose larger
 * dimension is at most max_dim (and above every smaller rule's) run on the
 * register-panel kernel with items_per_lane x waves x 64 item slots per
 * workgroup (waves wavefronts of 64 lanes, each lane holding items_per_lane
 * items of the panel in registers); items_per_lane = 0 sends them to the
 * LDS-panel kernel.  Variants exist for r = 16 with items_per_lane = 2 and
 * waves 1 .. 8 (up to 1024 items).  Every variant computes the same results;
 * only speed differs. */
typedef struct {
    int32_t max_dim, r, items_per_lane, waves;
} lra_batch_rule;

/* Replace the process-wide bin table of lra_cur_batched and
 * lra_cur_batched_points (count <= 64 rules, applied in increasing max_dim);
 * count = 0 restores the built-in table, which the project's tuner
 * (paper_1710_07946_amd/tune_batched.py, timing every variant per bin on this
 * device) writes at build time.  LRA_EINVAL for a malformed rule,
 * LRA_EUNSUPPORTED for a variant that is not compiled. */
lra_status lra_batch_set_rules(const lra_batch_rule *rules, int32_t count);

/* Copy up to `cap` rules of the current table to `out` (host); returns the
 * number of rules in the table. */
int32_t lra_batch_get_rules(lra_batch_rule *out, int32_t cap);

/* Refinement of a CUR LRA by its leverage scores (section on refining an
 * LRA with leverage scores: the scores of a crude LRA stand in for those of
 * W; Algorithm algcurlevsc with them, Algorithm algsmplex for the draws;
 * canonical nucleus of Algorithm algcnnncl).  The crude LRA is the CUR of
 * the r rows I0 and r columns J0 (device arrays, e.g. from lra_cur):
 *   column scores q_j = R_j^T (R R^T)^{-1} R_j of R = W[I0, :] and row
 *   scores of C = W[:, J0] likewise (Cholesky factor of the Gram matrix, sums
 *   in increasing item order);
 *   J = l draws by q (first column whose running sum exceeds u S, u the
 *   53-bit uniform from SplitMix64 stream 8 output t), I = k draws by the
 *   row scores (stream 9), both sorted ascending, duplicates kept;
 *   U = D M_r^+ Dbar with D = diag(1 / sqrt(l q_j / S)), Dbar likewise,
 *   M = Dbar W[I, J] D and M_r^+ the pseudo-inverse of M's rank-r SVD
 *   truncation.
 * Outputs (device): I_out int64[k], J_out int64[l], U_out double[l * k]
 * (row-major, W ~ W[:, J] U W[I, :]); info (device, may be NULL):
 * nucleus_rank, det_log_abs = log of the kept singular values' product of M.
 * 1 <= r <= min(m, n, 64); r <= k, l <= 256.  The call copies I0 and J0 to
 * the host and synchronizes `stream` to check them (LRA_EINVAL when out of
 * range); a non-finite entry read gives status LRA_EINVAL, a rank-deficient
 * factor LRA_ESINGULAR (in info), with I = J = -1 and U = NaN.  Scratch:
 * 8 (2 + r) (n + m) bytes + 1152 KiB of the stream's cached workspace (the
 * FP64 copy of C and R, scores, running sums, Gram matrices and factors,
 * and the nucleus's rotations when k or l exceeds 64). */
lra_status lra_cur_leverage(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r,
                            const int64_t *I0, const int64_t *J0, int32_t k, int32_t l, uint64_t seed,
                            int64_t *I_out, int64_t *J_out, double *U_out, lra_info *info, hipStream_t stream);

/* CUR with uniform leverage scores for many blocks (Algorithm algcurlevsc
 * with p_j = 1/n and pbar_i = 1/m: the superfast case of the section on
 * leverage scores for random and average inputs; sampling by Algorithm
 * algsmplex; nucleus by Algorithm algcnnncl).  For block b (seed + b):
 *   J = l column draws from [0, n) with replacement (stream 8),
 *   I = k row draws from [0, m) with replacement (stream 9), both sorted
 *   ascending with duplicates kept;
 *   U = D M_r^+ Dbar, M = Dbar W[I, J] D, D = sqrt(n / l), Dbar = sqrt(m / k),
 *   M_r^+ the pseudo-inverse of M's rank-r SVD truncation (one-sided Jacobi;
 *   the r largest singular values above max(1e-14, max(k, l) 2^-52) times the
 *   largest).
 * Only the k l entries of W[I, J] are read.  `blocks` is a HOST array;
 * outputs (device) are packed: I_out int64[count * k], J_out int64[count * l],
 * U_out double[count * l * k] (each l x k row-major, W ~ W[:, J] U W[I, :]),
 * infos lra_info[count] (may be NULL: status, nucleus_rank, det_log_abs =
 * log of the kept singular values' product of M).  A non-finite generator
 * entry gives that block status LRA_EINVAL, I = J = -1 and U = NaN.
 * 1 <= r <= min(k, l); k, l <= 64 (k > m or l > n allowed: draws repeat).
 * Asynchronous on `stream`. */
lra_status lra_cur_uniform_batched(const void *base, lra_dtype dt, const lra_block *blocks, int64_t count, int32_t r,
                                   int32_t k, int32_t l, uint64_t seed, int64_t *I_out, int64_t *J_out, double *U_out,
                                   lra_info *infos, hipStream_t stream);

/* C-A whose step subalgorithm is the leverage-score sampling of DMM08 on
 * every vertical and horizontal sketch (Section "Testing C-A acceleration of
 * the algorithms of DMM08", Tables 7 and 8; sampling of Algorithm
 * algcurlevsc by Algorithm algsmplex; scores of eq. eqlevsc with beta = 1
 * taken of the sketch), for many blocks, one workgroup per block.  Block b
 * (seed + b):
 *   J = l uniform column draws with replacement (stream 8), D = sqrt(n / l);
 *   iteration t = 0 .. iters - 1:
 *     I = k draws by the rank-r row scores of the sketch W[:, J] D (stream
 *       16 + 2t), Dbar = diag(1 / sqrt(k p_i));
 *     J = l draws by the rank-r column scores of Dbar W[I, :] (stream
 *       17 + 2t), D = diag(1 / sqrt(l p_j));
 *   U = D M_r^+ Dbar, M = Dbar W[I, J] D (truncated pseudo-inverse as in
 *   lra_cur_uniform_batched).
 * Rank-r scores: p_i proportional to |row i of the sketch's r dominant left
 * singular vectors|^2, those with squared singular value above 1e-13 times
 * the largest; draws u_t = (x >> 11) 2^-53 (SplitMix64 output t), the first
 * item whose running sum of scores exceeds u_t S.  I, J sorted ascending,
 * duplicates kept.  Outputs (device) packed as for lra_cur_uniform_batched:
 * I_out int64[count * k], J_out int64[count * l], U_out double[count * l * k];
 * infos (device, may be NULL): status, sweeps_run = iters, nucleus_rank,
 * det_log_abs of M.  A non-finite entry read gives that block LRA_EINVAL, a
 * zero sketch LRA_ESINGULAR, with I = J = -1 and U = NaN.
 * 1 <= r <= min(k, l, m, n) per block; k, l <= 64; iters >= 1.  Scratch:
 * 16 max(m, n) bytes per workgroup of the stream's cached workspace.
 * Asynchronous on `stream`. */
lra_status lra_cur_dmm_batched(const void *base, lra_dtype dt, const lra_block *blocks, int64_t count, int32_t r,
                               int32_t k, int32_t l, int32_t iters, uint64_t seed, int64_t *I_out, int64_t *J_out,
                               double *U_out, lra_info *infos, hipStream_t stream);

/* One far-field interaction block given by its two point sets: rows are the
 * m points starting at point x_off of the point buffer, columns the n points
 * starting at point y_off. */
typedef struct {
    int64_t x_off, y_off, m, n;
} lra_pts_block;

/* C-A CUR of many far-field blocks K_ij = 1 / |x_i - y_j| of planar point
 * sets, with every entry evaluated on the fly in FP64 from the points (the
 * superfast setting of the Superfast Multipole Method discussion, Section
 * "Some Implications and Extensions of Our Study": only the O((m + n) r)
 * entries that the C-A iterations read are ever formed; none is stored).
 *   pts     device double[npts * 2], point p = (pts[2p], pts[2p + 1]);
 *   blocks  HOST array of `count` descriptors; each block needs
 *           0 <= x_off, x_off + m <= npts, 0 <= y_off, y_off + n <= npts and
 *           r <= min(m, n) (else LRA_EINVAL, nothing launched).
 * Entry: dx = x_i0 - y_j0, dy = x_i1 - y_j1, K_ij = 1 / sqrt(dx dx + dy dy),
 * each operation rounded once in FP64.  A block with coinciding points gets
 * a non-finite entry and the status LRA_EINVAL in its info.  Scheduling,
 * seeds (seed + b), outputs and the unsupported options are those of
 * lra_cur_batched. */
lra_status lra_cur_batched_points(const double *pts, int64_t npts, const lra_pts_block *blocks, int64_t count,
                                  int32_t r, int32_t sweeps, uint64_t seed, const lra_opts *opts, int64_t *I_out,
                                  int64_t *J_out, double *U_out, lra_info *infos, hipStream_t stream);

/* Moments of the residual E = W - C U R of a CUR (C = W[:, J], R = W[I, :],
 * U r x r as returned by lra_cur), for the a-posteriori error estimate of
 * Section 4 (a random q x s submatrix of E whose entries are treated as
 * samples of one variable) or for the exact relative error.
 *   q = s = 0     every entry of W;
 *   1..256 each   q rows and s columns drawn (distinct, seeded SplitMix64
 *                 streams 3 and 4 of `seed`).
 *   I, J  device int64[r]; U device double[r * r];
 *   prec  lra_prec: LRA_PREC_PLAIN computes C (U R), e = w - C U R and the
 *         sums in FP64.  LRA_PREC_MIXED forms C (U R) in BF16 x 3 with FP32
 *         accumulation (each entry off by at most about 2^-16 sum_a |C_ia|
 *         |Z_aj|, Z = U R), e and the sums over each 64-column slice of a
 *         row in FP32 (relative error about 1e-6), the totals in FP64.
 *   moments  device double[4]: sum e, sum e^2, sum |e|, sum w^2 over the
 *            entries used (relative Frobenius error = sqrt(m[1] / m[3])).
 * An entry of I or J outside the matrix is not read; it makes the moments NaN.
 * Asynchronous on `stream`.  LRA_EUNSUPPORTED when more than 128 * 65535
 * rows are used. */
lra_status lra_residual(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r, const int64_t *I,
                        const int64_t *J, const double *U, int32_t q, int32_t s, uint64_t seed, int32_t prec,
                        double *moments, hipStream_t stream);

/* Result of the a-posteriori test (device-resident). */
typedef struct {
    int64_t K;         /* entries in the sample, q s */
    double mean;       /* (1/K) sum g_i over the sampled error entries g_i */
    double mean_abs;   /* (1/K) sum |g_i| */
    double var;        /* (1/K) sum (g_i - mean)^2 */
    double threshold;  /* tau^2 ((K - 1) - z sqrt(2 (K - 1))) / K */
    int32_t accept;    /* 1 when var <= threshold */
    int32_t reserved;
} lra_posterior;

/* Superfast a-posteriori check of a CUR (Section 4, the subsection on LRA of a
 * matrix filled with i.i.d. values of a single variable): the K = q s entries
 * g_i of a random q x s submatrix of E = W - C U R (rows and columns drawn as
 * by lra_residual, streams 3 and 4 of `seed`) are taken as observed values of
 * one Gaussian variable, and the customary one-sided test for its variance
 * decides whether the LRA meets the tolerance tau on the error entries' standard
 * deviation: accept (reject sigma^2 >= tau^2) when K var <= tau^2 ((K - 1) -
 * z sqrt(2 (K - 1))), the normal form of the chi-square test, with level
 * Phi(-z) (z = 1.645: 5 %); in the paper's terms the variance may deviate from
 * its observed value by the relative amount t = z sqrt(2 / (K - 1)).  mean,
 * mean_abs (the printed average of |g_i|) and var are reported; var is formed
 * from the sample's moments, sum e^2 / K - mean^2.
 *   1 <= q, s <= 256, q s >= 2; tau > 0 and z finite (else LRA_EINVAL);
 *   prec as lra_residual; I, J, U as lra_cur returns them; out device.
 * Cost O((q + s) r^2 + q s r): only q r + r s + q s entries of W are read.
 * Asynchronous on `stream`. */
lra_status lra_posterior_test(const void *W, lra_dtype dt, int64_t m, int64_t n, int64_t lda, int32_t r,
                              const int64_t *I, const int64_t *J, const double *U, int32_t q, int32_t s,
                              uint64_t seed, int32_t prec, double tau, double z, lra_posterior *out,
                              hipStream_t stream);

/* Adjoint of the CUR reconstruction at fixed index sets, for `count` blocks
 * of equal shape (the paper has no adjoint; this is the derivative of
 * W' = C G^{-1} R with the generator G = W[I, J] as an independent input):
 *   L_b = sum over (i, j) in Omega_b of (a_ij - (C_b G_b^{-1} R_b)_ij)^2,
 *   dC = Ebar Z^T, dR = G^{-T} C^T Ebar, dG = -G^{-T} C^T Ebar Z^T,
 *   with Z = G^{-1} R and Ebar = -2 (a - C Z) on Omega.
 * All pointers are device pointers, FP64 row-major, blocks packed one after
 * another: C count x m x r, R count x r x n, G count x r x r.  Omega has nnz
 * entries per block given as om_row / om_col (int32, sorted by row then
 * column), col_order (int32, the stable permutation that sorts the entries
 * by column) and a_om (the values of W there).  Outputs: loss[count],
 * dC, dR, dG (shapes of C, R, G), status[count]: LRA_OK, LRA_ESINGULAR when
 * G_b is singular, LRA_EINVAL when an Omega index of block b lies outside
 * the block, om_row is not sorted or col_order does not visit the columns
 * in order (then loss[b] is NaN and that block's gradients are not written).
 * m, n and nnz must be below 2^31.  Deterministic: every sum runs in a
 * fixed order. */
lra_status lra_cur_adjoint(int64_t count, int64_t m, int64_t n, int32_t r, const double *C, const double *R,
                           const double *G, int64_t nnz, const int32_t *om_row, const int32_t *om_col,
                           const int32_t *col_order, const double *a_om, double *loss, double *dC, double *dR,
                           double *dG, int32_t *status, hipStream_t stream);

/* Measurement helper (not part of the method): the one-way latency of an
 * exchange between two workgroups on different XCDs through device-scope
 * atomics, the accesses of the team selections, averaged over `rounds`
 * (>= 2) hand-offs.  Synchronizes `stream`; *ns_out (host) receives the
 * nanoseconds per hand-off.  LRA_EDEVICE if a hand-off did not arrive within
 * 100 ms. */
lra_status lra_probe_exchange(int32_t rounds, double *ns_out, hipStream_t stream);

/* Free every cached workspace of the calling process. */
void lra_release(void);

/* Static description of a status code. */
const char *lra_strerror(lra_status s);

#ifdef __cplusplus
}
#endif

#endif /* LRA_CUR_H */
