/*
 * lra_oracle.c -- plain, slow FP64 CPU oracle for cross-approximation (C-A)
 * CUR low-rank approximation, written from Pan, Luan, Svadlenka and Zhao,
 * "Superfast Accurate Low Rank Approximation" (arXiv 1710.07946).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU product path
 * never links, loads or calls it, and the two share no code, header, table or
 * helper: the only thing both sides follow is the published definition of the
 * SplitMix64 generator (Steele, Lea and Flood, OOPSLA 2014), which each side
 * implements on its own.
 *
 * Every routine takes the paper's steps in the paper's order, with no blocking,
 * fusion or reordering.  Where the paper is silent or ambiguous the reading
 * taken is stated at the routine (tie-breaks, thresholds, scaling).
 *
 * Conventions
 *   - matrices are dense row-major, element (i,j) at p[i*ld + j];
 *   - A is read through orc_get(), which upcasts FP32 / BF16 exactly to FP64;
 *   - index sets are 0-based int64; outputs are sorted ascending;
 *   - status: 0 ok, 1 invalid argument, 2 singular (rank deficient panel).
 *
 * Parity pins for every routine live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ESINGULAR 2

#define ORC_F64 0
#define ORC_F32 1
#define ORC_BF16 2

/* ------------------------------------------------------------------------ */
/* Random numbers: SplitMix64 in counter form.                               */
/* The i-th output (0-based) of the SplitMix64 sequence started at state     */
/* `seed` is mix(seed + (i+1)*gamma).  Independent streams are obtained by   */
/* offsetting the counter by stream * 2^40.                                  */
/* ------------------------------------------------------------------------ */
static uint64_t orc_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_rng_u64(uint64_t seed, uint64_t stream, uint64_t i) {
    const uint64_t gamma = 0x9e3779b97f4a7c15ULL;
    return orc_mix64(seed + gamma * ((stream << 40) + i + 1));
}

/* k distinct integers in [0, n), in draw order.  Each draw is reduced modulo
 * n after rejecting the top 2^64 mod n values (so every residue is equally
 * likely); a value already drawn is skipped.  Used for the random initial
 * column set of C-A (Tests 2 of the experiments section draw a random initial
 * index set) and for sampling the columns of the SRHT multiplier (App. B,
 * "sample l columns uniformly at random and without replacement"). */
int orc_draw_distinct(uint64_t seed, uint64_t stream, int64_t n, int64_t k, int64_t *out) {
    if (n <= 0 || k < 0 || k > n || (k > 0 && !out)) return ORC_EINVAL;
    uint64_t un = (uint64_t)n;
    uint64_t rem = (0 - un) % un;         /* 2^64 mod n */
    uint64_t lim = 0 - rem;               /* accept u < lim (all u if rem == 0) */
    uint64_t ctr = 0;
    int64_t got = 0;
    while (got < k) {
        uint64_t u = orc_rng_u64(seed, stream, ctr++);
        if (rem != 0 && u >= lim) continue;
        int64_t v = (int64_t)(u % un);
        int dup = 0;
        for (int64_t q = 0; q < got; q++)
            if (out[q] == v) { dup = 1; break; }
        if (!dup) out[got++] = v;
    }
    return ORC_OK;
}

/* Rademacher sign of the random diagonal D of the SRHT multiplier: the paper
 * takes D uniform on the complex unit circle; for real inputs the reading
 * taken is a uniform +-1 (App. B, randomized Hadamard transform). */
double orc_sign(uint64_t seed, int64_t c) {
    return (orc_rng_u64(seed, 1, (uint64_t)c) >> 63) ? -1.0 : 1.0;
}

/* ------------------------------------------------------------------------ */
/* Element access with exact upcast.                                         */
/* ------------------------------------------------------------------------ */
static double orc_get(const void *A, int dtype, int64_t lda, int64_t i, int64_t j) {
    int64_t o = i * lda + j;
    if (dtype == ORC_F64) return ((const double *)A)[o];
    if (dtype == ORC_F32) return (double)((const float *)A)[o];
    uint32_t bits = ((uint32_t)((const uint16_t *)A)[o]) << 16;
    float f;
    memcpy(&f, &bits, 4);
    return (double)f;
}

static void orc_note_margin(double *mm, double v1, double v2) {
    /* relative gap between the winning value and the runner-up */
    if (!mm) return;
    double g = (v1 > 0) ? (v1 - v2) / v1 : 0.0;
    if (v2 < 0) g = 1.0; /* no runner-up: nothing was decided */
    if (g < *mm) *mm = g;
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* Stage 1 of the iterative C-A by recursive LUP (App. D, Algorithm alggos): */
/* LU factorization with partial pivoting of a tall panel P (items x r).     */
/* The paper factors an r x n matrix with column pivoting; a tall panel is   */
/* its transpose, so here rows are pivoted.  Pivot k is the not-yet-pivoted  */
/* item with the largest |P[i][k]| after k elimination steps; among equal    */
/* magnitudes the lowest item index wins (reading: the paper is silent on   */
/* ties).  Rows stay in place: after the call, LU[piv[k]][j] holds U[k][j]   */
/* for j >= k and the multiplier L[k][j] for j < k; every other item holds   */
/* its r multipliers L21.  A zero pivot means the panel has rank k < r.      */
/* ------------------------------------------------------------------------ */
int orc_panel_lu(const double *P, int64_t items, int r, int64_t *piv, double *LU, int32_t *rank,
                 double *min_margin) {
    if (!P || !piv || !LU || r < 1 || items < r) return ORC_EINVAL;
    memcpy(LU, P, sizeof(double) * (size_t)items * (size_t)r);
    char *done = (char *)calloc((size_t)items, 1);
    if (!done) return ORC_EINVAL;
    int st = ORC_OK;
    if (rank) *rank = r;
    for (int k = 0; k < r; k++) {
        int64_t best = -1;
        double v1 = -1.0, v2 = -1.0;
        for (int64_t i = 0; i < items; i++) {
            if (done[i]) continue;
            double a = fabs(LU[i * r + k]);
            if (a > v1) { v2 = v1; v1 = a; best = i; }
            else if (a > v2) v2 = a;
        }
        if (v1 == 0.0) { st = ORC_ESINGULAR; if (rank) *rank = k; break; }
        orc_note_margin(min_margin, v1, v2);
        piv[k] = best;
        done[best] = 1;
        const double *prow = LU + best * r;
        for (int64_t i = 0; i < items; i++) {
            if (done[i]) continue;
            double *row = LU + i * r;
            double l = row[k] / prow[k];
            row[k] = l;
            for (int j = k + 1; j < r; j++) row[j] -= l * prow[j];
        }
    }
    free(done);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Dominant (locally maximal volume) r x r submatrix of a tall panel.        */
/* App. D, Algorithm alggos (stages 1-2) for the start, then the swaps of    */
/* Algorithm algdomin, in transposed (tall) form:                            */
/*   1. LUP of the panel gives the basis I (piv) and, for the remaining      */
/*      items, B = P * P[I,:]^{-1} = L21 * L11^{-1} (stage 2 of alggos;      */
/*      basis rows of B are unit rows);                                      */
/*   2. find the entry of largest magnitude of B among non-basis items; if   */
/*      it is at most 1 + delta stop (the paper stops at 1; a threshold a    */
/*      little above 1 guards against rounding, App. D, before GE96);        */
/*   3. otherwise item i enters the basis in slot j (the paper's "swap"),    */
/*      which multiplies |det P[I,:]| by |B[i][j]|, and B is updated by the  */
/*      rank-one formula B -= B[:,j] (B[i,:] - e_j^T) / B[i][j] that follows */
/*      from the Sherman-Morrison identity; go to 2.                         */
/* Reading of the garbled stage 3 of alggos: "go to stage 1" is taken as     */
/* the swap of algdomin with a rank-one update (no re-factorization), which  */
/* matches the (n - r) r flops per iteration stated after algdomin.          */
/* Ties in step 2: lowest item, then lowest slot.                            */
/* Outputs: slots[j] = item in basis slot j; B_out (items x r) if non-NULL;  */
/* trace of swaps (item, slot, B value) if non-NULL.                         */
/* ------------------------------------------------------------------------ */
int orc_maxvol(const double *P, int64_t items, int r, double delta, int32_t max_swaps,
               int64_t *slots, double *B_out, int64_t *trace_idx, double *trace_val,
               int32_t *swaps_out, int32_t *converged_out, int32_t *rank_out, double *min_margin) {
    if (!P || !slots || r < 1 || items < r || max_swaps < 0) return ORC_EINVAL;
    double *B = (double *)malloc(sizeof(double) * (size_t)items * (size_t)r);
    char *inb = (char *)calloc((size_t)items, 1);
    double *brow = (double *)malloc(sizeof(double) * (size_t)r);
    if (!B || !inb || !brow) { free(B); free(inb); free(brow); return ORC_EINVAL; }
    int32_t rank = r;
    int st = orc_panel_lu(P, items, r, slots, B, &rank, min_margin);
    if (rank_out) *rank_out = rank;
    if (swaps_out) *swaps_out = 0;
    if (converged_out) *converged_out = 0;
    if (st != ORC_OK) { free(B); free(inb); free(brow); return st; }

    /* L11[k][j] (j < k) is stored in the pivot row of step k. */
    double *L11 = (double *)calloc((size_t)r * (size_t)r, sizeof(double));
    for (int k = 0; k < r; k++)
        for (int j = 0; j < k; j++) L11[k * r + j] = B[slots[k] * r + j];
    for (int k = 0; k < r; k++) inb[slots[k]] = 1;
    /* B_i = l_i L11^{-1}: solve x L11 = l_i by column-oriented back        */
    /* substitution: for k = r-1 down to 1, x_k is final and is eliminated   */
    /* from every x_j with j < k.                                             */
    for (int64_t i = 0; i < items; i++) {
        if (inb[i]) continue;
        double *x = B + i * r;
        for (int k = r - 1; k >= 1; k--) {
            const double xk = x[k];
            for (int j = 0; j < k; j++) x[j] -= xk * L11[k * r + j];
        }
    }
    for (int k = 0; k < r; k++) {
        double *x = B + slots[k] * r;
        for (int j = 0; j < r; j++) x[j] = (j == k) ? 1.0 : 0.0;
    }
    free(L11);

    int32_t swaps = 0, conv = 0;
    const double thr = 1.0 + delta;
    for (;;) {
        int64_t bi = -1;
        int bj = -1;
        double v1 = -1.0, v2 = -1.0;
        for (int64_t i = 0; i < items; i++) {
            if (inb[i]) continue;
            for (int j = 0; j < r; j++) {
                double a = fabs(B[i * r + j]);
                if (a > v1) { v2 = v1; v1 = a; bi = i; bj = j; }
                else if (a > v2) v2 = a;
            }
        }
        if (bi < 0) { conv = 1; break; } /* items == r: nothing to swap */
        if (min_margin) {
            double g = fabs(v1 - thr) / thr;
            if (g < *min_margin) *min_margin = g;
        }
        if (v1 <= thr) { conv = 1; break; }
        if (swaps >= max_swaps) { conv = 0; break; }
        orc_note_margin(min_margin, v1, v2);
        double pv = B[bi * r + bj];
        if (trace_idx) { trace_idx[2 * swaps] = bi; trace_idx[2 * swaps + 1] = bj; }
        if (trace_val) trace_val[swaps] = pv;
        memcpy(brow, B + bi * r, sizeof(double) * (size_t)r);
        brow[bj] -= 1.0; /* B[i,:] - e_j^T */
        for (int64_t i = 0; i < items; i++) {
            if (i == bi) continue;
            double f = B[i * r + bj] / pv;
            if (f == 0.0) continue;
            for (int j = 0; j < r; j++) B[i * r + j] -= f * brow[j];
        }
        for (int j = 0; j < r; j++) B[bi * r + j] = (j == bj) ? 1.0 : 0.0;
        inb[slots[bj]] = 0;
        inb[bi] = 1;
        slots[bj] = bi;
        swaps++;
    }
    if (B_out) memcpy(B_out, B, sizeof(double) * (size_t)items * (size_t)r);
    if (swaps_out) *swaps_out = swaps;
    if (converged_out) *converged_out = conv;
    free(B); free(inb); free(brow);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Abridged SRHT sketch (App. B).  H_{N,d} is the recursion (eqrfd) stopped  */
/* at depth d with H_s = I_s, N = 2^d s, i.e. the Kronecker product          */
/* H_{2^d} (x) I_s: entry (a s + e, b s + e') is (-1)^{popcount(a & b)} if   */
/* e = e' and 0 otherwise (the printed H_{n,1}, H_{n,2} are the cases d=1,2). */
/* The multiplier is D H_{N,d} with l of its N columns sampled uniformly     */
/* without replacement (the random permutation P is absorbed by the uniform */
/* sampling) and scaled by sqrt(N/l); the factor 2^{-d/2} makes H_{N,d}      */
/* orthogonal.  Inputs with a dimension that is not a multiple of 2^d are    */
/* zero-padded to N.                                                         */
/*   side 0 (post-multiplication, m < n):  Y = W M_S, items = rows of W;     */
/*   side 1 (pre-multiplication, m >= n; Section 11 remark on m > n, and     */
/*          either form for m = n):                                          */
/*          Y = M_S^T W, items = columns of W.                               */
/* Output Y is items x l row-major; samples[q] is the q-th sampled column.   */
/* ------------------------------------------------------------------------ */
int orc_sketch(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int side, int d, int l,
               uint64_t seed, double *Y, int64_t *samples) {
    if (!A || !Y || !samples || d < 0 || d > 20 || l < 1 || m < 1 || n < 1 || lda < n) return ORC_EINVAL;
    int64_t dim = side ? m : n;      /* the dimension the multiplier acts on */
    int64_t items = side ? n : m;
    int64_t q2 = (int64_t)1 << d;
    int64_t s = (dim + q2 - 1) / q2;
    int64_t N = q2 * s;
    if (l > N) return ORC_EINVAL;
    int st = orc_draw_distinct(seed, 2, N, l, samples);
    if (st) return st;
    /* 2^{-d/2} sqrt(N/l) = sqrt(s/l) since N = 2^d s */
    double scale = sqrt((double)s / (double)l);
    for (int64_t it = 0; it < items; it++) {
        for (int q = 0; q < l; q++) {
            int64_t t = samples[q];
            int64_t b = t / s, e = t % s;
            double acc = 0.0;
            for (int64_t a = 0; a < q2; a++) {
                int64_t c = a * s + e;
                if (c >= dim) continue;
                double h = (__builtin_popcountll((uint64_t)(a & b)) & 1) ? -1.0 : 1.0;
                double w = side ? orc_get(A, dtype, lda, c, it) : orc_get(A, dtype, lda, it, c);
                acc += w * orc_sign(seed, c) * h;
            }
            Y[it * l + q] = scale * acc;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Abridged randomized Fourier sketch (App. B, the d-abridged DFT Omega_{N,d} */
/* of eq. (eqfd): the decimation-in-frequency recursion stopped after d      */
/* stages, Omega_s replaced by I_s, N = 2^d s).  Carrying the recursion out  */
/* with the stage twiddles omega_{2q}^i, i < q (the printed diag(omega_n^i)_ */
/* {i<n} has the wrong size: a length-2q stage multiplies the difference    */
/* half by the 2q-th roots of unity), output (k, e) of the abridged         */
/* transform is sum over a of x_{a s + e} omega_N^{k (a s + e)}, omega_N =   */
/* exp(2 pi i / N): column b s + e of the multiplier has the 2^d entries     */
/* omega_N^{b j} at rows j = a s + e (its rows and columns are orthogonal,  */
/* squared norm 2^d; completing every class e with an s-point DFT yields    */
/* the N-point DFT).  D: for a real input, the uniform law on the complex   */
/* unit circle is read as uniform on {1, i, -1, -i}: D_j = i^{t_j}, t_j the */
/* top two bits of SplitMix64 stream 1 at j.  l columns sampled as for the  */
/* SRHT (stream 2, distinct), scale sqrt(s / l).  Complex arithmetic in its */
/* real form: sampled column q contributes Re y_q as coordinate q and Im y_q */
/* as coordinate l + q of a real items x 2l sketch, so that the real QRP of  */
/* the seed runs on it (W real: W M = W Re M + i W Im M).  Sides as for     */
/* orc_sketch; dimensions padded to N with zeros.                           */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* cos and sin of 2 pi m / N for integers 0 <= m < N, evaluated in a fixed   */
/* order of IEEE operations (so that any implementation written from this   */
/* definition gives the same bits): the octant o = floor(8 m / N) and the    */
/* remainder rem = 8 m - o N are exact integers; the angle inside the       */
/* octant is x = (pi/4) rem / N (or (pi/4) (N - rem) / N from the octant's  */
/* far end for odd o), in [0, pi/4]; cos x and sin x are the Taylor series  */
/* through x^20 and x^21 by Horner's rule in x^2, with coefficients from    */
/* the recurrences a_k = -a_{k-1} / ((2k - 1) 2k), b_k = -b_{k-1} /         */
/* (2k (2k + 1)); then the octant's symmetry.  pi/4 is the double nearest   */
/* to it.  The truncation error is below 1e-23.                            */
/* ------------------------------------------------------------------------ */
static void orc_cos_sin_small(double x, double *c, double *s) {
    double a[11], b[11];
    a[0] = 1.0;
    b[0] = 1.0;
    for (int k = 1; k < 11; k++) {
        a[k] = -a[k - 1] / (double)((2 * k - 1) * (2 * k));
        b[k] = -b[k - 1] / (double)((2 * k) * (2 * k + 1));
    }
    double x2 = x * x;
    double pc = a[10], ps = b[10];
    for (int k = 9; k >= 0; k--) {
        pc = pc * x2 + a[k];
        ps = ps * x2 + b[k];
    }
    *c = pc;
    *s = x * ps;
}

void orc_unit_root(int64_t m, int64_t N, double *c_out, double *s_out) {
    const double pi4 = 0x1.921fb54442d18p-1;
    int64_t u = 8 * m;
    int64_t o = u / N;
    int64_t rem = u - o * N;
    double c, s;
    if ((o & 1) == 0) {
        orc_cos_sin_small((pi4 * (double)rem) / (double)N, &c, &s);
        switch (o / 2) {
        case 0: *c_out = c; *s_out = s; break;
        case 1: *c_out = -s; *s_out = c; break;
        case 2: *c_out = -c; *s_out = -s; break;
        default: *c_out = s; *s_out = -c; break;
        }
    } else {
        orc_cos_sin_small((pi4 * (double)(N - rem)) / (double)N, &c, &s);
        switch ((o + 1) / 2) {
        case 1: *c_out = s; *s_out = c; break;
        case 2: *c_out = -c; *s_out = s; break;
        case 3: *c_out = -s; *s_out = -c; break;
        default: *c_out = c; *s_out = -s; break;
        }
    }
}

int orc_sketch_fourier(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int side, int d, int l,
                       uint64_t seed, double *Y, int64_t *samples) {
    if (!A || !Y || !samples || d < 0 || d > 20 || l < 1 || m < 1 || n < 1 || lda < n) return ORC_EINVAL;
    int64_t dim = side ? m : n;
    int64_t items = side ? n : m;
    int64_t q2 = (int64_t)1 << d;
    int64_t s = (dim + q2 - 1) / q2;
    int64_t N = q2 * s;
    if (l > N) return ORC_EINVAL;
    int st = orc_draw_distinct(seed, 2, N, l, samples);
    if (st) return st;
    const double scale = sqrt((double)s / (double)l);
    for (int64_t it = 0; it < items; it++) {
        for (int q = 0; q < l; q++) {
            int64_t t = samples[q];
            int64_t b = t / s, e = t % s;
            double re = 0.0, im = 0.0;
            for (int64_t a = 0; a < q2; a++) {
                int64_t j = a * s + e;
                if (j >= dim) continue;
                double w = side ? orc_get(A, dtype, lda, j, it) : orc_get(A, dtype, lda, it, j);
                /* omega_N^{b j} times i^{t_j} (orc_unit_root for the root) */
                int64_t mexp = (int64_t)(((unsigned __int128)b * (unsigned __int128)j) % (unsigned __int128)N);
                double c, sn;
                orc_unit_root(mexp, N, &c, &sn);
                int tq = (int)(orc_rng_u64(seed, 1, (uint64_t)j) >> 62);
                double cr, ci;  /* (c + i sn) i^tq */
                if (tq == 0) { cr = c; ci = sn; }
                else if (tq == 1) { cr = -sn; ci = c; }
                else if (tq == 2) { cr = -c; ci = -sn; }
                else { cr = sn; ci = -c; }
                re += w * cr;
                im += w * ci;
            }
            Y[it * 2 * l + q] = scale * re;
            Y[it * 2 * l + l + q] = scale * im;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Quasi-Gaussian multipliers made of random bidiagonal factors (the        */
/* section on pre-processing with quasi Gaussian matrices, eq. (def11)):    */
/* G_q = B_1 P_1 B_2 P_2 ... B_q P_q with B_i cyclic bidiagonal (ones on     */
/* the diagonal, a random sign s_{i,j} at row j, column (j - 1) mod N) and   */
/* P_i a random permutation.  Readings: P_i e_c = e_{pi_i(c)} with pi_i a   */
/* four-round Feistel network on [0, 2^b), b = the even bit count with      */
/* 2^b >= N (at least 2), round function the low b/2 bits of SplitMix64      */
/* stream 6 at index (4 (i - 1) + round) 2^32 + right half, and cycle       */
/* walking back into [0, N) (Black and Rogaway, 2002); s_{i,j} = -1 when the */
/* top bit of stream 7 at index (i - 1) N + j is set, else +1.              */
/* ------------------------------------------------------------------------ */
int64_t orc_feistel(uint64_t seed, int factor, int64_t N, int64_t x) {
    int b = 2;
    while (((int64_t)1 << b) < N) b += 2;
    const int half = b / 2;
    const uint64_t mask = ((uint64_t)1 << half) - 1;
    uint64_t y = (uint64_t)x;
    do {
        uint64_t L = y >> half, R = y & mask;
        for (int rd = 0; rd < 4; rd++) {
            const uint64_t key = ((uint64_t)(4 * (factor - 1) + rd) << 32) | R;
            const uint64_t f = orc_rng_u64(seed, 6, key) & mask;
            const uint64_t nl = R, nr = L ^ f;
            L = nl;
            R = nr;
        }
        y = (L << half) | R;
    } while ((int64_t)y >= N);
    return (int64_t)y;
}

/* Column c of G_q: start from e_c and apply B_q P_q first, B_1 P_1 last;   */
/* B e_p = e_p + s_{(p+1) mod N} e_{(p+1) mod N}.  The terms (position,      */
/* integer coefficient) come out merged, without zeros, in ascending         */
/* position order; *cnt <= 2^q.                                              */
int orc_bidiag_column(uint64_t seed, int64_t N, int q, int64_t c, int64_t *pos, int64_t *coef, int *cnt) {
    if (!pos || !coef || !cnt || q < 0 || q > 6 || N < 2 || c < 0 || c >= N) return ORC_EINVAL;
    int k = 1;
    pos[0] = c;
    coef[0] = 1;
    for (int i = q; i >= 1; i--) {
        int64_t np[64], nc[64];
        int nk = 0;
        for (int t = 0; t < k; t++) {
            const int64_t p = orc_feistel(seed, i, N, pos[t]);
            const int64_t p1 = (p + 1) % N;
            const int64_t s = (orc_rng_u64(seed, 7, (uint64_t)((i - 1) * N + p1)) >> 63) ? -1 : 1;
            np[nk] = p;
            nc[nk++] = coef[t];
            np[nk] = p1;
            nc[nk++] = coef[t] * s;
        }
        /* merge equal positions, ascending (insertion sort of <= 64 terms) */
        for (int a = 1; a < nk; a++) {
            int64_t kp = np[a], kc = nc[a];
            int b2 = a - 1;
            while (b2 >= 0 && np[b2] > kp) { np[b2 + 1] = np[b2]; nc[b2 + 1] = nc[b2]; b2--; }
            np[b2 + 1] = kp;
            nc[b2 + 1] = kc;
        }
        k = 0;
        for (int a = 0; a < nk; a++) {
            if (k > 0 && pos[k - 1] == np[a]) coef[k - 1] += nc[a];
            else { pos[k] = np[a]; coef[k] = nc[a]; k++; }
        }
        int z = 0;
        for (int a = 0; a < k; a++)
            if (coef[a] != 0) { pos[z] = pos[a]; coef[z] = coef[a]; z++; }
        k = z;
    }
    *cnt = k;
    return ORC_OK;
}

/* Sketch with l sampled columns of G_q (distinct draws, stream 2, in draw  */
/* order), in the two forms of orc_sketch: side 0, Y = W G_q S (items =     */
/* rows); side 1, Y = (G_q S)^T W (items = columns), G_q of order m.  Each   */
/* entry sums coef * w over the column's terms in ascending position order. */
/* No scale factor (a common factor cannot change a QRP decision).          */
int orc_sketch_bidiag(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int side, int q, int l,
                      uint64_t seed, double *Y, int64_t *samples) {
    if (!A || !Y || !samples || q < 0 || q > 6 || l < 1 || m < 1 || n < 1 || lda < n) return ORC_EINVAL;
    const int64_t dim = side ? m : n;
    const int64_t items = side ? n : m;
    if (dim < 2 || l > dim) return ORC_EINVAL;
    int st = orc_draw_distinct(seed, 2, dim, l, samples);
    if (st) return st;
    int64_t pos[64], coef[64];
    for (int t = 0; t < l; t++) {
        int cnt = 0;
        orc_bidiag_column(seed, dim, q, samples[t], pos, coef, &cnt);
        for (int64_t it = 0; it < items; it++) {
            double acc = 0.0;
            for (int k = 0; k < cnt; k++) {
                const double w = side ? orc_get(A, dtype, lda, pos[k], it) : orc_get(A, dtype, lda, it, pos[k]);
                acc += (double)coef[k] * w;
            }
            Y[it * l + t] = acc;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Greedy expansion by Householder reflections (App. D, Algorithm alg1tor):  */
/* the columns of a w x items matrix Z (stored item-major: item it is the    */
/* w-vector Z[it*w .. it*w+w-1]) are chosen one at a time.  At step g the   */
/* chosen item is the unchosen one whose coordinates g..w-1 have the largest */
/* 2-norm (recomputed from the current vectors, not downdated; ties to the  */
/* lowest item); a Householder reflection acting on coordinates g..w-1 then  */
/* maps that part of the chosen vector onto a multiple of e_1 and is applied */
/* to every unchosen vector.  This is greedy QR with column pivoting; the    */
/* paper uses it (or GE96) at stage 2 of Algorithm algrhtcur to pick rows of */
/* the sketch.  Z is modified in place.                                      */
/* ------------------------------------------------------------------------ */
int orc_qrp(double *Z, int64_t items, int w, int k, int64_t *piv, int32_t *rank, double *min_margin) {
    if (!Z || !piv || w < 1 || k < 1 || k > w || items < k) return ORC_EINVAL;
    char *used = (char *)calloc((size_t)items, 1);
    double *v = (double *)malloc(sizeof(double) * (size_t)w);
    if (!used || !v) { free(used); free(v); return ORC_EINVAL; }
    int st = ORC_OK;
    if (rank) *rank = k;
    for (int g = 0; g < k; g++) {
        int64_t best = -1;
        double v1 = -1.0, v2 = -1.0;
        for (int64_t it = 0; it < items; it++) {
            if (used[it]) continue;
            const double *z = Z + it * w;
            double s = 0.0;
            for (int c = g; c < w; c++) s += z[c] * z[c];
            if (s > v1) { v2 = v1; v1 = s; best = it; }
            else if (s > v2) v2 = s;
        }
        if (v1 <= 0.0) { st = ORC_ESINGULAR; if (rank) *rank = g; break; }
        orc_note_margin(min_margin, v1, v2);
        piv[g] = best;
        used[best] = 1;
        double *x = Z + best * w;
        double nx = sqrt(v1);
        double alpha = (x[g] >= 0.0) ? -nx : nx;
        int len = w - g;
        for (int c = 0; c < len; c++) v[c] = x[g + c];
        v[0] -= alpha;
        double vtv = 0.0;
        for (int c = 0; c < len; c++) vtv += v[c] * v[c];
        if (vtv > 0.0) {
            for (int64_t it = 0; it < items; it++) {
                if (used[it]) continue;
                double *z = Z + it * w;
                double s = 0.0;
                for (int c = 0; c < len; c++) s += v[c] * z[g + c];
                double f = 2.0 * s / vtv;
                for (int c = 0; c < len; c++) z[g + c] -= f * v[c];
            }
        }
        x[g] = alpha;
        for (int c = g + 1; c < w; c++) x[c] = 0.0;
    }
    free(used); free(v);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Iterative refinement of an approximate inverse X of G (the refinement of  */
/* the nucleus in Section 3): `steps` times T = I - G X, then X <- X + X T,  */
/* every sum in increasing index order.  With E = I - G X, one step leaves   */
/* I - G (X + X E) = E - (I - E) E = E^2: the residual is squared.           */
/* ------------------------------------------------------------------------ */
int orc_refine_inverse(const double *G, int r, double *X, int steps) {
    if (!G || !X || r < 1 || steps < 0) return ORC_EINVAL;
    double *T = (double *)malloc(sizeof(double) * (size_t)r * (size_t)r);
    double *X2 = (double *)malloc(sizeof(double) * (size_t)r * (size_t)r);
    for (int it = 0; it < steps; it++) {
        for (int i = 0; i < r; i++)       /* T = I - G X */
            for (int j = 0; j < r; j++) {
                double s = (i == j) ? 1.0 : 0.0;
                for (int q = 0; q < r; q++) s -= G[i * r + q] * X[q * r + j];
                T[i * r + j] = s;
            }
        for (int i = 0; i < r; i++)       /* X + X T */
            for (int j = 0; j < r; j++) {
                double s = X[i * r + j];
                for (int q = 0; q < r; q++) s += X[i * r + q] * T[q * r + j];
                X2[i * r + j] = s;
            }
        memcpy(X, X2, sizeof(double) * (size_t)r * (size_t)r);
    }
    free(T); free(X2);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Nucleus U = G^{-1} of an r x r generator (Section 3, Algorithm algcnnncl  */
/* with k = l = r, where the truncated pseudo-inverse is the inverse,        */
/* Remark reklr_kl).  Gauss-Jordan style: LU with partial pivoting (ties to  */
/* the lowest row) then r triangular solves for the unit vectors.  Optional  */
/* iterative refinement X <- X + X (I - G X).  log|det G| is returned.       */
/* ------------------------------------------------------------------------ */
int orc_inverse(const double *G, int r, double *U, int refine_steps, double *logdet) {
    if (!G || !U || r < 1) return ORC_EINVAL;
    double *LU = (double *)malloc(sizeof(double) * (size_t)r * (size_t)r);
    int *p = (int *)malloc(sizeof(int) * (size_t)r);
    double *col = (double *)malloc(sizeof(double) * (size_t)r);
    memcpy(LU, G, sizeof(double) * (size_t)r * (size_t)r);
    for (int i = 0; i < r; i++) p[i] = i;
    double ld = 0.0;
    int st = ORC_OK;
    for (int k = 0; k < r; k++) {
        int best = k;
        double bv = fabs(LU[p[k] * r + k]);
        for (int i = k + 1; i < r; i++) {
            double a = fabs(LU[p[i] * r + k]);
            if (a > bv || (a == bv && p[i] < p[best])) { bv = a; best = i; }
        }
        if (bv == 0.0) { st = ORC_ESINGULAR; break; }
        int t = p[k]; p[k] = p[best]; p[best] = t;
        double pk = LU[p[k] * r + k];
        ld += log(fabs(pk));
        for (int i = k + 1; i < r; i++) {
            double l = LU[p[i] * r + k] / pk;
            LU[p[i] * r + k] = l;
            for (int j = k + 1; j < r; j++) LU[p[i] * r + j] -= l * LU[p[k] * r + j];
        }
    }
    if (st == ORC_OK) {
        /* solve G x = e_c for every column c: L y = P e_c, U x = y */
        for (int c = 0; c < r; c++) {
            for (int i = 0; i < r; i++) {
                double s = (p[i] == c) ? 1.0 : 0.0;
                for (int j = 0; j < i; j++) s -= LU[p[i] * r + j] * col[j];
                col[i] = s;
            }
            for (int i = r - 1; i >= 0; i--) {
                double s = col[i];
                for (int j = i + 1; j < r; j++) s -= LU[p[i] * r + j] * col[j];
                col[i] = s / LU[p[i] * r + i];
            }
            for (int i = 0; i < r; i++) U[i * r + c] = col[i];
        }
        orc_refine_inverse(G, r, U, refine_steps);
    }
    if (logdet) *logdet = ld;
    free(LU); free(p); free(col);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Truncated pseudo-inverse by one-sided Jacobi (Hestenes) SVD: the nucleus   */
/* of Algorithm algcnnncl when the generator is singular or too badly         */
/* conditioned for the LU inverse.  The columns of A = G are orthogonalised   */
/* by plane rotations (V accumulates them); pairs are visited in round-robin  */
/* order (position 0 fixed, the others rotating; a dummy position pads odd r);*/
/* a pair is rotated unless |a_p . a_q| <= 1e-15 sqrt(|a_p|^2 |a_q|^2); sweeps */
/* repeat until one applies no rotation (at most 60).  Then sigma_j = |a_j|,  */
/* and G^+ = sum over sigma_j > rtol * max sigma of v_j a_j^T / sigma_j^2     */
/* (j increasing).  All sums run in increasing index order.  *rank_out gets   */
/* the number of singular values kept.                                        */
/* ------------------------------------------------------------------------ */
static void orc_pair(int t, int k, int rp, int *p, int *q) {
    int a = (k == 0) ? 0 : ((k - 1 + t) % (rp - 1)) + 1;
    int kk = rp - 1 - k;
    int b = ((kk - 1 + t) % (rp - 1)) + 1;
    *p = a < b ? a : b;
    *q = a < b ? b : a;
}

int orc_pinv_jacobi(const double *G, int r, double rtol, double *X, int *rank_out) {
    if (!G || !X || r < 1) return ORC_EINVAL;
    double *A = (double *)malloc(sizeof(double) * (size_t)r * (size_t)r);
    double *V = (double *)calloc((size_t)r * (size_t)r, sizeof(double));
    double *sg = (double *)malloc(sizeof(double) * (size_t)r);
    memcpy(A, G, sizeof(double) * (size_t)r * (size_t)r);
    for (int i = 0; i < r; i++) V[i * r + i] = 1.0;
    const int rp = r + (r & 1);
    for (int sweep = 0; sweep < 60 && r > 1; sweep++) {
        int rotated = 0;
        for (int t = 0; t < rp - 1; t++) {
            for (int k = 0; k < rp / 2; k++) {
                int pc, qc;
                orc_pair(t, k, rp, &pc, &qc);
                if (qc >= r) continue;  /* paired with the padding position */
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = 0; i < r; i++) {
                    al += A[i * r + pc] * A[i * r + pc];
                    be += A[i * r + qc] * A[i * r + qc];
                    ga += A[i * r + pc] * A[i * r + qc];
                }
                if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
                double ze = (be - al) / (2.0 * ga);
                double tt = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
                double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
                for (int i = 0; i < r; i++) {
                    double x = A[i * r + pc], y = A[i * r + qc];
                    A[i * r + pc] = c * x - sn * y;
                    A[i * r + qc] = sn * x + c * y;
                    x = V[i * r + pc];
                    y = V[i * r + qc];
                    V[i * r + pc] = c * x - sn * y;
                    V[i * r + qc] = sn * x + c * y;
                }
                rotated = 1;
            }
        }
        if (!rotated) break;
    }
    double smax = 0.0;
    for (int j = 0; j < r; j++) {
        double s2 = 0.0;
        for (int i = 0; i < r; i++) s2 += A[i * r + j] * A[i * r + j];
        sg[j] = sqrt(s2);
        if (sg[j] > smax) smax = sg[j];
    }
    int rank = 0;
    for (int j = 0; j < r; j++) rank += (sg[j] > rtol * smax) ? 1 : 0;
    for (int a = 0; a < r; a++)
        for (int b = 0; b < r; b++) {
            double acc = 0.0;
            for (int j = 0; j < r; j++)
                if (sg[j] > rtol * smax) acc += V[a * r + j] * A[b * r + j] / (sg[j] * sg[j]);
            X[a * r + b] = acc;
        }
    if (rank_out) *rank_out = rank;
    free(A); free(V); free(sg);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Nucleus (Algorithm algcnnncl with k = l = r): the LU inverse of G with    */
/* `refine_steps` refinement steps; when a pivot is exactly zero or the      */
/* ratio of the largest to the smallest pivot magnitude exceeds 1e14 (a      */
/* cheap condition estimate from the same factors), the truncated            */
/* pseudo-inverse with relative truncation 1e-14 instead.  *rank_out: r for  */
/* the inverse, the kept rank for the pseudo-inverse; *logdet: log |det G|   */
/* (-inf when a pivot is zero).                                              */
/* ------------------------------------------------------------------------ */
int orc_nucleus(const double *G, int r, int refine_steps, double *U, double *logdet, int *rank_out) {
    if (!G || !U || r < 1) return ORC_EINVAL;
    double ld = 0.0;
    int st = orc_inverse(G, r, U, refine_steps, &ld);
    int fallback = (st == ORC_ESINGULAR);
    if (st == ORC_OK) {
        /* pivot magnitudes of the same elimination */
        double *LU = (double *)malloc(sizeof(double) * (size_t)r * (size_t)r);
        int *p = (int *)malloc(sizeof(int) * (size_t)r);
        memcpy(LU, G, sizeof(double) * (size_t)r * (size_t)r);
        for (int i = 0; i < r; i++) p[i] = i;
        double pmax = 0.0, pmin = INFINITY;
        for (int k = 0; k < r; k++) {
            int best = k;
            double bv = fabs(LU[p[k] * r + k]);
            for (int i = k + 1; i < r; i++) {
                double a = fabs(LU[p[i] * r + k]);
                if (a > bv || (a == bv && p[i] < p[best])) { bv = a; best = i; }
            }
            int t = p[k]; p[k] = p[best]; p[best] = t;
            double pk = LU[p[k] * r + k];
            if (fabs(pk) > pmax) pmax = fabs(pk);
            if (fabs(pk) < pmin) pmin = fabs(pk);
            for (int i = k + 1; i < r; i++) {
                double l = LU[p[i] * r + k] / pk;
                LU[p[i] * r + k] = l;
                for (int j = k + 1; j < r; j++) LU[p[i] * r + j] -= l * LU[p[k] * r + j];
            }
        }
        free(LU); free(p);
        fallback = pmax > 1e14 * pmin;
    } else if (st != ORC_ESINGULAR) {
        return st;
    }
    if (fallback) {
        st = orc_pinv_jacobi(G, r, 1e-14, U, rank_out);
        if (logdet) *logdet = (st == ORC_OK && *rank_out == r) ? ld : -INFINITY;
        return st;
    }
    if (rank_out) *rank_out = r;
    if (logdet) *logdet = ld;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* C-A CUR driver (Section 1.3 and Fig. 4: alternating vertical m x r and    */
/* horizontal r x n sketches; Section 13, Tests 2: random initial set, a few */
/* C-A loops, nucleus U = W_{I,J}^{-1}, W' = C U R as in eq. (eqtsts1)).     */
/*   column step: C = W[:, J] (J ascending), I = dominant rows of C;         */
/*   row step:    R = W[I, :] (I ascending), J = dominant columns of R.      */
/* One sweep is a column step followed by a row step; the loop stops early   */
/* once a sweep reproduces the previous sweep's sets (a fixed point, after   */
/* which further sweeps change nothing).  With pre-processing the start set  */
/* comes from greedy QRP on the abridged-SRHT sketch (Algorithm algrhtcur,   */
/* stage 2, with C-A replacing stage 3 as its remark rerfnhmt suggests):     */
/* post-multiplication yields rows I0 and one row step turns them into J0;   */
/* pre-multiplication yields J0 directly.                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    double delta;
    int32_t max_swaps;
    int32_t preprocess;   /* 0 none, 1 abridged SRHT, 2 random bidiagonal factors, 3 abridged SRFT */
    int32_t ah_depth;
    int32_t ah_samples;
    int32_t refine_steps;
    const int64_t *init_cols; /* optional r start columns */
} orc_opts;

typedef struct {
    int32_t sweeps_run, swaps_total, converged, rank_found;
    int32_t nucleus_rank, pad;   /* rank kept by the nucleus (r unless the pseudo-inverse truncated) */
    double min_margin, det_log_abs;
} orc_info;

static int orc_step(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int r, int rows,
                    const int64_t *set_in, const orc_opts *o, int64_t *set_out, orc_info *info) {
    /* rows = 1: column step (panel = W[:, set_in], items = rows of W);
       rows = 0: row step    (panel = W[set_in, :]^T, items = columns of W). */
    int64_t items = rows ? m : n;
    double *P = (double *)malloc(sizeof(double) * (size_t)items * (size_t)r);
    if (!P) return ORC_EINVAL;
    for (int64_t it = 0; it < items; it++)
        for (int j = 0; j < r; j++)
            P[it * r + j] = rows ? orc_get(A, dtype, lda, it, set_in[j]) : orc_get(A, dtype, lda, set_in[j], it);
    int32_t sw = 0, conv = 0, rk = r;
    int st = orc_maxvol(P, items, r, o->delta, o->max_swaps, set_out, NULL, NULL, NULL, &sw, &conv, &rk,
                        &info->min_margin);
    free(P);
    info->swaps_total += sw;
    if (st == ORC_ESINGULAR) info->rank_found = rk;
    if (st == ORC_OK && !conv) info->converged = 0;
    if (st == ORC_OK) qsort(set_out, (size_t)r, sizeof(int64_t), cmp_i64);
    return st;
}

void orc_default_opts(orc_opts *o) {
    o->delta = 0.01;
    o->max_swaps = -1; /* -1: 16 r */
    o->preprocess = 0;
    o->ah_depth = 3;
    o->ah_samples = 0; /* 0: 2 r */
    o->refine_steps = 0;
    o->init_cols = NULL;
}

static int orc_finite_scan(const void *A, int dtype, int64_t lda, int64_t rows0, int64_t nrows,
                           int64_t cols0, int64_t ncols) {
    for (int64_t i = rows0; i < rows0 + nrows; i++)
        for (int64_t j = cols0; j < cols0 + ncols; j++)
            if (!isfinite(orc_get(A, dtype, lda, i, j))) return 0;
    return 1;
}

int orc_ca_cur(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int r, int sweeps, uint64_t seed,
               const orc_opts *opts_in, int64_t *I_out, int64_t *J_out, double *U_out, orc_info *info_out) {
    orc_opts o;
    if (opts_in) o = *opts_in; else orc_default_opts(&o);
    if (o.max_swaps < 0) o.max_swaps = 16 * r;
    if (o.ah_samples <= 0) o.ah_samples = 2 * r;
    orc_info info = {0, 0, 1, 0, 0, 0, 1.0, 0.0};
    info.rank_found = r;
    if (!A || !I_out || !J_out || !U_out || r < 1 || sweeps < 1 || m < 1 || n < 1 || lda < n ||
        (int64_t)r > (m < n ? m : n) || dtype < 0 || dtype > 2 || !(o.delta >= 0.0) ||
        (o.preprocess != 0 && o.preprocess != 1 && o.preprocess != 2 && o.preprocess != 3)) {
        if (info_out) *info_out = info;
        return ORC_EINVAL;
    }
    int64_t *I = (int64_t *)malloc(sizeof(int64_t) * (size_t)r);
    int64_t *J = (int64_t *)malloc(sizeof(int64_t) * (size_t)r);
    int64_t *Ip = (int64_t *)malloc(sizeof(int64_t) * (size_t)r);
    int64_t *Jp = (int64_t *)malloc(sizeof(int64_t) * (size_t)r);
    int st = ORC_OK;

    if (o.preprocess == 1 || o.preprocess == 2 || o.preprocess == 3) {
        /* pre-multiplication for m >= n (the paper allows either form when   */
        /* m = n; this one yields the start columns directly)                */
        int side = (m >= n) ? 1 : 0;
        int64_t items = side ? n : m;
        int l = o.ah_samples;
        int wy = o.preprocess == 3 ? 2 * l : l;  /* real width of the sketch */
        if (wy < r) { st = ORC_EINVAL; goto done; }
        double *Y = (double *)malloc(sizeof(double) * (size_t)items * (size_t)wy);
        int64_t *smp = (int64_t *)malloc(sizeof(int64_t) * (size_t)l);
        st = o.preprocess == 1   ? orc_sketch(A, dtype, m, n, lda, side, o.ah_depth, l, seed, Y, smp)
             : o.preprocess == 2 ? orc_sketch_bidiag(A, dtype, m, n, lda, side, o.ah_depth, l, seed, Y, smp)
                                 : orc_sketch_fourier(A, dtype, m, n, lda, side, o.ah_depth, l, seed, Y, smp);
        int32_t rk = r;
        if (st == ORC_OK) {
            for (int64_t q = 0; q < items * wy; q++)
                if (!isfinite(Y[q])) { st = ORC_EINVAL; break; }
        }
        if (st == ORC_OK) st = orc_qrp(Y, items, wy, r, side ? J : I, &rk, &info.min_margin);
        if (st == ORC_ESINGULAR) info.rank_found = rk;
        free(Y); free(smp);
        if (st) goto done;
        if (!side) {
            qsort(I, (size_t)r, sizeof(int64_t), cmp_i64);
            for (int a = 0; a < r; a++)
                if (!orc_finite_scan(A, dtype, lda, I[a], 1, 0, n)) { st = ORC_EINVAL; goto done; }
            st = orc_step(A, dtype, m, n, lda, r, 0, I, &o, J, &info);
            if (st) goto done;
        } else {
            qsort(J, (size_t)r, sizeof(int64_t), cmp_i64);
        }
    } else if (o.init_cols) {
        for (int a = 0; a < r; a++) {
            if (o.init_cols[a] < 0 || o.init_cols[a] >= n) { st = ORC_EINVAL; goto done; }
            for (int b = 0; b < a; b++)
                if (o.init_cols[b] == o.init_cols[a]) { st = ORC_EINVAL; goto done; }
            J[a] = o.init_cols[a];
        }
        qsort(J, (size_t)r, sizeof(int64_t), cmp_i64);
    } else {
        orc_draw_distinct(seed, 0, n, r, J);
        qsort(J, (size_t)r, sizeof(int64_t), cmp_i64);
    }

    for (int s = 0; s < sweeps; s++) {
        for (int a = 0; a < r; a++)
            if (!orc_finite_scan(A, dtype, lda, 0, m, J[a], 1)) { st = ORC_EINVAL; goto done; }
        st = orc_step(A, dtype, m, n, lda, r, 1, J, &o, I, &info);
        if (st) goto done;
        for (int a = 0; a < r; a++)
            if (!orc_finite_scan(A, dtype, lda, I[a], 1, 0, n)) { st = ORC_EINVAL; goto done; }
        st = orc_step(A, dtype, m, n, lda, r, 0, I, &o, J, &info);
        if (st) goto done;
        info.sweeps_run = s + 1;
        if (s > 0 && !memcmp(I, Ip, sizeof(int64_t) * (size_t)r) && !memcmp(J, Jp, sizeof(int64_t) * (size_t)r))
            break;
        memcpy(Ip, I, sizeof(int64_t) * (size_t)r);
        memcpy(Jp, J, sizeof(int64_t) * (size_t)r);
    }

    {
        double *G = (double *)malloc(sizeof(double) * (size_t)r * (size_t)r);
        for (int a = 0; a < r; a++)
            for (int b = 0; b < r; b++) G[a * r + b] = orc_get(A, dtype, lda, I[a], J[b]);
        int nr = r;
        st = orc_nucleus(G, r, o.refine_steps, U_out, &info.det_log_abs, &nr);
        info.nucleus_rank = nr;
        free(G);
    }
    memcpy(I_out, I, sizeof(int64_t) * (size_t)r);
    memcpy(J_out, J, sizeof(int64_t) * (size_t)r);
done:
    free(I); free(J); free(Ip); free(Jp);
    if (st != ORC_OK) info.converged = 0;
    if (info_out) *info_out = info;
    return st;
}

/* ------------------------------------------------------------------------ */
/* Relative Frobenius error ||W - C U R||_F / ||W||_F of a CUR LRA with      */
/* C = W[:, J], R = W[I, :] and U (r x r, J-order x I-order), eq. (eqcur0).  */
/* Plain triple loop; out_err2 / out_norm2 receive the two squared sums.     */
/* ------------------------------------------------------------------------ */
int orc_residual(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I,
                 const int64_t *J, const double *U, double *out_err2, double *out_norm2) {
    if (!A || !I || !J || !U || r < 1 || m < 1 || n < 1 || lda < n) return ORC_EINVAL;
    /* UR = U * W[I,:]  (r x n) */
    double *UR = (double *)calloc((size_t)r * (size_t)n, sizeof(double));
    for (int a = 0; a < r; a++)
        for (int b = 0; b < r; b++) {
            double u = U[a * r + b];
            for (int64_t j = 0; j < n; j++) UR[a * n + j] += u * orc_get(A, dtype, lda, I[b], j);
        }
    double e2 = 0.0, w2 = 0.0;
    double *c = (double *)malloc(sizeof(double) * (size_t)r);
    for (int64_t i = 0; i < m; i++) {
        for (int a = 0; a < r; a++) c[a] = orc_get(A, dtype, lda, i, J[a]);
        for (int64_t j = 0; j < n; j++) {
            double x = 0.0;
            for (int a = 0; a < r; a++) x += c[a] * UR[a * n + j];
            double w = orc_get(A, dtype, lda, i, j);
            e2 += (w - x) * (w - x);
            w2 += w * w;
        }
    }
    free(UR); free(c);
    if (out_err2) *out_err2 = e2;
    if (out_norm2) *out_norm2 = w2;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Loss and gradients of the CUR reconstruction at fixed index sets (plain   */
/* calculus; the paper has no adjoint):                                      */
/*   L(C, R, G) = sum_{(i,j) in Omega} (a_ij - (C G^{-1} R)_ij)^2.           */
/* With Z = G^{-1} R and Ebar = -2 (a - C Z) on Omega:                       */
/*   dC = Ebar Z^T,  dZ = C^T Ebar,  dR = G^{-T} dZ,  dG = -G^{-T} dZ Z^T.   */
/* C is m x r, R is r x n, G is r x r, all FP64 row-major; Omega is COO.     */
/* ------------------------------------------------------------------------ */
int orc_cur_adjoint(const double *C, const double *R, const double *G, int64_t m, int64_t n, int r,
                    const int64_t *oi, const int64_t *oj, const double *aval, int64_t nnz,
                    double *loss, double *dC, double *dR, double *dG) {
    if (!C || !R || !G || r < 1 || m < 1 || n < 1 || nnz < 0) return ORC_EINVAL;
    double *Gi = (double *)malloc(sizeof(double) * (size_t)r * (size_t)r);
    int st = orc_inverse(G, r, Gi, 0, NULL);
    if (st) { free(Gi); return st; }
    double *Z = (double *)calloc((size_t)r * (size_t)n, sizeof(double));
    double *dZ = (double *)calloc((size_t)r * (size_t)n, sizeof(double));
    for (int a = 0; a < r; a++)
        for (int b = 0; b < r; b++)
            for (int64_t j = 0; j < n; j++) Z[a * n + j] += Gi[a * r + b] * R[b * n + j];
    if (dC) memset(dC, 0, sizeof(double) * (size_t)m * (size_t)r);
    double L = 0.0;
    for (int64_t q = 0; q < nnz; q++) {
        int64_t i = oi[q], j = oj[q];
        if (i < 0 || i >= m || j < 0 || j >= n) { st = ORC_EINVAL; break; }
        double x = 0.0;
        for (int a = 0; a < r; a++) x += C[i * r + a] * Z[a * n + j];
        double e = aval[q] - x;
        L += e * e;
        double eb = -2.0 * e;
        for (int a = 0; a < r; a++) {
            if (dC) dC[i * r + a] += eb * Z[a * n + j];
            dZ[a * n + j] += eb * C[i * r + a];
        }
    }
    if (st == ORC_OK) {
        if (loss) *loss = L;
        if (dR) {
            for (int a = 0; a < r; a++)
                for (int64_t j = 0; j < n; j++) {
                    double s = 0.0;
                    for (int b = 0; b < r; b++) s += Gi[b * r + a] * dZ[b * n + j];
                    dR[a * n + j] = s;
                }
        }
        if (dG) {
            /* T = dZ Z^T (r x r), dG = -Gi^T T */
            double *T = (double *)calloc((size_t)r * (size_t)r, sizeof(double));
            for (int a = 0; a < r; a++)
                for (int b = 0; b < r; b++) {
                    double s = 0.0;
                    for (int64_t j = 0; j < n; j++) s += dZ[a * n + j] * Z[b * n + j];
                    T[a * r + b] = s;
                }
            for (int a = 0; a < r; a++)
                for (int b = 0; b < r; b++) {
                    double s = 0.0;
                    for (int c = 0; c < r; c++) s += Gi[c * r + a] * T[c * r + b];
                    dG[a * r + b] = -s;
                }
            free(T);
        }
    }
    free(Gi); free(Z); free(dZ);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Residual moments over all entries (q = 0) or over a random q x s          */
/* submatrix of E = W - C U R (a-posteriori estimation, Section 4: sample a  */
/* q x s submatrix of the error matrix, qs >= 100 or so, and use the observed */
/* statistics of its entries).  Rows are q distinct draws from stream 3,     */
/* columns s distinct draws from stream 4 of SplitMix64(seed).               */
/* out[0] = sum e, out[1] = sum e^2, out[2] = sum |e|, out[3] = sum w^2.     */
/* ------------------------------------------------------------------------ */
int orc_residual_moments(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I,
                         const int64_t *J, const double *U, int64_t q, int64_t s, uint64_t seed, double *out) {
    if (!A || !I || !J || !U || !out || r < 1 || m < 1 || n < 1 || lda < n || q < 0 || s < 0 || q > m || s > n ||
        ((q == 0) != (s == 0)))
        return ORC_EINVAL;
    int64_t nq = q ? q : m, ns = s ? s : n;
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)nq);
    int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)ns);
    if (q) {
        orc_draw_distinct(seed, 3, m, q, rows);
        orc_draw_distinct(seed, 4, n, s, cols);
    } else {
        for (int64_t i = 0; i < m; i++) rows[i] = i;
        for (int64_t j = 0; j < n; j++) cols[j] = j;
    }
    /* UR = U * W[I, cols]  (r x ns) */
    double *UR = (double *)calloc((size_t)r * (size_t)ns, sizeof(double));
    for (int a = 0; a < r; a++)
        for (int b = 0; b < r; b++) {
            double u = U[a * r + b];
            for (int64_t c = 0; c < ns; c++) UR[a * ns + c] += u * orc_get(A, dtype, lda, I[b], cols[c]);
        }
    double se = 0.0, se2 = 0.0, sabs = 0.0, sw2 = 0.0;
    double *cr = (double *)malloc(sizeof(double) * (size_t)r);
    for (int64_t ii = 0; ii < nq; ii++) {
        for (int a = 0; a < r; a++) cr[a] = orc_get(A, dtype, lda, rows[ii], J[a]);
        for (int64_t c = 0; c < ns; c++) {
            double x = 0.0;
            for (int a = 0; a < r; a++) x += cr[a] * UR[a * ns + c];
            double w = orc_get(A, dtype, lda, rows[ii], cols[c]);
            double e = w - x;
            se += e;
            se2 += e * e;
            sabs += fabs(e);
            sw2 += w * w;
        }
    }
    out[0] = se;
    out[1] = se2;
    out[2] = sabs;
    out[3] = sw2;
    free(rows); free(cols); free(UR); free(cr);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Superfast a-posteriori test (Section 4, the subsection on matrices       */
/* filled with i.i.d. values of one variable): the K = q s entries g_i of a  */
/* random q x s submatrix of E = W - C U R (rows from stream 3, columns from */
/* stream 4, as orc_residual_moments) are taken as observed values of one   */
/* Gaussian variable; then a customary test for its variance.               */
/*   mean_abs = (1/K) sum |g_i|      (the observed average as printed)       */
/*   mean     = (1/K) sum g_i                                               */
/*   var      = (1/K) sum (g_i - mean)^2                                     */
/* Reading: the centre of the printed variance is the sample mean (the      */
/* printed average of |g_i| would bias it upwards for a centred variable).  */
/* Test of H0: sigma^2 >= tau^2 against sigma^2 < tau^2 at the one-sided    */
/* normal level z of the chi-square statistic K var / sigma^2 (mean K - 1,  */
/* variance 2 (K - 1)): accept the LRA (reject H0) iff                       */
/*   K var <= tau^2 ((K - 1) - z sqrt(2 (K - 1))),                          */
/* i.e. var <= (1 - t) tau^2 (K - 1) / K with the paper's relative         */
/* deviation t = z sqrt(2 / (K - 1)).                                        */
/* out: [K, mean, mean_abs, var, threshold on var, accept (1 or 0)].        */
/* ------------------------------------------------------------------------ */
int orc_posterior_test(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I,
                       const int64_t *J, const double *U, int64_t q, int64_t s, uint64_t seed, double tau, double z,
                       double *out) {
    if (!A || !I || !J || !U || !out || r < 1 || m < 1 || n < 1 || lda < n || q < 1 || s < 1 || q > m || s > n ||
        q * s < 2 || !(tau > 0.0) || !isfinite(tau) || !isfinite(z))
        return ORC_EINVAL;
    const int64_t K = q * s;
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)q);
    int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)s);
    orc_draw_distinct(seed, 3, m, q, rows);
    orc_draw_distinct(seed, 4, n, s, cols);
    /* the sampled entries of E, entry (a, c) at g[a s + c] */
    double *g = (double *)malloc(sizeof(double) * (size_t)K);
    for (int64_t a = 0; a < q; a++)
        for (int64_t c = 0; c < s; c++) {
            double x = 0.0; /* (C U R)[rows[a], cols[c]] = sum_i C[rows[a], i] (U R)[i, cols[c]] */
            for (int i = 0; i < r; i++) {
                double ur = 0.0;
                for (int j = 0; j < r; j++) ur += U[i * r + j] * orc_get(A, dtype, lda, I[j], cols[c]);
                x += orc_get(A, dtype, lda, rows[a], J[i]) * ur;
            }
            g[a * s + c] = orc_get(A, dtype, lda, rows[a], cols[c]) - x;
        }
    double sum = 0.0, sabs = 0.0;
    for (int64_t k = 0; k < K; k++) {
        sum += g[k];
        sabs += fabs(g[k]);
    }
    const double mean = sum / (double)K;
    double ss = 0.0;
    for (int64_t k = 0; k < K; k++) ss += (g[k] - mean) * (g[k] - mean);
    const double var = ss / (double)K;
    const double dof = (double)(K - 1);
    const double thr = tau * tau * (dof - z * sqrt(2.0 * dof)) / (double)K;
    out[0] = (double)K;
    out[1] = mean;
    out[2] = sabs / (double)K;
    out[3] = var;
    out[4] = thr;
    out[5] = var <= thr ? 1.0 : 0.0;
    free(rows); free(cols); free(g);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Far-field interaction block of two planar point sets (the Superfast      */
/* Multipole discussion in Section "Some Implications and Extensions of Our */
/* Study": generators of blocks K_ij = 1/|x_i - y_j| between well separated */
/* clusters).  Written out in FP64, each operation rounded once:            */
/* dx = x_i0 - y_j0, dy = x_i1 - y_j1, K_ij = 1 / sqrt(dx*dx + dy*dy).      */
/* x: m points, y: n points, as (p0, p1) pairs; K row-major m x n.          */
/* ------------------------------------------------------------------------ */
int orc_fmm_entries(const double *x, int64_t m, const double *y, int64_t n, double *K) {
    if (!x || !y || !K || m < 1 || n < 1) return ORC_EINVAL;
    for (int64_t i = 0; i < m; i++) {
        for (int64_t j = 0; j < n; j++) {
            const double dx = x[2 * i] - y[2 * j];
            const double dy = x[2 * i + 1] - y[2 * j + 1];
            K[i * n + j] = 1.0 / sqrt(dx * dx + dy * dy);
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Cynical CUR and its combination with C-A loops (Section 1.3, the cynical */
/* algorithms of Fig. 3; Section 13, Tests 3 and Tests 4 with k = l = 4r).  */
/*   L: k distinct random columns (stream 0 of `seed`), ascending.           */
/*   loops = 0 (Tests 3): K: k distinct random rows (stream 5), ascending.   */
/*   loops >= 1 (Tests 4 for loops = 1): `loops` C-A loops at rank k from L  */
/*     (column step: K = dominant rows of W[:, L]; row step: L = dominant    */
/*     columns of W[K, :]), stopping early at a fixed point.                 */
/*   Then the k x k sketch S = W[K, L]: C-A at rank r on S (orc_ca_cur with  */
/*   seed + 1, `sweeps` loops), an r x r submatrix of locally maximal volume  */
/*   in S, mapped back: I = K[I_S], J = L[J_S]; U = W[I, J]^{-1}.            */
/* The paper's inner routine (Algorithms 1 and 2 of its reference P00) is   */
/* not given in the paper; C-A on the sketch, which ends in a set that is    */
/* dominant in its rows and in its columns, stands in for it.  info          */
/* describes the inner C-A; swaps_total counts both phases.                  */
/* ------------------------------------------------------------------------ */
int orc_cynical(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int r, int k, int loops,
                int sweeps, uint64_t seed, const orc_opts *opts_in, int64_t *I_out, int64_t *J_out, double *U_out,
                orc_info *info_out) {
    orc_opts o;
    if (opts_in) o = *opts_in; else orc_default_opts(&o);
    if (o.max_swaps < 0) o.max_swaps = 16 * k;
    orc_info info = {0, 0, 1, 0, 0, 0, 1.0, 0.0};
    info.rank_found = r;
    if (!A || !I_out || !J_out || !U_out || r < 1 || k < r || loops < 0 || sweeps < 1 || m < 1 || n < 1 ||
        lda < n || (int64_t)k > (m < n ? m : n) || dtype < 0 || dtype > 2 || !(o.delta >= 0.0) ||
        o.preprocess != 0 || o.init_cols) {
        if (info_out) *info_out = info;
        return ORC_EINVAL;
    }
    int64_t *K = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    int64_t *L = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    int64_t *Kp = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    int64_t *Lp = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    double *S = (double *)malloc(sizeof(double) * (size_t)k * (size_t)k);
    int64_t *Is = (int64_t *)malloc(sizeof(int64_t) * (size_t)r);
    int64_t *Js = (int64_t *)malloc(sizeof(int64_t) * (size_t)r);
    int st = ORC_OK;
    int32_t outer_swaps = 0;
    orc_draw_distinct(seed, 0, n, k, L);
    qsort(L, (size_t)k, sizeof(int64_t), cmp_i64);
    if (loops == 0) {
        orc_draw_distinct(seed, 5, m, k, K);
        qsort(K, (size_t)k, sizeof(int64_t), cmp_i64);
    }
    for (int s = 0; s < loops; s++) {
        orc_info oi = {0, 0, 1, 0, 0, 0, 1.0, 0.0};
        oi.rank_found = k;
        for (int a = 0; a < k; a++)
            if (!orc_finite_scan(A, dtype, lda, 0, m, L[a], 1)) { st = ORC_EINVAL; goto done; }
        st = orc_step(A, dtype, m, n, lda, k, 1, L, &o, K, &oi);
        if (st == ORC_OK) {
            for (int a = 0; a < k; a++)
                if (!orc_finite_scan(A, dtype, lda, K[a], 1, 0, n)) { st = ORC_EINVAL; goto done; }
            st = orc_step(A, dtype, m, n, lda, k, 0, K, &o, L, &oi);
        }
        outer_swaps += oi.swaps_total;
        if (oi.min_margin < info.min_margin) info.min_margin = oi.min_margin;
        if (st) {
            if (st == ORC_ESINGULAR) info.rank_found = oi.rank_found;
            goto done;
        }
        if (s > 0 && !memcmp(K, Kp, sizeof(int64_t) * (size_t)k) && !memcmp(L, Lp, sizeof(int64_t) * (size_t)k))
            break;
        memcpy(Kp, K, sizeof(int64_t) * (size_t)k);
        memcpy(Lp, L, sizeof(int64_t) * (size_t)k);
    }
    for (int a = 0; a < k; a++)
        for (int b = 0; b < k; b++) S[a * k + b] = orc_get(A, dtype, lda, K[a], L[b]);
    {
        orc_opts oi = o;
        oi.max_swaps = opts_in ? opts_in->max_swaps : -1;
        orc_info ii;
        st = orc_ca_cur(S, 0, k, k, k, r, sweeps, seed + 1, &oi, Is, Js, U_out, &ii);
        double mm = info.min_margin;
        info = ii;
        if (mm < info.min_margin) info.min_margin = mm;
        info.swaps_total += outer_swaps;
        if (st == ORC_OK) {
            for (int a = 0; a < r; a++) {
                I_out[a] = K[Is[a]];
                J_out[a] = L[Js[a]];
            }
        }
    }
done:
    free(K); free(L); free(Kp); free(Lp); free(S); free(Is); free(Js);
    if (st != ORC_OK) info.converged = 0;
    if (info_out) *info_out = info;
    return st;
}

/* ------------------------------------------------------------------------ */
/* The pre-processed matrix W' = W M of Tests 2 with abridged randomized    */
/* Hadamard pre-processing (Section 13; Appendix B for the multiplier):     */
/* M = D (H_{2^d} (x) I_s), N = 2^d s >= n, W zero-padded to N columns, D   */
/* the Rademacher signs of stream 1 (orc_sign), no scale.  Entry (i, b s + e) */
/* sums W[i][a s + e] D[a s + e] (-1)^{popcount(a & b)} over a = 0 .. 2^d-1 */
/* in order.  Wp is m x N row-major.                                        */
/* ------------------------------------------------------------------------ */
int orc_hadamard_apply(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int d, uint64_t seed,
                       double *Wp) {
    if (!A || !Wp || d < 0 || d > 20 || m < 1 || n < 1 || lda < n) return ORC_EINVAL;
    const int64_t q2 = (int64_t)1 << d;
    const int64_t s = (n + q2 - 1) / q2;
    const int64_t N = q2 * s;
    for (int64_t i = 0; i < m; i++) {
        for (int64_t j = 0; j < N; j++) {
            const int64_t b = j / s, e = j % s;
            double acc = 0.0;
            for (int64_t a = 0; a < q2; a++) {
                const int64_t c = a * s + e;
                if (c >= n) continue;
                const double h = (__builtin_popcountll((uint64_t)(a & b)) & 1) ? -1.0 : 1.0;
                acc += orc_get(A, dtype, lda, i, c) * orc_sign(seed, c) * h;
            }
            Wp[i * N + j] = acc;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Truncated pseudo-inverse of a k x l generator (Section 3, Algorithm      */
/* algcnnncl: U = W_{k,l,r}^+, the pseudo-inverse of the rank-r SVD          */
/* truncation).  One-sided Jacobi (Hestenes) SVD of G (k x l, row-major):   */
/* its l columns are rotated in round-robin pair order (orc_pair, a dummy   */
/* position for odd l) until a sweep rotates nothing (at most 60); a pair   */
/* is rotated unless |a_p . a_q| <= k eps sqrt(|a_p|^2 |a_q|^2), eps =       */
/* 2^-52 (the usual one-sided Jacobi test, scaled by the column length, so  */
/* that rounding in the dot products cannot keep a converged pair turning), */
/* or one of its columns is negligible, |a|^2 <= (k eps)^2 times the largest */
/* squared column norm at the start of the sweep (a column at the rounding  */
/* level of G, e.g. after duplicate columns cancel), or the rotation's sine  */
/* is zero.  Then                                                           */
/* sigma_j = |a_j|; the kept set is the r largest sigma_j (ties to the      */
/* lower j) among those above max(1e-14, max(k, l) eps) max sigma (the      */
/* usual numerical-rank tolerance, and at least the negligible-column       */
/* level, so a column left at rounding level is never kept); X (l x k,      */
/* row-major) =                                                             */
/* sum over kept j (increasing) of v_j a_j^T / sigma_j^2.  *rank_out gets   */
/* the number kept and *logvol the sum of their logs, log v_{2,r}(G) of     */
/* eq. (eqvol) when all r are kept.                                         */
/* ------------------------------------------------------------------------ */
int orc_pinv_trunc(const double *G, int k, int l, int r, double *X, int *rank_out, double *logvol) {
    if (!G || !X || k < 1 || l < 1 || r < 1 || r > (k < l ? k : l)) return ORC_EINVAL;
    double *A = (double *)malloc(sizeof(double) * (size_t)k * (size_t)l);
    double *V = (double *)calloc((size_t)l * (size_t)l, sizeof(double));
    double *sg = (double *)malloc(sizeof(double) * (size_t)l);
    char *keep = (char *)calloc((size_t)l, 1);
    memcpy(A, G, sizeof(double) * (size_t)k * (size_t)l);
    for (int j = 0; j < l; j++) V[j * l + j] = 1.0;
    const int lp = l + (l & 1);
    const double tol = (double)k * 0x1p-52;
    for (int sweep = 0; sweep < 60 && l > 1; sweep++) {
        int rotated = 0;
        double big = 0.0;
        for (int j = 0; j < l; j++) {
            double s2 = 0.0;
            for (int i = 0; i < k; i++) s2 += A[i * l + j] * A[i * l + j];
            if (s2 > big) big = s2;
        }
        for (int t = 0; t < lp - 1; t++) {
            for (int s = 0; s < lp / 2; s++) {
                int pc, qc;
                orc_pair(t, s, lp, &pc, &qc);
                if (qc >= l) continue;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = 0; i < k; i++) {
                    al += A[i * l + pc] * A[i * l + pc];
                    be += A[i * l + qc] * A[i * l + qc];
                    ga += A[i * l + pc] * A[i * l + qc];
                }
                if (ga == 0.0 || fabs(ga) <= tol * sqrt(al * be)) continue;
                if (al <= tol * tol * big || be <= tol * tol * big) continue;
                double ze = (be - al) / (2.0 * ga);
                double tt = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
                double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
                if (sn == 0.0) continue;
                for (int i = 0; i < k; i++) {
                    double x = A[i * l + pc], y = A[i * l + qc];
                    A[i * l + pc] = c * x - sn * y;
                    A[i * l + qc] = sn * x + c * y;
                }
                for (int i = 0; i < l; i++) {
                    double x = V[i * l + pc], y = V[i * l + qc];
                    V[i * l + pc] = c * x - sn * y;
                    V[i * l + qc] = sn * x + c * y;
                }
                rotated = 1;
            }
        }
        if (!rotated) break;
    }
    double smax = 0.0;
    for (int j = 0; j < l; j++) {
        double s2 = 0.0;
        for (int i = 0; i < k; i++) s2 += A[i * l + j] * A[i * l + j];
        sg[j] = sqrt(s2);
        if (sg[j] > smax) smax = sg[j];
    }
    /* a singular value counts only above the rounding level of the process:
       max(1e-14, max(k, l) eps) times the largest, never below the level at
       which the rotation test leaves a column as negligible */
    const double thr = fmax(1e-14, (double)(k > l ? k : l) * 0x1p-52);
    int kept = 0;
    double lv = 0.0;
    for (int j = 0; j < l; j++) {
        int above = 0;  /* sigma values ranked before j */
        for (int i = 0; i < l; i++)
            if (sg[i] > sg[j] || (sg[i] == sg[j] && i < j)) above++;
        if (above < r && sg[j] > thr * smax) { keep[j] = 1; kept++; lv += log(sg[j]); }
    }
    for (int a = 0; a < l; a++)
        for (int b = 0; b < k; b++) {
            double acc = 0.0;
            for (int j = 0; j < l; j++)
                if (keep[j]) acc += V[a * l + j] * A[b * l + j] / (sg[j] * sg[j]);
            X[a * k + b] = acc;
        }
    if (rank_out) *rank_out = kept;
    if (logvol) *logvol = lv;
    free(A); free(V); free(sg); free(keep);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Lower Cholesky factor Ch (r x r) of S S^T + e e^T, S = Rp[:, set[0..g-1]] */
/* (Rp item-major, r per item), e = Rp[:, extra] or nothing (extra < 0).     */
/* Returns 0 when the matrix is not positive definite.                      */
/* ------------------------------------------------------------------------ */
static int orc_gram_chol(const double *Rp, int r, const int64_t *set, int g, int64_t extra, double *Ch) {
    for (int a = 0; a < r; a++)
        for (int b = 0; b <= a; b++) {
            double s = 0.0;
            for (int q = 0; q < g; q++) s += Rp[set[q] * r + a] * Rp[set[q] * r + b];
            if (extra >= 0) s += Rp[extra * r + a] * Rp[extra * r + b];
            for (int c = 0; c < b; c++) s -= Ch[a * r + c] * Ch[b * r + c];
            if (a == b) {
                if (!(s > 0.0)) return 0;
                Ch[a * r + a] = sqrt(s);
            } else {
                Ch[a * r + b] = s / Ch[b * r + b];
            }
        }
    return 1;
}

/* y^T (L L^T)^{-1} y for y = Rp[:, it], by one forward solve L z = y.      */
static double orc_qform(const double *Rp, int r, const double *Ch, int64_t it, double *z) {
    double s = 0.0;
    for (int a = 0; a < r; a++) {
        double x = Rp[it * r + a];
        for (int c = 0; c < a; c++) x -= Ch[a * r + c] * z[c];
        z[a] = x / Ch[a * r + a];
        s += z[a] * z[a];
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Choice of k items whose vectors span a submatrix of large r-projective   */
/* volume (Section "Extension of the maximization of the r-projective      */
/* volume", Algorithm algprjvlm transposed as its remark reprvtov allows;   */
/* Appendix, Algorithms alg1tor and algrup and the expansion-contraction   */
/* recipe after them as its black box).  P (items x w, item-major) holds    */
/* one w-vector per item: a row of W[:, J] in a column step, a column of    */
/* W[I, :] in a row step.                                                   */
/*  1. Rank-revealing QRP of the w x items matrix P^T, truncated at r: r    */
/*     greedy Householder steps (orc_qrp).  Its first r rows R' (r x items) */
/*     are Q_r^T P^T, Q_r the first r columns of the orthogonal factor.     */
/*  2. Algorithm alg1tor on R': r greedy Householder steps over all items.  */
/*  3. Algorithm algrup: for g = r .. k-1 add the unchosen item y (column   */
/*     of R') maximising y^T (S S^T)^{-1} y, S = R'[:, chosen]: by eq. (eqb) */
/*     the factor 1 + y^T (S S^T)^{-1} y multiplies v_2(S)^2 when y joins.   */
/*  4. Refinement with p = 1: expand by the item b of step 3's rule, then   */
/*     contract by the member s (other than b) of smallest y_s^T (S' S'^T)^-1 */
/*     y_s, S' = S with b, whose removal multiplies v_2^2 by 1 minus that    */
/*     (eq. (eqa)).  The exchange is made while the product of the two       */
/*     factors exceeds 1 + delta (the threshold of the swaps of Algorithm    */
/*     algdomin) and at most max_swaps times (*converged = 0 when the cap    */
/*     stops a profitable exchange).                                         */
/* Every quadratic form is recomputed from a Cholesky factor of the Gram    */
/* matrix; ties go to the lowest item.  out[0..k-1] receives the items (an  */
/* exchange puts b in s's place).  Every decision's margin (gap to the      */
/* runner-up, relative; for the stop test |gain - (1 + delta)| / (1 +       */
/* delta)) goes into *min_margin.  Status: singular when step 1 or 2 meets  */
/* a zero remaining norm (*rank = step).                                    */
/* ------------------------------------------------------------------------ */
int orc_projective_select(const double *P, int64_t items, int w, int r, int k, double delta, int32_t max_swaps,
                          int64_t *out, int32_t *rank, double *min_margin, int32_t *swaps, int32_t *converged) {
    if (!P || !out || w < 1 || r < 1 || r > w || k < r || (int64_t)k > items || !(delta >= 0.0) || max_swaps < 0)
        return ORC_EINVAL;
    double *Z = (double *)malloc(sizeof(double) * (size_t)items * (size_t)w);
    double *Rp = (double *)malloc(sizeof(double) * (size_t)items * (size_t)r);
    double *Y = (double *)malloc(sizeof(double) * (size_t)items * (size_t)r);
    double *Ch = (double *)malloc(sizeof(double) * (size_t)r * (size_t)r);
    double *z = (double *)malloc(sizeof(double) * (size_t)r);
    char *used = (char *)calloc((size_t)items, 1);
    int64_t *piv = (int64_t *)malloc(sizeof(int64_t) * (size_t)r);
    int st = ORC_OK;
    int32_t sw = 0, conv = 1;
    if (rank) *rank = r;
    /* 1: R' from r steps of QRP on P^T */
    memcpy(Z, P, sizeof(double) * (size_t)items * (size_t)w);
    st = orc_qrp(Z, items, w, r, piv, rank, min_margin);
    if (st) goto out;
    for (int64_t it = 0; it < items; it++)
        for (int c = 0; c < r; c++) Rp[it * r + c] = Z[it * w + c];
    /* 2: alg1tor on R' */
    memcpy(Y, Rp, sizeof(double) * (size_t)items * (size_t)r);
    st = orc_qrp(Y, items, r, r, out, rank, min_margin);
    if (st) goto out;
    for (int g = 0; g < r; g++) used[out[g]] = 1;
    /* 3: algrup */
    for (int g = r; g < k; g++) {
        if (!orc_gram_chol(Rp, r, out, g, -1, Ch)) { st = ORC_ESINGULAR; if (rank) *rank = g; goto out; }
        int64_t best = -1;
        double v1 = -1.0, v2 = -1.0;
        for (int64_t it = 0; it < items; it++) {
            if (used[it]) continue;
            double q = orc_qform(Rp, r, Ch, it, z);
            if (q > v1) { v2 = v1; v1 = q; best = it; }
            else if (q > v2) v2 = q;
        }
        orc_note_margin(min_margin, v1, v2);
        out[g] = best;
        used[best] = 1;
    }
    /* 4: expansion-contraction exchanges */
    while ((int64_t)k < items) {
        if (!orc_gram_chol(Rp, r, out, k, -1, Ch)) { st = ORC_ESINGULAR; if (rank) *rank = k; goto out; }
        int64_t b = -1;
        double v1 = -1.0, v2 = -1.0;
        for (int64_t it = 0; it < items; it++) {
            if (used[it]) continue;
            double q = orc_qform(Rp, r, Ch, it, z);
            if (q > v1) { v2 = v1; v1 = q; b = it; }
            else if (q > v2) v2 = q;
        }
        orc_note_margin(min_margin, v1, v2);
        const double grow = 1.0 + v1;
        if (!orc_gram_chol(Rp, r, out, k, b, Ch)) { st = ORC_ESINGULAR; if (rank) *rank = k; goto out; }
        int64_t s = -1;
        double c1 = -1.0, c2 = -1.0;  /* contraction factors 1 - y^T (S' S'^T)^{-1} y */
        for (int64_t it = 0; it < items; it++) {
            if (!used[it]) continue;
            double c = 1.0 - orc_qform(Rp, r, Ch, it, z);
            if (c > c1) { c2 = c1; c1 = c; s = it; }
            else if (c > c2) c2 = c;
        }
        orc_note_margin(min_margin, c1, c2);
        const double gain = grow * c1;
        if (min_margin) {
            double mg = fabs(gain - (1.0 + delta)) / (1.0 + delta);
            if (mg < *min_margin) *min_margin = mg;
        }
        if (!(gain > 1.0 + delta)) break;
        if (sw >= max_swaps) { conv = 0; break; }
        for (int g = 0; g < k; g++)
            if (out[g] == s) { out[g] = b; break; }
        used[s] = 0;
        used[b] = 1;
        sw++;
    }
out:
    if (swaps) *swaps = sw;
    if (converged) *converged = conv;
    free(Z); free(Rp); free(Y); free(Ch); free(z); free(used); free(piv);
    return st;
}

/* ------------------------------------------------------------------------ */
/* C-A with k x l generators of large r-projective volume (Section 1.3 and  */
/* Fig. 4 with k x l sketches; Theorem th3 bounds the error of the          */
/* canonical CUR of such a generator).  J: l distinct random columns        */
/* (stream 0), ascending.  A sweep is a column step (I = the k rows that    */
/* orc_projective_select picks from W[:, J]) and a row step (J = the l      */
/* columns it picks from W[I, :]^T), sets sorted; the loop stops early at a */
/* fixed point.  Nucleus U = W[I, J]_r^+ (l x k, J-order x I-order) by      */
/* orc_pinv_trunc; info.det_log_abs = log v_{2,r}(W[I, J]); swaps_total     */
/* counts the exchanges of every step (delta and max_swaps per step, the    */
/* cap defaulting to 16 r when negative).                                   */
/* ------------------------------------------------------------------------ */
int orc_projective_cur(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int r, int k, int l, int sweeps,
                       uint64_t seed, double delta, int32_t max_swaps, int64_t *I_out, int64_t *J_out, double *U_out,
                       orc_info *info_out) {
    orc_info info = {0, 0, 1, 0, 0, 0, 1.0, 0.0};
    info.rank_found = r;
    if (max_swaps < 0) max_swaps = 16 * r;
    if (!A || !I_out || !J_out || !U_out || r < 1 || k < r || l < r || sweeps < 1 || m < 1 || n < 1 || lda < n ||
        (int64_t)k > m || (int64_t)l > n || dtype < 0 || dtype > 2 || !(delta >= 0.0)) {
        if (info_out) *info_out = info;
        return ORC_EINVAL;
    }
    int64_t *I = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    int64_t *J = (int64_t *)malloc(sizeof(int64_t) * (size_t)l);
    int64_t *Ip = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    int64_t *Jp = (int64_t *)malloc(sizeof(int64_t) * (size_t)l);
    int64_t wmax = (m > n ? m : n) * (int64_t)(k > l ? k : l);
    double *P = (double *)malloc(sizeof(double) * (size_t)wmax);
    double *G = (double *)malloc(sizeof(double) * (size_t)k * (size_t)l);
    int st = ORC_OK;
    orc_draw_distinct(seed, 0, n, l, J);
    qsort(J, (size_t)l, sizeof(int64_t), cmp_i64);
    for (int s = 0; s < sweeps; s++) {
        int32_t rk = r;
        for (int b = 0; b < l; b++)
            if (!orc_finite_scan(A, dtype, lda, 0, m, J[b], 1)) { st = ORC_EINVAL; goto done; }
        for (int64_t i = 0; i < m; i++)
            for (int b = 0; b < l; b++) P[i * l + b] = orc_get(A, dtype, lda, i, J[b]);
        int32_t sw = 0, cv = 1;
        st = orc_projective_select(P, m, l, r, k, delta, max_swaps, I, &rk, &info.min_margin, &sw, &cv);
        info.swaps_total += sw;
        if (!cv) info.converged = 0;
        if (st) { if (st == ORC_ESINGULAR) info.rank_found = rk; goto done; }
        qsort(I, (size_t)k, sizeof(int64_t), cmp_i64);
        for (int a = 0; a < k; a++)
            if (!orc_finite_scan(A, dtype, lda, I[a], 1, 0, n)) { st = ORC_EINVAL; goto done; }
        for (int64_t j = 0; j < n; j++)
            for (int a = 0; a < k; a++) P[j * k + a] = orc_get(A, dtype, lda, I[a], j);
        st = orc_projective_select(P, n, k, r, l, delta, max_swaps, J, &rk, &info.min_margin, &sw, &cv);
        info.swaps_total += sw;
        if (!cv) info.converged = 0;
        if (st) { if (st == ORC_ESINGULAR) info.rank_found = rk; goto done; }
        qsort(J, (size_t)l, sizeof(int64_t), cmp_i64);
        info.sweeps_run = s + 1;
        if (s > 0 && !memcmp(I, Ip, sizeof(int64_t) * (size_t)k) && !memcmp(J, Jp, sizeof(int64_t) * (size_t)l))
            break;
        memcpy(Ip, I, sizeof(int64_t) * (size_t)k);
        memcpy(Jp, J, sizeof(int64_t) * (size_t)l);
    }
    for (int a = 0; a < k; a++)
        for (int b = 0; b < l; b++) G[a * l + b] = orc_get(A, dtype, lda, I[a], J[b]);
    {
        int nr = r;
        st = orc_pinv_trunc(G, k, l, r, U_out, &nr, &info.det_log_abs);
        info.nucleus_rank = nr;
    }
    memcpy(I_out, I, sizeof(int64_t) * (size_t)k);
    memcpy(J_out, J, sizeof(int64_t) * (size_t)l);
done:
    free(I); free(J); free(Ip); free(Jp); free(P); free(G);
    if (st != ORC_OK) info.converged = 0;
    if (info_out) *info_out = info;
    return st;
}

/* ------------------------------------------------------------------------ */
/* k i.i.d. uniform draws from [0, n) WITH replacement, in draw order: the   */
/* accepted outputs of the stream (the top 2^64 mod n values rejected, as in */
/* orc_draw_distinct), reduced modulo n.  This is the sampling matrix of     */
/* Algorithm algsmplex (exactly k columns, each drawn with probability p_i)  */
/* for uniform leverage scores p_i = 1/n.                                    */
/* ------------------------------------------------------------------------ */
int orc_draw_uniform(uint64_t seed, uint64_t stream, int64_t n, int64_t k, int64_t *out) {
    if (n <= 0 || k < 0 || (k > 0 && !out)) return ORC_EINVAL;
    uint64_t un = (uint64_t)n;
    uint64_t rem = (0 - un) % un;
    uint64_t lim = 0 - rem;
    uint64_t ctr = 0;
    int64_t got = 0;
    while (got < k) {
        uint64_t u = orc_rng_u64(seed, stream, ctr++);
        if (rem != 0 && u >= lim) continue;
        out[got++] = (int64_t)(u % un);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* CUR LRA with uniform leverage scores (Algorithm algcurlevsc with        */
/* p_j = 1/n and pbar_i = 1/m, the superfast case of the section on          */
/* leverage scores for random and average inputs):                          */
/*   stage 2: J = l uniform draws with replacement (stream 8),              */
/*            D = diag(1 / sqrt(l p_j)) = sqrt(n / l) I_l;                   */
/*   stage 4: I = k uniform draws with replacement (stream 9),              */
/*            Dbar = sqrt(m / k) I_k;                                        */
/*   stage 6: M = Dbar W[I, J] D, U = D M_r^+ Dbar.                          */
/* Reading: M^+ is the canonical nucleus of the k x l generator, the pseudo- */
/* inverse of its rank-r SVD truncation (orc_pinv_trunc), r being the       */
/* numerical rank the algorithm assumes of W.  I and J are returned sorted   */
/* ascending, duplicates kept (U's rows and columns follow that order).     */
/* Only the k l entries of W[I, J] are read; a non-finite one is EINVAL.    */
/* info.det_log_abs = log v_{2,r}(M), info.nucleus_rank = values kept.      */
/* ------------------------------------------------------------------------ */
int orc_uniform_cur(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int r, int k, int l, uint64_t seed,
                    int64_t *I_out, int64_t *J_out, double *U_out, orc_info *info_out) {
    orc_info info = {0, 0, 1, 0, 0, 0, 1.0, 0.0};
    info.rank_found = r;
    if (!A || !I_out || !J_out || !U_out || r < 1 || k < r || l < r || m < 1 || n < 1 || lda < n || dtype < 0 ||
        dtype > 2) {
        if (info_out) *info_out = info;
        return ORC_EINVAL;
    }
    orc_draw_uniform(seed, 8, n, l, J_out);
    orc_draw_uniform(seed, 9, m, k, I_out);
    qsort(J_out, (size_t)l, sizeof(int64_t), cmp_i64);
    qsort(I_out, (size_t)k, sizeof(int64_t), cmp_i64);
    double *M = (double *)malloc(sizeof(double) * (size_t)k * (size_t)l);
    const double dn = sqrt((double)n / (double)l), dm = sqrt((double)m / (double)k);
    int st = ORC_OK;
    for (int a = 0; a < k && st == ORC_OK; a++)
        for (int b = 0; b < l; b++) {
            double w = orc_get(A, dtype, lda, I_out[a], J_out[b]);
            if (!isfinite(w)) { st = ORC_EINVAL; break; }
            M[a * l + b] = (dm * w) * dn;
        }
    if (st == ORC_OK) {
        int nr = r;
        st = orc_pinv_trunc(M, k, l, r, U_out, &nr, &info.det_log_abs);
        info.nucleus_rank = nr;
        for (int64_t e = 0; e < (int64_t)l * k; e++) U_out[e] = (dn * U_out[e]) * dm;
    }
    free(M);
    if (st != ORC_OK) info.converged = 0;
    if (info_out) *info_out = info;
    return st;
}

/* ------------------------------------------------------------------------ */
/* Leverage scores of the items of a panel P (items x r, item-major) with   */
/* respect to its column space: q_i = P_i (P^T P)^{-1} P_i^T, formed as      */
/* |L^{-1} P_i^T|^2 with L the lower Cholesky factor of the Gram matrix      */
/* P^T P (every entry summed over the items in increasing order, the solve  */
/* and the norm in increasing index order).  cdf[i] = q_0 + ... + q_i in    */
/* that order.  Status singular when the Gram matrix is not positive        */
/* definite.                                                                */
/* ------------------------------------------------------------------------ */
static int orc_leverage(const double *P, int64_t items, int r, double *q, double *cdf) {
    double *Gm = (double *)calloc((size_t)r * (size_t)r, sizeof(double));
    double *L = (double *)calloc((size_t)r * (size_t)r, sizeof(double));
    double *z = (double *)malloc(sizeof(double) * (size_t)r);
    int st = ORC_OK;
    for (int a = 0; a < r; a++)
        for (int b = 0; b <= a; b++) {
            double s = 0.0;
            for (int64_t i = 0; i < items; i++) s += P[i * r + a] * P[i * r + b];
            Gm[a * r + b] = s;
        }
    for (int a = 0; a < r && st == ORC_OK; a++)
        for (int b = 0; b <= a; b++) {
            double s = Gm[a * r + b];
            for (int c = 0; c < b; c++) s -= L[a * r + c] * L[b * r + c];
            if (a == b) {
                if (!(s > 0.0)) { st = ORC_ESINGULAR; break; }
                L[a * r + a] = sqrt(s);
            } else {
                L[a * r + b] = s / L[b * r + b];
            }
        }
    double acc = 0.0;
    for (int64_t i = 0; i < items && st == ORC_OK; i++) {
        double s = 0.0;
        for (int a = 0; a < r; a++) {
            double x = P[i * r + a];
            for (int c = 0; c < a; c++) x -= L[a * r + c] * z[c];
            z[a] = x / L[a * r + a];
            s += z[a] * z[a];
        }
        q[i] = s;
        acc += s;
        cdf[i] = acc;
    }
    free(Gm); free(L); free(z);
    return st;
}

/* k i.i.d. draws by scores (Algorithm algsmplex, exactly k items, item i    */
/* with probability q_i / S, S = cdf[items - 1]): draw t takes u_t = (x >>   */
/* 11) 2^-53 from SplitMix64 output t of `stream` and picks the first item   */
/* i with cdf[i] > u_t S.                                                    */
static void orc_sample_scores(const double *cdf, int64_t items, uint64_t seed, uint64_t stream, int k, int64_t *out) {
    const double S = cdf[items - 1];
    for (int t = 0; t < k; t++) {
        const double u = (double)(orc_rng_u64(seed, stream, (uint64_t)t) >> 11) * 0x1p-53;
        const double target = u * S;
        int64_t lo = 0, hi = items - 1;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > target) hi = mid; else lo = mid + 1;
        }
        out[t] = lo;
    }
}

/* ------------------------------------------------------------------------ */
/* Refinement of a CUR LRA by its leverage scores (section on refining an   */
/* LRA with leverage scores: the scores of a crude LRA W' stand in for     */
/* those of W; Algorithm algcurlevsc with them, sampling by Algorithm       */
/* algsmplex).  The crude LRA is the CUR of (I0, J0) (r rows and columns):  */
/* W' = C U R with C = W[:, J0], R = W[I0, :], so its column space is that  */
/* of C and its row space that of R.                                        */
/*   column scores q_j of R^T and row scores qbar_i of C (orc_leverage);    */
/*   J = l draws by q (stream 8), I = k draws by qbar (stream 9), sorted;   */
/*   D = diag(1 / sqrt(l q_j / S)), Dbar = diag(1 / sqrt(k qbar_i / Sbar)); */
/*   M = Dbar W[I, J] D (entry (dbar_a w) d_b), U = D M_r^+ Dbar (entry     */
/*   (d_b x) dbar_a), M_r^+ by orc_pinv_trunc (the canonical nucleus, R29). */
/* Reading: the scores are taken with beta = 1 from the crude LRA's own     */
/* factors (their leverage scores are those of W' when U is nonsingular).   */
/* I, J (k and l entries) sorted ascending, duplicates kept; U is l x k.    */
/* ------------------------------------------------------------------------ */
int orc_leverage_cur(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int r, const int64_t *I0,
                     const int64_t *J0, int k, int l, uint64_t seed, int64_t *I_out, int64_t *J_out, double *U_out,
                     orc_info *info_out) {
    orc_info info = {0, 0, 1, 0, 0, 0, 1.0, 0.0};
    info.rank_found = r;
    if (!A || !I0 || !J0 || !I_out || !J_out || !U_out || r < 1 || k < r || l < r || m < 1 || n < 1 || lda < n ||
        (int64_t)r > (m < n ? m : n) || dtype < 0 || dtype > 2) {
        if (info_out) *info_out = info;
        return ORC_EINVAL;
    }
    double *Pr = (double *)malloc(sizeof(double) * (size_t)n * (size_t)r);   /* R^T, n x r */
    double *Pc = (double *)malloc(sizeof(double) * (size_t)m * (size_t)r);   /* C, m x r */
    double *qc = (double *)malloc(sizeof(double) * (size_t)n), *cc = (double *)malloc(sizeof(double) * (size_t)n);
    double *qr = (double *)malloc(sizeof(double) * (size_t)m), *cr = (double *)malloc(sizeof(double) * (size_t)m);
    double *M = (double *)malloc(sizeof(double) * (size_t)k * (size_t)l);
    double *dl = (double *)malloc(sizeof(double) * (size_t)l), *dk = (double *)malloc(sizeof(double) * (size_t)k);
    int st = ORC_OK;
    for (int a = 0; a < r && st == ORC_OK; a++) {
        if (I0[a] < 0 || I0[a] >= m || J0[a] < 0 || J0[a] >= n) st = ORC_EINVAL;
    }
    for (int64_t j = 0; j < n && st == ORC_OK; j++)
        for (int a = 0; a < r; a++) {
            double w = orc_get(A, dtype, lda, I0[a], j);
            if (!isfinite(w)) { st = ORC_EINVAL; break; }
            Pr[j * r + a] = w;
        }
    for (int64_t i = 0; i < m && st == ORC_OK; i++)
        for (int a = 0; a < r; a++) {
            double w = orc_get(A, dtype, lda, i, J0[a]);
            if (!isfinite(w)) { st = ORC_EINVAL; break; }
            Pc[i * r + a] = w;
        }
    if (st == ORC_OK) st = orc_leverage(Pr, n, r, qc, cc);
    if (st == ORC_OK) st = orc_leverage(Pc, m, r, qr, cr);
    if (st == ORC_OK) {
        orc_sample_scores(cc, n, seed, 8, l, J_out);
        orc_sample_scores(cr, m, seed, 9, k, I_out);
        qsort(J_out, (size_t)l, sizeof(int64_t), cmp_i64);
        qsort(I_out, (size_t)k, sizeof(int64_t), cmp_i64);
        const double S = cc[n - 1], Sb = cr[m - 1];
        for (int b = 0; b < l; b++) dl[b] = 1.0 / sqrt(((double)l * qc[J_out[b]]) / S);
        for (int a = 0; a < k; a++) dk[a] = 1.0 / sqrt(((double)k * qr[I_out[a]]) / Sb);
        for (int a = 0; a < k && st == ORC_OK; a++)
            for (int b = 0; b < l; b++) {
                double w = orc_get(A, dtype, lda, I_out[a], J_out[b]);
                if (!isfinite(w)) { st = ORC_EINVAL; break; }
                M[a * l + b] = (dk[a] * w) * dl[b];
            }
    }
    if (st == ORC_OK) {
        int nr = r;
        st = orc_pinv_trunc(M, k, l, r, U_out, &nr, &info.det_log_abs);
        info.nucleus_rank = nr;
        for (int b = 0; b < l; b++)
            for (int a = 0; a < k; a++) U_out[b * k + a] = (dl[b] * U_out[b * k + a]) * dk[a];
    }
    if (st == ORC_ESINGULAR) info.rank_found = 0;
    free(Pr); free(Pc); free(qc); free(cc); free(qr); free(cr); free(M); free(dl); free(dk);
    if (st != ORC_OK) info.converged = 0;
    if (info_out) *info_out = info;
    return st;
}

/* Leverage scores and their running sums, exported for the pins. */
int orc_leverage_scores(const double *P, int64_t items, int r, double *q, double *cdf) {
    if (!P || !q || !cdf || items < 1 || r < 1) return ORC_EINVAL;
    return orc_leverage(P, items, r, q, cdf);
}

/* ------------------------------------------------------------------------ */
/* Rank-r leverage scores of the items of a sketch P (items x w, item-      */
/* major, w >= r): eq. eqlevsc with beta = 1, p_i = |u_i^(r)|^2 / r, u_i^(r) */
/* row i of the items x r factor of P's r dominant left singular vectors.   */
/* Plain one-sided Jacobi (Hestenes) SVD of P: cyclic sweeps over the       */
/* column pairs (a, b), a < b, in row order; a pair is rotated when         */
/* |g| > w eps sqrt(al be) (al = |p_a|^2, be = |p_b|^2, g = p_a . p_b) so   */
/* that it becomes orthogonal; sweeps until none rotates (at most 80).      */
/* Then sigma_a = |p_a|; kept are the r largest (ties to the lower index)   */
/* among those with sigma_a^2 > 1e-13 sigma_max^2, and q_i = the sum over   */
/* the kept, largest first, of (P_ia / sigma_a)^2 (so the q_i sum to the     */
/* number kept).  Reading: a sketch of numerical rank below r (a row drawn   */
/* twice) gives the scores of its whole dominant subspace; 1e-13 lies far    */
/* above the rounding level of sigma^2 however it is computed and far below */
/* the top singular values of the inputs the method is meant for.           */
/* cdf[i] = q_0 + ... + q_i.  ESINGULAR when nothing is kept (P = 0).        */
/* ------------------------------------------------------------------------ */
static int orc_top_scores(const double *P, int64_t items, int w, int r, double *q, double *cdf) {
    double *B = (double *)malloc(sizeof(double) * (size_t)items * (size_t)w);   /* column-major copy */
    double *sig = (double *)malloc(sizeof(double) * (size_t)w);
    int *top = (int *)malloc(sizeof(int) * (size_t)w);
    for (int a = 0; a < w; a++)
        for (int64_t i = 0; i < items; i++) B[(size_t)a * items + i] = P[i * w + a];
    const double tol = (double)w * 0x1p-52;
    for (int sweep = 0; sweep < 80; sweep++) {
        int rotated = 0;
        for (int a = 0; a < w - 1; a++)
            for (int b = a + 1; b < w; b++) {
                double *x = B + (size_t)a * items, *y = B + (size_t)b * items;
                double al = 0.0, be = 0.0, g = 0.0;
                for (int64_t i = 0; i < items; i++) {
                    al += x[i] * x[i];
                    be += y[i] * y[i];
                    g += x[i] * y[i];
                }
                if (g == 0.0 || fabs(g) <= tol * sqrt(al * be)) continue;
                const double ze = (be - al) / (2.0 * g);
                const double t = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                if (s == 0.0) continue;
                for (int64_t i = 0; i < items; i++) {
                    const double u = x[i], v = y[i];
                    x[i] = c * u - s * v;
                    y[i] = s * u + c * v;
                }
                rotated = 1;
            }
        if (!rotated) break;
    }
    for (int a = 0; a < w; a++) {
        double s2 = 0.0;
        for (int64_t i = 0; i < items; i++) s2 += B[(size_t)a * items + i] * B[(size_t)a * items + i];
        sig[a] = sqrt(s2);
    }
    /* the r largest, largest first (selection; ties to the lower index) */
    double smax = 0.0;
    for (int a = 0; a < w; a++) smax = sig[a] > smax ? sig[a] : smax;
    int kept = 0;
    for (int t = 0; t < r; t++) {
        int best = -1;
        for (int a = 0; a < w; a++) {
            int used = 0;
            for (int u = 0; u < t; u++) used |= top[u] == a;
            if (!used && (best < 0 || sig[a] > sig[best])) best = a;
        }
        top[t] = best;
        if (sig[best] * sig[best] > 1e-13 * (smax * smax)) kept = t + 1;
    }
    int st = kept > 0 ? ORC_OK : ORC_ESINGULAR;
    double acc = 0.0;
    for (int64_t i = 0; i < items && st == ORC_OK; i++) {
        double s = 0.0;
        for (int t = 0; t < kept; t++) {
            const double u = B[(size_t)top[t] * items + i] / sig[top[t]];
            s += u * u;
        }
        q[i] = s;
        acc += s;
        cdf[i] = acc;
    }
    free(B); free(sig); free(top);
    return st;
}

/* Rank-r scores of a sketch, exported for the pins. */
int orc_sketch_scores(const double *P, int64_t items, int w, int r, double *q, double *cdf) {
    if (!P || !q || !cdf || items < 1 || w < 1 || r < 1 || r > w) return ORC_EINVAL;
    return orc_top_scores(P, items, w, r, q, cdf);
}

/* Distance of the draws of orc_sample_scores from the nearest boundary of  */
/* the items they picked, relative to S: min over t of min(cdf[i_t] - u_t S, */
/* u_t S - cdf[i_t - 1]) / S (cdf[-1] = 0).  A draw whose u_t S moves by     */
/* less than this keeps its item.                                           */
static double orc_sample_margin(const double *cdf, int64_t items, uint64_t seed, uint64_t stream, int k,
                                const int64_t *picked) {
    const double S = cdf[items - 1];
    double mg = 1.0;
    for (int t = 0; t < k; t++) {
        const double u = (double)(orc_rng_u64(seed, stream, (uint64_t)t) >> 11) * 0x1p-53;
        const double target = u * S;
        const int64_t i = picked[t];
        const double hi = (cdf[i] - target) / S, lo = (target - (i > 0 ? cdf[i - 1] : 0.0)) / S;
        const double d = hi < lo ? hi : lo;
        mg = d < mg ? d : mg;
    }
    return mg;
}

/* Pairs (index, scale) sorted by index, for keeping each drawn item's     */
/* rescaling factor beside it.                                              */
typedef struct {
    int64_t idx;
    double scale;
} orc_drawn;

static int cmp_drawn(const void *a, const void *b) {
    const int64_t x = ((const orc_drawn *)a)->idx, y = ((const orc_drawn *)b)->idx;
    return (x > y) - (x < y);
}

/* One half-step of C-A with DMM08 sampling: scores of the sketch P (items x */
/* w) by orc_top_scores, then cnt draws by them (Algorithm algsmplex,        */
/* orc_sample_scores on `stream`), sorted ascending with duplicates kept,    */
/* and each draw's rescaling 1 / sqrt(cnt q_i / S) of Algorithm algsmplex.  */
static int orc_dmm_half(const double *P, int64_t items, int w, int r, int cnt, uint64_t seed, uint64_t stream,
                        int64_t *set, double *scale, double *margin) {
    double *q = (double *)malloc(sizeof(double) * (size_t)items);
    double *cdf = (double *)malloc(sizeof(double) * (size_t)items);
    orc_drawn *dr = (orc_drawn *)malloc(sizeof(orc_drawn) * (size_t)cnt);
    int st = orc_top_scores(P, items, w, r, q, cdf);
    if (st == ORC_OK) {
        orc_sample_scores(cdf, items, seed, stream, cnt, set);
        const double mg = orc_sample_margin(cdf, items, seed, stream, cnt, set);
        *margin = mg < *margin ? mg : *margin;
        const double S = cdf[items - 1];
        for (int t = 0; t < cnt; t++) {
            dr[t].idx = set[t];
            dr[t].scale = 1.0 / sqrt(((double)cnt * q[set[t]]) / S);
        }
        qsort(dr, (size_t)cnt, sizeof(orc_drawn), cmp_drawn);
        for (int t = 0; t < cnt; t++) {
            set[t] = dr[t].idx;
            scale[t] = dr[t].scale;
        }
    }
    free(q); free(cdf); free(dr);
    return st;
}

/* ------------------------------------------------------------------------ */
/* C-A whose step subalgorithm is the leverage-score sampling of DMM08      */
/* applied to every vertical and horizontal sketch (Section "Testing C-A    */
/* acceleration of the algorithms of DMM08", Tables 7 and 8: eight C-A      */
/* iterations; the sampling is that of Algorithm algcurlevsc with Algorithm */
/* algsmplex, the scores those of eq. eqlevsc with beta = 1 taken of the     */
/* sketch in place of W).                                                    */
/*   start: J = l uniform draws (stream 8), D = sqrt(n / l) I (uniform       */
/*          scores, as in orc_uniform_cur);                                 */
/*   iteration t = 0 .. iters - 1:                                          */
/*     rows:    sketch W[:, J] D (m x l); its rank-r row scores; k draws     */
/*              (stream 16 + 2t) -> I sorted, Dbar = diag(1/sqrt(k p_i));    */
/*     columns: sketch Dbar W[I, :] (k x n); its rank-r column scores; l     */
/*              draws (stream 17 + 2t) -> J sorted, D = diag(1/sqrt(l p_j)); */
/*   nucleus: M = Dbar W[I, J] D, U = D M_r^+ Dbar (orc_pinv_trunc).         */
/* Readings: the sketches are rescaled as Algorithm algcurlevsc rescales C   */
/* before its row scores (stage 3 takes them of (C D)^T), on both sides;     */
/* draws are Exactly(k) / Exactly(l) (Algorithm algsmplex), so every step    */
/* returns k rows and l columns; one iteration is a row step then a column  */
/* step, so the last two steps are Algorithm algcurlevsc applied to W^T      */
/* with the row scores of the last vertical sketch.                          */
/* info: sweeps_run = iters, nucleus_rank, det_log_abs = log v_{2,r}(M),    */
/* min_margin = the smallest relative distance of a draw from the boundary  */
/* of the item it picked (orc_sample_margin) over all steps.  A non-finite  */
/* entry read is EINVAL; a zero sketch is ESINGULAR.                        */
/* ------------------------------------------------------------------------ */
int orc_dmm_ca(const void *A, int dtype, int64_t m, int64_t n, int64_t lda, int r, int k, int l, int iters,
               uint64_t seed, int64_t *I_out, int64_t *J_out, double *U_out, orc_info *info_out) {
    orc_info info = {0, 0, 1, 0, 0, 0, 1.0, 0.0};
    info.rank_found = r;
    if (!A || !I_out || !J_out || !U_out || r < 1 || k < r || l < r || iters < 1 || m < 1 || n < 1 || lda < n ||
        (int64_t)r > (m < n ? m : n) || dtype < 0 || dtype > 2) {
        info.converged = 0;
        if (info_out) *info_out = info;
        return ORC_EINVAL;
    }
    double *P = (double *)malloc(sizeof(double) * (size_t)(m > n ? m : n) * (size_t)(k > l ? k : l));
    double *dl = (double *)malloc(sizeof(double) * (size_t)l), *dk = (double *)malloc(sizeof(double) * (size_t)k);
    double *M = (double *)malloc(sizeof(double) * (size_t)k * (size_t)l);
    int st = ORC_OK;
    orc_draw_uniform(seed, 8, n, l, J_out);
    qsort(J_out, (size_t)l, sizeof(int64_t), cmp_i64);
    for (int b = 0; b < l; b++) dl[b] = sqrt((double)n / (double)l);
    double margin = 1.0;
    for (int t = 0; t < iters && st == ORC_OK; t++) {
        for (int64_t i = 0; i < m && st == ORC_OK; i++)
            for (int b = 0; b < l; b++) {
                const double w = orc_get(A, dtype, lda, i, J_out[b]);
                if (!isfinite(w)) { st = ORC_EINVAL; break; }
                P[i * l + b] = w * dl[b];
            }
        if (st == ORC_OK) st = orc_dmm_half(P, m, l, r, k, seed, 16 + 2 * (uint64_t)t, I_out, dk, &margin);
        for (int64_t j = 0; j < n && st == ORC_OK; j++)
            for (int a = 0; a < k; a++) {
                const double w = orc_get(A, dtype, lda, I_out[a], j);
                if (!isfinite(w)) { st = ORC_EINVAL; break; }
                P[j * k + a] = dk[a] * w;
            }
        if (st == ORC_OK) st = orc_dmm_half(P, n, k, r, l, seed, 17 + 2 * (uint64_t)t, J_out, dl, &margin);
        info.sweeps_run = t + 1;
    }
    for (int a = 0; a < k && st == ORC_OK; a++)
        for (int b = 0; b < l; b++) {
            const double w = orc_get(A, dtype, lda, I_out[a], J_out[b]);
            if (!isfinite(w)) { st = ORC_EINVAL; break; }
            M[a * l + b] = (dk[a] * w) * dl[b];
        }
    if (st == ORC_OK) {
        int nr = r;
        st = orc_pinv_trunc(M, k, l, r, U_out, &nr, &info.det_log_abs);
        info.nucleus_rank = nr;
        for (int b = 0; b < l; b++)
            for (int a = 0; a < k; a++) U_out[b * k + a] = (dl[b] * U_out[b * k + a]) * dk[a];
    }
    info.min_margin = margin;
    if (st == ORC_ESINGULAR) info.rank_found = 0;
    if (st != ORC_OK) info.converged = 0;
    free(P); free(dl); free(dk); free(M);
    if (info_out) *info_out = info;
    return st;
}
