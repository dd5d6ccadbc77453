/*
 * ftgemm_oracle.c -- plain CPU oracle for the fault-tolerant GEMM.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the GPU path must compute.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * library (libftgemm) never links, loads or calls it, and the two share no
 * code, header, table or helper.
 *
 * Source of the method: Wu, Zhai, Huang, Jian, Chen, "FT-GEMM: A Fault
 * Tolerant High Performance GEMM Implementation on x86 CPUs" (HPDC'23 poster).
 *   - Section 2.1 (Implementation of DGEMM): C = alpha*A*B + beta*C computed
 *     block by block; blocks of the output are the unit of work.
 *   - Section 2.2 (FT-DGEMM): the two checksum vectors of C are encoded while
 *     C is scaled by beta, the operand checksums are formed while A and B are
 *     staged (each staged element of B feeds B's own checksum and the
 *     encoded row checksum of C; each staged element of A feeds the encoded
 *     column checksum of C), and the reference checksums are the sums of the
 *     computed output; comparing the two verifies the multiplication.
 *   - Section 2.3 (Parallel FT-DGEMM): the output is split into independent
 *     parts, each carrying its own slice of the checksums.
 *   - Section 1 (Introduction): fail-continue soft errors in compute logic are
 *     the fault model; Huang and Abraham's ABFT is the underlying scheme.
 *
 * Notation (the reading taken of Section 2.2, where the paper never writes a
 * formula): e is the all-ones vector, X^c = X e (one entry per row) and
 * X^r = e^T X (one entry per column).  Everything here is FP64 and
 * column-major, in the BLAS convention: op(A) is m x k, op(B) is k x n.
 *
 * One-sided mode (one_sided = 1; the ranked extension "one-sided checksum plus
 * recompute on detection" for the low-precision formats): only the column
 * checksum C^c = C e of each tile is encoded and compared, one entry per row;
 * any disagreeing row has the tile computed again, since one side can
 * neither place the faulty column nor tell a data fault from a checksum
 * fault.  Faults aimed at the row checksum have no entry to land on.
 *
 * Weighted mode (weighted = 1; the ranked extension "weighted checksum
 * vectors locate two errors"): each tile also carries a weighted row
 * checksum per column, weights w_i = i + 1 over the tile's local rows.  A
 * single error at local row r of column j shows as (r + 1) times the plain
 * residual of column j on it, which locates the error without pairing
 * residuals by size and confirms every correction (see ft_tile).
 *
 * Pins (tests/test_oracle_*.py): the checksum identities e^T(AB) = (e^T A)B
 * and (AB)e = A(Be) bit-exactly on small-integer data; brute-force location
 * of single injected errors; bit-exact recovery of integer data; GEMM against
 * numpy's matmul; BLAS special cases; exhaustive decoders against torch; the
 * hand-worked example in tests/golden/.  The detection threshold is a
 * reading (the paper gives none): its value is pinned by hand-worked values
 * of every term of the bound (tests/golden/threshold_example.txt), and its
 * magnitude by tile residuals that the tests form with their own FP32 and
 * FP64 accumulation, which must lie within [1e-4, 1) of it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Number formats (inputs of the low-precision GEMMs), decoded from their    */
/* bit-level definitions.                                                    */
/* ------------------------------------------------------------------------- */

/* bfloat16: 1 sign bit, 8 exponent bits (bias 127), 7 fraction bits. */
double oracle_bf16_value(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int e = (h >> 7) & 0xff;
    int f = h & 0x7f;
    double v;
    if (e == 0xff)
        v = (f == 0) ? INFINITY : NAN;
    else if (e == 0)
        v = ldexp((double)f, -126 - 7);            /* subnormal: 0.f * 2^-126 */
    else
        v = ldexp((double)(128 + f), e - 127 - 7); /* 1.f * 2^(e-127) */
    return sign ? -v : v;
}

/* OCP FP8 E4M3 ("fn": finite, no infinities): 1 sign, 4 exponent bits
 * (bias 7), 3 fraction bits; exponent 15 with fraction 7 is NaN, so the
 * largest finite magnitude is 1.75 * 2^8 = 448. */
double oracle_e4m3_value(uint8_t b)
{
    int sign = (b >> 7) & 1;
    int e = (b >> 3) & 0xf;
    int f = b & 0x7;
    double v;
    if (e == 0xf && f == 0x7)
        v = NAN;
    else if (e == 0)
        v = ldexp((double)f, -6 - 3);              /* subnormal: 0.f * 2^-6 */
    else
        v = ldexp((double)(8 + f), e - 7 - 3);     /* 1.f * 2^(e-7) */
    return sign ? -v : v;
}

void oracle_decode_bf16(const uint16_t *src, double *dst, int64_t n)
{
    for (int64_t t = 0; t < n; ++t)
        dst[t] = oracle_bf16_value(src[t]);
}

void oracle_decode_e4m3(const uint8_t *src, double *dst, int64_t n)
{
    for (int64_t t = 0; t < n; ++t)
        dst[t] = oracle_e4m3_value(src[t]);
}

/* ------------------------------------------------------------------------- */
/* Plain GEMM (Section 2.1): C_out = alpha * op(A) op(B) + beta * C_in.     */
/* beta == 0 means C_in is not read (BLAS convention), so NaNs in it do not */
/* reach the result.                                                        */
/* ------------------------------------------------------------------------- */

static inline double opA(const double *A, int64_t lda, int ta, int64_t i, int64_t p)
{
    return ta ? A[p + i * lda] : A[i + p * lda];
}

static inline double opB(const double *B, int64_t ldb, int tb, int64_t p, int64_t j)
{
    return tb ? B[j + p * ldb] : B[p + j * ldb];
}

void oracle_gemm(int ta, int tb, int64_t m, int64_t n, int64_t k,
                 double alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb, double beta,
                 const double *Cin, int64_t ldc, double *Cout, int64_t ldo)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        double *col = Cout + j * ldo;
        for (int64_t i = 0; i < m; ++i)
            col[i] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            double b = opB(B, ldb, tb, p, j);
            for (int64_t i = 0; i < m; ++i)
                col[i] += opA(A, lda, ta, i, p) * b;
        }
        for (int64_t i = 0; i < m; ++i)
            col[i] = (beta == 0.0) ? alpha * col[i]
                                   : alpha * col[i] + beta * Cin[i + j * ldc];
    }
}

/* Selected entries only, one dot product each (used to check large runs on
 * sampled outputs). */
void oracle_gemm_entries(int ta, int tb, int64_t k, double alpha,
                         const double *A, int64_t lda, const double *B,
                         int64_t ldb, double beta, const double *Cin,
                         int64_t ldc, const int64_t *rows, const int64_t *cols,
                         int64_t count, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = rows[t], j = cols[t];
        double s = 0.0;
        for (int64_t p = 0; p < k; ++p)
            s += opA(A, lda, ta, i, p) * opB(B, ldb, tb, p, j);
        out[t] = (beta == 0.0) ? alpha * s : alpha * s + beta * Cin[i + j * ldc];
    }
}

/* ------------------------------------------------------------------------- */
/* Fault-tolerant GEMM, tile by tile (Sections 2.2 and 2.3).                 */
/* ------------------------------------------------------------------------- */

enum { INJ_ADD = 0, INJ_BITFLIP = 1 };
enum { TGT_ACC = 0, TGT_ROW_CHECKSUM = 1, TGT_COL_CHECKSUM = 2, TGT_WEIGHTED_CHECKSUM = 3 };
enum { KIND_CORRECTED = 1, KIND_CHECKSUM_ONLY = 2, KIND_RECOMPUTED = 3,
       KIND_UNCORRECTABLE = 4 };
/* Largest number of elements rebuilt along one line of a tile. */
#define MAX_LINE_FIXES 4

/* One planned soft error.  It lands after the inner-dimension step (of
 * length bk) that contains k_index has been accumulated.  TGT_ACC hits the
 * accumulator of C(row, col); TGT_ROW_CHECKSUM hits the encoded row checksum
 * entry of column col; TGT_COL_CHECKSUM the encoded column checksum entry of
 * row row. */
typedef struct {
    int64_t row, col, k_index;
    int32_t mode, target;
    double delta;
    int32_t bit, pad;
} oracle_injection;

typedef struct {
    int64_t tile_m, tile_n;
    int64_t row, col;          /* located element, -1 where not applicable */
    int32_t kind, nbad_rows, nbad_cols, pad;
    double d_row, d_col;       /* residuals of the row / column checksum   */
    double tau_row, tau_col;   /* thresholds they were held to             */
    double before, after;      /* element value before / after correction  */
} oracle_record;

typedef struct {
    int64_t row, col, k_index;
    int32_t applied, pad;
    double before, after;      /* the perturbed quantity, before and after */
} oracle_echo;

typedef struct {
    int32_t ta, tb;
    int64_t m, n, k, lda, ldb, ldc;
    double alpha, beta;        /* alpha already carries any input scales   */
    int64_t tm, tn, bk;        /* verification tile and inner step          */
    int32_t acc_bits;          /* 64: FP64 accumulators; 32: FP32           */
    int32_t correct;           /* 0: detect and classify only               */
    double lambda;             /* threshold multiplier                      */
    double mma_grid;           /* 0, or the truncation grid of a matrix     */
    int32_t mma_group;         /* instruction's group sums (see threshold)  */
    int32_t one_sided;         /* 1: only the column checksum (one entry    */
                               /* per row), recompute on any disagreement   */
    int32_t weighted;          /* 1: also a weighted row checksum per column */
                               /* (weights i + 1), see ft_tile              */
    int64_t slice_k;           /* 0, or the inner length of each slice of a */
                               /* split inner dimension (see ft_tile_split) */
} oracle_params;

/* Flip one bit of an accumulator held at the given precision. */
static double flip_bit(double v, int bit, int acc_bits)
{
    if (acc_bits == 32) {
        float f = (float)v;
        uint32_t u;
        memcpy(&u, &f, 4);
        u ^= (uint32_t)1u << bit;
        memcpy(&f, &u, 4);
        return (double)f;
    }
    uint64_t u;
    memcpy(&u, &v, 8);
    u ^= (uint64_t)1u << bit;
    memcpy(&v, &u, 8);
    return v;
}

/* Unit roundoff of the accumulation: FP32 or FP64. */
static double unit_roundoff(const oracle_params *P)
{
    return (P->acc_bits == 32) ? ldexp(1.0, -24) : ldexp(1.0, -53);
}

/* Rounding-error threshold of one checksum entry.
 *
 * The paper gives no threshold; the reading taken is a probabilistic
 * rounding-error bound (Higham and Mary's sqrt(n) model, lambda standard
 * deviations) built only from input norms, so a corrupted accumulator can
 * never inflate its own threshold.  For the row checksum of column j of a
 * tile with rows I (|I| = h), with u the unit roundoff of the arithmetic:
 *
 *   tau_j = lambda * ( |alpha| * ||b_j|| * [ (u sqrt(k) + u) ||A_I||_F
 *                                           + u (sqrt(k) ||x|| + sqrt(h) ||A_I||_F) ]
 *                      + 2 u |beta| ||Cin(I, j)|| )
 *
 * where b_j is column j of op(B) over all k, x = e^T op(A)(I, :) is the
 * tile's operand checksum, and the four terms bound the accumulation of the
 * products, the rounding of the output, the encoding product x^T b_j, and
 * the rounding inside x.  The column checksum entry of row i swaps the roles
 * of A and B.
 *
 * Multiplier units that do not add their products exactly (mma_grid > 0):
 * products are summed in groups of g = mma_group consecutive inner indices,
 * each product cut to a multiple of mma_grid * 2^E, 2^E the binade of the
 * group's largest product.  A product's error is then below mma_grid times
 * that largest product, so the squared errors of a group are at most g times
 * the sum of its squared products, and over the h entries of the checksum
 * (the same random-walk reading)
 *
 *   sqrt(sum_i sum_p e_ip^2) <= mma_grid sqrt(g) sqrt(sum_i sum_p a_ip^2 b_pj^2)
 *                            <= mma_grid sqrt(g) sqrt(h) max|A_I| ||b_j||,
 *
 * which adds lambda |alpha| mma_grid sqrt(g) sqrt(h) max|A_I| ||b_j|| to
 * tau_j (and the mirror image, with max|B_J| and ||a_i||, to tau_i). */
static double threshold(double lambda, double u, int64_t k, int64_t h,
                        double alpha, double nrm_vec, double frob_tile,
                        double nrm_chk, double beta, double nrm_cin)
{
    double sk = sqrt((double)k);
    double sh = sqrt((double)h);
    double prod = (u * sk + u) * frob_tile + u * (sk * nrm_chk + sh * frob_tile);
    return lambda * (fabs(alpha) * nrm_vec * prod + 2.0 * u * fabs(beta) * nrm_cin);
}

/* Accumulate one tile, applying the injections aimed at its accumulators
 * after the step that contains their k_index.  acc is h x w, column-major. */
static void tile_accumulate(const oracle_params *P, const double *A,
                            const double *B, int64_t i0, int64_t j0, int64_t h,
                            int64_t w, double *acc,
                            const oracle_injection *inj, int64_t ninj,
                            oracle_echo *echo)
{
    for (int64_t t = 0; t < h * w; ++t)
        acc[t] = 0.0;
    int64_t nsteps = (P->k + P->bk - 1) / P->bk;
    for (int64_t s = 0; s < nsteps; ++s) {
        int64_t p0 = s * P->bk, p1 = p0 + P->bk < P->k ? p0 + P->bk : P->k;
        for (int64_t jj = 0; jj < w; ++jj)
            for (int64_t p = p0; p < p1; ++p) {
                double b = opB(B, P->ldb, P->tb, p, j0 + jj);
                for (int64_t ii = 0; ii < h; ++ii)
                    acc[ii + jj * h] += opA(A, P->lda, P->ta, i0 + ii, p) * b;
            }
        for (int64_t q = 0; inj && q < ninj; ++q) {
            const oracle_injection *f = &inj[q];
            if (f->target != TGT_ACC || f->k_index / P->bk != s)
                continue;
            if (f->row < i0 || f->row >= i0 + h || f->col < j0 || f->col >= j0 + w)
                continue;
            double *a = &acc[(f->row - i0) + (f->col - j0) * h];
            double before = *a;
            *a = (f->mode == INJ_ADD) ? *a + f->delta : flip_bit(*a, f->bit, P->acc_bits);
            if (echo) {
                echo[q].applied = 1;
                echo[q].before = before;
                echo[q].after = *a;
            }
        }
    }
}

/* Encoded checksums (Pr, Pc) and thresholds (tr, tc) of one tile of h rows
 * starting at i0 and w columns starting at j0. */
static void tile_encode(const oracle_params *P, const double *A, const double *B,
                        const double *Cin, int64_t i0, int64_t j0, int64_t h,
                        int64_t w, double *Pr, double *Pc, double *tr, double *tc)
{
    const int64_t k = P->k;
    const double u = unit_roundoff(P);
    const double alpha = P->alpha, beta = P->beta;
    double *x = malloc(sizeof(double) * (k > 0 ? k : 1));
    double *y = malloc(sizeof(double) * (k > 0 ? k : 1));
    double *nb = malloc(sizeof(double) * w), *na = malloc(sizeof(double) * h);
    double *gc = malloc(sizeof(double) * w), *gr = malloc(sizeof(double) * h);

    /* Operand checksums of the tile: x = e^T op(A)(I,:), y = op(B)(:,J) e. */
    for (int64_t p = 0; p < k; ++p) {
        double sx = 0.0, sy = 0.0;
        for (int64_t ii = 0; ii < h; ++ii)
            sx += opA(A, P->lda, P->ta, i0 + ii, p);
        for (int64_t jj = 0; jj < w; ++jj)
            sy += opB(B, P->ldb, P->tb, p, j0 + jj);
        x[p] = sx;
        y[p] = sy;
    }
    /* Encoded checksums of C (Section 2.2): the product part from the
     * operand checksums, the beta part from the input C. */
    for (int64_t jj = 0; jj < w; ++jj) {
        double s = 0.0, c = 0.0;
        for (int64_t p = 0; p < k; ++p)
            s += x[p] * opB(B, P->ldb, P->tb, p, j0 + jj);
        if (beta != 0.0)
            for (int64_t ii = 0; ii < h; ++ii)
                c += Cin[(i0 + ii) + (j0 + jj) * P->ldc];
        Pr[jj] = alpha * s + beta * c;
    }
    for (int64_t ii = 0; ii < h; ++ii) {
        double s = 0.0, c = 0.0;
        for (int64_t p = 0; p < k; ++p)
            s += opA(A, P->lda, P->ta, i0 + ii, p) * y[p];
        if (beta != 0.0)
            for (int64_t jj = 0; jj < w; ++jj)
                c += Cin[(i0 + ii) + (j0 + jj) * P->ldc];
        Pc[ii] = alpha * s + beta * c;
    }
    /* Norms for the thresholds. */
    double fa = 0.0, fb = 0.0, nx = 0.0, ny = 0.0;
    for (int64_t ii = 0; ii < h; ++ii) {
        double s = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            double a = opA(A, P->lda, P->ta, i0 + ii, p);
            s += a * a;
        }
        na[ii] = sqrt(s);
        fa += s;
    }
    for (int64_t jj = 0; jj < w; ++jj) {
        double s = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            double b = opB(B, P->ldb, P->tb, p, j0 + jj);
            s += b * b;
        }
        nb[jj] = sqrt(s);
        fb += s;
    }
    for (int64_t p = 0; p < k; ++p) {
        nx += x[p] * x[p];
        ny += y[p] * y[p];
    }
    fa = sqrt(fa); fb = sqrt(fb); nx = sqrt(nx); ny = sqrt(ny);
    double ma = 0.0, mb = 0.0;  /* largest magnitudes of the tile's operands */
    if (P->mma_grid > 0.0) {
        for (int64_t p = 0; p < k; ++p) {
            for (int64_t ii = 0; ii < h; ++ii)
                ma = fmax(ma, fabs(opA(A, P->lda, P->ta, i0 + ii, p)));
            for (int64_t jj = 0; jj < w; ++jj)
                mb = fmax(mb, fabs(opB(B, P->ldb, P->tb, p, j0 + jj)));
        }
    }
    const double trunc = P->mma_grid * sqrt((double)(P->mma_group > 0 ? P->mma_group : 1));
    for (int64_t jj = 0; jj < w; ++jj) {
        double s = 0.0;
        if (beta != 0.0)
            for (int64_t ii = 0; ii < h; ++ii) {
                double c = Cin[(i0 + ii) + (j0 + jj) * P->ldc];
                s += c * c;
            }
        gc[jj] = sqrt(s);
    }
    for (int64_t ii = 0; ii < h; ++ii) {
        double s = 0.0;
        if (beta != 0.0)
            for (int64_t jj = 0; jj < w; ++jj) {
                double c = Cin[(i0 + ii) + (j0 + jj) * P->ldc];
                s += c * c;
            }
        gr[ii] = sqrt(s);
    }
    for (int64_t jj = 0; jj < w; ++jj)
        tr[jj] = threshold(P->lambda, u, k, h, alpha, nb[jj], fa, nx, beta, gc[jj]) +
                 P->lambda * fabs(alpha) * trunc * sqrt((double)h) * ma * nb[jj];
    for (int64_t ii = 0; ii < h; ++ii)
        tc[ii] = threshold(P->lambda, u, k, w, alpha, na[ii], fb, ny, beta, gr[ii]) +
                 P->lambda * fabs(alpha) * trunc * sqrt((double)w) * mb * na[ii];

    free(x); free(y); free(nb); free(na); free(gc); free(gr);
}

/* Weighted row checksums of one tile (the weighted mode): with local row
 * weights w_i = i + 1 (i = 0 .. h-1 within the tile),
 *   Pw_j = alpha sum_p x'_p B(p, j) + beta sum_i w_i Cin(i, j),  x'_p = sum_i w_i A(i, p),
 * and their thresholds: the row-checksum bound with A_I replaced by W A_I
 * (W = diag(w)), x by x' and Cin(I, j) by W Cin(I, j). */
static void tile_encode_weighted(const oracle_params *P, const double *A, const double *B,
                                 const double *Cin, int64_t i0, int64_t j0, int64_t h,
                                 int64_t w, double *Pw, double *tw)
{
    const int64_t k = P->k;
    const double u = unit_roundoff(P);
    const double alpha = P->alpha, beta = P->beta;
    double *xw = malloc(sizeof(double) * (k > 0 ? k : 1));
    for (int64_t p = 0; p < k; ++p) {
        double s = 0.0;
        for (int64_t ii = 0; ii < h; ++ii)
            s += (double)(ii + 1) * opA(A, P->lda, P->ta, i0 + ii, p);
        xw[p] = s;
    }
    double fwa = 0.0, nxw = 0.0, ma = 0.0;
    for (int64_t ii = 0; ii < h; ++ii)
        for (int64_t p = 0; p < k; ++p) {
            const double a = (double)(ii + 1) * opA(A, P->lda, P->ta, i0 + ii, p);
            fwa += a * a;
            ma = fmax(ma, fabs(a));
        }
    for (int64_t p = 0; p < k; ++p) nxw += xw[p] * xw[p];
    fwa = sqrt(fwa);
    nxw = sqrt(nxw);
    const double trunc = P->mma_grid * sqrt((double)(P->mma_group > 0 ? P->mma_group : 1));
    for (int64_t jj = 0; jj < w; ++jj) {
        double s = 0.0, c = 0.0, c2 = 0.0, nb = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            const double b = opB(B, P->ldb, P->tb, p, j0 + jj);
            s += xw[p] * b;
            nb += b * b;
        }
        if (beta != 0.0)
            for (int64_t ii = 0; ii < h; ++ii) {
                const double cw = (double)(ii + 1) * Cin[(i0 + ii) + (j0 + jj) * P->ldc];
                c += cw;
                c2 += cw * cw;
            }
        Pw[jj] = alpha * s + beta * c;
        tw[jj] = threshold(P->lambda, u, k, h, alpha, sqrt(nb), fwa, nxw, beta, sqrt(c2)) +
                 P->lambda * fabs(alpha) * trunc * sqrt((double)h) * ma * sqrt(nb);
    }
    free(xw);
}

/* Thresholds of one tile, exported for the fault planner's guard band. */
void oracle_tile_thresholds(const oracle_params *P, const double *A, const double *B,
                            const double *Cin, int64_t tile_m, int64_t tile_n,
                            double *tr, double *tc)
{
    const int64_t i0 = tile_m * P->tm, j0 = tile_n * P->tn;
    const int64_t h = (P->m - i0 < P->tm) ? P->m - i0 : P->tm;
    const int64_t w = (P->n - j0 < P->tn) ? P->n - j0 : P->tn;
    double *Pr = malloc(sizeof(double) * w), *Pc = malloc(sizeof(double) * h);
    tile_encode(P, A, B, Cin, i0, j0, h, w, Pr, Pc, tr, tc);
    free(Pr); free(Pc);
}

/* One tile of the fault-tolerant GEMM.  Writes the tile of Cout (and of
 * Craw, the output before correction, when given) and at most one record.
 * Returns 1 when a record was produced. */
static int ft_tile(const oracle_params *P, const double *A, const double *B,
                   const double *Cin, double *Cout, int64_t ldo, double *Craw,
                   int64_t tile_m, int64_t tile_n,
                   const oracle_injection *inj, int64_t ninj,
                   oracle_echo *echo, oracle_record *rec, double *max_ratio,
                   int local, double *pub, double *pub_tau)
{
    /* local: Cout and Craw hold only this tile (leading dimension ldo).
     * pub / pub_tau (may be NULL): the tile's final encoded checksums and
     * their thresholds, row checksums (one per column) first, then the
     * column checksums (one per row); an entry found to be a checksum fault
     * is replaced by the reference sum of the verified output. */
    const int64_t i0 = tile_m * P->tm, j0 = tile_n * P->tn;
    const int64_t oi = local ? 0 : i0, oj = local ? 0 : j0;
    const int64_t h = (P->m - i0 < P->tm) ? P->m - i0 : P->tm;
    const int64_t w = (P->n - j0 < P->tn) ? P->n - j0 : P->tn;
    const double alpha = P->alpha, beta = P->beta;

    double *acc = malloc(sizeof(double) * h * w);
    double *out = malloc(sizeof(double) * h * w);
    double *Pr = malloc(sizeof(double) * w), *Pc = malloc(sizeof(double) * h);
    double *Rr = malloc(sizeof(double) * w), *Rc = malloc(sizeof(double) * h);
    double *tr = malloc(sizeof(double) * w), *tc = malloc(sizeof(double) * h);
    const int wt = P->weighted && !P->one_sided;
    double *Pw = malloc(sizeof(double) * w), *tw = malloc(sizeof(double) * w);
    double *dw = malloc(sizeof(double) * w);

    int recomputed = 0, produced = 0;
    int attempt_faults = 1;
    for (;;) {
        /* Encoding (Section 2.2), then the planned faults on the encoded
         * checksums -- on the first attempt only. */
        tile_encode(P, A, B, Cin, i0, j0, h, w, Pr, Pc, tr, tc);
        if (wt) tile_encode_weighted(P, A, B, Cin, i0, j0, h, w, Pw, tw);

        /* Faults aimed at the encoded checksums. */
        for (int64_t q = 0; attempt_faults && inj && q < ninj; ++q) {
            const oracle_injection *f = &inj[q];
            if (f->target == TGT_ROW_CHECKSUM && !P->one_sided && f->col >= j0 &&
                f->col < j0 + w && f->row >= i0 && f->row < i0 + h) {
                double before = Pr[f->col - j0];
                Pr[f->col - j0] = (f->mode == INJ_ADD) ? before + f->delta
                                                       : flip_bit(before, f->bit, 64);
                if (echo) { echo[q].applied = 1; echo[q].before = before; echo[q].after = Pr[f->col - j0]; }
            } else if (f->target == TGT_COL_CHECKSUM && f->row >= i0 && f->row < i0 + h &&
                       f->col >= j0 && f->col < j0 + w) {
                double before = Pc[f->row - i0];
                Pc[f->row - i0] = (f->mode == INJ_ADD) ? before + f->delta
                                                       : flip_bit(before, f->bit, 64);
                if (echo) { echo[q].applied = 1; echo[q].before = before; echo[q].after = Pc[f->row - i0]; }
            } else if (f->target == TGT_WEIGHTED_CHECKSUM && wt && f->row >= i0 &&
                       f->row < i0 + h && f->col >= j0 && f->col < j0 + w) {
                double before = Pw[f->col - j0];
                Pw[f->col - j0] = before + f->delta;
                if (echo) { echo[q].applied = 1; echo[q].before = before; echo[q].after = Pw[f->col - j0]; }
            }
        }

        /* Multiplication (with the planned faults on the first attempt) and
         * the beta pass. */
        tile_accumulate(P, A, B, i0, j0, h, w, acc,
                        attempt_faults ? inj : NULL, ninj, attempt_faults ? echo : NULL);
        for (int64_t jj = 0; jj < w; ++jj)
            for (int64_t ii = 0; ii < h; ++ii) {
                double a = alpha * acc[ii + jj * h];
                out[ii + jj * h] = (beta == 0.0)
                    ? a : a + beta * Cin[(i0 + ii) + (j0 + jj) * P->ldc];
            }
        if (Craw && attempt_faults)
            for (int64_t jj = 0; jj < w; ++jj)
                for (int64_t ii = 0; ii < h; ++ii)
                    Craw[(oi + ii) + (oj + jj) * ldo] = out[ii + jj * h];

        /* Reference checksums: sums of the computed output. */
        for (int64_t jj = 0; jj < w; ++jj) {
            double s = 0.0;
            for (int64_t ii = 0; ii < h; ++ii)
                s += out[ii + jj * h];
            Rr[jj] = s;
        }
        for (int64_t ii = 0; ii < h; ++ii) {
            double s = 0.0;
            for (int64_t jj = 0; jj < w; ++jj)
                s += out[ii + jj * h];
            Rc[ii] = s;
        }
        /* Weighted reference sums and their residuals. */
        for (int64_t jj = 0; wt && jj < w; ++jj) {
            double s = 0.0;
            for (int64_t ii = 0; ii < h; ++ii)
                s += (double)(ii + 1) * out[ii + jj * h];
            dw[jj] = s - Pw[jj];
        }

        /* Verify.  The comparison is written so that NaN residuals flag. */
        int64_t nbad_c = 0, nbad_r = 0, jbad = -1, ibad = -1;
        for (int64_t jj = 0; !P->one_sided && jj < w; ++jj) {
            double d = Rr[jj] - Pr[jj];
            if (!(fabs(d) <= tr[jj])) {
                if (nbad_c++ == 0) jbad = jj;
            } else if (tr[jj] > 0.0 && fabs(d) / tr[jj] > *max_ratio) {
                *max_ratio = fabs(d) / tr[jj];
            }
        }
        for (int64_t ii = 0; ii < h; ++ii) {
            double d = Rc[ii] - Pc[ii];
            if (!(fabs(d) <= tc[ii])) {
                if (nbad_r++ == 0) ibad = ii;
            } else if (tc[ii] > 0.0 && fabs(d) / tc[ii] > *max_ratio) {
                *max_ratio = fabs(d) / tc[ii];
            }
        }
        if (nbad_c == 0 && nbad_r == 0) {
            if (recomputed && rec) {
                /* the record of the failed attempt is kept, kind updated */
                rec->kind = KIND_RECOMPUTED;
            }
            break;
        }
        if (recomputed) {
            /* still inconsistent without any injected fault */
            if (rec) rec->kind = KIND_UNCORRECTABLE;
            break;
        }
        produced = 1;
        if (rec) {
            rec->tile_m = tile_m; rec->tile_n = tile_n;
            rec->row = ibad >= 0 ? i0 + ibad : -1;
            rec->col = jbad >= 0 ? j0 + jbad : -1;
            rec->nbad_rows = (int32_t)nbad_r; rec->nbad_cols = (int32_t)nbad_c;
            rec->d_row = jbad >= 0 ? Rr[jbad] - Pr[jbad] : 0.0;
            rec->d_col = ibad >= 0 ? Rc[ibad] - Pc[ibad] : 0.0;
            rec->tau_row = jbad >= 0 ? tr[jbad] : 0.0;
            rec->tau_col = ibad >= 0 ? tc[ibad] : 0.0;
            rec->before = (ibad >= 0 && jbad >= 0) ? out[ibad + jbad * h] : 0.0;
            rec->after = rec->before;
        }
        if (!P->correct) {
            if (rec) rec->kind = P->one_sided ? KIND_RECOMPUTED
                               : (nbad_r == 1 && nbad_c == 1) ? KIND_CORRECTED
                               : (nbad_r + nbad_c == 1) ? KIND_CHECKSUM_ONLY
                                                        : KIND_RECOMPUTED;
            break;
        }
        if (P->one_sided) {
            /* With one side the faulty column is unknown, and a checksum
             * fault looks like a data fault: the tile is computed again. */
        } else if (nbad_r == 1 && nbad_c == 1) {
            /* Locate at the crossing of the flagged row and column; rebuild
             * the element from the encoded row checksum and the rest of its
             * column (this also repairs NaN / Inf values), then confirm it
             * against the encoded column checksum of its row. */
            double sr = 0.0, sc = 0.0;
            for (int64_t ii = 0; ii < h; ++ii)
                if (ii != ibad) sr += out[ii + jbad * h];
            for (int64_t jj = 0; jj < w; ++jj)
                if (jj != jbad) sc += out[ibad + jj * h];
            double fixed = Pr[jbad] - sr;
            /* Weighted mode: a finite error at (ibad, jbad) shows as
             * (ibad + 1) times its column residual on the weighted checksum. */
            const double dcol = Rr[jbad] - Pr[jbad];
            const int wok = !wt || !isfinite(dcol) || !isfinite(dw[jbad]) ||
                fabs(dw[jbad] - (double)(ibad + 1) * dcol) <=
                    tw[jbad] + (double)(ibad + 1) * tr[jbad];
            if (wok && fabs(sc + fixed - Pc[ibad]) <= tc[ibad]) {
                out[ibad + jbad * h] = fixed;
                if (rec) { rec->kind = KIND_CORRECTED; rec->after = fixed; }
                break;
            }
        } else if ((nbad_r == 1 && nbad_c >= 2 && nbad_c <= MAX_LINE_FIXES) ||
                   (nbad_c == 1 && nbad_r >= 2 && nbad_r <= MAX_LINE_FIXES)) {
            /* Several errors on one line: the flagged row (one flagged row,
             * up to MAX_LINE_FIXES flagged columns) or the flagged column.
             * Each element where the line crosses a flagged entry x of the
             * other side loses that entry's residual, out - (R_x - P_x) (the
             * classical ABFT correction), and the line is confirmed by its
             * own residual: after the corrections it is d_line - sum_x d_x.
             * A residual that is not finite cannot be subtracted: such a
             * line fails to confirm and the tile is computed again. */
            const int by_row = (nbad_r == 1);
            const int64_t line = by_row ? ibad : jbad;
            const int64_t len = by_row ? w : h;
            double sumd = 0.0;
            for (int64_t x = 0; x < len; ++x) {
                const double d = by_row ? Rr[x] - Pr[x] : Rc[x] - Pc[x];
                if (!(fabs(d) <= (by_row ? tr[x] : tc[x]))) sumd += d;
            }
            const double dl = by_row ? Rc[line] - Pc[line] : Rr[line] - Pr[line];
            /* Weighted mode: along a row, each crossing column x shows
             * (line + 1) d_x on its weighted checksum; along a column, the
             * column's weighted residual is the weighted sum of the rows'. */
            int wok = 1;
            if (wt && by_row) {
                for (int64_t x = 0; x < len; ++x) {
                    const double d = Rr[x] - Pr[x];
                    if (fabs(d) <= tr[x]) continue;
                    if (!(fabs(dw[x] - (double)(line + 1) * d) <=
                          tw[x] + (double)(line + 1) * tr[x])) wok = 0;
                }
            } else if (wt) {
                double sw = 0.0, tsum = tw[line];
                for (int64_t x = 0; x < len; ++x) {
                    const double d = Rc[x] - Pc[x];
                    if (fabs(d) <= tc[x]) continue;
                    sw += (double)(x + 1) * d;
                    tsum += (double)(x + 1) * tc[x];
                }
                if (!(fabs(dw[line] - sw) <= tsum)) wok = 0;
            }
            if (wok && fabs(dl - sumd) <= (by_row ? tc[line] : tr[line])) {
                for (int64_t x = 0; x < len; ++x) {
                    const double d = by_row ? Rr[x] - Pr[x] : Rc[x] - Pc[x];
                    if (fabs(d) <= (by_row ? tr[x] : tc[x])) continue;
                    const int64_t ii = by_row ? line : x, jj = by_row ? x : line;
                    out[ii + jj * h] -= d;
                }
                if (rec) {
                    /* the record names the first rebuilt element */
                    rec->kind = KIND_CORRECTED;
                    rec->after = out[ibad + jbad * h];
                }
                break;
            }
        } else if (nbad_r == nbad_c && nbad_r >= 2 && nbad_r <= MAX_LINE_FIXES) {
            /* As many flagged rows as flagged columns: errors in distinct
             * rows and columns.  An error shows as the same residual on its
             * row and on its column, so each flagged row is paired with the
             * flagged column whose residual agrees with its own within the
             * two thresholds.  When every row finds exactly one such column
             * and no column is found twice, each crossing loses its
             * column's residual (as a line correction does).  Otherwise --
             * errors of equal size, errors sharing lines, a checksum fault
             * among them, a residual that is not finite -- the tile is
             * computed again. */
            int64_t rows[MAX_LINE_FIXES], cols[MAX_LINE_FIXES], mate[MAX_LINE_FIXES];
            int64_t nr = 0, nc = 0;
            for (int64_t ii = 0; ii < h; ++ii)
                if (!(fabs(Rc[ii] - Pc[ii]) <= tc[ii])) rows[nr++] = ii;
            for (int64_t jj = 0; jj < w; ++jj)
                if (!(fabs(Rr[jj] - Pr[jj]) <= tr[jj])) cols[nc++] = jj;
            int paired = 1;
            unsigned taken = 0;
            if (wt) {
                /* Weighted mode: each flagged column locates its error's
                 * row from the ratio of its weighted to its plain residual
                 * (row + 1); the row must be flagged, taken once, and carry
                 * the same residual.  Equal errors need no pairing by size;
                 * two errors in one column give a ratio that does not fit. */
                for (int64_t a = 0; a < nr; ++a) mate[a] = -1;
                for (int64_t b = 0; b < nc && paired; ++b) {
                    const double dc = Rr[cols[b]] - Pr[cols[b]];
                    const double ratio = dw[cols[b]] / dc;
                    if (!isfinite(ratio) || !isfinite(dc)) { paired = 0; break; }
                    const int64_t r = (int64_t)llround(ratio) - 1;
                    int64_t a = -1;
                    for (int64_t q = 0; q < nr; ++q) if (rows[q] == r) a = q;
                    if (a < 0 || mate[a] >= 0) { paired = 0; break; }
                    if (!(fabs(dw[cols[b]] - (double)(r + 1) * dc) <=
                          tw[cols[b]] + (double)(r + 1) * tr[cols[b]]) ||
                        !(fabs((Rc[r] - Pc[r]) - dc) <= tc[r] + tr[cols[b]])) {
                        paired = 0;
                        break;
                    }
                    mate[a] = b;
                }
            } else
            for (int64_t a = 0; a < nr && paired; ++a) {
                const double dr = Rc[rows[a]] - Pc[rows[a]];
                int64_t found = 0;
                for (int64_t b = 0; b < nc; ++b) {
                    const double dc = Rr[cols[b]] - Pr[cols[b]];
                    if (fabs(dr - dc) <= tc[rows[a]] + tr[cols[b]]) { ++found; mate[a] = b; }
                }
                if (found != 1 || (taken >> mate[a]) & 1u) paired = 0;
                else taken |= 1u << mate[a];
            }
            if (paired) {
                const double before = out[rows[0] + cols[mate[0]] * h];
                for (int64_t a = 0; a < nr; ++a) {
                    const int64_t jj = cols[mate[a]];
                    out[rows[a] + jj * h] -= Rr[jj] - Pr[jj];
                }
                /* the record names the first flagged row's element */
                jbad = cols[mate[0]];
                if (rec) {
                    rec->kind = KIND_CORRECTED;
                    rec->col = j0 + jbad;
                    rec->d_row = Rr[jbad] - Pr[jbad];
                    rec->tau_row = tr[jbad];
                    rec->before = before;
                    rec->after = out[ibad + jbad * h];
                }
                break;
            }
        } else if (nbad_r + nbad_c == 1) {
            /* A single encoded checksum entry disagrees while every sum on
             * the other side matches.  A data error of size D shows as D on
             * both sides, each up to its own rounding, so it can hide on the
             * other side only if |D| <= 2 tau there, which puts the flagged
             * residual within its own tau plus twice the largest tau of the
             * other side.  Beyond that bound the fault hit the checksum path
             * and the data is left as it is; within it the tile is computed
             * again.  (Several entries on one side with none on the other
             * cannot come from one checksum fault: such a tile is computed
             * again below.) */
            const int by_col = (nbad_c == 1);
            const double d = by_col ? Rr[jbad] - Pr[jbad] : Rc[ibad] - Pc[ibad];
            double other = 0.0;
            for (int64_t x = 0; x < (by_col ? h : w); ++x)
                other = fmax(other, by_col ? tc[x] : tr[x]);
            const double bound = (by_col ? tr[jbad] : tc[ibad]) + 2.0 * other;
            if (!(fabs(d) <= bound)) {
                if (rec) rec->kind = KIND_CHECKSUM_ONLY;
                if (by_col) Pr[jbad] = Rr[jbad]; else Pc[ibad] = Rc[ibad];
                break;
            }
        }
        /* Several faults, or a correction that does not verify: compute the
         * tile again (the planned faults are not repeated). */
        recomputed = 1;
        attempt_faults = 0;
    }

    for (int64_t jj = 0; jj < w; ++jj)
        for (int64_t ii = 0; ii < h; ++ii)
            Cout[(oi + ii) + (oj + jj) * ldo] = out[ii + jj * h];
    if (pub)
        for (int64_t x = 0; x < w + h; ++x) {
            pub[x] = x < w ? Pr[x] : Pc[x - w];
            pub_tau[x] = x < w ? tr[x] : tc[x - w];
        }

    free(acc); free(out); free(Pr); free(Pc); free(Rr); free(Rc); free(tr); free(tc);
    free(Pw); free(tw); free(dw);
    return produced;
}

/* Encoded and reference checksums of one fault-free tile, exported so the
 * tests can hold the two against each other (the checksum identities). */
void oracle_tile_checksums(const oracle_params *P, const double *A, const double *B,
                           const double *Cin, int64_t tile_m, int64_t tile_n,
                           double *Pr, double *Pc, double *Rr, double *Rc)
{
    const int64_t i0 = tile_m * P->tm, j0 = tile_n * P->tn;
    const int64_t h = (P->m - i0 < P->tm) ? P->m - i0 : P->tm;
    const int64_t w = (P->n - j0 < P->tn) ? P->n - j0 : P->tn;
    double *tr = malloc(sizeof(double) * w), *tc = malloc(sizeof(double) * h);
    double *acc = malloc(sizeof(double) * h * w);
    tile_encode(P, A, B, Cin, i0, j0, h, w, Pr, Pc, tr, tc);
    tile_accumulate(P, A, B, i0, j0, h, w, acc, NULL, 0, NULL);
    for (int64_t jj = 0; jj < w; ++jj) {
        double s = 0.0;
        for (int64_t ii = 0; ii < h; ++ii) {
            double a = P->alpha * acc[ii + jj * h];
            s += (P->beta == 0.0) ? a : a + P->beta * Cin[(i0 + ii) + (j0 + jj) * P->ldc];
        }
        Rr[jj] = s;
    }
    for (int64_t ii = 0; ii < h; ++ii) {
        double s = 0.0;
        for (int64_t jj = 0; jj < w; ++jj) {
            double a = P->alpha * acc[ii + jj * h];
            s += (P->beta == 0.0) ? a : a + P->beta * Cin[(i0 + ii) + (j0 + jj) * P->ldc];
        }
        Rc[ii] = s;
    }
    free(tr); free(tc); free(acc);
}

/* One output tile of a split inner dimension (the parts of Section 2.3
 * taken along k).  The inner range is cut into slices of slice_k indices
 * (the last one shorter); each slice's partial product
 * W_s = op(A)(I, K_s) op(B)(K_s, J) is computed, verified and corrected as a
 * tile of its own (alpha 1, beta 0) with the faults whose k_index lies in it
 * (checksum faults past the end go to the last slice).  Checksums are
 * linear, so the encoded checksums of the result are alpha times the sum of
 * the slices' (each slice's checksum-fault entry replaced by its verified
 * reference sum) plus beta times the sums of C_in; the result
 * out = alpha sum_s W_s + beta C_in is verified against them, with the
 * slices' thresholds times |alpha| plus lambda u ((S + 3) sum|out| +
 * 2 |beta| ||C_in||) for the rounding of the reduction itself (S terms,
 * alpha, the beta term, the reference sum), and classified as a single tile
 * is; a reduction that does not verify is formed again from the slices.
 * Returns the number of records (slices first, in order, then the
 * reduction); at most rec_room are written. */
static int ft_tile_split(const oracle_params *P, const double *A, const double *B,
                         const double *Cin, double *Cout, int64_t ldo, double *Craw,
                         int64_t tile_m, int64_t tile_n,
                         const oracle_injection *inj, int64_t ninj, oracle_echo *echo,
                         oracle_record *recs, int rec_room, double *max_ratio)
{
    const int64_t i0 = tile_m * P->tm, j0 = tile_n * P->tn;
    const int64_t h = (P->m - i0 < P->tm) ? P->m - i0 : P->tm;
    const int64_t w = (P->n - j0 < P->tn) ? P->n - j0 : P->tn;
    const int64_t S = (P->k + P->slice_k - 1) / P->slice_k;
    const double alpha = P->alpha, beta = P->beta;
    const double u = ldexp(1.0, -53);
    double *W = calloc((size_t)(h * w), sizeof(double));      /* sum of the slices */
    double *Wraw = calloc((size_t)(h * w), sizeof(double));
    double *Ws = malloc(sizeof(double) * h * w), *Wr = malloc(sizeof(double) * h * w);
    double *pub = malloc(sizeof(double) * (w + h)), *ptau = malloc(sizeof(double) * (w + h));
    double *Psum = calloc((size_t)(w + h), sizeof(double));
    double *Tsum = calloc((size_t)(w + h), sizeof(double));
    oracle_injection *li = malloc(sizeof(oracle_injection) * (ninj > 0 ? ninj : 1));
    oracle_echo *le = malloc(sizeof(oracle_echo) * (ninj > 0 ? ninj : 1));
    int64_t *map = malloc(sizeof(int64_t) * (ninj > 0 ? ninj : 1));
    int nrec = 0;

    for (int64_t s = 0; s < S; ++s) {
        const int64_t kb = s * P->slice_k;
        const int64_t len = (P->k - kb < P->slice_k) ? P->k - kb : P->slice_k;
        oracle_params Ps = *P;
        Ps.k = len;
        Ps.alpha = 1.0;
        Ps.beta = 0.0;
        Ps.slice_k = 0;
        const double *As = P->ta ? A + kb : A + kb * P->lda;
        const double *Bs = P->tb ? B + kb * P->ldb : B + kb;
        int64_t nl = 0;
        for (int64_t q = 0; inj && q < ninj; ++q) {
            const oracle_injection *f = &inj[q];
            const int in = f->k_index >= kb &&
                           (f->k_index < kb + len || (f->target != TGT_ACC && s == S - 1));
            if (!in) continue;
            li[nl] = *f;
            li[nl].k_index = f->k_index - kb;
            le[nl].applied = 0;
            map[nl++] = q;
        }
        oracle_record r;
        memset(&r, 0, sizeof r);
        double mr = 0.0;
        const int got = ft_tile(&Ps, As, Bs, Cin, Ws, h, Wr, tile_m, tile_n, li, nl, le,
                                &r, &mr, 1, pub, ptau);
        if (mr > *max_ratio) *max_ratio = mr;
        for (int64_t q = 0; echo && q < nl; ++q)
            if (le[q].applied) {
                echo[map[q]].applied = 1;
                echo[map[q]].before = le[q].before;
                echo[map[q]].after = le[q].after;
            }
        if (got) {
            if (nrec < rec_room) recs[nrec] = r;
            ++nrec;
        }
        for (int64_t t = 0; t < h * w; ++t) { W[t] += Ws[t]; Wraw[t] += Wr[t]; }
        for (int64_t x = 0; x < w + h; ++x) { Psum[x] += pub[x]; Tsum[x] += ptau[x]; }
    }

    /* The verified reduction. */
    double *out = malloc(sizeof(double) * h * w);
    for (int64_t jj = 0; jj < w; ++jj)
        for (int64_t ii = 0; ii < h; ++ii) {
            const double c = Cin[(i0 + ii) + (j0 + jj) * P->ldc];
            double v = alpha * W[ii + jj * h], vr = alpha * Wraw[ii + jj * h];
            if (beta != 0.0) { v = v + beta * c; vr = vr + beta * c; }
            out[ii + jj * h] = v;
            if (Craw) Craw[(i0 + ii) + (j0 + jj) * ldo] = vr;
        }
    double *Pe = malloc(sizeof(double) * (w + h)), *Re = malloc(sizeof(double) * (w + h));
    double *Te = malloc(sizeof(double) * (w + h)), *De = malloc(sizeof(double) * (w + h));
    for (int64_t x = 0; x < w + h; ++x) {
        const int col = x < w;           /* row checksum of a column */
        const int64_t e = col ? x : x - w, len = col ? h : w;
        double R = 0.0, a = 0.0, cs = 0.0, c2 = 0.0;
        for (int64_t y = 0; y < len; ++y) {
            const int64_t ii = col ? y : e, jj = col ? e : y;
            const double v = out[ii + jj * h];
            R += v;
            a += fabs(v);
            if (beta != 0.0) {
                const double c = Cin[(i0 + ii) + (j0 + jj) * P->ldc];
                cs += c;
                c2 += c * c;
            }
        }
        double Pv = alpha * Psum[x];
        if (beta != 0.0) Pv += beta * cs;
        Pe[x] = Pv;
        Re[x] = R;
        Te[x] = fabs(alpha) * Tsum[x] +
                P->lambda * u * ((double)(S + 3) * a + 2.0 * fabs(beta) * sqrt(c2));
        De[x] = R - Pv;
    }
    int64_t nbad_c = 0, nbad_r = 0, jbad = -1, ibad = -1;
    for (int64_t x = 0; x < w + h; ++x)
        if (!(fabs(De[x]) <= Te[x])) {
            if (x < w) { if (nbad_c++ == 0) jbad = x; }
            else if (nbad_r++ == 0) ibad = x - w;
        }
    if (nbad_c || nbad_r) {
        oracle_record r;
        memset(&r, 0, sizeof r);
        r.tile_m = tile_m; r.tile_n = tile_n;
        r.row = ibad >= 0 ? i0 + ibad : -1;
        r.col = jbad >= 0 ? j0 + jbad : -1;
        r.nbad_rows = (int32_t)nbad_r; r.nbad_cols = (int32_t)nbad_c;
        r.d_row = jbad >= 0 ? De[jbad] : 0.0;
        r.tau_row = jbad >= 0 ? Te[jbad] : 0.0;
        r.d_col = ibad >= 0 ? De[w + ibad] : 0.0;
        r.tau_col = ibad >= 0 ? Te[w + ibad] : 0.0;
        /* Formed again from the same slices the sums come out the same:
         * whatever does not verify here stays uncorrectable. */
        r.kind = KIND_UNCORRECTABLE;
        if (nbad_r == 1 && nbad_c == 1) {
            double sr = 0.0, sc = 0.0;
            for (int64_t ii = 0; ii < h; ++ii)
                if (ii != ibad) sc += out[ii + jbad * h];
            for (int64_t jj = 0; jj < w; ++jj)
                if (jj != jbad) sr += out[ibad + jj * h];
            const double fixed = Pe[jbad] - sc;
            if (fabs(sr + fixed - Pe[w + ibad]) <= Te[w + ibad]) {
                r.kind = KIND_CORRECTED;
                r.before = out[ibad + jbad * h];
                r.after = fixed;
                out[ibad + jbad * h] = fixed;
            }
        } else if (nbad_r + nbad_c == 1) {
            const int by_col = (nbad_c == 1);
            const double d = by_col ? De[jbad] : De[w + ibad];
            double other = 0.0;
            for (int64_t x = 0; x < (by_col ? h : w); ++x)
                other = fmax(other, by_col ? Te[w + x] : Te[x]);
            if (!(fabs(d) <= (by_col ? Te[jbad] : Te[w + ibad]) + 2.0 * other))
                r.kind = KIND_CHECKSUM_ONLY;
        }
        if (nrec < rec_room) recs[nrec] = r;
        ++nrec;
    }
    for (int64_t jj = 0; jj < w; ++jj)
        for (int64_t ii = 0; ii < h; ++ii)
            Cout[(i0 + ii) + (j0 + jj) * ldo] = out[ii + jj * h];

    free(W); free(Wraw); free(Ws); free(Wr); free(pub); free(ptau); free(Psum); free(Tsum);
    free(li); free(le); free(map); free(out); free(Pe); free(Re); free(Te); free(De);
    return nrec;
}

/* Weighted encoded checksums, their thresholds and the weighted reference
 * sums of one fault-free tile (pins of the weighted mode). */
void oracle_tile_weighted(const oracle_params *P, const double *A, const double *B,
                          const double *Cin, int64_t tile_m, int64_t tile_n,
                          double *Pw, double *tw, double *Rw)
{
    const int64_t i0 = tile_m * P->tm, j0 = tile_n * P->tn;
    const int64_t h = (P->m - i0 < P->tm) ? P->m - i0 : P->tm;
    const int64_t w = (P->n - j0 < P->tn) ? P->n - j0 : P->tn;
    double *acc = malloc(sizeof(double) * h * w);
    tile_encode_weighted(P, A, B, Cin, i0, j0, h, w, Pw, tw);
    tile_accumulate(P, A, B, i0, j0, h, w, acc, NULL, 0, NULL);
    for (int64_t jj = 0; jj < w; ++jj) {
        double s = 0.0;
        for (int64_t ii = 0; ii < h; ++ii) {
            double a = P->alpha * acc[ii + jj * h];
            if (P->beta != 0.0) a = a + P->beta * Cin[(i0 + ii) + (j0 + jj) * P->ldc];
            s += (double)(ii + 1) * a;
        }
        Rw[jj] = s;
    }
    free(acc);
}

/* Fault-tolerant GEMM over the tile grid.  tiles: list of tile indices
 * (tile_m + tile_n * tiles_m) to process, or NULL for all tiles.  Records of
 * detected faults go to rec (at most rec_cap are stored; the return value is
 * the number produced).  echo (ninj entries, may be NULL) reports the value of
 * each injected quantity before and after the fault.  Craw (may be NULL)
 * receives the output before correction. */
int64_t oracle_ftgemm(const oracle_params *P, const double *A, const double *B,
                      const double *Cin, double *Cout, int64_t ldo, double *Craw,
                      const oracle_injection *inj, int64_t ninj,
                      const int64_t *tiles, int64_t ntiles,
                      oracle_record *rec, int64_t rec_cap, oracle_echo *echo,
                      double *max_ratio)
{
    if (P->m <= 0 || P->n <= 0)
        return 0;
    const int64_t tiles_m = (P->m + P->tm - 1) / P->tm;
    const int64_t tiles_n = (P->n + P->tn - 1) / P->tn;
    const int64_t total = tiles ? ntiles : tiles_m * tiles_n;
    int64_t nrec = 0;
    double mr = 0.0;
    if (echo)
        for (int64_t q = 0; q < ninj; ++q) {
            echo[q].row = inj[q].row; echo[q].col = inj[q].col;
            echo[q].k_index = inj[q].k_index; echo[q].applied = 0;
            echo[q].before = echo[q].after = 0.0;
        }
    const int split = P->slice_k > 0 && P->slice_k < P->k;
    const int room = split ? (int)((P->k + P->slice_k - 1) / P->slice_k) + 1 : 1;
#pragma omp parallel for schedule(dynamic, 1) reduction(max : mr)
    for (int64_t t = 0; t < total; ++t) {
        int64_t id = tiles ? tiles[t] : t;
        oracle_record *r = calloc((size_t)room, sizeof(oracle_record));
        double local = 0.0;
        int got = split
            ? ft_tile_split(P, A, B, Cin, Cout, ldo, Craw, id % tiles_m, id / tiles_m,
                            inj, ninj, echo, r, room, &local)
            : ft_tile(P, A, B, Cin, Cout, ldo, Craw, id % tiles_m, id / tiles_m,
                      inj, ninj, echo, r, &local, 0, NULL, NULL);
        if (local > mr) mr = local;
        for (int g = 0; g < got && g < room; ++g) {
            int64_t slot;
#pragma omp atomic capture
            slot = nrec++;
            if (rec && slot < rec_cap)
                rec[slot] = r[g];
        }
        free(r);
    }
    if (max_ratio)
        *max_ratio = mr;
    return nrec;
}

/* Threads the OpenMP loops use from now on (the CPU baseline is timed at
 * one thread and at all of them); returns the previous setting. */
#ifdef _OPENMP
#include <omp.h>
#endif
int32_t oracle_set_threads(int32_t n)
{
#ifdef _OPENMP
    const int32_t prev = (int32_t)omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return prev;
#else
    (void)n;
    return 1;
#endif
}

/* Sizes of the structures, so the Python side can check its mirror. */
int64_t oracle_sizeof(int which)
{
    switch (which) {
    case 0: return (int64_t)sizeof(oracle_injection);
    case 1: return (int64_t)sizeof(oracle_record);
    case 2: return (int64_t)sizeof(oracle_echo);
    case 3: return (int64_t)sizeof(oracle_params);
    default: return -1;
    }
}
