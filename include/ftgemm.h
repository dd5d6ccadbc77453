/*
 * ftgemm.h -- C ABI of libftgemm, a fault-tolerant GEMM for AMD MI355X (gfx950).
 *
 * The library computes C = alpha * op(A) * op(B) + beta * C with
 * algorithm-based fault tolerance fused into the kernel, following
 * "FT-GEMM: A Fault Tolerant High Performance GEMM Implementation on x86
 * CPUs" (Wu, Zhai, Huang, Jian, Chen; HPDC'23):
 *   - the two checksum vectors of each output tile are encoded while C is
 *     scaled by beta (Section 2.2);
 *   - the operand checksums are formed from the operand values as they are
 *     staged for the multiplication, and feed the encoded checksums of C
 *     (Section 2.2; Section 2.3 for the split of the work into independent
 *     parts, here one output tile per GPU workgroup);
 *   - the reference checksums are the sums of the computed tile, taken from
 *     registers before it is written (Section 2.2);
 *   - a single soft error per tile (the fail-continue fault model of
 *     Section 1) is located at the crossing of the disagreeing row and
 *     column and rebuilt before C is written; a tile with several errors
 *     is computed again.
 *
 * Conventions shared by every entry point:
 *   - Matrices are column-major (BLAS).  op(X) = X for FTGEMM_OP_N and X^T
 *     for FTGEMM_OP_T.  op(A) is m x k, op(B) is k x n, C is m x n.
 *     lda >= max(1, transA == N ? m : k), ldb >= max(1, transB == N ? k : n),
 *     ldc >= max(1, m).  The kernels address what one tile reads in one
 *     inner-dimension step of an operand (and, for F64, the tile's part of
 *     C) with 32-bit offsets, so a leading dimension that makes it span
 *     2 GiB or more is refused as invalid (for F64 about 2.1 million
 *     elements for the operand whose tile spans 128 stored columns, and
 *     for ldc; see the library's argument check).
 *   - A, B and C are device pointers owned by the caller; C is read (unless
 *     beta == 0) and written.  Nothing is retained after the call returns.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL is the
 *     default stream), except that a call asked for a report waits for the
 *     stream before it returns, the report then being complete.
 *   - Arguments are checked on the host before any HIP call.  An invalid
 *     one returns FTGEMM_ERR_INVALID_ARG and ftgemm_last_invalid_arg()
 *     gives its 1-based BLAS position (1 transA, 2 transB, 3 m, 4 n, 5 k,
 *     6 alpha, 7 A, 8 lda, 9 B, 10 ldb, 11 beta, 12 C, 13 ldc, 14 the
 *     report / descriptor), as xerbla does.
 *   - Quick returns: m == 0 or n == 0, or (alpha == 0 or k == 0) with
 *     beta == 1, do nothing.  alpha == 0 or k == 0 otherwise only scales C
 *     by beta (beta == 0 stores zeros and never reads C).
 *   - Faults found on the device never fail a call (the fail-continue
 *     model): they show up in the report only.  The status covers host-side
 *     argument, launch and memory errors.
 *   - Calls that ask for a report share one device-side report area per
 *     GPU: such calls must not overlap on one GPU (issue them on one stream,
 *     or synchronise in between).
 */
#ifndef FTGEMM_H
#define FTGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { FTGEMM_OP_N = 0, FTGEMM_OP_T = 1 } ftgemm_op;

/* Input type.  F64: A, B, C are double.  BF16: A, B are bfloat16 (raw
 * 16-bit codes), C is float.  FP8_E4M3: A, B are OCP E4M3 (finite) codes
 * with per-tensor scales scaleA, scaleB (value = code * scale), C is float.
 * The low-precision types accumulate in FP32 on the matrix cores; the
 * checksum comparison and the correction are done in FP64. */
typedef enum { FTGEMM_F64 = 0, FTGEMM_BF16 = 1, FTGEMM_FP8_E4M3 = 2 } ftgemm_dtype;

typedef enum {
    FTGEMM_OK = 0,
    FTGEMM_ERR_INVALID_ARG = 1,
    FTGEMM_ERR_UNSUPPORTED = 2,
    FTGEMM_ERR_HIP = 3,
    FTGEMM_ERR_NO_MEMORY = 4
} ftgemm_status;

/* Outcome of a tile whose checksums disagreed. */
enum {
    FTGEMM_KIND_CORRECTED = 1,      /* one element located and rebuilt          */
    FTGEMM_KIND_CHECKSUM_ONLY = 2,  /* one encoded checksum entry was wrong;
                                       the data was left as computed           */
    FTGEMM_KIND_RECOMPUTED = 3,     /* several errors: the tile was computed
                                       again and then verified clean           */
    FTGEMM_KIND_UNCORRECTABLE = 4   /* still inconsistent after recomputation   */
};

/* Fault injection (test hook): mode and target. */
enum { FTGEMM_INJ_ADD = 0, FTGEMM_INJ_BITFLIP = 1 };
enum {
    FTGEMM_TGT_ACC = 0,
    FTGEMM_TGT_ROW_CHECKSUM = 1,
    FTGEMM_TGT_COL_CHECKSUM = 2,
    FTGEMM_TGT_WEIGHTED_CHECKSUM = 3  /* weighted mode (abft 4) only */
};

/* One detection.  row / col are global indices into C (-1 where the kind
 * has none: a checksum-only record names the row of a disagreeing column
 * checksum entry, or the column of a disagreeing row checksum entry).
 * d_* are the residuals (reference minus encoded) of the row checksum of
 * column `col` and of the column checksum of row `row`, tau_* the
 * thresholds they were held to; before / after are the element of C before
 * and after correction. */
typedef struct {
    int32_t problem;
    int32_t kind;
    int32_t tile_m, tile_n;
    int64_t row, col;
    int32_t nbad_rows, nbad_cols;
    double d_row, d_col;
    double tau_row, tau_col;
    double before, after;
} ftgemm_fault_record;

/* Echo of one injected fault as applied on the device: the perturbed
 * quantity (an accumulator before alpha is applied, or an encoded checksum
 * entry) before and after the fault. */
typedef struct {
    int32_t problem;
    int32_t applied;
    int64_t row, col, k_index;
    double before, after;
} ftgemm_injection_echo;

/* Per-call report.  The caller sets the capacities and the two arrays
 * (host memory it owns; NULL with capacity 0 is allowed); the library fills
 * the rest.  Records beyond a capacity are dropped but still counted. */
typedef struct {
    uint64_t tiles_verified;
    uint64_t detected;          /* tiles whose checksums disagreed          */
    uint64_t corrected, checksum_only, recomputed, uncorrectable;
    double max_ratio;           /* largest |residual| / threshold over the
                                   checksum entries that passed: the margin
                                   of the rounding-error threshold          */
    uint32_t record_count, echo_count;
    uint32_t record_capacity, echo_capacity;
    ftgemm_fault_record *records;
    ftgemm_injection_echo *echoes;
} ftgemm_report;

/* One planned soft error (test hook).  It lands after the inner-dimension
 * step containing k_index has been accumulated (ACC target), or on the
 * encoded checksum entry of column `col` (ROW_CHECKSUM) / row `row`
 * (COL_CHECKSUM) of the tile holding C(row, col), or on the weighted row
 * checksum entry of column `col` (WEIGHTED_CHECKSUM; applied in the
 * weighted mode only, elsewhere it has no entry to land on).  BITFLIP flips bit `bit`
 * of the accumulator in its own precision (FP64 for F64, FP32 otherwise);
 * checksum targets take ADD only.  `problem` selects the problem of a
 * batched call (0 otherwise). */
typedef struct {
    int32_t problem;
    int32_t mode;
    int32_t target;
    int32_t bit;
    int64_t row, col, k_index;
    double delta;
} ftgemm_injection;

/* A GEMM described in full, for ftgemm_gemm_ex and ftgemm_gemm_batched.
 * abft selects the fault tolerance:
 *   0  the same kernel with every checksum operation compiled out (the
 *      plain-GEMM baseline);
 *   1  row and column checksums of every tile (Section 2.2): a single
 *      error per tile, two to four on one row or one column of it, or two
 *      to four in distinct rows and columns (each flagged row paired with
 *      the flagged column of equal residual), is located and corrected
 *      (the record names the first flagged row and its element's column);
 *      patterns that cannot be told apart are computed again;
 *   2  one-sided (BF16 / FP8 single calls only; FTGEMM_ERR_UNSUPPORTED for
 *      F64 and in batches): only the column checksum C e of each tile is
 *      kept, one entry per row, and a tile with any disagreeing row is
 *      computed again (records: kind RECOMPUTED, col -1).  Faults planned
 *      on the row checksum have no entry to land on and are not applied.
 *   3  unfused (F64 single calls only; FTGEMM_ERR_UNSUPPORTED for BF16 /
 *      FP8 and in batches): the comparison the fusion is measured against
 *      (Section 2.2).  The same 128 x 128 tile checksums and thresholds as
 *      mode 1, formed by separate passes over A, B and C around the
 *      checksum-free GEMM (segment sums, two thin GEMMs for the encoded
 *      parts, a compare kernel); detection only: every inconsistent tile
 *      gets one record of kind UNCORRECTABLE and the output is left as
 *      computed.  Planned faults: additions on accumulators (applied to the
 *      finished output as alpha * delta) and on either checksum; bit flips
 *      are not applied.  Its workspace ((m + n) k / 128 + 8 m n / 128
 *      doubles, plus the thin GEMMs' split slices) is grown on demand and
 *      kept.
 *   4  weighted (F64 single calls only; FTGEMM_ERR_UNSUPPORTED for BF16 /
 *      FP8, in batches and without allocation): mode 1 plus a weighted
 *      row checksum per column of each tile, sum_i (i + 1) C(i, j) over
 *      the tile's local rows i, encoded the same way (from the weighted
 *      column sums of the staged A tile, and C_in in the beta pass) and
 *      held to the column's threshold with A, the operand checksum and
 *      C_in weighted alike.  A single error at local row r of column j
 *      shows as r + 1 times the column's residual on it: every correction
 *      of mode 1 is confirmed by it, and errors in distinct rows and
 *      columns are paired by it (each flagged column names its row) rather
 *      than by their sizes, so equal errors are corrected too.  The inner
 *      dimension is never split.
 * BF16 / FP8 single calls with abft 2, and with abft 1 when the output
 * holds at least 256 tiles, take the threshold norms of the rows of op(A)
 * and columns of op(B), and the FP32 operand checksums of every tile
 * ((tiles_m + tiles_n) k floats), in one pass over A and B before the
 * product, using the library's workspace (batches compute them in the
 * tiles).  Other values of abft are rejected (argument position 14). */
typedef struct {
    ftgemm_dtype dtype;
    ftgemm_op transA, transB;
    int32_t abft;
    int64_t m, n, k, lda, ldb, ldc;
    double alpha, beta;
    double scaleA, scaleB;          /* FP8 only; ignored otherwise */
    const void *A;
    const void *B;
    void *C;
} ftgemm_gemm_desc;

/* FP64 fault-tolerant GEMM (Sections 2.2 and 2.3):
 *   C = alpha * op(A) * op(B) + beta * C, A/B/C double, device pointers.
 * report: NULL, or filled after the stream synchronises. */
ftgemm_status ftgemm_gemm(ftgemm_op transA, ftgemm_op transB, int64_t m, int64_t n,
                          int64_t k, double alpha, const double *A, int64_t lda,
                          const double *B, int64_t ldb, double beta, double *C,
                          int64_t ldc, ftgemm_report *report, void *stream);

/* Any input type, with or without the fault tolerance (desc->abft). */
ftgemm_status ftgemm_gemm_ex(const ftgemm_gemm_desc *desc, ftgemm_report *report,
                             void *stream);

/* `count` independent GEMMs (Section 2.3's independent parts, taken to
 * whole problems), each with its own checksums, in one persistent launch
 * replayed from a captured HIP graph.
 *   problems: host array of `count` descriptors (device data pointers); all
 *     must share dtype, abft and the two transposes (otherwise
 *     FTGEMM_ERR_UNSUPPORTED).  An invalid descriptor returns
 *     FTGEMM_ERR_INVALID_ARG with the position of its bad field.
 *   reports: NULL or a host array of `count` reports, one per problem; the
 *     fault plan's `problem` field is the index in `problems`.
 * Tiles: 128 x 128 for FP64 problems (inner step 32).  A BF16 / FP8
 * problem takes 128 x 128 tiles, or 256 x 128 tiles when it has at least
 * m* rows; m* (none, 1024, 512 or 256) and the work order (cost-ordered
 * single queue, given order, or one queue per XCD) are tuned by timing the
 * candidates on the batch itself, the first time a batch of its shape is
 * seen with every beta 0 (C is then write-only, so the trial runs are
 * harmless), and remembered for that shape, in the tuning table too (see
 * ftgemm_load_tune_table); other batches of an unknown shape take the
 * defaults (no 256-row tiles, cost order).  ftgemm_batch_tiling tells the
 * rows each problem's tiles take.  The device arrays of per-problem
 * arguments and the captured graph belong to the library and are reused
 * while the batch's size and the plan stay the same. */
ftgemm_status ftgemm_gemm_batched(int32_t count, const ftgemm_gemm_desc *problems,
                                  ftgemm_report *reports, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * same call as ftgemm_gemm_ex, and the same kernels, with nothing
 * allocated.  The device memory it needs besides A, B and C -- the report
 * counters, 1024 record slots, and the fault plan with its echo slots -- is
 * a fixed 128 KiB array per GPU inside the library, which each GPU the
 * library runs on keeps until the process ends.  So that nothing grows with
 * the problem, the FP64 inner dimension is never split (slower on outputs
 * of few tiles) and BF16 / FP8 tiles form their threshold norms and operand
 * checksums themselves, with no pass over A and B before the product (C is
 * the same; a rebuilt element may differ from ftgemm_gemm_ex's in its last
 * FP32 bits).  Fault-tolerant FP8 tiles have 128 rows here (those sums do
 * not fit a 256-row FP8 tile), unless the tuning table says otherwise.  Refused with FTGEMM_ERR_UNSUPPORTED: abft 2 and 3 (their
 * workspace grows with the problem), abft 4 and an armed fault plan longer than
 * 256 entries.  Records beyond 1024 are dropped (still counted).  Every
 * call on a GPU shares that GPU's array and keeps the last call's contents
 * in it: calls that overlap on one GPU (on different streams, or from
 * different threads without synchronising) race and must not be issued.
 * A report, when asked for, is filled before the call returns (it waits for
 * the stream), through host staging inside the library. */
ftgemm_status ftgemm_gemm_ex_noalloc(const ftgemm_gemm_desc *desc, ftgemm_report *report,
                                     void *stream);

/* The same problems launched one by one (the baseline the persistent
 * launch is measured against). */
ftgemm_status ftgemm_gemm_batched_loop(int32_t count, const ftgemm_gemm_desc *problems,
                                       ftgemm_report *reports, void *stream);

/* Rows of the tiles each of `count` problems takes in ftgemm_gemm_batched
 * now (128 or 256; see there), into tile_rows[count].  Errors: count < 0
 * (position 1), problems NULL (2), tile_rows NULL (3). */
ftgemm_status ftgemm_batch_tiling(int32_t count, const ftgemm_gemm_desc *problems,
                                  int32_t *tile_rows);

/* Replace the tuning table with the one in the text file `path` (NULL: an
 * empty table).  Its lines, '#' starting a comment:
 *   tile <dtype> <abft> <rows>   single BF16 (1) / FP8 (2) calls in mode
 *                                abft (0..2) take tiles of rows = 128 or 256
 *                                instead of the default choice
 *   batch_mstar <m>              in low-precision batches, problems of at
 *                                least m rows take 256-row tiles (the
 *                                threshold is then not tuned; -1: tuned)
 *   batch <sig> <order> <m>      a batch tuned before (written by the
 *                                library: shape signature, work order,
 *                                threshold, -1 for none)
 * Batches tuned from then on are appended to the file.  Without a call, the
 * file the environment variable FTGEMM_TUNE_TABLE names (if any) is read at
 * first use.  Errors: the file cannot be read or has a malformed line
 * (position 1; the table is left unchanged). */
ftgemm_status ftgemm_load_tune_table(const char *path);

/* Arm the fault plan (test hook): it applies to every following call until
 * replaced; n == 0 clears it.  The plan is copied. */
ftgemm_status ftgemm_set_fault_plan(const ftgemm_injection *plan, int32_t n);

/* Verification tile (tm x tn), inner step bk and split of the inner
 * dimension chosen for a fault-tolerant call on a problem: FP64 128 x 128;
 * BF16 256 x 128 once the output holds at least 256 such tiles, else
 * 128 x 128; FP8 128 x 128 (a call without fault tolerance may use 256-row
 * tiles there too; nothing is verified then).  Batches use 128 x 128 for
 * every low-precision problem.  split_k > 1 (FP64 only) means the inner
 * dimension is cut into split_k slices run in one launch: each slice
 * verifies and corrects its partial product as its own tile (its faults are
 * those whose k_index falls in it; records carry the tile, once per slice
 * that found something), and a verified reduction then forms C.  The
 * report's tiles_verified counts split_k + 1 verifications per tile. */
ftgemm_status ftgemm_query_tiling(ftgemm_dtype dtype, int64_t m, int64_t n, int64_t k,
                                  int32_t *tm, int32_t *tn, int32_t *bk,
                                  int32_t *split_k);

/* The same for the call a descriptor describes (its dtype, abft, m, n, k;
 * the other fields are not read): in the one-sided mode FP8 also takes
 * 256 x 128 tiles from 256 tiles on.  Errors: desc NULL or its fields out of
 * range (position 1), an output pointer NULL (position 2); one-sided F64
 * and unfused or weighted BF16 / FP8 return FTGEMM_ERR_UNSUPPORTED.  The
 * unfused mode reports the tiling of its checksum-free product (its
 * verification tiles are 128 x 128, as the F64 kernel's); the weighted mode
 * reports split_k 1. */
ftgemm_status ftgemm_query_tiling_ex(const ftgemm_gemm_desc *desc, int32_t *tm, int32_t *tn,
                                     int32_t *bk, int32_t *split_k);

/* 1-based position of the argument rejected by the last call on this
 * thread that returned FTGEMM_ERR_INVALID_ARG (0 if none). */
int32_t ftgemm_last_invalid_arg(void);

const char *ftgemm_status_string(ftgemm_status status);

/* Frees the library's device workspace (report areas, fault plans, batched
 * descriptors, captured graphs) on every GPU it touched. */
void ftgemm_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* FTGEMM_H */
