// ftgemm_kernels.h -- launchers of the libftgemm kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "ftgemm_device.h"

namespace ftg {

// FP64 tile kernel (one 128 x 128 output tile per workgroup).
// weighted: the weighted mode (also a weighted row checksum per column;
// never splits the inner dimension)
hipError_t launch_f64(const GemmArgs &g, bool ta, bool tb, bool abft, hipStream_t stream,
                      bool weighted = false);
void tiling_f64(int *tm, int *tn, int *bk);

// BF16 / FP8 E4M3 tile kernel (FP32 accumulation and output, one tm x 128
// output tile per workgroup, tm = 128 or 256 as tiling_lp chose).  mode: 0
// without checksums, 1 fault-tolerant, 2 one-sided.  pre: the threshold
// norms come from g's line norms (set by the caller; required by mode 2)
// instead of the tiles.
hipError_t launch_lp(const GemmArgs &g, bool fp8, bool ta, bool tb, int mode, bool pre, int tm,
                     hipStream_t stream);
// Tile of an m x n low-precision output in a mode (batched: the batched
// kernel's tile; in_tile: the operand checksums and norms are formed in the
// tiles, with no pass before the product).
constexpr int64_t kLargeTileMin = 256;  // 256-row tiles from this many tiles on
void tiling_lp(bool fp8, int mode, int64_t m, int64_t n, bool batched, bool in_tile, int *tm,
               int *tn, int *bk);

// Squared norms and largest magnitudes of the lines of a column-major R x Cn
// matrix of BF16 / E4M3 codes: of each row (along_rows; R results) or of
// each column (Cn results).  Row sums use part (at least 2 R doubles; more
// lets the columns be split into more chunks).  seg (may be null) receives,
// in the same pass, FP32 sums over segments of seg_len lines across the
// other index: along_rows, of each column over seg_len consecutive rows at
// seg[(row / seg_len) * seg_ld + column]; otherwise of each row over
// seg_len consecutive columns at seg[(column / seg_len) * seg_ld + row].
// seg_len: a power-of-two multiple of 16 bytes of elements, at most 64 of
// them; seg_ld at least Cn (along_rows) or R.
hipError_t launch_line_norms(const void *X, int64_t ld, int64_t R, int64_t Cn, bool fp8,
                             bool along_rows, double *nrm2, double *amax, double *part,
                             int64_t part_cap, float *seg, int seg_len, int64_t seg_ld,
                             hipStream_t stream);

// Unfused FP64 fault tolerance (detection only).  Segment sums of a
// column-major R x Cn matrix of doubles over L consecutive rows (down; one
// result per segment and column, at out[g + c * ldo]) or columns (across;
// at out[r + g * ldo]); transpose swaps the two output indices; square sums
// squares; out2 (may be null) receives the sums of squares in the same pass.
hipError_t launch_seg_sums(const double *Z, int64_t ld, int64_t R, int64_t Cn, int64_t L,
                           bool down, bool square, double *out, double *out2, int64_t ldo,
                           bool transpose, hipStream_t stream);
// Output faults: C(row, col) += alpha * delta for the plan's ADD faults on
// accumulators.
hipError_t launch_uf_inject(double *C, int64_t m, int64_t n, int64_t ldc, double alpha,
                            const ftgemm_injection *plan, int nplan, ftgemm_injection_echo *echo,
                            int problem, hipStream_t stream);
// Per 128 x 128 tile: entries of the tile's rows (Pc, Rc, cc, cc2: m x
// tiles_n, leading dimension m) and columns (Pr, Rr, cr, cr2: tiles_m x n,
// leading dimension tiles_m) verified against the thresholds built from the
// line norms and |x_I|^2 (xn2), |y_J|^2 (yn2).
struct UfArgs {
    const double *Pr, *Pc, *Rr, *Rc, *cr, *cc, *cr2, *cc2;
    const double *row_nrm2, *col_nrm2, *xn2, *yn2;
    int64_t m, n, k;
    int32_t tiles_m, tiles_n, problem, nplan;
    double alpha, beta;
    DevCounters *counters;
    ftgemm_fault_record *records;
    uint32_t record_cap;
    unsigned int *rec_slot;
    const ftgemm_injection *plan;
    ftgemm_injection_echo *echo;
};
hipError_t launch_uf_compare(const UfArgs &a, hipStream_t stream);

// Verified reduction of a split inner dimension (FP64): C = alpha * sum_s
// W_s + beta * C, checked against the slices' encoded checksums.
struct ReduceArgs {
    double *C;
    const double *wsp;   // nslices partial products, each m x n, leading dimension m
    const double *chk;   // the slices' encoded checksums and thresholds
    int64_t m, n, ldc;
    double alpha, beta;
    int32_t nslices, tiles_m, tiles_n, problem;
    DevCounters *counters;
    ftgemm_fault_record *records;
    uint32_t record_cap;
    unsigned int *rec_slot;
};
hipError_t launch_splitk_reduce(const ReduceArgs &r, bool abft, hipStream_t stream);

// C = beta * C over an m x n column-major matrix of double (f64) or float.
hipError_t launch_scale(void *C, bool f64, int64_t m, int64_t n, int64_t ldc, double beta,
                        hipStream_t stream);

// Clear a report area: counters, the first n echo slots and naux words of
// auxiliary counters (record slots, the batched work queue).
hipError_t launch_clear_report(DevCounters *ct, int ncounters, ftgemm_injection_echo *echo,
                               int nech, unsigned int *aux, int naux, hipStream_t stream);

// Batched persistent launch: the tiles of many problems, pulled from a work
// queue by a fixed grid of workgroups.
struct WorkItem {
    int32_t problem, tile_m, tile_n, pad;
};
constexpr int kMaxQueues = 8;
struct BatchArgs {
    const GemmArgs *probs;   // one per problem (device)
    const WorkItem *items;   // in the order they are handed out (device)
    unsigned int *queue;     // per queue: next item to hand out; zero at launch
    int32_t nqueues;         // 1, or one per XCD
    int32_t qbegin[kMaxQueues + 1];  // queue q hands out items [qbegin[q], qbegin[q + 1])
    int32_t rows;            // low precision: 128 or 256 when every problem's tiles
                             // have that many rows, 0 when mixed
};
hipError_t launch_f64_batched(const BatchArgs &b, bool ta, bool tb, bool abft, int grid,
                              hipStream_t stream);

// The no-allocation entry point: device scratch of kNoAllocBytes per GPU
// (a file-scope array of ftgemm_noalloc.hip) holding the counters,
// kNoAllocRecords record slots and kNoAllocPlan fault-plan and echo slots.
constexpr size_t kNoAllocBytes = 128 * 1024;
constexpr int kNoAllocRecords = 1024;
constexpr int kNoAllocPlan = 256;
ftgemm_status run_noalloc(const ftgemm_gemm_desc &d, ftgemm_report *rep, hipStream_t stream,
                          unsigned char *scratch, size_t bytes);
hipError_t launch_lp_batched(const BatchArgs &b, bool fp8, bool ta, bool tb, bool abft, int grid,
                             hipStream_t stream);

}  // namespace ftg
