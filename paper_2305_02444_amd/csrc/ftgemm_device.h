// ftgemm_device.h -- device-side building blocks shared by the libftgemm
// kernels (gfx950, wave64): launch arguments, the device report layout,
// lane reductions, the tile schedule, the rounding-error threshold and the
// fault hook.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ftgemm.h"

namespace ftg {

constexpr int kWave = 64;
constexpr int kMaxTileFaults = 4;  // planned faults honoured per tile

// Device-side report counters of one call (or one problem of a batch).
struct DevCounters {
    unsigned long long tiles_verified;
    unsigned long long detected;
    unsigned long long corrected, checksum_only, recomputed, uncorrectable;
    unsigned long long max_ratio_bits;  // non-negative double, compared as bits
    unsigned int record_count;
    unsigned int pad;
};

// Everything one GEMM needs on the device.  Passed by value to the
// single-problem kernels, and as an array for the batched kernel.
struct GemmArgs {
    const void *A;
    const void *B;
    void *C;
    int64_t m, n, k, lda, ldb, ldc;
    double alpha, beta;                 // alpha already carries FP8 scales
    int32_t problem;
    int32_t tiles_m, tiles_n;           // verification grid
    int32_t tile_rows;                  // rows of its tiles (low-precision batches: 128 or 256)
    int64_t k_base;                     // first inner index (split-k slices)
    // fault tolerance (ignored by the plain kernels)
    DevCounters *counters;
    ftgemm_fault_record *records;
    uint32_t record_cap;
    unsigned int *rec_slot;             // record slots, shared by all problems
    int32_t nplan;
    const ftgemm_injection *plan;
    ftgemm_injection_echo *echo;        // one slot per plan entry
    // split inner dimension (FP64): nslices > 1 runs slice s of every tile
    // in workgroup s * tiles + tile; the slice covers inner indices
    // [s * slice_k, min(k, (s + 1) * slice_k)), writes its verified partial
    // product to wsp + s * m * n (leading dimension m) and its encoded
    // checksums and thresholds to chk (layout: see slice_chk_index).
    int32_t nslices;
    int32_t slice_last;                 // set per workgroup: last slice
    int64_t slice_k;
    double *wsp;
    double *chk;
    // one-sided low-precision mode: squared norms and largest magnitudes of
    // the rows of op(A) (m each) and the columns of op(B) (n each), over
    // the whole inner dimension, computed before the product
    const double *row_nrm2, *row_max, *col_nrm2, *col_max;
    // with the norms above (low precision): the operand checksums of every
    // tile, taken in the same pass -- xsum[tile_m * ldxs + p] = sum over the
    // tile's rows i of op(A)(i, p), ysum[tile_n * ldxs + p] = sum over the
    // tile's columns j of op(B)(p, j), FP32 (null: formed in the tiles)
    const float *xsum, *ysum;
    int64_t ldxs;
};

// Slice checksum workspace: for slice s and tile t (tile_m + tile_n *
// tiles_m), 2 * (tm + tn) doubles: encoded checksums of the tile's rows
// (tm) and columns (tn), then their thresholds.
__device__ __host__ __forceinline__ int64_t slice_chk_index(int64_t s, int64_t tile,
                                                            int64_t ntiles, int tm, int tn)
{
    return (s * ntiles + tile) * 2 * (tm + tn);
}

// ---------------------------------------------------------------------------
// Lane reductions.  DPP moves only exchange 32-bit values, so doubles go
// through their two halves.  Every lane of the reduced group ends with the
// same bits (each step adds a value to its mirror image, and FP addition is
// commutative), which keeps results bitwise reproducible.
// ---------------------------------------------------------------------------
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = (int)__double2loint(v), hi = (int)__double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, kCtrl, 0xf, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, kCtrl, 0xf, 0xf, false));
}

template <int kCtrl>
__device__ __forceinline__ float dpp_f32(float v)
{
    const int x = __float_as_int(v);
    return __int_as_float(__builtin_amdgcn_update_dpp(x, x, kCtrl, 0xf, 0xf, false));
}

// DPP controls (GFX9 encoding).
constexpr int kQuadXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;

// Sum over each row of 16 lanes; all 16 lanes receive the sum.
__device__ __forceinline__ double sum16(double v)
{
    v += dpp_f64<kQuadXor1>(v);
    v += dpp_f64<kQuadXor2>(v);
    v += dpp_f64<kRowHalfMirror>(v);
    v += dpp_f64<kRowMirror>(v);
    return v;
}

__device__ __forceinline__ float sum16f(float v)
{
    v += dpp_f32<kQuadXor1>(v);
    v += dpp_f32<kQuadXor2>(v);
    v += dpp_f32<kRowHalfMirror>(v);
    v += dpp_f32<kRowMirror>(v);
    return v;
}

// v_permlane16_swap / v_permlane32_swap (gfx950) exchange rows of 16 lanes
// (odd rows of the first operand with even rows of the second) or halves of
// 32 lanes; with both operands equal to v, the two results hold v and its
// partner in every lane, so their sum is the pair sum, bitwise the same in
// both lanes.
__device__ __forceinline__ double pair_sum16(double v)
{
    const int lo = (int)__double2loint(v), hi = (int)__double2hiint(v);
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}

__device__ __forceinline__ double pair_sum32(double v)
{
    const int lo = (int)__double2loint(v), hi = (int)__double2hiint(v);
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}

__device__ __forceinline__ float pair_sum16f(float v)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
}

__device__ __forceinline__ float pair_sum32f(float v)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
}

// Sum over the four rows of 16 (lanes l, l^16, l^32, l^48).
__device__ __forceinline__ double sum_rows(double v)
{
    return pair_sum32(pair_sum16(v));
}

__device__ __forceinline__ double sum64(double v)
{
    return sum_rows(sum16(v));
}

__device__ __forceinline__ double max64(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o));
    return v;
}

// ---------------------------------------------------------------------------
// Buffer loads.  A raw buffer resource carries a base address and an extent
// in bytes; a load whose per-lane offset falls outside the extent returns 0.
// Operand tiles are fetched through such resources so that rows or columns
// past the end of a matrix read as zeros without per-element branches, and
// lanes that must not load get kOob as their offset.
// ---------------------------------------------------------------------------
constexpr int kRsrcWord3 = 0x00020000;  // gfx9: raw (untyped) buffer
constexpr uint32_t kOob = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint64_t bytes)
{
    const uint32_t ext = bytes > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)ext, kRsrcWord3);
}

__device__ __forceinline__ double buf_load_f64(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// ---------------------------------------------------------------------------
// Tile schedule.  Workgroups are dispatched round-robin over the 8 XCDs of
// an MI355X, and each XCD has its own L2.  Consecutive logical tiles are
// therefore gathered onto one XCD, and the logical order walks groups of
// kGroupM tile rows column by column, so the tiles an XCD runs together
// share their A row panels and B column panels in its L2.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;
constexpr int kGroupM = 8;

__device__ __forceinline__ void map_tile(int wg, int tiles_m, int tiles_n, int &tile_m,
                                         int &tile_n)
{
    const int nt = tiles_m * tiles_n;
    const int q = nt / kXcds, r = nt % kXcds;
    const int x = wg % kXcds, idx = wg / kXcds;
    const int logical = x * q + (x < r ? x : r) + idx;
    const int per_group = kGroupM * tiles_n;
    const int group = logical / per_group;
    const int first_m = group * kGroupM;
    const int gsize = (tiles_m - first_m) < kGroupM ? (tiles_m - first_m) : kGroupM;
    const int in_group = logical % per_group;
    tile_m = first_m + in_group % gsize;
    tile_n = in_group / gsize;
}

// ---------------------------------------------------------------------------
// Rounding-error threshold of one checksum entry.  A probabilistic bound
// (errors of a length-n sum grow like sqrt(n) unit roundoffs; lambda is the
// number of standard deviations) built only from input norms, so a faulty
// accumulator cannot raise its own threshold:
//   tau = lambda * ( |alpha| * nv * [ (u sqrt(k) + u) F + u (sqrt(k) nc + sqrt(h) F) ]
//                    + 2 u |beta| ncin )
// nv: norm of the matching column of op(B) (row of op(A)) over all of k;
// F: Frobenius norm of the tile's rows of op(A) (columns of op(B)); nc:
// norm of the operand checksum vector; h: the tile extent being summed;
// ncin: norm of the matching part of C_in.  The four terms cover the
// products' accumulation, the rounding of the output, the encoding product
// and the rounding inside the operand checksum.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ft_threshold(double lambda, double u, double sqrt_k,
                                               double sqrt_h, double alpha, double nv,
                                               double F, double nc, double beta,
                                               double ncin)
{
    const double prod = (u * sqrt_k + u) * F + u * (sqrt_k * nc + sqrt_h * F);
    return lambda * (fabs(alpha) * nv * prod + 2.0 * u * fabs(beta) * ncin);
}

constexpr double kLambda = 8.0;

// Errors confined to one row (column) of a tile are rebuilt from the other
// side's checksums when the other side flags at most this many entries;
// the line's own checksum confirms them.
constexpr int kMaxLineFixes = 4;

// threadIdx.x as a value the compiler cannot tie to earlier reads: indices
// derived from it after a long loop are formed again from this rather than
// kept alive (and spilled to scratch) across the loop.
__device__ __forceinline__ int fresh_tid()
{
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Raise a non-negative double kept as bits (the order of the bit patterns is
// the order of the values).  Many workgroups report into one address; most
// values do not raise it, so the current value is read first and the atomic
// is issued only when needed.
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long *addr, double v)
{
    if (!(v > 0.0)) return;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    if (__atomic_load_n(addr, __ATOMIC_RELAXED) < bits) atomicMax(addr, bits);
}

__device__ __forceinline__ double flip_bit_f64(double v, int bit)
{
    return __longlong_as_double(__double_as_longlong(v) ^ (1ll << bit));
}

__device__ __forceinline__ float flip_bit_f32(float v, int bit)
{
    return __int_as_float(__float_as_int(v) ^ (1 << bit));
}

// A fault planned for the current tile, in tile-local coordinates.
struct TileFault {
    int32_t idx;       // index in the plan (echo slot)
    int32_t row, col;  // tile-local
    int32_t kstep;     // inner-dimension step after which it lands
    int32_t mode, target, bit, pad;
    double delta;
};

// Collect (in plan order) the planned faults that fall in the tile
// [i0, i0 + tm) x [j0, j0 + tn).  Run by one whole wave; lane 0 writes.
__device__ __forceinline__ int gather_tile_faults(const GemmArgs &g, int64_t i0, int64_t j0,
                                                  int tm, int tn, int bk, int64_t k_base,
                                                  TileFault *out)
{
    const int lane = threadIdx.x & 63;
    int n = 0;
    for (int base = 0; base < g.nplan && n < kMaxTileFaults; base += kWave) {
        const int idx = base + lane;
        bool hit = false;
        if (idx < g.nplan) {
            const ftgemm_injection f = g.plan[idx];
            // accumulator faults land in the slice holding their inner
            // index; with a split inner dimension, so do checksum faults
            // (the last slice takes indices past the end)
            const bool in_slice = f.k_index >= k_base &&
                                  (f.k_index < k_base + g.k ||
                                   (f.target != FTGEMM_TGT_ACC && g.slice_last));
            hit = f.problem == g.problem && f.row >= i0 && f.row < i0 + tm && f.col >= j0 &&
                  f.col < j0 + tn && f.row < g.m && f.col < g.n &&
                  ((f.target != FTGEMM_TGT_ACC && g.nslices <= 1) || in_slice);
        }
        unsigned long long mask = __ballot(hit);
        while (mask && n < kMaxTileFaults) {
            const int b = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            if (lane == 0) {
                const ftgemm_injection f = g.plan[base + b];
                TileFault t;
                t.idx = base + b;
                t.row = (int32_t)(f.row - i0);
                t.col = (int32_t)(f.col - j0);
                t.kstep = (int32_t)((f.k_index - k_base) / bk);
                t.mode = f.mode;
                t.target = f.target;
                t.bit = f.bit;
                t.pad = 0;
                t.delta = f.delta;
                out[n] = t;
            }
            ++n;
        }
    }
    return n;
}

}  // namespace ftg
