// ftgemm_norms.hip -- the input norms of the one-sided low-precision mode:
// for every row of op(A) and every column of op(B), the sum of squares and
// the largest magnitude over the whole inner dimension (the quantities the
// rounding-error threshold of each checksum entry is built from; they do not
// depend on the output tile, so they are taken once, in one pass over A and
// B, instead of in every tile).  Inputs are BF16 or E4M3 codes, widened
// exactly; sums in FP32 per thread, then FP64.
//
// The same pass can also take the operand checksums of every output tile
// (FT-GEMM, Section 2.2: x = e^T A_I, y = B_J e), the sums of each inner
// index over the tile's rows of op(A) or columns of op(B).  They depend only
// on the operands and the tile grid, so the product's tiles then read them
// (one value per inner index and step) instead of summing their staged
// operand registers at every step.  Sums in FP32, as the tiles form them.
#include "ftgemm_device.h"
#include "ftgemm_kernels.h"

namespace ftg {
namespace norms {

constexpr int NT = 256;
typedef int i32x4 __attribute__((ext_vector_type(4)));

// EPV consecutive elements of one column from byte offset off of a column
// resource: one 16-byte load when all `live` of them are wanted, else
// element by element (nothing past the live ones is read).
template <bool FP8>
__device__ __forceinline__ i32x4 load_run(__amdgpu_buffer_rsrc_t rs, int off, int live)
{
    constexpr int EB = FP8 ? 1 : 2, EPV = 16 / EB, PG = 4 / EB;
    if (live >= EPV) return __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    i32x4 v = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < EPV; ++e) {
        if (e >= live) break;
        const unsigned x = FP8 ? (unsigned)__builtin_amdgcn_raw_buffer_load_b8(rs, off + e, 0, 0)
                               : (unsigned)__builtin_amdgcn_raw_buffer_load_b16(rs, off + 2 * e, 0, 0);
        v[e / PG] |= (int)(x << (8 * EB * (e % PG)));
    }
    return v;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t column(const char *X, int64_t ld, int64_t c,
                                                         int64_t R, int EB)
{
    const int64_t bytes = R * EB;
    return make_rsrc(X + c * ld * EB, (uint64_t)(bytes < 0x7FFFFFFF ? bytes : 0x7FFFFFFF));
}

template <bool FP8>
__device__ __forceinline__ float widen(unsigned dw, int e)
{
    if (FP8) {
        switch (e & 3) {
        case 0: return __builtin_amdgcn_cvt_f32_fp8((int)dw, 0);
        case 1: return __builtin_amdgcn_cvt_f32_fp8((int)dw, 1);
        case 2: return __builtin_amdgcn_cvt_f32_fp8((int)dw, 2);
        default: return __builtin_amdgcn_cvt_f32_fp8((int)dw, 3);
        }
    }
    return __uint_as_float((e & 1) ? (dw & 0xffff0000u) : (dw << 16));
}

// Along each stored row (R rows, Cn columns, leading dimension ld): block
// (bx, by) covers 64 row vectors of EPV rows (one 16-byte load each) and
// the column chunk [by * cc, (by + 1) * cc); its 4 waves take every 4th
// column.  Partials go to part[by][row] (sum of squares) and
// part[nchunks + by][row] (largest magnitude).
// seg (may be null): the sums of each column over segments of SL EPV
// consecutive rows (SL lanes; a power of two, at most 64), at
// seg[(row / (SL EPV)) * ldo + column].
template <bool FP8>
__global__ __launch_bounds__(NT) void rows_kernel(const char *X, int64_t ld, int64_t R,
                                                   int64_t Cn, int64_t cc, double *part,
                                                   int nchunks, float *seg, int SL, int64_t ldo)
{
    constexpr int EB = FP8 ? 1 : 2, EPV = 16 / EB, PG = 4 / EB;
    __shared__ float ssum[4][64 * EPV], smax[4][64 * EPV];
    const int t = threadIdx.x, rv = t & 63;
    const int cp = __builtin_amdgcn_readfirstlane(t >> 6);  // wave: every 4th column
    const int64_t r0 = ((int64_t)blockIdx.x * 64 + rv) * EPV;
    const int64_t c0 = (int64_t)blockIdx.y * cc;
    const int64_t c1 = c0 + cc < Cn ? c0 + cc : Cn;
    float s[EPV], mx[EPV];
#pragma unroll
    for (int e = 0; e < EPV; ++e) { s[e] = 0.0f; mx[e] = 0.0f; }
    const int live = (int)(R - r0 < EPV ? (R - r0 > 0 ? R - r0 : 0) : EPV);
    for (int64_t c = c0 + cp; c < c1; c += 4) {
        const __amdgpu_buffer_rsrc_t rs = column(X, ld, c, R, EB);
        const i32x4 v = live > 0 ? load_run<FP8>(rs, (int)(r0 * EB), live) : (i32x4){0, 0, 0, 0};
        float cs = 0.0f;  // this lane's part of the column's segment sum
#pragma unroll
        for (int e = 0; e < EPV; ++e) {
            const float x = e < live ? widen<FP8>((unsigned)v[e / PG], e % PG) : 0.0f;
            s[e] = fmaf(x, x, s[e]);
            mx[e] = fmaxf(mx[e], fabsf(x));
            cs += x;
        }
        if (seg) {  // uniform: the whole wave takes the branch
            for (int msk = 1; msk < SL; msk <<= 1) cs += __shfl_xor(cs, msk);
            if ((rv & (SL - 1)) == 0 && live > 0)
                seg[(r0 / ((int64_t)SL * EPV)) * ldo + c] = cs;
        }
    }
#pragma unroll
    for (int e = 0; e < EPV; ++e) {
        ssum[cp][rv * EPV + e] = s[e];
        smax[cp][rv * EPV + e] = mx[e];
    }
    __syncthreads();
    for (int i = t; i < 64 * EPV; i += NT) {
        const int64_t r = (int64_t)blockIdx.x * 64 * EPV + i;
        if (r >= R) continue;
        const double sum = ((double)ssum[0][i] + (double)ssum[1][i]) +
                           ((double)ssum[2][i] + (double)ssum[3][i]);
        const float m = fmaxf(fmaxf(smax[0][i], smax[1][i]), fmaxf(smax[2][i], smax[3][i]));
        part[(int64_t)blockIdx.y * R + r] = sum;
        part[((int64_t)nchunks + blockIdx.y) * R + r] = (double)m;
    }
}

// Partials of the column chunks: 64 rows per workgroup, its 4 waves taking
// every 4th chunk, then the waves' sums added in a fixed order.
__global__ __launch_bounds__(NT) void rows_finish(const double *part, int nchunks, int64_t R,
                                                  double *nrm2, double *amax)
{
    __shared__ double ssum[4][64], smax[4][64];
    const int t = threadIdx.x, rl = t & 63, cg = t >> 6;
    const int64_t r = (int64_t)blockIdx.x * 64 + rl;
    double s = 0.0, m = 0.0;
    if (r < R) {
#pragma unroll 4
        for (int c = cg; c < nchunks; c += 4) {
            s += part[(int64_t)c * R + r];
            m = fmax(m, part[((int64_t)nchunks + c) * R + r]);
        }
    }
    ssum[cg][rl] = s;
    smax[cg][rl] = m;
    __syncthreads();
    if (cg == 0 && r < R) {
        nrm2[r] = (ssum[0][rl] + ssum[1][rl]) + (ssum[2][rl] + ssum[3][rl]);
        amax[r] = fmax(fmax(smax[0][rl], smax[1][rl]), fmax(smax[2][rl], smax[3][rl]));
    }
}

// Along each stored column: one block per column, 16-byte loads down it.
template <bool FP8>
__global__ __launch_bounds__(NT) void cols_kernel(const char *X, int64_t ld, int64_t R,
                                                   int64_t Cn, double *nrm2, double *amax)
{
    constexpr int EB = FP8 ? 1 : 2, EPV = 16 / EB, PG = 4 / EB;
    __shared__ double ssum[NT / 64], smax[NT / 64];
    const int t = threadIdx.x;
    const int64_t c = blockIdx.x;
    const __amdgpu_buffer_rsrc_t rs = column(X, ld, c, R, EB);
    float s = 0.0f, mx = 0.0f;
    for (int64_t r0 = (int64_t)t * EPV; r0 < R; r0 += (int64_t)NT * EPV) {
        const int live = (int)(R - r0 < EPV ? R - r0 : EPV);
        const i32x4 v = load_run<FP8>(rs, (int)(r0 * EB), live);
#pragma unroll
        for (int e = 0; e < EPV; ++e) {
            const float x = e < live ? widen<FP8>((unsigned)v[e / PG], e % PG) : 0.0f;
            s = fmaf(x, x, s);
            mx = fmaxf(mx, fabsf(x));
        }
    }
    const double ws = sum64((double)s), wm = max64((double)mx);
    if ((t & 63) == 0) { ssum[t >> 6] = ws; smax[t >> 6] = wm; }
    __syncthreads();
    if (t == 0) {
        nrm2[c] = (ssum[0] + ssum[1]) + (ssum[2] + ssum[3]);
        amax[c] = fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
    }
}

// Sums of each stored row over segments of L consecutive columns:
// out[(column / L) * ldo + row].  Block (bx, by): 64 row vectors of EPV rows
// (one 16-byte load each) and column segment by; its 4 waves take every 4th
// column of the segment, and the waves' sums are added in a fixed order.
template <bool FP8>
__global__ __launch_bounds__(NT) void seg_across_kernel(const char *X, int64_t ld, int64_t R,
                                                        int64_t Cn, int L, float *out,
                                                        int64_t ldo)
{
    constexpr int EB = FP8 ? 1 : 2, EPV = 16 / EB, PG = 4 / EB;
    __shared__ float ssum[4][64 * EPV];
    const int t = threadIdx.x, rv = t & 63;
    const int cp = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t r0 = ((int64_t)blockIdx.x * 64 + rv) * EPV;
    const int64_t c0 = (int64_t)blockIdx.y * L;
    const int64_t c1 = c0 + L < Cn ? c0 + L : Cn;
    float s[EPV];
#pragma unroll
    for (int e = 0; e < EPV; ++e) s[e] = 0.0f;
    const int live = (int)(R - r0 < EPV ? (R - r0 > 0 ? R - r0 : 0) : EPV);
#pragma unroll 4
    for (int64_t c = c0 + cp; c < c1; c += 4) {
        const __amdgpu_buffer_rsrc_t rs = column(X, ld, c, R, EB);
        const i32x4 v = live > 0 ? load_run<FP8>(rs, (int)(r0 * EB), live) : (i32x4){0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < EPV; ++e)
            s[e] += e < live ? widen<FP8>((unsigned)v[e / PG], e % PG) : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < EPV; ++e) ssum[cp][rv * EPV + e] = s[e];
    __syncthreads();
    for (int i = t; i < 64 * EPV; i += NT) {
        const int64_t r = (int64_t)blockIdx.x * 64 * EPV + i;
        if (r >= R) continue;
        out[(int64_t)blockIdx.y * ldo + r] = (ssum[0][i] + ssum[1][i]) + (ssum[2][i] + ssum[3][i]);
    }
}

template <bool FP8>
hipError_t lines(const void *X, int64_t ld, int64_t R, int64_t Cn, bool along_rows,
                 double *nrm2, double *amax, double *part, int64_t part_cap, float *seg,
                 int seg_len, int64_t seg_ld, hipStream_t stream)
{
    constexpr int EPV = FP8 ? 16 : 8;
    if (seg && (seg_len <= 0 || seg_len % EPV != 0 || seg_len > 64 * EPV ||
                ((seg_len / EPV) & (seg_len / EPV - 1)) != 0 || seg_ld < (along_rows ? Cn : R)))
        return hipErrorInvalidValue;
    if (R <= 0 || Cn <= 0) return hipSuccess;
    if (!along_rows) {
        hipLaunchKernelGGL(cols_kernel<FP8>, dim3((unsigned)Cn), dim3(NT), 0, stream,
                           (const char *)X, ld, R, Cn, nrm2, amax);
        if (seg)
            hipLaunchKernelGGL(seg_across_kernel<FP8>,
                               dim3((unsigned)((R + 64 * EPV - 1) / (64 * EPV)),
                                    (unsigned)((Cn + seg_len - 1) / seg_len)),
                               dim3(NT), 0, stream, (const char *)X, ld, R, Cn, seg_len, seg,
                               seg_ld);
        return hipGetLastError();
    }
    const int64_t rblocks = (R + 64 * EPV - 1) / (64 * EPV);
    int64_t nchunks = (1024 + rblocks - 1) / rblocks;  // about 1024 workgroups
    if (nchunks > Cn) nchunks = Cn;
    if (nchunks * 2 * R > part_cap) nchunks = part_cap / (2 * R);
    if (nchunks < 1) return hipErrorInvalidValue;
    const int64_t cc = (Cn + nchunks - 1) / nchunks;
    nchunks = (Cn + cc - 1) / cc;
    hipLaunchKernelGGL(rows_kernel<FP8>, dim3((unsigned)rblocks, (unsigned)nchunks), dim3(NT), 0,
                       stream, (const char *)X, ld, R, Cn, cc, part, (int)nchunks, seg,
                       seg_len / EPV, seg_ld);
    hipLaunchKernelGGL(rows_finish, dim3((unsigned)((R + 63) / 64)), dim3(NT), 0, stream,
                       part, (int)nchunks, R, nrm2, amax);
    return hipGetLastError();
}

}  // namespace norms

hipError_t launch_line_norms(const void *X, int64_t ld, int64_t R, int64_t Cn, bool fp8,
                             bool along_rows, double *nrm2, double *amax, double *part,
                             int64_t part_cap, float *seg, int seg_len, int64_t seg_ld,
                             hipStream_t stream)
{
    return fp8 ? norms::lines<true>(X, ld, R, Cn, along_rows, nrm2, amax, part, part_cap, seg,
                                    seg_len, seg_ld, stream)
               : norms::lines<false>(X, ld, R, Cn, along_rows, nrm2, amax, part, part_cap, seg,
                                     seg_len, seg_ld, stream);
}

}  // namespace ftg
