// ftgemm_unfused.hip -- the unfused form of the FP64 fault-tolerant GEMM, the
// comparison the paper's fusion is measured against (Section 2.2): the same
// per-tile checksums and thresholds as the fused kernel, but formed by
// separate passes over memory around an unchanged (checksum-free) GEMM, and
// detection only (the output is left as computed).
//
// Segment sums (one kernel, two directions) give the operand checksums
// x_I = e^T op(A)(I, :) and y_J = op(B)(:, J) e, the C_in and output sums of
// every tile line, and the squared norms; the encoded product parts
// x_I op(B) and op(A) y_J are plain GEMMs; a compare kernel per tile then
// verifies every row and column entry.
#include "ftgemm_device.h"
#include "ftgemm_kernels.h"

namespace ftg {
namespace uf {

constexpr int NT = 256;
constexpr int T = 128;                         // verification tile
constexpr double kU = 1.1102230246251565e-16;  // 2^-53

// down: S(g, c) = sum over rows [L g, L g + L) of f(Z(r, c)), one wave per
// (g, c) pair; stored at out[g + c * ldo] (tr: out[c + g * ldo]).
__global__ __launch_bounds__(NT) void seg_down(const double *Z, int64_t ld, int64_t R,
                                               int64_t Cn, int64_t L, int sq, double *out,
                                               int64_t ldo, int tr)
{
    const int lane = threadIdx.x & 63;
    const int64_t nseg = (R + L - 1) / L;
    const int64_t total = nseg * Cn;
    for (int64_t pr = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6); pr < total;
         pr += (int64_t)gridDim.x * (NT / 64)) {
        const int64_t g = pr % nseg, c = pr / nseg;
        const int64_t r0 = g * L, r1 = r0 + L < R ? r0 + L : R;
        double s = 0.0;
        for (int64_t r = r0 + lane; r < r1; r += 64) {
            const double v = Z[r + c * ld];
            s += sq ? v * v : v;
        }
        s = sum64(s);
        if (lane == 0) out[tr ? c + g * ldo : g + c * ldo] = s;
    }
}

// across: S(r, g) = sum over columns [L g, L g + L) of f(Z(r, c)), one
// thread per row (block.y = g); stored at out[r + g * ldo] (tr: out[g + r * ldo]).
__global__ __launch_bounds__(NT) void seg_across(const double *Z, int64_t ld, int64_t R,
                                                 int64_t Cn, int64_t L, int sq, double *out,
                                                 int64_t ldo, int tr)
{
    const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t g = blockIdx.y;
    if (r >= R) return;
    const int64_t c0 = g * L, c1 = c0 + L < Cn ? c0 + L : Cn;
    double s = 0.0;
    for (int64_t c = c0; c < c1; ++c) {
        const double v = Z[r + c * ld];
        s += sq ? v * v : v;
    }
    out[tr ? g + r * ldo : r + g * ldo] = s;
}

// Planned faults on the output (accumulator faults, ADD only: the output
// changes by alpha * delta); one thread walks the plan.
__global__ void inject_kernel(double *C, int64_t m, int64_t n, int64_t ldc, double alpha,
                              const ftgemm_injection *plan, int nplan,
                              ftgemm_injection_echo *echo, int problem)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int q = 0; q < nplan; ++q) {
        const ftgemm_injection f = plan[q];
        if (f.problem != problem || f.target != FTGEMM_TGT_ACC || f.mode != FTGEMM_INJ_ADD)
            continue;
        if (f.row < 0 || f.row >= m || f.col < 0 || f.col >= n) continue;
        double *p = C + f.row + f.col * ldc;
        ftgemm_injection_echo e;
        e.problem = problem;
        e.applied = 1;
        e.row = f.row;
        e.col = f.col;
        e.k_index = f.k_index;
        e.before = *p;
        *p = *p + alpha * f.delta;
        e.after = *p;
        echo[q] = e;
    }
}

// One workgroup per tile (I, J): threads 0..127 hold the column-checksum
// entries of the tile's rows, 128..255 the row-checksum entries of its
// columns.
__global__ __launch_bounds__(NT) void compare_kernel(UfArgs a)
{
    __shared__ double wsum[NT / 64], wratio[NT / 64];
    __shared__ double dd[2][T], tt[2][T];
    __shared__ int nb[2], fi[2];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int I = (int)(blockIdx.x % (unsigned)a.tiles_m), J = (int)(blockIdx.x / (unsigned)a.tiles_m);
    const int64_t i0 = (int64_t)I * T, j0 = (int64_t)J * T;
    const int h = (int)(a.m - i0 < T ? a.m - i0 : T), wd = (int)(a.n - j0 < T ? a.n - j0 : T);
    const bool is_row = t < T;
    const int x = is_row ? t : t - T;
    const bool live = x < (is_row ? h : wd);
    const double nv2 = live ? (is_row ? a.row_nrm2[i0 + x] : a.col_nrm2[j0 + x]) : 0.0;
    const double f = sum64(nv2);
    if (lane == 0) wsum[w] = f;
    if (t == 0) { nb[0] = nb[1] = 0; fi[0] = fi[1] = T; }
    __syncthreads();
    const double fa = sqrt(wsum[0] + wsum[1]), fb = sqrt(wsum[2] + wsum[3]);
    const double sqk = sqrt((double)a.k);
    double ratio = 0.0;
    if (live) {
        double P, R, c2 = 0.0;
        if (is_row) {
            const int64_t e = (i0 + x) + (int64_t)J * a.m;  // (i, J) of the m x tiles_n parts
            P = a.alpha * a.Pc[e];
            R = a.Rc[e];
            if (a.beta != 0.0) { P += a.beta * a.cc[e]; c2 = a.cc2[e]; }
        } else {
            const int64_t e = I + (j0 + x) * (int64_t)a.tiles_m;  // (I, j) of the tiles_m x n parts
            P = a.alpha * a.Pr[e];
            R = a.Rr[e];
            if (a.beta != 0.0) { P += a.beta * a.cr[e]; c2 = a.cr2[e]; }
        }
        for (int q = 0; q < a.nplan; ++q) {
            const ftgemm_injection fq = a.plan[q];
            if (fq.problem != a.problem || fq.mode != FTGEMM_INJ_ADD) continue;
            const bool hit = is_row
                ? fq.target == FTGEMM_TGT_COL_CHECKSUM && fq.row == i0 + x && fq.col >= j0 &&
                      fq.col < j0 + wd
                : fq.target == FTGEMM_TGT_ROW_CHECKSUM && fq.col == j0 + x && fq.row >= i0 &&
                      fq.row < i0 + h;
            if (!hit) continue;
            ftgemm_injection_echo e;
            e.problem = a.problem; e.applied = 1; e.row = fq.row; e.col = fq.col;
            e.k_index = fq.k_index; e.before = P; P += fq.delta; e.after = P;
            a.echo[q] = e;
        }
        const double tau = is_row
            ? ft_threshold(kLambda, kU, sqk, sqrt((double)wd), a.alpha, sqrt(nv2), fb,
                           sqrt(a.yn2[J]), a.beta, sqrt(c2))
            : ft_threshold(kLambda, kU, sqk, sqrt((double)h), a.alpha, sqrt(nv2), fa,
                           sqrt(a.xn2[I]), a.beta, sqrt(c2));
        const double d = R - P;
        dd[is_row ? 0 : 1][x] = d;
        tt[is_row ? 0 : 1][x] = tau;
        if (!(fabs(d) <= tau)) {
            atomicAdd(&nb[is_row ? 0 : 1], 1);
            atomicMin(&fi[is_row ? 0 : 1], x);
        } else if (tau > 0.0) {
            ratio = fabs(d) / tau;
        }
    }
    ratio = max64(ratio);
    if (lane == 0) wratio[w] = ratio;
    __syncthreads();
    if (t != 0) return;
    DevCounters *ct = a.counters;
    atomic_max_nonneg(&ct->max_ratio_bits,
                      fmax(fmax(wratio[0], wratio[1]), fmax(wratio[2], wratio[3])));
    atomicAdd(&ct->tiles_verified, 1ull);
    if (nb[0] == 0 && nb[1] == 0) return;
    // detected, and left as computed
    atomicAdd(&ct->detected, 1ull);
    atomicAdd(&ct->uncorrectable, 1ull);
    atomicAdd(&ct->record_count, 1u);
    const unsigned slot = atomicAdd(a.rec_slot, 1u);
    if (slot >= a.record_cap) return;
    ftgemm_fault_record rc;
    rc.problem = a.problem;
    rc.kind = FTGEMM_KIND_UNCORRECTABLE;
    rc.tile_m = I;
    rc.tile_n = J;
    rc.row = nb[0] ? i0 + fi[0] : -1;
    rc.col = nb[1] ? j0 + fi[1] : -1;
    rc.nbad_rows = nb[0];
    rc.nbad_cols = nb[1];
    rc.d_row = nb[1] ? dd[1][fi[1]] : 0.0;   // row checksum (entry of a column)
    rc.tau_row = nb[1] ? tt[1][fi[1]] : 0.0;
    rc.d_col = nb[0] ? dd[0][fi[0]] : 0.0;   // column checksum (entry of a row)
    rc.tau_col = nb[0] ? tt[0][fi[0]] : 0.0;
    rc.before = 0.0;
    rc.after = 0.0;
    a.records[slot] = rc;
}

}  // namespace uf

hipError_t launch_seg_sums(const double *Z, int64_t ld, int64_t R, int64_t Cn, int64_t L,
                           bool down, bool square, double *out, int64_t ldo, bool transpose,
                           hipStream_t stream)
{
    if (R <= 0 || Cn <= 0) return hipSuccess;
    if (L < 1) return hipErrorInvalidValue;
    const int64_t nseg = down ? (R + L - 1) / L : (Cn + L - 1) / L;
    if (down) {
        int64_t blocks = (nseg * Cn + uf::NT / 64 - 1) / (uf::NT / 64);
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(uf::seg_down, dim3((unsigned)blocks), dim3(uf::NT), 0, stream, Z, ld,
                           R, Cn, L, (int)square, out, ldo, (int)transpose);
    } else {
        if (nseg > 65535) return hipErrorInvalidValue;
        hipLaunchKernelGGL(uf::seg_across, dim3((unsigned)((R + uf::NT - 1) / uf::NT), (unsigned)nseg),
                           dim3(uf::NT), 0, stream, Z, ld, R, Cn, L, (int)square, out, ldo,
                           (int)transpose);
    }
    return hipGetLastError();
}

hipError_t launch_uf_inject(double *C, int64_t m, int64_t n, int64_t ldc, double alpha,
                            const ftgemm_injection *plan, int nplan, ftgemm_injection_echo *echo,
                            int problem, hipStream_t stream)
{
    if (nplan <= 0) return hipSuccess;
    hipLaunchKernelGGL(uf::inject_kernel, dim3(1), dim3(64), 0, stream, C, m, n, ldc, alpha, plan,
                       nplan, echo, problem);
    return hipGetLastError();
}

hipError_t launch_uf_compare(const UfArgs &a, hipStream_t stream)
{
    const unsigned grid = (unsigned)a.tiles_m * (unsigned)a.tiles_n;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(uf::compare_kernel, dim3(grid), dim3(uf::NT), 0, stream, a);
    return hipGetLastError();
}

}  // namespace ftg
