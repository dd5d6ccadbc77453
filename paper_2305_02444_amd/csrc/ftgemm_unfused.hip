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
// (g, c) pair, four pairs in flight per wave; stored at out[g + c * ldo]
// (tr: out[c + g * ldo]); with out2, the sums of squares go there too.
__global__ __launch_bounds__(NT) void seg_down(const double *Z, int64_t ld, int64_t R,
                                               int64_t Cn, int64_t L, int sq, double *out,
                                               double *out2, int64_t ldo, int tr)
{
    constexpr int P = 4;
    const int lane = threadIdx.x & 63;
    const int64_t nseg = (R + L - 1) / L;
    const int64_t total = nseg * Cn;
    const int64_t stride = (int64_t)gridDim.x * (NT / 64) * P;
    for (int64_t base = ((int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6)) * P; base < total;
         base += stride) {
        double s[P], s2[P];
        int64_t r0[P], r1[P], col[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int64_t pr = base + j < total ? base + j : total - 1;
            const int64_t g = pr % nseg;
            col[j] = pr / nseg;
            r0[j] = g * L;
            r1[j] = r0[j] + L < R ? r0[j] + L : R;
            s[j] = 0.0;
            s2[j] = 0.0;
        }
        for (int64_t o = lane; o < L; o += 64) {
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const int64_t r = r0[j] + o;
                const double v = r < r1[j] ? Z[r + col[j] * ld] : 0.0;
                s[j] += sq ? v * v : v;
                s2[j] += v * v;
            }
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const double a = sum64(s[j]);
            const double b = out2 ? sum64(s2[j]) : 0.0;
            if (lane == 0 && base + j < total) {
                const int64_t g = (base + j) % nseg, c = col[j];
                const int64_t at = tr ? c + g * ldo : g + c * ldo;
                out[at] = a;
                if (out2) out2[at] = b;
            }
        }
    }
}

// across: S(r, g) = sum over columns [L g, L g + L) of f(Z(r, c)), one
// thread per row (block.y = g); stored at out[r + g * ldo] (tr: out[g + r * ldo]);
// with out2, the sums of squares go there too.
__global__ __launch_bounds__(NT) void seg_across(const double *Z, int64_t ld, int64_t R,
                                                 int64_t Cn, int64_t L, int sq, double *out,
                                                 double *out2, int64_t ldo, int tr)
{
    const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t g = blockIdx.y;
    if (r >= R) return;
    const int64_t c0 = g * L, c1 = c0 + L < Cn ? c0 + L : Cn;
    double s = 0.0, s2 = 0.0;
    for (int64_t c = c0; c < c1; ++c) {
        const double v = Z[r + c * ld];
        s += sq ? v * v : v;
        s2 += v * v;
    }
    const int64_t at = tr ? g + r * ldo : r + g * ldo;
    out[at] = s;
    if (out2) out2[at] = s2;
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

// A workgroup verifies tiles (I, J) in turn (grid-stride): threads 0..127
// hold the column-checksum entries of the tile's rows, 128..255 the
// row-checksum entries of its columns.  The tile count and the largest
// ratio go to the counters once per workgroup.
__global__ __launch_bounds__(NT) void compare_kernel(UfArgs a)
{
    __shared__ double wsum[NT / 64], wratio[NT / 64];
    __shared__ double dd[2][T], tt[2][T];
    __shared__ int nb[2], fi[2];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const bool is_row = t < T;
    const int x = is_row ? t : t - T;
    const double sqk = sqrt((double)a.k);
    const int64_t ntiles = (int64_t)a.tiles_m * a.tiles_n;
    double ratio = 0.0;
    unsigned long long seen = 0;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int I = (int)(tile % a.tiles_m), J = (int)(tile / a.tiles_m);
        const int64_t i0 = (int64_t)I * T, j0 = (int64_t)J * T;
        const int h = (int)(a.m - i0 < T ? a.m - i0 : T), wd = (int)(a.n - j0 < T ? a.n - j0 : T);
        const bool live = x < (is_row ? h : wd);
        const double nv2 = live ? (is_row ? a.row_nrm2[i0 + x] : a.col_nrm2[j0 + x]) : 0.0;
        const double f = sum64(nv2);
        __syncthreads();  // the previous tile's readers of wsum, nb, fi, dd, tt are done
        if (lane == 0) wsum[w] = f;
        if (t == 0) { nb[0] = nb[1] = 0; fi[0] = fi[1] = T; }
        __syncthreads();
        const double fa = sqrt(wsum[0] + wsum[1]), fb = sqrt(wsum[2] + wsum[3]);
        if (live) {
            double P, R, c2 = 0.0;
            if (is_row) {
                const int64_t e = (i0 + x) + (int64_t)J * a.m;  // (i, J): m x tiles_n parts
                P = a.alpha * a.Pc[e];
                R = a.Rc[e];
                if (a.beta != 0.0) { P += a.beta * a.cc[e]; c2 = a.cc2[e]; }
            } else {
                const int64_t e = I + (j0 + x) * (int64_t)a.tiles_m;  // (I, j): tiles_m x n
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
                ratio = fmax(ratio, fabs(d) / tau);
            }
        }
        __syncthreads();
        ++seen;
        if (t != 0 || (nb[0] == 0 && nb[1] == 0)) continue;
        // detected, and left as computed
        DevCounters *ct = a.counters;
        atomicAdd(&ct->detected, 1ull);
        atomicAdd(&ct->uncorrectable, 1ull);
        atomicAdd(&ct->record_count, 1u);
        const unsigned slot = atomicAdd(a.rec_slot, 1u);
        if (slot >= a.record_cap) continue;
        ftgemm_fault_record rc;
        rc.problem = a.problem;
        rc.kind = FTGEMM_KIND_UNCORRECTABLE;
        rc.tile_m = I;
        rc.tile_n = J;
        rc.row = nb[0] ? i0 + fi[0] : -1;
        rc.col = nb[1] ? j0 + fi[1] : -1;
        rc.nbad_rows = nb[0];
        rc.nbad_cols = nb[1];
        rc.d_row = nb[1] ? dd[1][fi[1]] : 0.0;  // row checksum (entry of a column)
        rc.tau_row = nb[1] ? tt[1][fi[1]] : 0.0;
        rc.d_col = nb[0] ? dd[0][fi[0]] : 0.0;  // column checksum (entry of a row)
        rc.tau_col = nb[0] ? tt[0][fi[0]] : 0.0;
        rc.before = 0.0;
        rc.after = 0.0;
        a.records[slot] = rc;
    }
    ratio = max64(ratio);
    __syncthreads();
    if (lane == 0) wratio[w] = ratio;
    __syncthreads();
    if (t != 0 || seen == 0) return;
    atomic_max_nonneg(&a.counters->max_ratio_bits,
                      fmax(fmax(wratio[0], wratio[1]), fmax(wratio[2], wratio[3])));
    atomicAdd(&a.counters->tiles_verified, seen);
}

}  // namespace uf

hipError_t launch_seg_sums(const double *Z, int64_t ld, int64_t R, int64_t Cn, int64_t L,
                           bool down, bool square, double *out, double *out2, int64_t ldo,
                           bool transpose, hipStream_t stream)
{
    if (R <= 0 || Cn <= 0) return hipSuccess;
    if (L < 1) return hipErrorInvalidValue;
    const int64_t nseg = down ? (R + L - 1) / L : (Cn + L - 1) / L;
    if (down) {
        constexpr int64_t per_block = uf::NT / 64 * 4;
        int64_t blocks = (nseg * Cn + per_block - 1) / per_block;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(uf::seg_down, dim3((unsigned)blocks), dim3(uf::NT), 0, stream, Z, ld,
                           R, Cn, L, (int)square, out, out2, ldo, (int)transpose);
    } else {
        if (nseg > 65535) return hipErrorInvalidValue;
        hipLaunchKernelGGL(uf::seg_across, dim3((unsigned)((R + uf::NT - 1) / uf::NT), (unsigned)nseg),
                           dim3(uf::NT), 0, stream, Z, ld, R, Cn, L, (int)square, out, out2, ldo,
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
    const int64_t ntiles = (int64_t)a.tiles_m * a.tiles_n;
    if (ntiles == 0) return hipSuccess;
    const unsigned grid = (unsigned)(ntiles < 1024 ? ntiles : 1024);
    hipLaunchKernelGGL(uf::compare_kernel, dim3(grid), dim3(uf::NT), 0, stream, a);
    return hipGetLastError();
}

}  // namespace ftg
