// ftgemm_splitk.hip -- verified reduction of a split inner dimension (FP64).
//
// When a problem has too few output tiles to fill the chip, the inner
// dimension is cut into slices: the tile kernel computes, verifies and, where
// needed, corrects the partial product of each slice (FT-GEMM, Section 2.2,
// applied to op(A)(:, K_s) op(B)(K_s, :)) and leaves it in a workspace
// together with the slice's encoded checksums and thresholds.  Checksums are
// linear, so the encoded checksums of the result are
//   Pr_j = alpha * sum_s Pr_j^(s) + beta * sum_i C_in(i, j)   (and Pc_i alike),
// which this kernel compares with the sums of what it writes,
//   C = alpha * sum_s W_s + beta * C_in,
// catching faults in the reduction and in the workspace between the two
// kernels.  One workgroup per 128 x 128 tile; the verification, location and
// reconstruction follow the tile kernel's.
#include "ftgemm_device.h"
#include "ftgemm_kernels.h"

namespace ftg {
namespace splitk {

constexpr int T = 128;   // tile (the tile kernel's verification tile)
constexpr int NT = 256;  // thread t < 128 owns row t, t >= 128 column t - 128
constexpr int LD = T + 1;
constexpr double U = 1.1102230246251565e-16;  // 2^-53

struct Smem {
    double tile[T][LD];  // [column][row]
    double P[2][T], tau[2][T], R[2][T], d[2][T];
    double red[4][2];
    int nbad[2], bad[2];
};

// C_in (when read) or the reduced output of this thread's elements: thread t
// handles rows t % 64 + 64 h (h = 0, 1) of columns t / 64 + 4 q (q < 32), so
// a wave reads 64 consecutive rows of one column.
template <bool kOut>
__device__ __forceinline__ void fill(const ReduceArgs &r, int64_t i0, int64_t j0, int hrows,
                                     int wcols, Smem &sm)
{
    const int t = threadIdx.x;
    const double *C = r.C;
    for (int q = 0; q < T / 4; ++q) {
        const int col = (t >> 6) + 4 * q;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = (t & 63) + 64 * h;
            double v = 0.0;
            if (row < hrows && col < wcols) {
                const int64_t off = (i0 + row) + (j0 + col) * r.m;
                const double cin = r.beta != 0.0 ? C[(i0 + row) + (j0 + col) * r.ldc] : 0.0;
                if (kOut) {
                    double w = 0.0;
                    for (int s = 0; s < r.nslices; ++s) w += r.wsp[off + (int64_t)s * r.m * r.n];
                    v = r.alpha * w;
                    if (r.beta != 0.0) v = v + r.beta * cin;
                } else {
                    v = cin;
                }
            }
            sm.tile[col][row] = v;
        }
    }
}

// sums over row t (t < 128) or column t - 128 of the staged tile: the sum,
// the sum of magnitudes and the sum of squares
__device__ __forceinline__ void line_sums(const Smem &sm, double &s, double &a, double &s2)
{
    const int t = threadIdx.x;
    s = a = s2 = 0.0;
    if (t < T) {
        for (int j = 0; j < T; ++j) {
            const double v = sm.tile[j][t];
            s += v; a += fabs(v); s2 += v * v;
        }
    } else {
        for (int i = 0; i < T; ++i) {
            const double v = sm.tile[t - T][i];
            s += v; a += fabs(v); s2 += v * v;
        }
    }
}

template <bool ABFT>
__global__ __launch_bounds__(NT) void reduce_kernel(ReduceArgs r)
{
    __shared__ Smem sm;
    const int t = threadIdx.x;
    int tm_, tn_;
    map_tile(blockIdx.x, r.tiles_m, r.tiles_n, tm_, tn_);
    const int64_t i0 = (int64_t)tm_ * T, j0 = (int64_t)tn_ * T;
    const int hrows = (int)(r.m - i0 < T ? r.m - i0 : T);
    const int wcols = (int)(r.n - j0 < T ? r.n - j0 : T);
    const int side = t < T ? 0 : 1;  // 0: row t, 1: column t - 128
    const int x = t & (T - 1);
    const bool live = x < (side ? wcols : hrows);
    const int64_t ntiles = (int64_t)r.tiles_m * r.tiles_n;
    const int64_t tile = tm_ + (int64_t)tn_ * r.tiles_m;

    double cs = 0.0, c2 = 0.0;
    if (ABFT && r.beta != 0.0) {
        fill<false>(r, i0, j0, hrows, wcols, sm);
        __syncthreads();
        double a;
        line_sums(sm, cs, a, c2);
        __syncthreads();
    }
    // encoded checksums and thresholds of this line, from the slices
    double P = 0.0, tau = 0.0;
    if (ABFT) {
        for (int s = 0; s < r.nslices; ++s) {
            const double *src = r.chk + slice_chk_index(s, tile, ntiles, T, T);
            P += src[t];  // rows [0, 128), columns [128, 256)
            tau += src[2 * T + t];
        }
        P = r.alpha * P;
        if (r.beta != 0.0) P += r.beta * cs;
    }
    if (t == 0) { sm.nbad[0] = sm.nbad[1] = 0; sm.bad[0] = sm.bad[1] = T; }

    int kind = 0, nr0 = 0, nc0 = 0, bi = -1, bj = -1;
    double before = 0.0, after = 0.0, keep[4] = {0, 0, 0, 0};
    for (int attempt = 0; attempt < 2; ++attempt) {
        fill<true>(r, i0, j0, hrows, wcols, sm);
        __syncthreads();
        if (!ABFT) break;
        double R, a, s2;
        line_sums(sm, R, a, s2);
        // slices' thresholds, plus the rounding of the S-term reduction, of
        // alpha, of the beta term and of the reference sum (lambda unit
        // roundoffs per term), plus the beta part's encoding
        const double th = fabs(r.alpha) * tau +
                          kLambda * U * ((r.nslices + 3) * a + 2.0 * fabs(r.beta) * sqrt(c2));
        const double d = R - P;
        sm.P[side][x] = P; sm.tau[side][x] = th; sm.R[side][x] = R; sm.d[side][x] = d;
        if (live && !(fabs(d) <= th)) {
            atomicAdd(&sm.nbad[side], 1);
            atomicMin(&sm.bad[side], x);
        }
        __syncthreads();
        const int nr = sm.nbad[0], nc = sm.nbad[1];
        if (nr == 0 && nc == 0) {
            if (attempt == 1) kind = FTGEMM_KIND_RECOMPUTED;
            break;
        }
        if (attempt == 1) { kind = FTGEMM_KIND_UNCORRECTABLE; break; }
        nr0 = nr; nc0 = nc;
        bi = nr ? sm.bad[0] : -1;
        bj = nc ? sm.bad[1] : -1;
        keep[0] = bj >= 0 ? sm.d[1][bj] : 0.0; keep[1] = bj >= 0 ? sm.tau[1][bj] : 0.0;
        keep[2] = bi >= 0 ? sm.d[0][bi] : 0.0; keep[3] = bi >= 0 ? sm.tau[0][bi] : 0.0;
        if (nr == 1 && nc == 1) {
            // rebuild from the column's encoded checksum, confirm with the row
            double sc = 0.0, sr = 0.0;
            if (t == 0) {
                for (int i = 0; i < T; ++i) if (i != bi) sc += sm.tile[bj][i];
                for (int j = 0; j < T; ++j) if (j != bj) sr += sm.tile[j][bi];
                const double fixed = sm.P[1][bj] - sc;
                const bool ok = fabs(sr + fixed - sm.P[0][bi]) <= sm.tau[0][bi];
                sm.red[0][0] = ok ? 1.0 : 0.0;
                sm.red[0][1] = sm.tile[bj][bi];
                if (ok) sm.tile[bj][bi] = fixed;
                sm.red[1][0] = fixed;
            }
            __syncthreads();
            if (sm.red[0][0] != 0.0) {
                kind = FTGEMM_KIND_CORRECTED;
                before = sm.red[0][1];
                after = sm.red[1][0];
                break;
            }
        } else if (nr + nc == 1) {
            // a checksum fault only beyond the entry's threshold plus twice
            // the other side's largest (a data error shows on both sides)
            if (t == 0) {
                const int side_o = nc == 1 ? 0 : 1;
                const int cnt = nc == 1 ? hrows : wcols;
                double o = 0.0;
                for (int x2 = 0; x2 < cnt; ++x2) o = fmax(o, sm.tau[side_o][x2]);
                const double dd = nc == 1 ? sm.d[1][bj] : sm.d[0][bi];
                const double own = nc == 1 ? sm.tau[1][bj] : sm.tau[0][bi];
                sm.red[2][0] = !(fabs(dd) <= own + 2.0 * o) ? 1.0 : 0.0;
            }
            __syncthreads();
            if (sm.red[2][0] != 0.0) {
                kind = FTGEMM_KIND_CHECKSUM_ONLY;
                break;
            }
        }
        __syncthreads();
        if (t == 0) { sm.nbad[0] = sm.nbad[1] = 0; sm.bad[0] = sm.bad[1] = T; }
        __syncthreads();
    }
    if (ABFT && t == 0) {
        DevCounters *ct = r.counters;
        atomicAdd(&ct->tiles_verified, 1ull);
        if (kind != 0) {
            atomicAdd(&ct->detected, 1ull);
            unsigned long long *which =
                kind == FTGEMM_KIND_CORRECTED ? &ct->corrected
                : kind == FTGEMM_KIND_CHECKSUM_ONLY ? &ct->checksum_only
                : kind == FTGEMM_KIND_RECOMPUTED ? &ct->recomputed
                                                 : &ct->uncorrectable;
            atomicAdd(which, 1ull);
            atomicAdd(&ct->record_count, 1u);
            const unsigned slot = atomicAdd(r.rec_slot, 1u);
            if (slot < r.record_cap) {
                ftgemm_fault_record rc;
                rc.problem = r.problem;
                rc.kind = kind;
                rc.tile_m = tm_;
                rc.tile_n = tn_;
                rc.row = bi >= 0 ? i0 + bi : -1;
                rc.col = bj >= 0 ? j0 + bj : -1;
                rc.nbad_rows = nr0;
                rc.nbad_cols = nc0;
                rc.d_row = keep[0]; rc.tau_row = keep[1];
                rc.d_col = keep[2]; rc.tau_col = keep[3];
                rc.before = kind == FTGEMM_KIND_CORRECTED ? before : 0.0;
                rc.after = kind == FTGEMM_KIND_CORRECTED ? after : 0.0;
                r.records[slot] = rc;
            }
        }
    }
    __syncthreads();
    double *C = r.C;
    for (int q = 0; q < T / 4; ++q) {
        const int col = (t >> 6) + 4 * q;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = (t & 63) + 64 * h;
            if (row < hrows && col < wcols)
                C[(i0 + row) + (j0 + col) * r.ldc] = sm.tile[col][row];
        }
    }
}

}  // namespace splitk

hipError_t launch_splitk_reduce(const ReduceArgs &r, bool abft, hipStream_t stream)
{
    const unsigned grid = (unsigned)r.tiles_m * (unsigned)r.tiles_n;
    if (grid == 0) return hipSuccess;
    if (abft)
        hipLaunchKernelGGL(splitk::reduce_kernel<true>, dim3(grid), dim3(splitk::NT), 0, stream, r);
    else
        hipLaunchKernelGGL(splitk::reduce_kernel<false>, dim3(grid), dim3(splitk::NT), 0, stream, r);
    return hipGetLastError();
}

}  // namespace ftg
