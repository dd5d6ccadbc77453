// ftgemm_f64.hip -- FP64 fault-tolerant GEMM tile for gfx950.
//
// One workgroup (4 waves, 2 x 2) owns a 128 x 128 output tile and walks the
// inner dimension in steps of 16.  Each step is staged HBM -> VGPR -> LDS
// (double-buffered, one barrier per step) and multiplied with
// v_mfma_f64_16x16x4_f64; every wave owns a 64 x 64 sub-tile.
//
// Fault tolerance (FT-GEMM, Section 2.2), all on values already in
// registers, so it adds no HBM traffic:
//   * operand checksums: the MFMA operand fragments a wave reads from LDS are
//     reused for x = e^T A_I (column sums of the A tile), y = B_J e (row sums
//     of the B tile) and the squared norms of A's rows / B's columns;
//   * encoded checksums of C: Pc_i += A(i,:) y and Pr_j += x B(:,j), one step
//     behind so that the partial sums produced by other waves are complete
//     (they travel through LDS and the step's single barrier);
//   * the encoding of C_in is fused into the beta pass of the epilogue, and
//     the reference checksums are summed from the accumulator registers
//     before anything is written (Section 2.2);
//   * verify, locate, rebuild and confirm one element per tile; a tile with
//     several disagreements is computed again (the same workgroup, C not yet
//     written).
// Work split between the waves (Section 2.3's partition, inside one tile):
// waves 0 and 3 handle the A-side checksums of rows 0-63 and 64-127, waves 1
// and 2 the B-side checksums of columns 0-63 and 64-127, so every wave does
// the same amount of checksum work next to the same amount of MFMA work.
#include "ftgemm_device.h"
#include "ftgemm_kernels.h"

namespace ftg {
namespace f64 {

constexpr int TM = 128, TN = 128, BK = 16, NT = 256;
constexpr int SA = TM + 1, SB = TN + 1;  // odd LDS strides: conflict-free transposed stores
constexpr double U = 1.1102230246251565e-16;  // 2^-53, unit roundoff of FP64

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64 operands and result, lane l = 16 q + c (q < 4, c < 16):
// A fragment holds A[c][q], B fragment holds B[q][c], and result register r
// holds D[4 r + q][c] (measured on gfx950).

struct Stage {
    double A[BK][SA];  // A tile, [p][i]
    double B[BK][SB];  // B tile, [p][j]
};

struct Epi {
    double ref_row[2][TM], ref_col[2][TN];    // partial sums of the output
    double cin_row[2][TM], cin_col[2][TN];    // partial sums of C_in
    double cin2_row[2][TM], cin2_col[2][TN];  // partial sums of squares of C_in
};

struct Smem {
    union {
        Stage st[2];
        Epi epi;
    } u;
    double xs[2][2][BK];  // [buffer][row half][p]: partial column sums of A
    double ys[2][2][BK];  // [buffer][col half][p]: partial row sums of B
    double enc_row[TM], enc_col[TN];  // product part of the encoded checksums
    double nrm_row[TM], nrm_col[TN];  // squared norms of A's rows / B's columns
    double fin_row[TM], fin_col[TN];  // full encoded checksums (with beta part)
    double tau_row[TM], tau_col[TN];
    double d_row[TM], d_col[TN];
    double red[4][2];
    double scal[4];  // |x|^2, |y|^2, |A_I|_F^2, |B_J|_F^2
    TileFault faults[kMaxTileFaults];
    int nfaults;
    int nbad_r, nbad_c, ibad, jbad;
};

// Fetches one step's part of a stored (column-major) operand: TR stored rows
// by 256 * 8 / TR stored columns.  Thread t takes stored row t % TR and
// columns t / TR + r * (256 / TR), r = 0..7, so 64-lane waves read runs of
// consecutive rows.  Stored rows past the matrix get an out-of-range offset;
// stored columns past it fall outside the resource's extent; both read 0.
template <int TR>
struct OpLoader {
    static constexpr int kCStep = NT / TR;
    const char *X;
    int64_t ld, R, total_bytes;
    int row, col0;
    uint32_t voff0, cstep_bytes;

    __device__ __forceinline__ void init(const double *x, int64_t ld_, int64_t rows,
                                         int64_t cols, int t)
    {
        X = (const char *)x;
        ld = ld_;
        R = rows;
        total_bytes = (rows > 0 && cols > 0) ? (ld_ * (cols - 1) + rows) * 8 : 0;
        row = t % TR;
        col0 = t / TR;
        voff0 = (uint32_t)((row + (int64_t)col0 * ld_) * 8);
        cstep_bytes = (uint32_t)(kCStep * ld_ * 8);
    }
    __device__ __forceinline__ int col(int r) const { return col0 + r * kCStep; }
    __device__ __forceinline__ void load(int64_t r0, int64_t c0, double v[8]) const
    {
        const int64_t first = r0 + c0 * ld;
        int64_t ext = total_bytes - first * 8;
        if (ext < 0) ext = 0;
        if (ext > 0x7FFFFFFF) ext = 0x7FFFFFFF;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(X + first * 8, (uint64_t)ext);
        const uint32_t off = (r0 + row < R) ? voff0 : kOob;
#pragma unroll
        for (int r = 0; r < 8; ++r)
            v[r] = buf_load_f64(rs, off + (uint32_t)r * cstep_bytes);
    }
};

template <bool TA, bool TB, bool ABFT>
__device__ void tile(const GemmArgs &g, int tile_m, int tile_n, Smem &sm)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int q = lane >> 4, c16 = lane & 15;
    const int64_t i0 = (int64_t)tile_m * TM, j0 = (int64_t)tile_n * TN;
    const double *__restrict__ A = (const double *)g.A;
    const double *__restrict__ B = (const double *)g.B;
    double *__restrict__ C = (double *)g.C;
    const int64_t m = g.m, n = g.n, k = g.k, lda = g.lda, ldb = g.ldb, ldc = g.ldc;
    const int nsteps = (int)((k + BK - 1) / BK);
    const int hrows = (int)(m - i0 < TM ? m - i0 : TM);
    const int wcols = (int)(n - j0 < TN ? n - j0 : TN);
    const bool use_c = g.beta != 0.0;

    // Staging.  Each thread fetches 8 elements of A and 8 of B per step
    // through buffer resources (see OpLoader); a wave's loads are contiguous
    // runs in memory and its LDS stores hit distinct banks.
    OpLoader<TA ? 16 : 128> la;
    OpLoader<TB ? 128 : 16> lb;
    la.init(A, lda, TA ? k : m, TA ? m : k, t);
    lb.init(B, ldb, TB ? n : k, TB ? k : n, t);
    double ra[8], rb[8];
    auto load = [&](int s) {
        const int64_t k0 = (int64_t)s * BK;
        if (!TA) la.load(i0, k0, ra); else la.load(k0, i0, ra);
        if (!TB) lb.load(k0, j0, rb); else lb.load(j0, k0, rb);
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            // A tile is [p][i]; B tile is [p][j]
            if (!TA) sm.u.st[buf].A[la.col(r)][la.row] = ra[r];
            else     sm.u.st[buf].A[la.row][la.col(r)] = ra[r];
            if (!TB) sm.u.st[buf].B[lb.row][lb.col(r)] = rb[r];
            else     sm.u.st[buf].B[lb.col(r)][lb.row] = rb[r];
        }
    };

    // Planned faults of this tile (test hook).
    int nf = 0;
    if (ABFT) {
        if (w == 0) {
            const int cnt = gather_tile_faults(g, i0, j0, TM, TN, BK,
                                               g.k_base, sm.faults);
            if (lane == 0) sm.nfaults = cnt;
        }
        __syncthreads();
        nf = sm.nfaults;
    }

    const bool a_side = (w == 0 || w == 3);  // waves holding A-side checksum work
    int kind = 0, first_nr = 0, first_nc = 0, first_i = -1, first_j = -1;
    double rec_d_row = 0, rec_d_col = 0, rec_t_row = 0, rec_t_col = 0, rec_before = 0,
           rec_after = 0;

    d4 acc[4][4];
#pragma unroll 1
    for (int attempt = 0; attempt < 2; ++attempt) {
        const bool faults_on = ABFT && attempt == 0 && nf > 0;
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                acc[mi][ni] = (d4){0.0, 0.0, 0.0, 0.0};
        double cs_acc[4] = {0, 0, 0, 0};  // Pc (A side) or Pr (B side) partials
        double cs_nrm[4] = {0, 0, 0, 0};  // row / column squared norms
        double vec_nrm = 0.0;             // |y|^2 (A side) or |x|^2 (B side)
        double prev[4][4];                // last step's checksum-side fragments

        load(0);
        // The steps run in segments that end where a planned fault lands, so
        // the fault hook sits outside the hot loop.
        int s = 0;
#pragma unroll 1
        while (s < nsteps) {
        int stop = nsteps - 1;
        if (faults_on)
            for (int f = 0; f < nf; ++f) {
                const int fs = sm.faults[f].kstep;
                if (sm.faults[f].target == FTGEMM_TGT_ACC && fs >= s && fs < stop) stop = fs;
            }
#pragma unroll 1
        for (; s <= stop; ++s) {
            const int buf = s & 1;
            store(buf);
            __syncthreads();
            if (s + 1 < nsteps)
                load(s + 1);

            // Encoded checksums, one step behind: the operand-checksum
            // partials of step s-1 from the other waves are complete now.
            if (ABFT && s > 0) {
                const int pb = (s - 1) & 1;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const double v = a_side
                        ? sm.ys[pb][0][4 * kk + q] + sm.ys[pb][1][4 * kk + q]
                        : sm.xs[pb][0][4 * kk + q] + sm.xs[pb][1][4 * kk + q];
                    vec_nrm += v * v;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        cs_acc[e] += prev[kk][e] * v;
                }
            }

#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                double fa[4], fb[4];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
                    fa[mi] = sm.u.st[buf].A[4 * kk + q][wm * 64 + 16 * mi + c16];
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    fb[ni] = sm.u.st[buf].B[4 * kk + q][wn * 64 + 16 * ni + c16];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
                        acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            fa[mi], fb[ni], acc[mi][ni], 0, 0, 0);
                if (ABFT) {
                    // operand checksums and norms from the fragments in hand:
                    // A side sums over its 64 rows, B side over its 64 columns
                    double part = 0.0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double v = a_side ? fa[e] : fb[e];
                        cs_nrm[e] += v * v;
                        part += v;
                        prev[kk][e] = v;
                    }
                    part = sum16(part);
                    if (c16 == 0) {
                        if (a_side) sm.xs[buf][wm][4 * kk + q] = part;
                        else        sm.ys[buf][wn][4 * kk + q] = part;
                    }
                }
            }

        }
            if (ABFT) {
                // Fault hook: accumulator faults land after step `stop`.
                if (faults_on) {
                    for (int f = 0; f < nf; ++f) {
                        const TileFault tf = sm.faults[f];
                        if (tf.target != FTGEMM_TGT_ACC || tf.kstep != stop)
                            continue;
                        // owner: wave, lane and register of C(row, col)
                        const int ow = (tf.row >> 6) + 2 * (tf.col >> 6);
                        const int ol = 16 * (tf.row & 3) + (tf.col & 15);
                        const int sel = ((tf.row & 63) >> 4) * 16 + ((tf.col & 63) >> 4) * 4 +
                                        ((tf.row & 15) >> 2);
                        if (w != ow) continue;
                        double before = 0.0;
#pragma unroll
                        for (int e = 0; e < 64; ++e)
                            if (sel == e) before = acc[e >> 4][(e >> 2) & 3][e & 3];
                        const double after = tf.mode == FTGEMM_INJ_ADD
                                                 ? before + tf.delta
                                                 : flip_bit_f64(before, tf.bit);
#pragma unroll
                        for (int e = 0; e < 64; ++e)
                            if (sel == e && lane == ol) acc[e >> 4][(e >> 2) & 3][e & 3] = after;
                        if (lane == ol) {
                            ftgemm_injection_echo ech;
                            ech.problem = g.problem;
                            ech.applied = 1;
                            ech.row = i0 + tf.row;
                            ech.col = j0 + tf.col;
                            ech.k_index = g.plan[tf.idx].k_index;
                            ech.before = before;
                            ech.after = after;
                            g.echo[tf.idx] = ech;
                        }
                    }
                }
            }
        }
        __syncthreads();

        if (!ABFT) {
            // Plain GEMM epilogue: the beta pass and the store.
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm * 64 + 16 * mi + 4 * r + q;
                        const int col = wn * 64 + 16 * ni + c16;
                        if (row < hrows && col < wcols) {
                            double *pc = C + (i0 + row) + (j0 + col) * ldc;
                            const double o = g.alpha * acc[mi][ni][r];
                            *pc = use_c ? o + g.beta * *pc : o;
                        }
                    }
            return;
        }

        // Last lagged update of the encoded checksums, then fold the four
        // rows of 16 lanes (each handled every fourth p).
        {
            const int pb = (nsteps - 1) & 1;
            if (a_side) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const double yv = sm.ys[pb][0][4 * kk + q] + sm.ys[pb][1][4 * kk + q];
                    vec_nrm += yv * yv;
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
                        cs_acc[mi] += prev[kk][mi] * yv;
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const double xv = sm.xs[pb][0][4 * kk + q] + sm.xs[pb][1][4 * kk + q];
                    vec_nrm += xv * xv;
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
                        cs_acc[ni] += xv * prev[kk][ni];
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                cs_acc[v] = sum_rows(cs_acc[v]);
                cs_nrm[v] = sum_rows(cs_nrm[v]);
            }
            vec_nrm = sum_rows(vec_nrm);
            if (q == 0) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (a_side) {
                        sm.enc_row[wm * 64 + 16 * v + c16] = cs_acc[v];
                        sm.nrm_row[wm * 64 + 16 * v + c16] = cs_nrm[v];
                    } else {
                        sm.enc_col[wn * 64 + 16 * v + c16] = cs_acc[v];
                        sm.nrm_col[wn * 64 + 16 * v + c16] = cs_nrm[v];
                    }
                }
            }
            if (lane == 0 && w == 0) sm.scal[1] = vec_nrm;  // |y|^2
            if (lane == 0 && w == 1) sm.scal[0] = vec_nrm;  // |x|^2
        }

        // Beta pass fused with the C_in part of the encoding (Section 2.2)
        // and the reference sums of the output.
        double col_o[4] = {0, 0, 0, 0}, col_c[4] = {0, 0, 0, 0}, col_c2[4] = {0, 0, 0, 0};
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double row_o = 0, row_c = 0, row_c2 = 0;
                const int row = wm * 64 + 16 * mi + 4 * r + q;
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) {
                    const int col = wn * 64 + 16 * ni + c16;
                    const bool ok = row < hrows && col < wcols;
                    const double cin = (use_c && ok) ? C[(i0 + row) + (j0 + col) * ldc] : 0.0;
                    double o = g.alpha * acc[mi][ni][r];
                    if (use_c) o = o + g.beta * cin;
                    o = ok ? o : 0.0;
                    acc[mi][ni][r] = o;
                    row_o += o; row_c += cin; row_c2 += cin * cin;
                    col_o[ni] += o; col_c[ni] += cin; col_c2[ni] += cin * cin;
                }
                row_o = sum16(row_o);
                if (use_c) { row_c = sum16(row_c); row_c2 = sum16(row_c2); }
                if (c16 == 0) {
                    sm.u.epi.ref_row[wn][row] = row_o;
                    sm.u.epi.cin_row[wn][row] = row_c;
                    sm.u.epi.cin2_row[wn][row] = row_c2;
                }
            }
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            col_o[ni] = sum_rows(col_o[ni]);
            if (use_c) { col_c[ni] = sum_rows(col_c[ni]); col_c2[ni] = sum_rows(col_c2[ni]); }
            if (q == 0) {
                const int col = wn * 64 + 16 * ni + c16;
                sm.u.epi.ref_col[wm][col] = col_o[ni];
                sm.u.epi.cin_col[wm][col] = col_c[ni];
                sm.u.epi.cin2_col[wm][col] = col_c2[ni];
            }
        }
        if (t == 0) { sm.nbad_r = 0; sm.nbad_c = 0; sm.ibad = TM; sm.jbad = TN; }
        __syncthreads();
        if (w == 0) sm.scal[2] = sum64(sm.nrm_row[lane] + sm.nrm_row[lane + 64]);
        if (w == 1) sm.scal[3] = sum64(sm.nrm_col[lane] + sm.nrm_col[lane + 64]);
        __syncthreads();

        // Verify: thread t < 128 checks row t, the others column t - 128.
        {
            const double sqk = sqrt((double)k);
            double ratio = 0.0;
            if (t < TM) {
                const int i = t;
                double P = g.alpha * sm.enc_row[i];
                if (use_c) P += g.beta * (sm.u.epi.cin_row[0][i] + sm.u.epi.cin_row[1][i]);
                if (faults_on)
                    for (int f = 0; f < nf; ++f) {
                        const TileFault tf = sm.faults[f];
                        if (tf.target == FTGEMM_TGT_COL_CHECKSUM && tf.row == i) {
                            ftgemm_injection_echo e;
                            e.problem = g.problem; e.applied = 1; e.row = i0 + tf.row;
                            e.col = j0 + tf.col; e.k_index = g.plan[tf.idx].k_index;
                            e.before = P; P += tf.delta; e.after = P;
                            g.echo[tf.idx] = e;
                        }
                    }
                const double R = sm.u.epi.ref_row[0][i] + sm.u.epi.ref_row[1][i];
                const double tau = ft_threshold(
                    kLambda, U, sqk, sqrt((double)wcols), g.alpha, sqrt(sm.nrm_row[i]),
                    sqrt(sm.scal[3]), sqrt(sm.scal[1]), g.beta,
                    sqrt(sm.u.epi.cin2_row[0][i] + sm.u.epi.cin2_row[1][i]));
                const double d = R - P;
                sm.fin_row[i] = P; sm.tau_row[i] = tau; sm.d_row[i] = d;
                if (i < hrows) {
                    if (!(fabs(d) <= tau)) {
                        atomicAdd(&sm.nbad_r, 1);
                        atomicMin(&sm.ibad, i);
                    } else if (tau > 0.0) {
                        ratio = fabs(d) / tau;
                    }
                }
            } else {
                const int j = t - TM;
                double P = g.alpha * sm.enc_col[j];
                if (use_c) P += g.beta * (sm.u.epi.cin_col[0][j] + sm.u.epi.cin_col[1][j]);
                if (faults_on)
                    for (int f = 0; f < nf; ++f) {
                        const TileFault tf = sm.faults[f];
                        if (tf.target == FTGEMM_TGT_ROW_CHECKSUM && tf.col == j) {
                            ftgemm_injection_echo e;
                            e.problem = g.problem; e.applied = 1; e.row = i0 + tf.row;
                            e.col = j0 + tf.col; e.k_index = g.plan[tf.idx].k_index;
                            e.before = P; P += tf.delta; e.after = P;
                            g.echo[tf.idx] = e;
                        }
                    }
                const double R = sm.u.epi.ref_col[0][j] + sm.u.epi.ref_col[1][j];
                const double tau = ft_threshold(
                    kLambda, U, sqk, sqrt((double)hrows), g.alpha, sqrt(sm.nrm_col[j]),
                    sqrt(sm.scal[2]), sqrt(sm.scal[0]), g.beta,
                    sqrt(sm.u.epi.cin2_col[0][j] + sm.u.epi.cin2_col[1][j]));
                const double d = R - P;
                sm.fin_col[j] = P; sm.tau_col[j] = tau; sm.d_col[j] = d;
                if (j < wcols) {
                    if (!(fabs(d) <= tau)) {
                        atomicAdd(&sm.nbad_c, 1);
                        atomicMin(&sm.jbad, j);
                    } else if (tau > 0.0) {
                        ratio = fabs(d) / tau;
                    }
                }
            }
            ratio = max64(ratio);
            if (lane == 0) atomic_max_nonneg(&g.counters->max_ratio_bits, ratio);
        }
        __syncthreads();

        const int nr = sm.nbad_r, nc = sm.nbad_c;
        if (nr == 0 && nc == 0) {
            if (attempt == 1) kind = FTGEMM_KIND_RECOMPUTED;
            break;
        }
        if (attempt == 1) {
            kind = FTGEMM_KIND_UNCORRECTABLE;
            break;
        }
        // First attempt disagreed: keep what the record needs.
        first_nr = nr; first_nc = nc;
        first_i = nr ? sm.ibad : -1;
        first_j = nc ? sm.jbad : -1;
        rec_d_row = first_j >= 0 ? sm.d_col[first_j] : 0.0;
        rec_t_row = first_j >= 0 ? sm.tau_col[first_j] : 0.0;
        rec_d_col = first_i >= 0 ? sm.d_row[first_i] : 0.0;
        rec_t_col = first_i >= 0 ? sm.tau_row[first_i] : 0.0;

        if (nr == 1 && nc == 1) {
            // Locate at the crossing; rebuild from the encoded checksum of
            // its column and the rest of the column (robust to Inf / NaN in
            // the faulty element); confirm with the rest of its row.
            const int is = first_i, js = first_j;
            double s_col = 0.0, s_row = 0.0;
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm * 64 + 16 * mi + 4 * r + q;
                        const int col = wn * 64 + 16 * ni + c16;
                        const double o = acc[mi][ni][r];
                        if (col == js && row != is) s_col += o;
                        if (row == is && col != js) s_row += o;
                    }
            s_col = sum64(s_col);
            s_row = sum64(s_row);
            if (lane == 0) { sm.red[w][0] = s_col; sm.red[w][1] = s_row; }
            __syncthreads();
            const double sc = ((sm.red[0][0] + sm.red[1][0]) + sm.red[2][0]) + sm.red[3][0];
            const double sr = ((sm.red[0][1] + sm.red[1][1]) + sm.red[2][1]) + sm.red[3][1];
            const double fixed = sm.fin_col[js] - sc;
            if (fabs(sr + fixed - sm.fin_row[is]) <= sm.tau_row[is]) {
                const int ow = (is >> 6) + 2 * (js >> 6);
                const int ol = 16 * (is & 3) + (js & 15);
                const int omi = (is & 63) >> 4, oni = (js & 63) >> 4, orr = (is & 15) >> 2;
                if (w == ow && lane == ol) {
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                if (mi == omi && ni == oni && r == orr) {
                                    rec_before = acc[mi][ni][r];
                                    acc[mi][ni][r] = fixed;
                                }
                }
                rec_after = fixed;
                kind = FTGEMM_KIND_CORRECTED;
                break;
            }
        } else if (nr + nc == 1) {
            kind = FTGEMM_KIND_CHECKSUM_ONLY;
            break;
        }
        // Several disagreements, or a rebuilt value that does not confirm:
        // compute the tile again.
        __syncthreads();
    }

    if (ABFT) {
        // the owner lane of a corrected element knows its old value
        if (kind == FTGEMM_KIND_CORRECTED) {
            const int ow = (first_i >> 6) + 2 * (first_j >> 6);
            const int ol = 16 * (first_i & 3) + (first_j & 15);
            if (w == ow && lane == ol) sm.red[0][0] = rec_before;
            __syncthreads();
            rec_before = sm.red[0][0];
        }
        if (t == 0) {
            DevCounters *ct = g.counters;
            atomicAdd(&ct->tiles_verified, 1ull);
            if (kind != 0) {
                atomicAdd(&ct->detected, 1ull);
                unsigned long long *which =
                    kind == FTGEMM_KIND_CORRECTED ? &ct->corrected
                    : kind == FTGEMM_KIND_CHECKSUM_ONLY ? &ct->checksum_only
                    : kind == FTGEMM_KIND_RECOMPUTED ? &ct->recomputed
                                                     : &ct->uncorrectable;
                atomicAdd(which, 1ull);
                const unsigned slot = atomicAdd(&ct->record_count, 1u);
                if (slot < g.record_cap) {
                    ftgemm_fault_record rc;
                    rc.problem = g.problem;
                    rc.kind = kind;
                    rc.tile_m = tile_m;
                    rc.tile_n = tile_n;
                    rc.row = first_i >= 0 ? i0 + first_i : -1;
                    rc.col = first_j >= 0 ? j0 + first_j : -1;
                    rc.nbad_rows = first_nr;
                    rc.nbad_cols = first_nc;
                    rc.d_row = rec_d_row;
                    rc.d_col = rec_d_col;
                    rc.tau_row = rec_t_row;
                    rc.tau_col = rec_t_col;
                    rc.before = kind == FTGEMM_KIND_CORRECTED ? rec_before : 0.0;
                    rc.after = kind == FTGEMM_KIND_CORRECTED ? rec_after : 0.0;
                    g.records[slot] = rc;
                }
            }
        }
        // Store the verified tile.
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wm * 64 + 16 * mi + 4 * r + q;
                    const int col = wn * 64 + 16 * ni + c16;
                    if (row < hrows && col < wcols)
                        C[(i0 + row) + (j0 + col) * ldc] = acc[mi][ni][r];
                }
    }
}

template <bool TA, bool TB, bool ABFT>
__global__ __launch_bounds__(NT) void kernel(GemmArgs g)
{
    __shared__ Smem sm;
    int tm_, tn_;
    map_tile(blockIdx.x, g.tiles_m, g.tiles_n, tm_, tn_);
    tile<TA, TB, ABFT>(g, tm_, tn_, sm);
}

}  // namespace f64

#define FTG_F64_CASE(ta, tb, ab) \
    hipLaunchKernelGGL((f64::kernel<ta, tb, ab>), dim3(grid), dim3(f64::NT), 0, stream, g)

hipError_t launch_f64(const GemmArgs &g, bool ta, bool tb, bool abft, hipStream_t stream)
{
    const unsigned grid = (unsigned)g.tiles_m * (unsigned)g.tiles_n;
    if (grid == 0) return hipSuccess;
    if (abft) {
        if (!ta && !tb) FTG_F64_CASE(false, false, true);
        else if (!ta && tb) FTG_F64_CASE(false, true, true);
        else if (ta && !tb) FTG_F64_CASE(true, false, true);
        else FTG_F64_CASE(true, true, true);
    } else {
        if (!ta && !tb) FTG_F64_CASE(false, false, false);
        else if (!ta && tb) FTG_F64_CASE(false, true, false);
        else if (ta && !tb) FTG_F64_CASE(true, false, false);
        else FTG_F64_CASE(true, true, false);
    }
    return hipGetLastError();
}

void tiling_f64(int *tm, int *tn, int *bk)
{
    *tm = f64::TM;
    *tn = f64::TN;
    *bk = f64::BK;
}

}  // namespace ftg
