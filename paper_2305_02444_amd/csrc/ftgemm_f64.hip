// ftgemm_f64.hip -- FP64 fault-tolerant GEMM tile for gfx950.
//
// One workgroup (8 waves, 2 x 4) owns a 128 x 128 output tile and walks the
// inner dimension in steps of 32.  Each step is staged HBM -> VGPR -> LDS
// (double-buffered, one barrier per step) and multiplied with
// v_mfma_f64_16x16x4_f64; every wave owns a 64 x 32 sub-tile, and the two
// waves on each SIMD hide each other's LDS and barrier latency.
//
// Fault tolerance (FT-GEMM, Section 2.2), on the staged operand values, so
// it adds no HBM traffic:
//   * every thread's 8 staged elements of a step share one inner index p;
//     before the step's barrier it adds them into the operand checksums
//     x_p = sum_i A(i,p) and y_p = sum_j B(p,j) (a short cross-lane
//     reduction finishes them in LDS);
//   * after the barrier, with x_p and y_p complete, the staged A registers
//     feed the encoded column checksums Pc_i += A(i,p) y_p and the squared
//     row norms of A, and the staged B tile in LDS feeds the encoded row
//     checksums Pr_j += x_p B(p,j) and the squared column norms of B (one
//     column and a quarter of the p per thread);
//   * the encoding of C_in is fused into the beta pass of the epilogue, and
//     the reference checksums are summed from the accumulator registers
//     before anything is written;
//   * verify, locate, rebuild and confirm (one error, errors on one line, or
//     errors in distinct rows and columns); a tile whose disagreements fit
//     none of these is computed again by the same workgroup (C is not
//     written until the tile verifies).
// The weighted mode adds a weighted row checksum per column (weights i + 1)
// that locates and confirms corrections.
#include "ftgemm_device.h"
#include "ftgemm_kernels.h"

#include <type_traits>

namespace ftg {
namespace f64 {

constexpr int TM = 128, TN = 128, BK = 32;
constexpr int WM = 2, WN = 4, NW = WM * WN, NT = 64 * NW;  // 8 waves, 512 threads
constexpr int EPT = TM * BK / NT;  // staged elements per thread per operand (8)
constexpr int S = 145;  // LDS row stride in doubles (odd; 128 + one pad per 8)
constexpr double U = 1.1102230246251565e-16;  // 2^-53, unit roundoff of FP64

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64 operands and result, lane l = 16 q + c (q < 4, c < 16):
// A fragment holds A[c][q], B fragment holds B[q][c], and result register r
// holds D[4 r + q][c] (measured on gfx950).
//
// Wave w = wm + 2 wn holds rows 64 wm .. +63 and columns 32 wn .. +31 as
// acc[mi][ni][r] = C(64 wm + 16 mi + 4 r + q, 32 wn + 16 ni + c), mi < 4,
// ni < 2, r < 4.

// LDS column of tile index i: one pad slot after every 8, so lanes that each
// store 4 consecutive elements spread over the banks, while 16 lanes that
// read 16 consecutive elements stay conflict-free.
__device__ __forceinline__ int phys(int i) { return i + (i >> 3); }

struct Stage {
    double A[BK][S];  // A tile, [p][phys(i)]
    double B[BK][S];  // B tile, [p][phys(j)]
};

struct Epi {
    double ref_row[WN][TM], ref_col[WM][TN];    // partial sums of the output
    double cin_row[WN][TM], cin_col[WM][TN];    // partial sums of C_in
    double cin2_row[WN][TM], cin2_col[WM][TN];  // partial sums of squares of C_in
    double enc_row[NW][TM], enc_col[NW][TN];    // product part of the encoded checksums
    double nrm_row[NW][TM], nrm_col[NW][TN];    // squared norms of A's rows / B's columns
    double fin_row[TM], fin_col[TN];            // full encoded checksums
    double tau_row[TM], tau_col[TN];
    double d_row[TM], d_col[TN];
    // weighted mode: weighted row checksums of the columns (weights i + 1)
    double enc_colw[NT / TN][TN];               // product part, partials
    double ref_colw[WM][TN], cin_colw[WM][TN], cin2_colw[WM][TN];
    double fin_colw[TN], tau_colw[TN], d_colw[TN];
};

struct Smem {
    union {
        Stage st[2];
        Epi epi;
    } u;
    // [buffer][p][partial]: column sums of the A tile (weighted mode, A not
    // transposed: the weighted sum in slot 1)
    alignas(16) double xs[2][BK][NW];
    double ys[2][BK][NW];  // [buffer][p][partial]: row sums of the B tile
    double xws[2][BK][NW]; // weighted mode: weighted column sums of the A tile
    double red[NW][2];
    double vnrm[2][BK];    // x_p^2, y_p^2 summed over the steps (slot per p)
    double vnrmw[BK];      // weighted mode: x'_p^2 summed over the steps
    alignas(16) double xfin[BK][2];  // weighted mode, A transposed: x_p, x'_p of the step
    double scal[6];        // |x|^2, |y|^2, |A_I|_F^2, |B_J|_F^2, |W A_I|_F^2, |x'|^2
    TileFault faults[kMaxTileFaults];
    int nfaults;
    double wratio[4];      // largest |d| / tau of the waves that verify
    int nbad_r, nbad_c, ibad, jbad;
    int bad_r[kMaxLineFixes], bad_c[kMaxLineFixes];  // the first flagged entries, any order
};

// Fetches one step's part of a stored (column-major) operand: 8 elements per
// thread, all at the same inner index p.
//   kContig: the operand's outer index (i of A, j of B) runs along the stored
//     rows (A not transposed, B transposed); thread t takes p = t / 16 and the
//     8 consecutive outer indices 8 (t % 16) .. +7 (four 16-byte loads);
//   otherwise: the inner index runs along the stored rows; thread t takes
//     p = t % 32 and the outer indices t / 32 + 16 r (scalar loads; 32
//     consecutive lanes read 32 consecutive p).
// Fetches go through a buffer resource whose extent ends with the matrix, so
// what lies past its end reads as 0.
template <bool kContig>
struct OpLoader {
    const char *X;
    int64_t ld, R, total_bytes;  // stored rows R, leading dimension ld
    int t;

    __device__ __forceinline__ void init(const double *x, int64_t ld_, int64_t rows,
                                         int64_t cols, int t_)
    {
        X = (const char *)x;
        ld = ld_;
        R = rows;
        total_bytes = (rows > 0 && cols > 0) ? (ld_ * (cols - 1) + rows) * 8 : 0;
        t = t_;
    }
    // inner index and outer indices of this thread's elements
    __device__ __forceinline__ int p() const { return kContig ? (t >> 4) : (t & 31); }
    __device__ __forceinline__ int o(int r) const
    {
        return kContig ? 8 * (t & 15) + r : (t >> 5) + 16 * r;
    }
    // the step at inner offset k0 of the tile whose outer offset is o0
    __device__ __forceinline__ void load(int64_t o0, int64_t k0, int64_t nouter,
                                         double v[EPT]) const
    {
        // stored (row, col) of the tile's first element
        const int64_t r0 = kContig ? o0 : k0, c0 = kContig ? k0 : o0;
        const int64_t first = r0 + c0 * ld;
        int64_t ext = total_bytes - first * 8;
        if (ext < 0) ext = 0;
        if (ext > 0x7FFFFFFF) ext = 0x7FFFFFFF;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(X + first * 8, (uint64_t)ext);
        if (kContig) {
            const uint32_t off = (uint32_t)((8 * (t & 15) + (int64_t)(t >> 4) * ld) * 8);
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const auto w4 =
                    __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 16 * h), 0, 0);
                v[2 * h] = __hiloint2double(w4[1], w4[0]);
                v[2 * h + 1] = __hiloint2double(w4[3], w4[2]);
            }
            // outer indices past the matrix but inside the leading dimension
            if (o0 + 128 > nouter) {
#pragma unroll
                for (int r = 0; r < EPT; ++r)
                    if (o0 + o(r) >= nouter) v[r] = 0.0;
            }
        } else {
            const bool ok = r0 + (t & 31) < R;
            const uint32_t base =
                ok ? (uint32_t)(((t & 31) + (int64_t)(t >> 5) * ld) * 8) : kOob;
            const uint32_t step = (uint32_t)(16 * ld * 8);
#pragma unroll
            for (int r = 0; r < EPT; ++r)
                v[r] = buf_load_f64(rs, base + (uint32_t)r * step);
        }
    }
    // Sum of this thread's 8 elements, completed across the threads sharing
    // its p: the full tile sum for kContig (the 16 lanes of one DPP row), a
    // per-wave partial otherwise (lanes l and l^32).  The result goes to
    // dst[p][slot]: slot 0 for kContig, the wave index otherwise.
    // Returns what this thread summed (for kContig, every thread of the p
    // has the full sum).
    __device__ __forceinline__ double sum_to(const double v[EPT], double (*dst)[NW]) const
    {
        double s = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
        if (kContig) {
            s = sum16(s);
            if ((t & 15) == 0) dst[t >> 4][0] = s;
        } else {
            s = pair_sum32(s);
            if ((t & 63) < 32) dst[t & 31][t >> 6] = s;
        }
        return s;
    }
    // The same with every element weighted by its outer index + 1 (the
    // weighted mode's x'_p = sum_i (i + 1) A(i, p)), into slot `slot` for
    // kContig (slot 1 sits beside x_p, so one read fetches both).
    __device__ __forceinline__ double wsum_to(const double v[EPT], double (*dst)[NW],
                                              int slot) const
    {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < EPT; ++r) s = fma((double)(o(r) + 1), v[r], s);
        if (kContig) {
            s = sum16(s);
            if ((t & 15) == 0) dst[t >> 4][slot] = s;
        } else {
            s = pair_sum32(s);
            if ((t & 63) < 32) dst[t & 31][t >> 6] = s;
        }
        return s;
    }
    // Per-outer-index partials accumulated by this thread over the steps,
    // completed across the threads that hold the same outer indices (the
    // other p), into dst[slot][outer]: 8 slots (one per wave) for kContig,
    // slot 0 otherwise.
    template <typename T>
    __device__ __forceinline__ void partials_to(const T a_in[EPT], double (*dst)[128]) const
    {
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            double a = (double)a_in[r];
            if (kContig) {
                a = sum_rows(a);
                if ((t & 48) == 0) dst[t >> 6][o(r)] = a;
            } else {
                a = pair_sum16(sum16(a));
                if ((t & 31) == 0) dst[0][o(r)] = a;
            }
        }
    }
    // the thread that accounts for p in |x|^2 / |y|^2
    __device__ __forceinline__ bool first_of_p() const
    {
        return kContig ? (t & 15) == 0 : t < 32;
    }
    static constexpr int kParts = kContig ? 1 : NW;      // partials of x_p / y_p
    static constexpr int kOuterParts = kContig ? NW : 1;  // partials per outer index
};

template <int kParts>
__device__ __forceinline__ double gather(const double (*src)[NW], int p)
{
    if (kParts == 1) return src[p][0];
    return ((src[p][0] + src[p][1]) + (src[p][2] + src[p][3])) +
           ((src[p][4] + src[p][5]) + (src[p][6] + src[p][7]));
}

// C_in for the beta pass, read through a buffer resource that starts at the
// tile and ends with C, so what lies past C's last element reads as 0; rows
// and columns past the tile's own inside C are read and must be dropped by
// the caller.  Offsets are 32-bit: the host limits ldc so that a tile spans
// less than 2 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t cin_rsrc(const double *C, int64_t ldc,
                                                           int64_t m, int64_t n, int64_t i0,
                                                           int64_t j0)
{
    const int64_t first = i0 + j0 * ldc;
    int64_t ext = (ldc * (n - 1) + m - first) * 8;
    if (ext < 0) ext = 0;
    if (ext > 0x7FFFFFFF) ext = 0x7FFFFFFF;
    return make_rsrc(C + first, (uint64_t)ext);
}

// The C_in elements under this thread's accumulators of row group mi (acc
// layout).  The beta passes fetch group mi + 1 before they work on group mi,
// so one group's wait overlaps the previous group's work.
__device__ __forceinline__ void load_cin(__amdgpu_buffer_rsrc_t rs, int64_t ldc, int mi, int wm,
                                         int wn, int q, int c16, double cv[2][4])
{
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = wm * 64 + 16 * mi + 4 * r + q;
            const int col = wn * 32 + 16 * ni + c16;
            cv[ni][r] = buf_load_f64(rs, (uint32_t)((row + (int64_t)col * ldc) * 8));
        }
}

// owner of tile element (row, col): wave, lane and flat register index
__device__ __forceinline__ int owner_wave(int row, int col) { return (row >> 6) + 2 * (col >> 5); }
__device__ __forceinline__ int owner_lane(int row, int col) { return 16 * (row & 3) + (col & 15); }
__device__ __forceinline__ int owner_reg(int row, int col)
{
    return ((row & 63) >> 4) * 8 + ((col & 31) >> 4) * 4 + ((row & 15) >> 2);
}

// WGT (with ABFT): the weighted mode -- a weighted row checksum per column
// (weights i + 1 over the tile's rows) locates and confirms corrections.
template <bool TA, bool TB, bool ABFT, bool WGT = false>
__device__ __forceinline__ void tile(const GemmArgs &g, int tile_m, int tile_n, Smem &sm)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int q = lane >> 4, c16 = lane & 15;
    const int64_t i0 = (int64_t)tile_m * TM, j0 = (int64_t)tile_n * TN;
    double *__restrict__ C = (double *)g.C;
    const int64_t m = g.m, n = g.n, k = g.k, ldc = g.ldc;
    const int nsteps = (int)((k + BK - 1) / BK);
    const int hrows = (int)(m - i0 < TM ? m - i0 : TM);
    const int wcols = (int)(n - j0 < TN ? n - j0 : TN);
    const bool use_c = g.beta != 0.0;

    // A not transposed: its rows (i) run along the stored rows (contiguous);
    // B transposed: its columns (j) do.
    OpLoader<!TA> la;
    OpLoader<TB> lb;
    // x_p (and x'_p) left as wave partials (A transposed): finished once
    // per step behind a second barrier, for the B-side sums read from LDS
    constexpr bool kFinish = ABFT && OpLoader<!TA>::kParts > 1;
    la.init((const double *)g.A, g.lda, TA ? k : m, TA ? m : k, t);
    lb.init((const double *)g.B, g.ldb, TB ? n : k, TB ? k : n, t);
    // Staged operand registers of one step.
    double ra[EPT], rb[EPT];
    auto load = [&](int s) {
        const int64_t k0 = (int64_t)s * BK;
        la.load(i0, k0, m, ra);
        lb.load(j0, k0, n, rb);
    };
    auto store = [&](int buf) {
        const int a_p = la.p(), b_p = lb.p();
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            sm.u.st[buf].A[a_p][phys(la.o(r))] = ra[r];
            sm.u.st[buf].B[b_p][phys(lb.o(r))] = rb[r];
        }
    };
    // (A not transposed: the squares of the step's x_p and, in the
    // weighted mode, x'_p of this thread's p go into vx, vxw)
    auto sums = [&](int buf, float &vx, float &vxw) {
        const double x = la.sum_to(ra, sm.xs[buf]);
        if (!kFinish) {
            const float fx = (float)x;
            vx = fmaf(fx, fx, vx);
        }
        if (WGT) {
            const double xw = kFinish ? la.wsum_to(ra, sm.xws[buf], 0)
                                      : la.wsum_to(ra, sm.xs[buf], 1);
            if (!kFinish) {
                const float fw = (float)xw;
                vxw = fmaf(fw, fw, vxw);
            }
        }
        lb.sum_to(rb, sm.ys[buf]);
    };

    // Planned faults of this tile (test hook).
    int nf = 0;
    if (ABFT) {
        if (w == 0) {
            const int cnt = gather_tile_faults(g, i0, j0, TM, TN, BK, g.k_base, sm.faults);
            if (lane == 0) sm.nfaults = cnt;
        }
        __syncthreads();
        nf = sm.nfaults;
    }

    int kind = 0, first_nr = 0, first_nc = 0, first_i = -1, first_j = -1;
    int npairs = 0;  // corrections left for the stored tile
    double rec_before = 0, rec_after = 0;

    d4 acc[4][2];
#pragma unroll 1
    for (int attempt = 0; attempt < 2; ++attempt) {
        const bool faults_on = ABFT && attempt == 0 && nf > 0;
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni)
                acc[mi][ni] = (d4){0.0, 0.0, 0.0, 0.0};
        // Checksum partials over the steps.  The A side comes from the
        // staged registers: this thread's 8 rows of A (A . y and the squared
        // row norms).  The B side comes from the staged B tile in LDS, one
        // register per sum instead of one per staged element: thread t
        // covers column j = t mod 128 and a quarter of each step's p, and
        // sums x_p B(p, j) (x'_p B(p, j) in the weighted mode) and B(p, j)^2.
        // The norms only scale the rounding-error threshold: the A side
        // squares its FP32-rounded values in FP32 (half the registers of one
        // double per staged element), the B side, one register in all, takes
        // one FP64 fma per element.
        double enc_a[EPT] = {}, enc_b = 0.0, enc_w = 0.0, nrm_b = 0.0;
        float nrm_a[EPT] = {};
        float vx = 0.0f, vy = 0.0f;  // x_p^2, y_p^2 over the steps
        float vxw = 0.0f;            // weighted mode: x'_p^2

        load(0);
        if (ABFT) sums(0, vx, vxw);
        if constexpr (!ABFT) {
            // Checksum-free steps: those with a next step, then the last one,
            // which fetches the beta pass's first two row groups of C_in into
            // the free operand registers instead (measured faster for this
            // kernel; the fault-tolerant loop below measured slower with the
            // same split).
            auto pstep = [&](const int s, auto last) {
                constexpr bool kLast = decltype(last)::value;
                const int buf = s & 1;
                store(buf);
                __syncthreads();
#pragma unroll
                for (int kk = 0; kk < BK / 4; ++kk) {
                    if (kk == 0) {
                        if constexpr (!kLast) {
                            load(s + 1);
                        } else if (use_c) {
                            const __amdgpu_buffer_rsrc_t crs = cin_rsrc(C, ldc, m, n, i0, j0);
                            load_cin(crs, ldc, 0, wm, wn, q, c16,
                                     reinterpret_cast<double (*)[4]>(ra));
                            load_cin(crs, ldc, 1, wm, wn, q, c16,
                                     reinterpret_cast<double (*)[4]>(rb));
                        }
                    }
                    double fa[4], fb[2];
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
                        fa[mi] = sm.u.st[buf].A[4 * kk + q][phys(wm * 64 + 16 * mi + c16)];
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni)
                        fb[ni] = sm.u.st[buf].B[4 * kk + q][phys(wn * 32 + 16 * ni + c16)];
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                        for (int ni = 0; ni < 2; ++ni)
                            acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                fa[mi], fb[ni], acc[mi][ni], 0, 0, 0);
                }
            };
#pragma unroll 1
            for (int s = 0; s < nsteps - 1; ++s) pstep(s, std::false_type{});
            if (nsteps > 0) pstep(nsteps - 1, std::true_type{});
        } else {
            // The steps run in segments that end where a planned fault lands, so
            // the fault hook sits outside the hot loop.
            int s = 0;
#pragma unroll 1
            while (s < nsteps) {
                int stop = nsteps - 1;
                if (faults_on)
                    for (int f = 0; f < nf; ++f) {
                        const int fs = sm.faults[f].kstep;
                        if (sm.faults[f].target == FTGEMM_TGT_ACC && fs >= s && fs < stop)
                            stop = fs;
                    }
#pragma unroll 1
                for (; s <= stop; ++s) {
                    const int buf = s & 1;
                    store(buf);
                    __syncthreads();
                    if constexpr (kFinish) {
                        // x_p and x'_p of the step summed once from their wave
                        // partials (each thread reads eight p per step)
                        if (t < BK) {
                            const double x = gather<NW>(sm.xs[buf], t);
                            sm.xfin[t][0] = x;
                            const float fx = (float)x;
                            vx = fmaf(fx, fx, vx);
                            if (WGT) {
                                const double xw = gather<NW>(sm.xws[buf], t);
                                sm.xfin[t][1] = xw;
                                const float fw = (float)xw;
                                vxw = fmaf(fw, fw, vxw);
                            }
                        }
                        __syncthreads();
                    }
                    // x_p, y_p of step s are complete; their gather is issued
                    // here and used after the step's first products.  In the
                    // weighted mode, waves 4-7 encode, and fetch the next
                    // step, three sub-steps after waves 0-3, so that the
                    // vector work of the two waves a SIMD holds (waves dealt
                    // round-robin) does not coincide (measured: 14% faster
                    // there; the plain two-sided mode measured 1% slower
                    // with it at 8192^3).
                    const int enc_kk =
                        WGT && __builtin_amdgcn_readfirstlane(threadIdx.x >> 8) ? 4 : 1;
                    double yv = 0.0;
                    if (ABFT) yv = gather<OpLoader<TB>::kParts>(sm.ys[buf], la.p());
#pragma unroll
                    for (int kk = 0; kk < BK / 4; ++kk) {
                        if (kk == (ABFT ? enc_kk : 0)) {
                            if (ABFT) {
                                // the encoded checksums and norms of step s,
                                // before ra/rb take step s + 1
#pragma unroll
                                for (int r = 0; r < EPT; ++r) {
                                    enc_a[r] += ra[r] * yv;
                                    // squares of the FP32-rounded values: two
                                    // instructions (convert, FP32 fma)
                                    const float fa = (float)ra[r];
                                    nrm_a[r] = fmaf(fa, fa, nrm_a[r]);
                                }
                                const float fy = (float)yv;
                                vy = fmaf(fy, fy, vy);
                            }
                            if (s + 1 < nsteps) load(s + 1);
                        }
                        if (ABFT) {
                            // the B side: one p of this thread's quarter per
                            // sub-step (x_p and x'_p read together)
                            const int pw = (t / TN) * (BK / 4) + kk;
                            const double bv = sm.u.st[buf].B[pw][phys(t & (TN - 1))];
                            const double2 xq = *reinterpret_cast<const double2 *>(
                                kFinish ? &sm.xfin[pw][0] : &sm.xs[buf][pw][0]);
                            enc_b = fma(xq.x, bv, enc_b);
                            if (WGT) enc_w = fma(xq.y, bv, enc_w);
                            nrm_b = fma(bv, bv, nrm_b);
                        }
                        double fa[4], fb[2];
#pragma unroll
                        for (int mi = 0; mi < 4; ++mi)
                            fa[mi] = sm.u.st[buf].A[4 * kk + q][phys(wm * 64 + 16 * mi + c16)];
#pragma unroll
                        for (int ni = 0; ni < 2; ++ni)
                            fb[ni] = sm.u.st[buf].B[4 * kk + q][phys(wn * 32 + 16 * ni + c16)];
#pragma unroll
                        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                            for (int ni = 0; ni < 2; ++ni)
                                acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                    fa[mi], fb[ni], acc[mi][ni], 0, 0, 0);
                        if (ABFT && kk == BK / 4 - 1 && s + 1 < nsteps) {
                            // operand checksums of step s + 1, published before
                            // its barrier
                            sums(buf ^ 1, vx, vxw);
                        }
                    }
                }
                if (ABFT && faults_on) {
                    // Fault hook: accumulator faults land after step `stop`.
                    for (int f = 0; f < nf; ++f) {
                        const TileFault tf = sm.faults[f];
                        if (tf.target != FTGEMM_TGT_ACC || tf.kstep != stop) continue;
                        if (w != owner_wave(tf.row, tf.col)) continue;
                        const int ol = owner_lane(tf.row, tf.col), sel = owner_reg(tf.row, tf.col);
                        double before = 0.0;
#pragma unroll
                        for (int e = 0; e < 32; ++e)
                            if (sel == e) before = acc[e >> 3][(e >> 2) & 1][e & 3];
                        const double after = tf.mode == FTGEMM_INJ_ADD ? before + tf.delta
                                                                       : flip_bit_f64(before, tf.bit);
#pragma unroll
                        for (int e = 0; e < 32; ++e)
                            if (sel == e && lane == ol) acc[e >> 3][(e >> 2) & 1][e & 3] = after;
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
        // From here on the lane-derived indices are formed again instead of
        // being carried across the main loop.
        const int t = fresh_tid(), lane = t & 63, w = t >> 6;
        const int wm = w & 1, wn = w >> 1, q = lane >> 4, c16 = lane & 15;
        la.t = t;
        lb.t = t;

        if (!ABFT) {
            // Plain GEMM epilogue: the beta pass and the store.
            // row groups 0 and 1 of C_in arrived in the operand registers;
            // 2 and 3 are fetched while the first two are written
            const __amdgpu_buffer_rsrc_t crs = cin_rsrc(C, ldc, m, n, i0, j0);
            double c2[2][4] = {}, c3[2][4] = {};
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
                if (use_c && mi < 2) load_cin(crs, ldc, mi + 2, wm, wn, q, c16, mi ? c3 : c2);
                const double (*cn)[4] = mi == 0   ? reinterpret_cast<const double (*)[4]>(ra)
                                        : mi == 1 ? reinterpret_cast<const double (*)[4]>(rb)
                                        : mi == 2 ? c2
                                                  : c3;
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm * 64 + 16 * mi + 4 * r + q;
                        const int col = wn * 32 + 16 * ni + c16;
                        if (row < hrows && col < wcols) {
                            const double o = g.alpha * acc[mi][ni][r];
                            C[(i0 + row) + (j0 + col) * ldc] =
                                use_c ? o + g.beta * cn[ni][r] : o;
                        }
                    }
            }
            return;
        }

        // The first row group of C_in is on its way while the partials are
        // published.
        const __amdgpu_buffer_rsrc_t crs = cin_rsrc(C, ldc, m, n, i0, j0);
        double cn[2][4] = {}, cx[2][4] = {};
        if (use_c) load_cin(crs, ldc, 0, wm, wn, q, c16, cn);

        // Publish the per-thread partials: rows of A from the A loader (the
        // other p completed in lanes); columns of B, one partial per quarter
        // of p.  The y_p gathered by the A loader's threads is the same for
        // every thread of a p: one thread per p accounts for it, and the
        // squares of x_p (x'_p) come from the threads that summed them, one
        // per p.
        la.partials_to(enc_a, sm.u.epi.enc_row);
        la.partials_to(nrm_a, sm.u.epi.nrm_row);
        if (la.first_of_p()) sm.vnrm[1][la.p()] = (double)vy;
        {
            const int jw = t & (TN - 1), qw = t / TN;
            sm.u.epi.enc_col[qw][jw] = enc_b;
            sm.u.epi.nrm_col[qw][jw] = nrm_b;
            if (WGT) sm.u.epi.enc_colw[qw][jw] = enc_w;
            const bool own = kFinish ? t < BK : la.first_of_p();
            const int pv = kFinish ? t : la.p();
            if (own) {
                sm.vnrm[0][pv] = (double)vx;
                if (WGT) sm.vnrmw[pv] = (double)vxw;
            }
        }

        // Beta pass fused with the C_in part of the encoding (Section 2.2)
        // and the reference sums of the output.
        // (row group mi + 1 of C_in is fetched while group mi is summed)
        double col_o[2] = {0, 0}, col_c[2] = {0, 0}, col_c2[2] = {0, 0};
        // weighted mode: the same column sums with row weights i + 1
        double col_ow[WGT ? 2 : 1] = {}, col_cw[WGT ? 2 : 1] = {}, col_cw2[WGT ? 2 : 1] = {};
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            if (use_c && mi + 1 < 4) load_cin(crs, ldc, mi + 1, wm, wn, q, c16, cx);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double row_o = 0, row_c = 0, row_c2 = 0;
                const int row = wm * 64 + 16 * mi + 4 * r + q;
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    const int col = wn * 32 + 16 * ni + c16;
                    const bool ok = row < hrows && col < wcols;
                    const double cin = (use_c && ok) ? cn[ni][r] : 0.0;
                    double o = g.alpha * acc[mi][ni][r];
                    if (use_c) o = o + g.beta * cin;
                    o = ok ? o : 0.0;
                    acc[mi][ni][r] = o;
                    row_o += o; row_c += cin; row_c2 += cin * cin;
                    col_o[ni] += o; col_c[ni] += cin; col_c2[ni] += cin * cin;
                    if (WGT) {
                        const double wr = (double)(row + 1), cw = wr * cin;
                        col_ow[ni] += wr * o; col_cw[ni] += cw; col_cw2[ni] += cw * cw;
                    }
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
            for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                for (int r = 0; r < 4; ++r) cn[ni][r] = cx[ni][r];
        }
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            col_o[ni] = sum_rows(col_o[ni]);
            if (use_c) { col_c[ni] = sum_rows(col_c[ni]); col_c2[ni] = sum_rows(col_c2[ni]); }
            if (q == 0) {
                const int col = wn * 32 + 16 * ni + c16;
                sm.u.epi.ref_col[wm][col] = col_o[ni];
                sm.u.epi.cin_col[wm][col] = col_c[ni];
                sm.u.epi.cin2_col[wm][col] = col_c2[ni];
            }
            if (WGT) {
                col_ow[ni] = sum_rows(col_ow[ni]);
                if (use_c) {
                    col_cw[ni] = sum_rows(col_cw[ni]);
                    col_cw2[ni] = sum_rows(col_cw2[ni]);
                }
                if (q == 0) {
                    const int col = wn * 32 + 16 * ni + c16;
                    sm.u.epi.ref_colw[wm][col] = col_ow[ni];
                    sm.u.epi.cin_colw[wm][col] = col_cw[ni];
                    sm.u.epi.cin2_colw[wm][col] = col_cw2[ni];
                }
            }
        }
        if (t == 0) { sm.nbad_r = 0; sm.nbad_c = 0; sm.ibad = TM; sm.jbad = TN; }
        __syncthreads();

        // Combine the partials in a fixed order: row i (its encoded checksum
        // and squared norm) in thread i, column j in thread 128 + j.
        const bool is_row = t < TM, is_col = t >= TM && t < TM + TN;
        const int x = is_row ? t : t - TM;
        double nrm2 = 0.0;
        if (is_row) {
            double e = 0, nr = 0;
#pragma unroll
            for (int v = 0; v < OpLoader<!TA>::kOuterParts; ++v) {
                e += sm.u.epi.enc_row[v][x];
                nr += sm.u.epi.nrm_row[v][x];
            }
            nrm2 = nr;
            sm.u.epi.fin_row[x] = e;
        } else if (is_col) {
            double e = 0, nr = 0, ew = 0;
            constexpr int parts = NT / TN;
#pragma unroll
            for (int v = 0; v < parts; ++v) {
                e += sm.u.epi.enc_col[v][x];
                nr += sm.u.epi.nrm_col[v][x];
                if (WGT) ew += sm.u.epi.enc_colw[v][x];
            }
            nrm2 = nr;
            sm.u.epi.fin_col[x] = e;
            if (WGT) sm.u.epi.fin_colw[x] = ew;
        }
        // Frobenius norms of the A and B tiles (waves 0-1 and 2-3), |x|, |y|;
        // weighted mode: |W A_I|_F (rows weighted by i + 1) and |x'|
        if (w < 4) {
            const double f = sum64(nrm2);
            if (lane == 0) sm.red[w][0] = f;
            if (WGT && w < 2) {
                const double wx = (double)(x + 1), fw = sum64(wx * wx * nrm2);
                if (lane == 0) sm.red[w][1] = fw;
            }
        }
        if (w == 4) {
            const double v2 = pair_sum16(sum16(sm.vnrm[lane >> 5][lane & 31]));
            if ((lane & 31) == 0) sm.red[4 + (lane >> 5)][0] = v2;
        }
        if (WGT && w == 5) {
            const double v2 = sum64(lane < BK ? sm.vnrmw[lane] : 0.0);
            if (lane == 0) sm.red[6][0] = v2;
        }
        __syncthreads();
        if (t == 0) {
            sm.scal[2] = sm.red[0][0] + sm.red[1][0];  // |A_I|_F^2
            sm.scal[3] = sm.red[2][0] + sm.red[3][0];  // |B_J|_F^2
            sm.scal[0] = sm.red[4][0];                 // |x|^2
            sm.scal[1] = sm.red[5][0];                 // |y|^2
            if (WGT) {
                sm.scal[4] = sm.red[0][1] + sm.red[1][1];  // |W A_I|_F^2
                sm.scal[5] = sm.red[6][0];                 // |x'|^2
            }
        }
        __syncthreads();

        // Verify: thread t < 128 checks row t, threads 128..255 column t - 128.
        {
            const double sqk = sqrt((double)k);
            double ratio = 0.0;
            if (is_row || is_col) {
                double P = g.alpha * (is_row ? sm.u.epi.fin_row[x] : sm.u.epi.fin_col[x]);
                double R = 0.0, cs = 0.0, c2 = 0.0;
                if (is_row) {
#pragma unroll
                    for (int v = 0; v < WN; ++v) {
                        R += sm.u.epi.ref_row[v][x];
                        cs += sm.u.epi.cin_row[v][x];
                        c2 += sm.u.epi.cin2_row[v][x];
                    }
                } else {
                    R = sm.u.epi.ref_col[0][x] + sm.u.epi.ref_col[1][x];
                    cs = sm.u.epi.cin_col[0][x] + sm.u.epi.cin_col[1][x];
                    c2 = sm.u.epi.cin2_col[0][x] + sm.u.epi.cin2_col[1][x];
                }
                if (use_c) P += g.beta * cs;
                if (faults_on)
                    for (int f = 0; f < nf; ++f) {
                        const TileFault tf = sm.faults[f];
                        const bool hit = is_row
                            ? (tf.target == FTGEMM_TGT_COL_CHECKSUM && tf.row == x)
                            : (tf.target == FTGEMM_TGT_ROW_CHECKSUM && tf.col == x);
                        if (hit) {
                            ftgemm_injection_echo e;
                            e.problem = g.problem; e.applied = 1; e.row = i0 + tf.row;
                            e.col = j0 + tf.col; e.k_index = g.plan[tf.idx].k_index;
                            e.before = P; P += tf.delta; e.after = P;
                            g.echo[tf.idx] = e;
                        }
                    }
                // row i: norm of A's row i, Frobenius norm of the B tile and
                // |y|, summed over the tile's columns; column j symmetrically
                const double tau = is_row
                    ? ft_threshold(kLambda, U, sqk, sqrt((double)wcols), g.alpha, sqrt(nrm2),
                                   sqrt(sm.scal[3]), sqrt(sm.scal[1]), g.beta, sqrt(c2))
                    : ft_threshold(kLambda, U, sqk, sqrt((double)hrows), g.alpha, sqrt(nrm2),
                                   sqrt(sm.scal[2]), sqrt(sm.scal[0]), g.beta, sqrt(c2));
                const double d = R - P;
                if (is_row) {
                    sm.u.epi.fin_row[x] = P; sm.u.epi.tau_row[x] = tau; sm.u.epi.d_row[x] = d;
                } else {
                    sm.u.epi.fin_col[x] = P; sm.u.epi.tau_col[x] = tau; sm.u.epi.d_col[x] = d;
                }
                if (WGT && is_col) {
                    // weighted row checksum of column x and its threshold:
                    // the column's bound with A_I, x and C_in(:, x) weighted
                    double Pw = g.alpha * sm.u.epi.fin_colw[x];
                    const double Rw = sm.u.epi.ref_colw[0][x] + sm.u.epi.ref_colw[1][x];
                    const double cw2 = sm.u.epi.cin2_colw[0][x] + sm.u.epi.cin2_colw[1][x];
                    if (use_c) Pw += g.beta * (sm.u.epi.cin_colw[0][x] + sm.u.epi.cin_colw[1][x]);
                    if (faults_on)
                        for (int f = 0; f < nf; ++f) {
                            const TileFault tf = sm.faults[f];
                            if (tf.target != FTGEMM_TGT_WEIGHTED_CHECKSUM || tf.col != x) continue;
                            ftgemm_injection_echo e;
                            e.problem = g.problem; e.applied = 1; e.row = i0 + tf.row;
                            e.col = j0 + tf.col; e.k_index = g.plan[tf.idx].k_index;
                            e.before = Pw; Pw += tf.delta; e.after = Pw;
                            g.echo[tf.idx] = e;
                        }
                    sm.u.epi.fin_colw[x] = Pw;
                    sm.u.epi.tau_colw[x] =
                        ft_threshold(kLambda, U, sqk, sqrt((double)hrows), g.alpha, sqrt(nrm2),
                                     sqrt(sm.scal[4]), sqrt(sm.scal[5]), g.beta, sqrt(cw2));
                    sm.u.epi.d_colw[x] = Rw - Pw;
                }
                if (x < (is_row ? hrows : wcols)) {
                    if (!(fabs(d) <= tau)) {
                        const int slot = atomicAdd(is_row ? &sm.nbad_r : &sm.nbad_c, 1);
                        if (slot < kMaxLineFixes) (is_row ? sm.bad_r : sm.bad_c)[slot] = x;
                        atomicMin(is_row ? &sm.ibad : &sm.jbad, x);
                    } else if (tau > 0.0) {
                        ratio = fabs(d) / tau;
                    }
                }
            }
            if (w < 4) {
                ratio = max64(ratio);
                if (lane == 0) sm.wratio[w] = ratio;
            }
        }
        __syncthreads();
        if (t == 0)
            atomic_max_nonneg(&g.counters->max_ratio_bits,
                              fmax(fmax(sm.wratio[0], sm.wratio[1]),
                                   fmax(sm.wratio[2], sm.wratio[3])));

        const int nr = sm.nbad_r, nc = sm.nbad_c;
        if (nr == 0 && nc == 0) {
            if (attempt == 1) kind = FTGEMM_KIND_RECOMPUTED;
            break;
        }
        if (attempt == 1) {
            kind = FTGEMM_KIND_UNCORRECTABLE;
            break;
        }
        // First attempt disagreed: keep what the record needs (the residuals
        // and thresholds stay in LDS until the record is written, unless the
        // tile is computed again).
        first_nr = nr; first_nc = nc;
        first_i = nr ? sm.ibad : -1;
        first_j = nc ? sm.jbad : -1;

        if (nr == 1 && nc == 1) {
            // Locate at the crossing; rebuild from the encoded checksum of
            // its column and the rest of the column (robust to Inf / NaN in
            // the faulty element); confirm with the rest of its row.
            const int is = first_i, js = first_j;
            double s_col = 0.0, s_row = 0.0;
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm * 64 + 16 * mi + 4 * r + q;
                        const int col = wn * 32 + 16 * ni + c16;
                        const double o = acc[mi][ni][r];
                        if (col == js && row != is) s_col += o;
                        if (row == is && col != js) s_row += o;
                    }
            s_col = sum64(s_col);
            s_row = sum64(s_row);
            if (lane == 0) { sm.red[w][0] = s_col; sm.red[w][1] = s_row; }
            __syncthreads();
            double sc = 0.0, sr = 0.0;
#pragma unroll
            for (int v = 0; v < NW; ++v) { sc += sm.red[v][0]; sr += sm.red[v][1]; }
            const double fixed = sm.u.epi.fin_col[js] - sc;
            // weighted mode: a finite error at (is, js) shows as is + 1 times
            // the column's residual on its weighted checksum
            bool wok = true;
            if (WGT) {
                const double dc = sm.u.epi.d_col[js], dw = sm.u.epi.d_colw[js];
                wok = !isfinite(dc) || !isfinite(dw) ||
                      fabs(dw - (double)(is + 1) * dc) <=
                          sm.u.epi.tau_colw[js] + (double)(is + 1) * sm.u.epi.tau_col[js];
            }
            if (wok && fabs(sr + fixed - sm.u.epi.fin_row[is]) <= sm.u.epi.tau_row[is]) {
                if (w == owner_wave(is, js)) {
                    const int ol = owner_lane(is, js), sel = owner_reg(is, js);
#pragma unroll
                    for (int e = 0; e < 32; ++e)
                        if (sel == e && lane == ol) {
                            rec_before = acc[e >> 3][(e >> 2) & 1][e & 3];
                            acc[e >> 3][(e >> 2) & 1][e & 3] = fixed;
                        }
                }
                rec_after = fixed;
                kind = FTGEMM_KIND_CORRECTED;
                break;
            }
        } else if ((nr == 1 && nc >= 2 && nc <= kMaxLineFixes) ||
                   (nc == 1 && nr >= 2 && nr <= kMaxLineFixes)) {
            // Several errors on one line: the flagged row (or column).  Each
            // element where it crosses a flagged entry of the other side
            // loses that entry's residual (the classical ABFT correction),
            // and the line is confirmed by its own residual, which after the
            // corrections is d_line - sum of the crossing residuals.  A
            // residual that is not finite cannot be subtracted: the line
            // fails to confirm and the tile is computed again.
            const bool by_row = nr == 1;
            const int line = by_row ? first_i : first_j;
            const int nfix = by_row ? nc : nr;
            double sumd = 0.0;
#pragma unroll
            for (int f = 0; f < kMaxLineFixes; ++f)
                if (f < nfix)
                    sumd += by_row ? sm.u.epi.d_col[sm.bad_c[f]] : sm.u.epi.d_row[sm.bad_r[f]];
            const double dl = by_row ? sm.u.epi.d_row[line] : sm.u.epi.d_col[line];
            // weighted mode: along a row, each flagged column shows line + 1
            // times its residual on its weighted checksum; along a column,
            // the column's weighted residual is the weighted sum of the
            // flagged rows' residuals
            bool wok = true;
            if (WGT) {
                if (by_row) {
                    const double wl = (double)(line + 1);
#pragma unroll
                    for (int f = 0; f < kMaxLineFixes; ++f)
                        if (f < nfix) {
                            const int xc = sm.bad_c[f];
                            if (!(fabs(sm.u.epi.d_colw[xc] - wl * sm.u.epi.d_col[xc]) <=
                                  sm.u.epi.tau_colw[xc] + wl * sm.u.epi.tau_col[xc]))
                                wok = false;
                        }
                } else {
                    double sw = 0.0, tsum = sm.u.epi.tau_colw[line];
#pragma unroll
                    for (int f = 0; f < kMaxLineFixes; ++f)
                        if (f < nfix) {
                            const int xr = sm.bad_r[f];
                            sw += (double)(xr + 1) * sm.u.epi.d_row[xr];
                            tsum += (double)(xr + 1) * sm.u.epi.tau_row[xr];
                        }
                    wok = fabs(sm.u.epi.d_colw[line] - sw) <= tsum;
                }
            }
            if (wok &&
                fabs(dl - sumd) <= (by_row ? sm.u.epi.tau_row[line] : sm.u.epi.tau_col[line])) {
                // each crossing's residual at its position along the line
                // (the encoded-sum partials are no longer needed)
                double *lfix = sm.u.epi.enc_row[0];
                for (int x = t; x < (by_row ? TN : TM); x += NT) lfix[x] = 0.0;
                __syncthreads();
                if (t < nfix) {
                    const int cf = by_row ? sm.bad_c[t] : sm.bad_r[t];
                    lfix[cf] = by_row ? sm.u.epi.d_col[cf] : sm.u.epi.d_row[cf];
                }
                __syncthreads();
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = wm * 64 + 16 * mi + 4 * r + q;
                            const int col = wn * 32 + 16 * ni + c16;
                            if ((by_row ? row : col) != line) continue;
                            const int at = by_row ? col : row;
                            const double d = lfix[at];
                            if (d == 0.0) continue;
                            const bool named = at == (by_row ? first_j : first_i);
                            if (named) rec_before = acc[mi][ni][r];
                            acc[mi][ni][r] -= d;
                            if (named) rec_after = acc[mi][ni][r];
                        }
                kind = FTGEMM_KIND_CORRECTED;
                break;
            }
        } else if (nr == nc && nr >= 2 && nr <= kMaxLineFixes) {
            // Errors in distinct rows and columns: each flagged row is paired
            // with the one flagged column whose residual agrees with its own
            // within the two thresholds; a one-to-one pairing is corrected
            // (each crossing loses its column's residual), anything else is
            // computed again.  The pairs go to a table by row in LDS (the
            // encoded-sum partials are no longer needed); the lanes that
            // hold the elements apply them to the stored tile (see below),
            // which keeps this rare path off the registers of the others.
            int *pcol = reinterpret_cast<int *>(sm.u.epi.enc_row[1]);
            double *pd = sm.u.epi.enc_row[0];
            if (WGT && t == 0) {
                // Weighted mode: each flagged column finds its error's row
                // from the ratio of its weighted to its plain residual
                // (row + 1); that row must be flagged, found once, carry the
                // same residual, and the weighted residual must fit.  Equal
                // errors need no pairing by size; two errors in one column
                // give a ratio that fits no row.
                bool ok = true;
                unsigned taken = 0;
                for (int b = 0; b < nc && ok; ++b) {
                    const int j = sm.bad_c[b];
                    const double dc = sm.u.epi.d_col[j], dw = sm.u.epi.d_colw[j];
                    const double ratio = dw / dc;
                    int a = -1, r = -1;
                    if (isfinite(dc) && isfinite(ratio)) {
                        const double rr = round(ratio);
                        if (rr >= 1.0 && rr <= (double)TM) r = (int)rr - 1;
                    }
                    for (int q2 = 0; q2 < nr; ++q2)
                        if (r >= 0 && sm.bad_r[q2] == r) a = q2;
                    if (a < 0 || ((taken >> a) & 1u)) { ok = false; break; }
                    const double wr = (double)(r + 1);
                    if (!(fabs(dw - wr * dc) <= sm.u.epi.tau_colw[j] + wr * sm.u.epi.tau_col[j]) ||
                        !(fabs(sm.u.epi.d_row[r] - dc) <= sm.u.epi.tau_row[r] + sm.u.epi.tau_col[j])) {
                        ok = false;
                        break;
                    }
                    taken |= 1u << a;
                    pcol[r] = j;
                    pd[r] = dc;
                }
                sm.red[3][0] = (double)(ok ? pcol[first_i] : -1);
            } else if (t == 0) {
                unsigned taken = 0;
                int named = -1;
                for (int a = 0; a < nr; ++a) {
                    const int i = sm.bad_r[a];
                    int found = 0, mate = 0, mb = 0;
                    for (int b = 0; b < nc; ++b) {
                        const int j = sm.bad_c[b];
                        if (fabs(sm.u.epi.d_row[i] - sm.u.epi.d_col[j]) <=
                            sm.u.epi.tau_row[i] + sm.u.epi.tau_col[j]) {
                            ++found;
                            mate = j;
                            mb = b;
                        }
                    }
                    if (found != 1 || ((taken >> mb) & 1u) || named == -2) {
                        named = -2;
                        continue;
                    }
                    taken |= 1u << mb;
                    pcol[i] = mate;
                    pd[i] = sm.u.epi.d_col[mate];
                    if (i == first_i) named = mate;
                }
                sm.red[3][0] = (double)(named >= 0 ? named : -1);
            }
            __syncthreads();
            const int named = (int)sm.red[3][0];
            if (named >= 0) {
                first_j = named;
                npairs = nr;
                kind = FTGEMM_KIND_CORRECTED;
                break;
            }
        } else if (nr + nc == 1) {
            // A lone disagreement.  A data error shows on both sides, each
            // up to its own rounding, so it stays below every threshold of
            // the other side only if it is at most twice the largest of
            // them; the flagged residual is then within its own threshold
            // plus that.  Beyond this bound only the checksum path can have
            // been hit and the data stays as it is; within it the tile is
            // computed again.
            const bool by_col = nc == 1;
            if (w == 0) {
                const double *tau_o = by_col ? sm.u.epi.tau_row : sm.u.epi.tau_col;
                const int cnt = by_col ? hrows : wcols;
                double o = 0.0;
                for (int x = lane; x < cnt; x += 64) o = fmax(o, tau_o[x]);
                o = max64(o);
                if (lane == 0) sm.red[3][0] = o;
            }
            __syncthreads();
            const double d = by_col ? sm.u.epi.d_col[first_j] : sm.u.epi.d_row[first_i];
            const double bound =
                (by_col ? sm.u.epi.tau_col[first_j] : sm.u.epi.tau_row[first_i]) +
                2.0 * sm.red[3][0];
            if (!(fabs(d) <= bound)) {
                kind = FTGEMM_KIND_CHECKSUM_ONLY;
                break;
            }
        }
        // Several disagreements, or a rebuilt value that does not confirm:
        // keep the first attempt's residuals for the record, then compute
        // the tile again.
        if (t == 0) {
            sm.red[0][0] = first_j >= 0 ? sm.u.epi.d_col[first_j] : 0.0;
            sm.red[0][1] = first_j >= 0 ? sm.u.epi.tau_col[first_j] : 0.0;
            sm.red[1][0] = first_i >= 0 ? sm.u.epi.d_row[first_i] : 0.0;
            sm.red[1][1] = first_i >= 0 ? sm.u.epi.tau_row[first_i] : 0.0;
        }
        __syncthreads();
    }

    if (ABFT) {
        const int t = fresh_tid(), lane = t & 63, w = t >> 6;
        const int wm = w & 1, wn = w >> 1, q = lane >> 4, c16 = lane & 15;
        if (kind == FTGEMM_KIND_CORRECTED && npairs == 0) {
            // the owner lane of a corrected element knows its old value
            __syncthreads();
            if (w == owner_wave(first_i, first_j) && lane == owner_lane(first_i, first_j)) {
                sm.red[2][0] = rec_before;
                sm.red[2][1] = rec_after;
            }
            __syncthreads();
            rec_before = sm.red[2][0];
            rec_after = sm.red[2][1];
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
                atomicAdd(&ct->record_count, 1u);
                const unsigned slot = atomicAdd(g.rec_slot, 1u);
                sm.red[3][1] = (double)slot;  // for a paired correction's values
                if (slot < g.record_cap) {
                    // residuals: from LDS of this attempt (corrected /
                    // checksum-only) or saved from the first attempt
                    const bool again = kind == FTGEMM_KIND_RECOMPUTED ||
                                       kind == FTGEMM_KIND_UNCORRECTABLE;
                    ftgemm_fault_record rc;
                    rc.problem = g.problem;
                    rc.kind = kind;
                    rc.tile_m = tile_m;
                    rc.tile_n = tile_n;
                    rc.row = first_i >= 0 ? i0 + first_i : -1;
                    rc.col = first_j >= 0 ? j0 + first_j : -1;
                    rc.nbad_rows = first_nr;
                    rc.nbad_cols = first_nc;
                    rc.d_row = again ? sm.red[0][0] : first_j >= 0 ? sm.u.epi.d_col[first_j] : 0.0;
                    rc.tau_row = again ? sm.red[0][1] : first_j >= 0 ? sm.u.epi.tau_col[first_j] : 0.0;
                    rc.d_col = again ? sm.red[1][0] : first_i >= 0 ? sm.u.epi.d_row[first_i] : 0.0;
                    rc.tau_col = again ? sm.red[1][1] : first_i >= 0 ? sm.u.epi.tau_row[first_i] : 0.0;
                    rc.before = kind == FTGEMM_KIND_CORRECTED ? rec_before : 0.0;
                    rc.after = kind == FTGEMM_KIND_CORRECTED ? rec_after : 0.0;
                    g.records[slot] = rc;
                }
            }
        }
        // Split inner dimension: publish this slice's encoded checksums and
        // thresholds for the verified reduction.  An entry that disagreed
        // alone (checksum-only) is replaced by the reference sum of the
        // verified data.
        if (g.nslices > 1 && t < TM + TN) {
            const bool row = t < TM;
            const int x = row ? t : t - TM;
            double P = row ? sm.u.epi.fin_row[x] : sm.u.epi.fin_col[x];
            const double tau = row ? sm.u.epi.tau_row[x] : sm.u.epi.tau_col[x];
            if (kind == FTGEMM_KIND_CHECKSUM_ONLY && x == (row ? first_i : first_j))
                P += row ? sm.u.epi.d_row[x] : sm.u.epi.d_col[x];
            double *dst = g.chk + slice_chk_index(0, tile_m + (int64_t)tile_n * g.tiles_m,
                                                  (int64_t)g.tiles_m * g.tiles_n, TM, TN);
            dst[t] = P;
            dst[TM + TN + t] = tau;
        }
        // Store the verified tile.
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wm * 64 + 16 * mi + 4 * r + q;
                    const int col = wn * 32 + 16 * ni + c16;
                    if (row < hrows && col < wcols)
                        C[(i0 + row) + (j0 + col) * ldc] = acc[mi][ni][r];
                }
        if (npairs > 0) {
            // Paired corrections: the lane that stored each element takes
            // the pair's residual off it in memory (its own store is ordered
            // before its atomics on the same address); the named element's
            // old and new values complete the record.
            const int *pcol = reinterpret_cast<const int *>(sm.u.epi.enc_row[1]);
            const double *pd = sm.u.epi.enc_row[0];
            for (int f = 0; f < npairs; ++f) {
                const int i = sm.bad_r[f], j = pcol[i];
                if (w != owner_wave(i, j) || lane != owner_lane(i, j)) continue;
                unsigned long long *a = reinterpret_cast<unsigned long long *>(
                    C + (i0 + i) + (j0 + j) * ldc);
                unsigned long long cur = atomicOr(a, 0ull);
                double before = __longlong_as_double((long long)cur), after = before - pd[i];
                for (int it = 0; it < 4; ++it) {
                    const unsigned long long prev =
                        atomicCAS(a, cur, (unsigned long long)__double_as_longlong(after));
                    if (prev == cur) break;
                    cur = prev;
                    before = __longlong_as_double((long long)cur);
                    after = before - pd[i];
                }
                if (i == first_i) {
                    sm.red[2][0] = before;
                    sm.red[2][1] = after;
                }
            }
            __syncthreads();
            const unsigned slot = (unsigned)sm.red[3][1];
            if (t == 0 && slot < g.record_cap) {
                g.records[slot].before = sm.red[2][0];
                g.records[slot].after = sm.red[2][1];
            }
        }
    }
}

template <bool TA, bool TB, bool ABFT, bool WGT = false>
__global__ __launch_bounds__(NT, 2) void kernel(GemmArgs g)
{
    __shared__ Smem sm;
    int tm_, tn_;
    if (WGT || g.nslices <= 1) {
        map_tile(blockIdx.x, g.tiles_m, g.tiles_n, tm_, tn_);
        tile<TA, TB, ABFT, WGT>(g, tm_, tn_, sm);
        return;
    }
    // Slice s of a split inner dimension: the partial product of the
    // slice's inner range (alpha 1, beta 0) into the workspace.
    const int ntiles = g.tiles_m * g.tiles_n;
    const int s = blockIdx.x / ntiles;
    map_tile(blockIdx.x - s * ntiles, g.tiles_m, g.tiles_n, tm_, tn_);
    GemmArgs gs = g;
    const int64_t kb = (int64_t)s * g.slice_k;
    gs.k = (g.k - kb < g.slice_k) ? g.k - kb : g.slice_k;
    gs.k_base = g.k_base + kb;
    gs.slice_last = s == g.nslices - 1;
    gs.A = (const double *)g.A + kb * (TA ? 1 : g.lda);
    gs.B = (const double *)g.B + kb * (TB ? g.ldb : 1);
    gs.C = g.wsp + s * g.m * g.n;
    gs.ldc = g.m;
    gs.alpha = 1.0;
    gs.beta = 0.0;
    gs.chk = g.chk + slice_chk_index(s, 0, ntiles, TM, TN);
    tile<TA, TB, ABFT>(gs, tm_, tn_, sm);
}


// Persistent batched kernel: workgroup w starts on queue w mod nqueues (with
// one queue per XCD, the XCD it runs on) and moves on to the others when it
// runs dry; every workgroup leaves once all queues are drained.
template <bool TA, bool TB, bool ABFT>
__global__ __launch_bounds__(NT, 2) void batched_kernel(BatchArgs b)
{
    __shared__ Smem sm;
    __shared__ int next;
    const int first = (int)(blockIdx.x % (unsigned)b.nqueues);
    for (int qi = 0; qi < b.nqueues; ++qi) {
        const int qq = (first + qi) % b.nqueues;
        const int end = b.qbegin[qq + 1];
        for (;;) {
            if (threadIdx.x == 0) next = b.qbegin[qq] + (int)atomicAdd(&b.queue[qq], 1u);
            __syncthreads();
            const int it = __builtin_amdgcn_readfirstlane(next);
            __syncthreads();
            if (it >= end) break;
            const WorkItem w = b.items[it];
            const GemmArgs g = b.probs[w.problem];
            tile<TA, TB, ABFT>(g, w.tile_m, w.tile_n, sm);
            __syncthreads();
        }
    }
}

}  // namespace f64

#define FTG_F64_CASE(ta, tb, ab) \
    hipLaunchKernelGGL((f64::kernel<ta, tb, ab>), dim3(grid), dim3(f64::NT), 0, stream, g)
#define FTG_F64_WCASE(ta, tb) \
    hipLaunchKernelGGL((f64::kernel<ta, tb, true, true>), dim3(grid), dim3(f64::NT), 0, stream, g)

hipError_t launch_f64(const GemmArgs &g, bool ta, bool tb, bool abft, hipStream_t stream,
                      bool weighted)
{
    const unsigned grid = (unsigned)g.tiles_m * (unsigned)g.tiles_n *
                          (unsigned)(g.nslices > 1 && !weighted ? g.nslices : 1);
    if (grid == 0) return hipSuccess;
    if (weighted) {
        if (!ta && !tb) FTG_F64_WCASE(false, false);
        else if (!ta && tb) FTG_F64_WCASE(false, true);
        else if (ta && !tb) FTG_F64_WCASE(true, false);
        else FTG_F64_WCASE(true, true);
    } else if (abft) {
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

hipError_t launch_f64_batched(const BatchArgs &b, bool ta, bool tb, bool abft, int grid,
                              hipStream_t stream)
{
#define FTG_F64_BCASE(x, y, z) \
    hipLaunchKernelGGL((f64::batched_kernel<x, y, z>), dim3(grid), dim3(f64::NT), 0, stream, b)
    if (abft) {
        if (!ta && !tb) FTG_F64_BCASE(false, false, true);
        else if (!ta && tb) FTG_F64_BCASE(false, true, true);
        else if (ta && !tb) FTG_F64_BCASE(true, false, true);
        else FTG_F64_BCASE(true, true, true);
    } else {
        if (!ta && !tb) FTG_F64_BCASE(false, false, false);
        else if (!ta && tb) FTG_F64_BCASE(false, true, false);
        else if (ta && !tb) FTG_F64_BCASE(true, false, false);
        else FTG_F64_BCASE(true, true, false);
    }
#undef FTG_F64_BCASE
    return hipGetLastError();
}

}  // namespace ftg
