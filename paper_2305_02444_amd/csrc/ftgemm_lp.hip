// ftgemm_lp.hip -- low-precision (BF16, FP8 E4M3) fault-tolerant GEMM tile
// for gfx950: matrix-core products accumulated in FP32, FP32 checksums,
// verification, location and correction in FP64, FP32 output.
//
// One workgroup of 8 waves owns a BM x 128 output tile (BM = 128: waves 2 x 4
// of 64 x 32; BM = 256: waves 4 x 2 of 64 x 64) and walks the inner dimension
// in steps of 128 bytes per row (64 BF16 or 128 FP8 values).
// Both operand tiles live in LDS with the inner index contiguous, the layout
// the MFMA operands want: v_mfma_f32_16x16x32_bf16 and
// v_mfma_f32_16x16x128_f8f6f4 (E4M3, unit block scales) read 8 / 32
// consecutive inner values per lane.  Operands whose outer index is the
// contiguous one in memory (A not transposed, B transposed) are transposed
// in registers while staged (pairs / quads of inner values per dword).
//
// Fault tolerance follows the FP64 kernel (FT-GEMM, Section 2.2): the staged
// operand registers feed the operand checksums x_p = sum_i A(i,p),
// y_p = sum_j B(p,j) and the norms before the step's barrier, and the
// encoded checksums Pc_i += A(i,p) y_p, Pr_j += x_p B(p,j) after it, all in
// FP32; the epilogue encodes C_in in the beta pass, sums the FP32 outputs in
// FP64, and verifies, locates, rebuilds and confirms in FP64.  The
// threshold's unit roundoff is FP32's.
#include "ftgemm_device.h"
#include "ftgemm_kernels.h"

namespace ftg {
namespace lp {

constexpr int TN = 128, BKB = 128;  // tile columns, inner step in bytes per row
constexpr int NW = 8, NT = 64 * NW;
constexpr int SROW = BKB + 16;      // LDS row stride in bytes

// Wave grid of a BM x TN tile: wave w = wm + WM wn holds rows 64 wm .. +63
// and columns WC wn .. +WC-1.
template <int BM>
struct Geo {
    static constexpr int WM = BM / 64;          // waves along the rows
    static constexpr int WN = NW / WM;          // waves along the columns
    static constexpr int WC = TN / WN;          // columns per wave
    static constexpr int NI = WC / 16;          // 16-column blocks per wave
    static constexpr int NA = BM / (16 * NW);   // 16-row A blocks per wave in A . y
    static constexpr int NREG = 16 * NI;        // accumulator values per lane
    static constexpr int kRW = BM / 64;         // waves that verify rows
    static constexpr int kVW = kRW + TN / 64;   // ... and columns after them
};
constexpr double U = 5.9604644775390625e-08;  // 2^-24, unit roundoff of FP32
// The FP8 matrix instructions do not add their products exactly: products
// are summed in groups of 8 consecutive inner indices, each cut (toward
// zero) to a multiple of 2^-14 times the binade of the group's largest
// product (measured on gfx950; BF16 products are added as in FP32).  The
// thresholds of the FP8 path carry the matching term
// lambda |alpha| 2^-14 sqrt(8) sqrt(h) max|A_I| ||b_j|| (rows: the mirror).
constexpr double kTruncGrid = 6.103515625e-05;  // 2^-14
constexpr int kTruncGroup = 8;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef int i4v __attribute__((ext_vector_type(4)));

// Result layout of both MFMAs (measured on gfx950): lane l = 16 q + c,
// register r holds D[4 q + r][c].  Wave (wm, wn) holds its block as
// acc[mi][ni][r] = C(64 wm + 16 mi + 4 q + r, WC wn + 16 ni + c).

template <bool FP8>
struct Elem {
    static constexpr int EB = FP8 ? 1 : 2;       // bytes per element
    static constexpr int BK = BKB / EB;          // inner values per step
    static constexpr int KV = 16 / EB;           // values per 16 bytes
    static constexpr int KPI = FP8 ? 128 : 32;   // inner values per MFMA
    static constexpr int NKK = BK / KPI;         // MFMAs along the inner step
};

// LDS rows hold 8 chunks of 16 bytes; chunk c of row r is stored at chunk
// c ^ ((r / 16) % 8).  With that the transposed 4-byte stores (8 rows apart
// per lane) spread over all banks instead of hitting 8 lanes per bank,
// while the 16-byte fragment reads of both formats stay conflict-free.
__device__ __forceinline__ int swz(int row, int chunk) { return chunk ^ ((row >> 4) & 7); }

// BF16 encodes on the matrix cores: each step's operand checksums x (of the
// A tile) and y (of the B tile), split exactly into three BF16 parts, are
// kept as XR extra rows of the staged tiles, and every wave multiplies them
// with its fragments of the other operand (x . B and A . y, accumulated in
// FP32 like the product).
constexpr int XR = 16;  // extra rows (3 parts, the rest zero)

template <int BM>
struct Stage {
    unsigned char A[BM + XR][SROW];  // A tile, [i][inner bytes]; rows BM.. x parts
    unsigned char B[TN + XR][SROW];  // B tile, [j][inner bytes]; rows TN.. y parts
};

template <int BM>
struct Epi {
    using G = Geo<BM>;
    double ref_row[G::WN][BM], ref_col[G::WM][TN];
    double cin_row[G::WN][BM], cin_col[G::WM][TN];
    double cin2_row[G::WN][BM], cin2_col[G::WM][TN];
    double enc_row[NW][BM], enc_col[NW][TN];
    double nrm_row[NW][BM], nrm_col[NW][TN];
    double fin_row[BM], fin_col[TN];
    double tau_row[BM], tau_col[TN];
    double d_row[BM], d_col[TN];
};

// Two staged steps.  (The BF16 checksum products trail the main product by
// one step; the fragments of the main rows they need are kept in registers
// from the step itself, and their extra rows are only rewritten after the
// next barrier, so a third stage is not needed.)
template <int BM>
struct Smem {
    union {
        Stage<BM> st[2];
        Epi<BM> epi;
    } u;
    float xs[2][128][NW];  // [buffer][p][partial]: column sums of the A tile
    float ys[2][128][NW];  // [buffer][p][partial]: row sums of the B tile
    float xc[128], yc[128];  // FP8: the step's x_p, y_p, combined once
    double red[NW][2];
    double wsum[NW][5];    // per wave: |x|^2, |y|^2, row / column norms^2, max|A|, max|B|
    double scal[6];
    TileFault faults[kMaxTileFaults];
    int nfaults;
    double wratio[NW];     // largest |d| / tau of the waves that verify
    int nbad_r, nbad_c, ibad, jbad;
    int bad_r[kMaxLineFixes], bad_c[kMaxLineFixes];  // the first flagged entries, any order
};

// E4M3 byte b (a constant after unrolling) of a dword, exactly widened
__device__ __forceinline__ float fp8_byte(int d, int b)
{
    switch (b & 3) {
    case 0: return __builtin_amdgcn_cvt_f32_fp8(d, 0);
    case 1: return __builtin_amdgcn_cvt_f32_fp8(d, 1);
    case 2: return __builtin_amdgcn_cvt_f32_fp8(d, 2);
    default: return __builtin_amdgcn_cvt_f32_fp8(d, 3);
    }
}

// element e of a dword (two BF16 or four E4M3 values), exactly widened
template <bool FP8>
__device__ __forceinline__ float elem_dw(int d, int e)
{
    if (FP8) return fp8_byte(d, e);
    return __uint_as_float((e & 1) ? ((unsigned)d & 0xffff0000u) : ((unsigned)d << 16));
}

// element e (0 .. KV-1) of a 16-byte chunk held in 4 dwords
template <bool FP8>
__device__ __forceinline__ float elem(const i4v &w, int e)
{
    return FP8 ? elem_dw<true>(w[e >> 2], e & 3) : elem_dw<false>(w[e >> 1], e & 1);
}

// Staging of one operand (OUTER = 128 or 256 outer indices) for one step;
// every thread handles OUTER / 4 bytes.
//   kInner (the inner index runs along the stored rows: A transposed, B not
//   transposed): thread t fetches 16 bytes (KV consecutive inner values) at
//   outer indices o = t / 8 + 64 r (r < OUTER / 64), inner chunk t % 8, and
//   stores them unchanged.
//   otherwise (the outer index runs along the stored rows): thread t fetches
//   the outer indices 8 (t % 16) + 128 g .. +7 (g < OUTER / 128) at the PG
//   (2 for BF16, 4 for FP8) consecutive inner indices PG (t / 16) .. +PG-1
//   as PG raw columns, and regroups them into one dword per outer index (its
//   inner pair or quad, the LDS layout) only when storing: nothing reads the
//   loaded registers before the next step's store, so the loads stay in
//   flight across the step's matrix products.
template <bool FP8, bool kInner, int OUTER>
struct LpLoader {
    using E = Elem<FP8>;
    static constexpr int PG = 4 / E::EB;               // inner values per dword
    static constexpr int kNP = kInner ? E::KV : PG;    // inner values per thread
    static constexpr int kParts = kInner ? NW : 1;     // partials of an operand checksum
    static constexpr int kGroups = OUTER / 128;        // otherwise: groups of 8 outer
    static constexpr int kOuter = kInner ? OUTER / 64 : 8 * kGroups;  // outer indices per thread
    static constexpr int kOuterParts = kInner ? 1 : NW;  // partials of a per-outer sum
    const char *X;
    int64_t ld, R, total_bytes;  // stored rows R, leading dimension ld (elements)
    int t;
    // kInner: raw 16-byte chunks; otherwise: raw columns, see col_dw
    i4v w[kInner ? kOuter : kOuter / 4];
    // otherwise: dword d of raw column b (inner p0 + b) of group g, holding
    // outer 8 g + d PG / 2 .. (BF16: 2 per dword, FP8: 4)
    __device__ __forceinline__ int col_dw(int g, int b, int d) const
    {
        return FP8 ? w[2 * g + (b >> 1)][2 * (b & 1) + d] : w[2 * g + b][d];
    }
    __device__ __forceinline__ void set_col_dw(int g, int b, int d, int v)
    {
        if (FP8)
            w[2 * g + (b >> 1)][2 * (b & 1) + d] = v;
        else
            w[2 * g + b][d] = v;
    }

    __device__ __forceinline__ void init(const void *x, int64_t ld_, int64_t rows, int64_t cols,
                                         int t_)
    {
        X = (const char *)x;
        ld = ld_;
        R = rows;
        total_bytes = (rows > 0 && cols > 0) ? (ld_ * (cols - 1) + rows) * E::EB : 0;
        t = t_;
    }
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int64_t r0, int64_t c0) const
    {
        const int64_t first = r0 + c0 * ld;
        int64_t ext = total_bytes - first * E::EB;
        if (ext < 0) ext = 0;
        if (ext > 0x7FFFFFFF) ext = 0x7FFFFFFF;
        return make_rsrc(X + first * E::EB, (uint64_t)ext);
    }
    __device__ __forceinline__ int outer(int r) const
    {
        return kInner ? (t >> 3) + 64 * r : 8 * (t & 15) + (r & 7) + 128 * (r >> 3);
    }
    __device__ __forceinline__ int p0() const { return kInner ? E::KV * (t & 7) : PG * (t >> 4); }

    // one element of the operand, zero outside the resource
    __device__ __forceinline__ unsigned load_elem(__amdgpu_buffer_rsrc_t rs, uint32_t off) const
    {
        if (FP8) return (unsigned)__builtin_amdgcn_raw_buffer_load_b8(rs, (int)off, 0, 0);
        return (unsigned)__builtin_amdgcn_raw_buffer_load_b16(rs, (int)off, 0, 0);
    }

    __device__ __forceinline__ void load(int64_t o0, int64_t k0, int64_t nouter, int64_t k)
    {
        if (kInner) {
            const __amdgpu_buffer_rsrc_t rs = rsrc(k0, o0);
            if (k - k0 >= E::BK) {
                // a full step (uniform): no chunk crosses the end of the
                // inner dimension, so no per-chunk checks (whose masks
                // would otherwise be held across the loop)
#pragma unroll
                for (int r = 0; r < kOuter; ++r)
                    w[r] = __builtin_amdgcn_raw_buffer_load_b128(
                        rs, (int)(uint32_t)((p0() + (int64_t)outer(r) * ld) * E::EB), 0, 0);
                return;
            }
            const int valid = (int)((k - k0) < E::BK ? (k - k0) : E::BK) - p0();
#pragma unroll
            for (int r = 0; r < kOuter; ++r) {
                const uint32_t off =
                    valid > 0 ? (uint32_t)((p0() + (int64_t)outer(r) * ld) * E::EB) : kOob;
                w[r] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
            }
            if (valid > 0 && valid < E::KV) {
                // a chunk that crosses the end of the inner dimension: element
                // by element, so nothing past the matrix is read into it
#pragma unroll
                for (int r = 0; r < kOuter; ++r) {
                    const uint32_t base = (uint32_t)((p0() + (int64_t)outer(r) * ld) * E::EB);
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        unsigned v = 0;
#pragma unroll
                        for (int e = 0; e < PG; ++e) {
                            const int idx = d * PG + e;
                            if (idx < valid)
                                v |= load_elem(rs, base + idx * E::EB) << (8 * E::EB * e);
                        }
                        w[r][d] = (int)v;
                    }
                }
            }
        } else {
            const __amdgpu_buffer_rsrc_t rs = rsrc(o0, k0);
            const uint32_t col = (uint32_t)(ld * E::EB);
#pragma unroll
            for (int g = 0; g < kGroups; ++g) {
                const uint32_t base = (uint32_t)((outer(8 * g) + (int64_t)p0() * ld) * E::EB);
                // raw columns: PG columns of 8 outer indices (16 or 8 bytes each)
#pragma unroll
                for (int b = 0; b < PG; ++b) {
                    if (!FP8) {
                        w[2 * g + b] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(base + b * col), 0, 0);
                    } else {
                        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(base + b * col), 0, 0);
                        set_col_dw(g, b, 0, (int)v[0]);
                        set_col_dw(g, b, 1, (int)v[1]);
                    }
                }
            }
            // Only the last tile along the outer index (a uniform test) can
            // hold chunks that cross the end of the matrix; its other tiles
            // skip the per-group checks, whose masks would otherwise be held
            // across the loop.
            if (nouter - o0 < OUTER) {
#pragma unroll
                for (int g = 0; g < kGroups; ++g) {
                    const uint32_t base =
                        (uint32_t)((outer(8 * g) + (int64_t)p0() * ld) * E::EB);
                    const int live = (int)(nouter - o0) - outer(8 * g);  // outer indices inside
                    if (live < 8) {
                        // the tile's last rows: element by element (a chunk
                        // that crosses the end of the matrix), zero past it
#pragma unroll
                        for (int b = 0; b < PG; ++b)
#pragma unroll
                            for (int d = 0; d < 8 / PG; ++d) {
                                unsigned v = 0;
#pragma unroll
                                for (int e = 0; e < PG; ++e) {
                                    const int idx = d * PG + e;
                                    if (idx < live)
                                        v |= load_elem(rs, base + b * col + idx * E::EB)
                                             << (8 * E::EB * e);
                                }
                                set_col_dw(g, b, d, (int)v);
                            }
                    }
                }
            }
        }
    }
    __device__ __forceinline__ void store(unsigned char (*dst)[SROW]) const
    {
        if (kInner) {
#pragma unroll
            for (int r = 0; r < kOuter; ++r)
                *(i4v *)&dst[outer(r)][16 * swz(outer(r), t & 7)] = w[r];
        } else {
            // regroup: one dword per outer index holding its PG inner values
#pragma unroll
            for (int g = 0; g < kGroups; ++g)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    unsigned v;
                    if (!FP8) {
                        // dword e / 2 of a column holds outer e (low half if e is even)
                        v = __builtin_amdgcn_perm((unsigned)col_dw(g, 1, e >> 1),
                                                  (unsigned)col_dw(g, 0, e >> 1),
                                                  (e & 1) ? 0x07060302u : 0x05040100u);
                    } else {
                        const int h = e >> 2, sb = e & 3;  // dword and byte of outer e in a column
                        const unsigned sel = (unsigned)(sb | ((sb + 4) << 8)) | 0x0c0c0000u;
                        const unsigned p01 = __builtin_amdgcn_perm((unsigned)col_dw(g, 1, h),
                                                                   (unsigned)col_dw(g, 0, h), sel);
                        const unsigned p23 = __builtin_amdgcn_perm((unsigned)col_dw(g, 3, h),
                                                                   (unsigned)col_dw(g, 2, h), sel);
                        v = __builtin_amdgcn_perm(p23, p01, 0x05040100u);
                    }
                    const int o = outer(8 * g + e);
                    *(int *)&dst[o][16 * swz(o, t >> 6) + 4 * ((t >> 4) & 3)] = (int)v;
                }
        }
    }
    // value of inner e (0 .. kNP-1) at outer slot r (0 .. kOuter-1)
    __device__ __forceinline__ float val(int r, int e) const
    {
        if (kInner) return elem<FP8>(w[r], e);
        const int g = r >> 3, o = r & 7;  // raw column e holds outer o of group g
        return FP8 ? elem_dw<true>(col_dw(g, e, o >> 2), o & 3)
                   : elem_dw<false>(col_dw(g, e, o >> 1), o & 1);
    }
    // This step's operand checksum over the tile's outer indices, into
    // dst[p][slot]: complete (otherwise, slot 0, the 16 lanes of a row share
    // p) or one partial per wave (kInner, slot = wave, over the 8 lanes
    // sharing the inner chunk).
    // (kNorms: the squared norms of this thread's outer indices are
    // accumulated in the same pass.)
    template <bool kNorms = false>
    __device__ __forceinline__ void sum_to(float (*dst)[NW], float (&nrm)[kOuter]) const
    {
        float v[kNP];
#pragma unroll
        for (int e = 0; e < kNP; ++e) {
            float s = 0.0f;
#pragma unroll
            for (int r = 0; r < kOuter; ++r) {
                const float x = val(r, e);
                s += x;
                if (kNorms) nrm[r] = fmaf(x, x, nrm[r]);
            }
            v[e] = s;
        }
        if constexpr (!kInner) {
#pragma unroll
            for (int e = 0; e < kNP; ++e) {
                const float s = sum16f(v[e]);
                if ((t & 15) == 0) dst[p0() + e][0] = s;
            }
        } else {
        // The 8 lanes holding this inner chunk (lane bits 3..5) reduce kNP
        // values by halving: each exchange step sends half of the values to
        // the partner and keeps the other half, so every lane ends with
        // kNP / 8 complete sums -- for inner index p0 + e_lane + i, e_lane =
        // (kNP / 2) b5 + (kNP / 4) b4 + (kNP / 8) b3.
        constexpr int H1 = kNP / 2, H2 = kNP / 4, H3 = kNP / 8;
        float u[H1], z[H2], f[H3];
#pragma unroll
        for (int i = 0; i < H1; ++i) {  // lanes l, l ^ 32
            const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(v[i]),
                                                            __float_as_int(v[i + H1]), false, false);
            u[i] = __int_as_float(r[0]) + __int_as_float(r[1]);
        }
#pragma unroll
        for (int i = 0; i < H2; ++i) {  // lanes l, l ^ 16
            const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(u[i]),
                                                            __float_as_int(u[i + H2]), false, false);
            z[i] = __int_as_float(r[0]) + __int_as_float(r[1]);
        }
        const bool b3 = (t & 8) != 0;
#pragma unroll
        for (int i = 0; i < H3; ++i) {  // lanes l, l ^ 8 (row_ror:8)
            const float keep = b3 ? z[i + H3] : z[i];
            const float send = b3 ? z[i] : z[i + H3];
            f[i] = keep + dpp_f32<0x128>(send);
        }
        const int e0 = ((t & 32) ? H1 : 0) + ((t & 16) ? H2 : 0) + (b3 ? H3 : 0);
#pragma unroll
        for (int i = 0; i < H3; ++i) dst[p0() + e0 + i][t >> 6] = f[i];
        }
    }
    // Encoded checksum (with the other operand's checksum v, indexed like
    // this thread's inner values) and squared norms over this step.
    // (FP8: amx tracks the largest magnitude for the truncation term.)
    // (kNrm false: the encoded checksum only.)
    // (kPk, FP8 without norms: packed conversions, below; the one-sided
    // tiles use them -- in the two-sided FP8 tile they measured slower)
    template <bool kNrm = true, bool kPk = false>
    __device__ __forceinline__ void encode(const float (&v)[kNP], float (&enc)[kOuter],
                                           float (&nrm)[kOuter], float &amx) const
    {
        static_assert(!(kPk && kNrm), "packed conversions take no norms");
        if (FP8 && kPk) {
            // two E4M3 codes of one 16-bit half per conversion: inner pairs
            // (e, e + 1) of a chunk, or outer pairs (r, r + 1) of a raw
            // column; each enc[r] still takes its terms in ascending e
            if (kInner) {
#pragma unroll
                for (int r = 0; r < kOuter; ++r)
#pragma unroll
                    for (int e = 0; e < kNP; e += 2) {
                        const int d = w[r][e >> 2];
                        const auto a = (e & 2) ? __builtin_amdgcn_cvt_pk_f32_fp8(d, true)
                                               : __builtin_amdgcn_cvt_pk_f32_fp8(d, false);
                        enc[r] = fmaf(a[0], v[e], enc[r]);
                        enc[r] = fmaf(a[1], v[e + 1], enc[r]);
                    }
            } else {
#pragma unroll
                for (int e = 0; e < kNP; ++e)
#pragma unroll
                    for (int r = 0; r < kOuter; r += 2) {
                        const int g = r >> 3, o = r & 7;
                        const int d = col_dw(g, e, o >> 2);
                        const auto a = (o & 2) ? __builtin_amdgcn_cvt_pk_f32_fp8(d, true)
                                               : __builtin_amdgcn_cvt_pk_f32_fp8(d, false);
                        enc[r] = fmaf(a[0], v[e], enc[r]);
                        enc[r + 1] = fmaf(a[1], v[e], enc[r + 1]);
                    }
            }
            return;
        }
#pragma unroll
        for (int r = 0; r < kOuter; ++r)
#pragma unroll
            for (int e = 0; e < kNP; ++e) {
                const float a = val(r, e);
                enc[r] = fmaf(a, v[e], enc[r]);
                if (kNrm) nrm[r] = fmaf(a, a, nrm[r]);
                if (FP8 && kNrm) amx = fmaxf(amx, fabsf(a));
            }
    }
    // Per-outer sums completed over the threads holding the same outer
    // index, into dst[part][outer].
    __device__ __forceinline__ void partials_to(const float (&a_in)[kOuter], double (*dst)[OUTER]) const
    {
#pragma unroll
        for (int r = 0; r < kOuter; ++r) {
            double a = (double)a_in[r];
            if (kInner) {
                // the 8 consecutive lanes holding the 8 inner chunks
                a += dpp_f64<kQuadXor1>(a);
                a += dpp_f64<kQuadXor2>(a);
                a += dpp_f64<kRowHalfMirror>(a);
                if ((t & 7) == 0) dst[0][outer(r)] = a;
            } else {
                a = sum_rows(a);  // the 4 inner groups of a wave
                if ((t & 48) == 0) dst[t >> 6][outer(r)] = a;
            }
        }
    }
};

// v as hi + mid + lo, three BF16 values (exact: each part takes the next
// 8 significant bits of the FP32 value), stored as element p of the extra
// rows first_row .. first_row + 2 of a staged tile.
__device__ __forceinline__ void put_parts(unsigned char (*tile)[SROW], int first_row, int p,
                                          float v)
{
    float r = v;
#pragma unroll
    for (int part = 0; part < 3; ++part) {
        const __bf16 h = (__bf16)r;
        r -= (float)h;
        const int row = first_row + part;
        *(__bf16 *)&tile[row][16 * swz(row, p >> 3) + 2 * (p & 7)] = h;
    }
}

template <int kParts>
__device__ __forceinline__ float gather_lp(const float (*src)[NW], int p)
{
    if (kParts == 1) return src[p][0];
    return ((src[p][0] + src[p][1]) + (src[p][2] + src[p][3])) +
           ((src[p][4] + src[p][5]) + (src[p][6] + src[p][7]));
}

// wave, lane and accumulator slot (acc[e / (4 NI)][(e / 4) % NI][e % 4])
// holding element (row, col) of a BM x TN tile
template <int BM>
__device__ __forceinline__ int owner_wave(int row, int col)
{
    return (row >> 6) + Geo<BM>::WM * (col / Geo<BM>::WC);
}
__device__ __forceinline__ int owner_lane(int row, int col)
{
    return 16 * ((row & 15) >> 2) + (col & 15);
}
template <int BM>
__device__ __forceinline__ int owner_reg(int row, int col)
{
    return ((row & 63) >> 4) * (4 * Geo<BM>::NI) + ((col % Geo<BM>::WC) >> 4) * 4 + (row & 3);
}

// C_in for the beta pass, read through a buffer resource that starts at the
// tile and ends with C, so what lies past C's last element reads as 0; rows
// and columns past the tile's own inside C are read and must be dropped by
// the caller.  Offsets are 32-bit: the host limits ldc so that a tile spans
// less than 2 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t cin_rsrc(const float *C, int64_t ldc, int64_t m,
                                                           int64_t n, int64_t i0, int64_t j0)
{
    const int64_t first = i0 + j0 * ldc;
    int64_t ext = (ldc * (n - 1) + m - first) * 4;
    if (ext < 0) ext = 0;
    if (ext > 0x7FFFFFFF) ext = 0x7FFFFFFF;
    return make_rsrc(C + first, (uint64_t)ext);
}

// The C_in elements under this thread's accumulators of row group mi (acc
// layout).  The epilogues fetch group mi + 1 before they work on group mi,
// so one group's wait overlaps the previous group's work (instead of one
// wait per row).
template <int BM>
__device__ __forceinline__ void load_cin(__amdgpu_buffer_rsrc_t rs, int64_t ldc, int mi, int wm,
                                         int wn, int q, int c16, float cv[Geo<BM>::NI][4])
{
#pragma unroll
    for (int ni = 0; ni < Geo<BM>::NI; ++ni)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = wm * 64 + 16 * mi + 4 * q + r;
            const int col = wn * Geo<BM>::WC + 16 * ni + c16;
            cv[ni][r] = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(
                           rs, (int)(uint32_t)((row + (int64_t)col * ldc) * 4), 0, 0));
        }
}

// Four outputs of one column, rows row0 .. row0 + 3 of the tile (each lane
// holds four consecutive rows of a column): one 16-byte store where all four
// lie inside the matrix and C's columns start on 16-byte boundaries (vec),
// else one store per element inside it.
__device__ __forceinline__ void store_rows4(float *C, int64_t ldc, int64_t i0, int64_t j0,
                                            int row0, int col, int hrows, int wcols, bool vec,
                                            const f4 v)
{
    if (col >= wcols) return;
    float *p = C + (i0 + row0) + (j0 + col) * ldc;
    if (vec && row0 + 4 <= hrows) {
        *reinterpret_cast<f4 *>(p) = v;
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (row0 + r < hrows) p[r] = v[r];
    }
}

// ONE: the one-sided mode -- only the column checksum of the tile (one
// entry per row, C^c = C e) is encoded and verified, and any disagreement has
// the tile computed again.  PRE (implied by ONE): the threshold norms come
// from g.row_nrm2 / g.col_nrm2 / g.row_max / g.col_max, taken before the
// product, instead of from the staged operands.
template <bool FP8, bool TA, bool TB, bool ABFT, int BM, bool ONE = false, bool PRE = false>
__device__ void tile(const GemmArgs &g, int tile_m, int tile_n, Smem<BM> &sm)
{
    using E = Elem<FP8>;
    using G = Geo<BM>;
    constexpr int NI = G::NI, NA = G::NA;
    constexpr bool kMma = !FP8;  // BF16: encoded checksums on the matrix cores
    constexpr bool kOne = ABFT && ONE;
    constexpr bool kPre = ABFT && (ONE || PRE);
    // with the operand checksums computed in the tiles, the checksum products
    // of step s run during step s + 1 (its x/y parts are complete only after
    // step s's barrier); with them taken before the product, the parts are
    // staged with the tiles and the products run in their own step, on the
    // wave's own fragments
    constexpr bool kLag = kMma && ABFT && !kPre;
    constexpr bool kInStep = kMma && ABFT && kPre;
    // kPre: the operand checksums x_p, y_p come from g.xsum, g.ysum (taken
    // with the norms before the product) instead of the staged registers
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w % G::WM, wn = w / G::WM;
    const int q = lane >> 4, c16 = lane & 15;
    const int64_t i0 = (int64_t)tile_m * BM, j0 = (int64_t)tile_n * TN;
    float *__restrict__ C = (float *)g.C;
    const int64_t m = g.m, n = g.n, k = g.k, ldc = g.ldc;
    const int nsteps = (int)((k + E::BK - 1) / E::BK);
    const int hrows = (int)(m - i0 < BM ? m - i0 : BM);
    const int wcols = (int)(n - j0 < TN ? n - j0 : TN);
    const bool use_c = g.beta != 0.0;

    // inner index along the stored rows: A transposed, B not transposed
    using LA = LpLoader<FP8, TA, BM>;
    using LB = LpLoader<FP8, !TB, TN>;
    LA la;
    LB lb;
    la.init(g.A, g.lda, TA ? k : m, TA ? m : k, t);
    lb.init(g.B, g.ldb, TB ? n : k, TB ? k : n, t);
    auto load = [&](int s) {
        const int64_t k0 = (int64_t)s * E::BK;
        la.load(i0, k0, m, k);
        lb.load(j0, k0, n, k);
    };
    // kPre: this step's x_p, y_p at p = s BK + t (threads t < BK; zero past k)
    float px = 0.0f, py = 0.0f;
    auto load_sums = [&](int s) {
        if (t < E::BK) {
            const int64_t p = (int64_t)s * E::BK + t;
            py = p < k ? g.ysum[(int64_t)tile_n * g.ldxs + p] : 0.0f;
            if (!kOne) px = p < k ? g.xsum[(int64_t)tile_m * g.ldxs + p] : 0.0f;
        }
    };

    int nf = 0;
    if (ABFT) {
        if (w == 0) {
            const int cnt = gather_tile_faults(g, i0, j0, BM, TN, E::BK, g.k_base, sm.faults);
            if (lane == 0) sm.nfaults = cnt;
        }
        __syncthreads();
        nf = sm.nfaults;
    }

    int kind = 0, first_nr = 0, first_nc = 0, first_i = -1, first_j = -1;
    int npairs = 0;  // corrections left for the stored tile
    double rec_before = 0, rec_after = 0;

    // Checksum products of a staged step (BF16): the x-part rows times this
    // wave's B block (columns WC wn + 16 wm ..), this wave's NA A blocks
    // (rows 64 wm + 16 (NA wn + h) ..) times the y-part rows.  The parts come
    // from the extra rows of the step's stage, the blocks from registers
    // (hb, ha) read while the step was the current one.
    auto check_products = [&](const Stage<BM> &st, int kk, const bf8v &hb, const bf8v (&ha)[NA],
                              f4 &acc_r, f4 (&acc_c)[NA]) {
        const bf8v fyb = *(const bf8v *)&st.B[TN + c16][16 * swz(TN + c16, 4 * kk + q)];
        if (!kOne) {
            const bf8v fxa = *(const bf8v *)&st.A[BM + c16][16 * swz(BM + c16, 4 * kk + q)];
            acc_r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fxa, hb, acc_r, 0, 0, 0);
        }
#pragma unroll
        for (int h = 0; h < NA; ++h)
            acc_c[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[h], fyb, acc_c[h], 0, 0, 0);
    };
    constexpr int kHold = kLag ? E::NKK : 1;
    bf8v hold_b[kHold], hold_a[kHold][NA];  // this wave's check blocks of the last step

    f4 acc[4][NI];
#pragma unroll 1
    for (int attempt = 0; attempt < 2; ++attempt) {
        const bool faults_on = ABFT && attempt == 0 && nf > 0;
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni)
                acc[mi][ni] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
        float enc_a[LA::kOuter] = {}, nrm_a[LA::kOuter] = {};
        float enc_b[LB::kOuter] = {}, nrm_b[LB::kOuter] = {};
        float vx = 0.0f, vy = 0.0f, amx_a = 0.0f, amx_b = 0.0f;
        float yv[LA::kNP], xv[LB::kNP];  // y at the A loader's p, x at the B loader's
        f4 acc_r = (f4){0.0f, 0.0f, 0.0f, 0.0f};  // x-part rows times this wave's B block
        f4 acc_c[NA];                             // this wave's A blocks times the y parts
#pragma unroll
        for (int h = 0; h < NA; ++h) acc_c[h] = (f4){0.0f, 0.0f, 0.0f, 0.0f};

        if (ABFT && kMma) {
            // clear the extra rows of both stages (the epilogue reuses the
            // memory); done before step 0's barrier
            constexpr int kRowChunks = XR * (SROW / 16);
            constexpr int kChunks = 2 * 2 * kRowChunks;
            for (int c = t; c < kChunks; c += NT) {
                const int st = c / (2 * kRowChunks), rem = c % (2 * kRowChunks);
                const int op = rem / kRowChunks, rr = rem % kRowChunks;
                unsigned char(*dst)[SROW] = op ? sm.u.st[st].B : sm.u.st[st].A;
                *(i4v *)&dst[(op ? TN : BM) + rr / (SROW / 16)][16 * (rr % (SROW / 16))] =
                    (i4v){0, 0, 0, 0};
            }
        }

        load(0);
        if (ABFT && kPre) {
            load_sums(0);
        } else if (ABFT) {
            if (!kOne) la.template sum_to<kMma>(sm.xs[0], nrm_a);
            lb.template sum_to<kMma>(sm.ys[0], nrm_b);
        }
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
                const int stg = s & 1;  // stage and checksum buffers of step s
                la.store(sm.u.st[stg].A);
                lb.store(sm.u.st[stg].B);
                if (kInStep && t < E::BK) {
                    // the parts of step s's x_p, y_p (taken before the
                    // product) go to the stage's extra rows with the tiles
                    vy = fmaf(py, py, vy);
                    put_parts(sm.u.st[stg].B, TN, t, py);
                    if (!kOne) {
                        vx = fmaf(px, px, vx);
                        put_parts(sm.u.st[stg].A, BM, t, px);
                    }
                }
                if (ABFT && kPre && !kMma && t < E::BK) {
                    // x_p, y_p of step s (taken before the product) are
                    // staged with the tiles, so the step's one barrier
                    // publishes them too: flat in this stage's partial
                    // buffers, which the sums from registers would use
                    vy = fmaf(py, py, vy);
                    (&sm.ys[stg][0][0])[t] = py;
                    if (!kOne) {
                        vx = fmaf(px, px, vx);
                        (&sm.xs[stg][0][0])[t] = px;
                    }
                }
                __syncthreads();
                if (kLag) {
                    // x_p, y_p of step s are complete: their parts go to the
                    // extra rows, for the checksum products of step s (run
                    // during step s + 1, after its barrier)
                    if (t < E::BK) {
                        const float yp = gather_lp<LB::kParts>(sm.ys[stg], t);
                        vy = fmaf(yp, yp, vy);
                        put_parts(sm.u.st[stg].B, TN, t, yp);
                        if (!kOne) {
                            const float xp = gather_lp<LA::kParts>(sm.xs[stg], t);
                            vx = fmaf(xp, xp, vx);
                            put_parts(sm.u.st[stg].A, BM, t, xp);
                        }
                    }
                } else if (ABFT && !kMma) {
                    // x_p, y_p of step s are complete: combined once (one
                    // thread per p; already staged when taken before the
                    // product), then the encoded checksums and norms of
                    // step s, before the registers take step s + 1
                    const float *ycs = kPre ? &sm.ys[stg][0][0] : sm.yc;
                    const float *xcs = kPre ? &sm.xs[stg][0][0] : sm.xc;
                    if (!kPre) {
                        if (t < E::BK) {
                            const float yp = gather_lp<LB::kParts>(sm.ys[stg], t);
                            vy = fmaf(yp, yp, vy);
                            sm.yc[t] = yp;
                            if (!kOne) {
                                const float xp = gather_lp<LA::kParts>(sm.xs[stg], t);
                                vx = fmaf(xp, xp, vx);
                                sm.xc[t] = xp;
                            }
                        }
                        __syncthreads();
                    }
#pragma unroll
                    for (int e = 0; e < LA::kNP; ++e) yv[e] = ycs[la.p0() + e];
                    la.template encode<!kPre, kOne>(yv, enc_a, nrm_a, amx_a);
                    if (!kOne) {
#pragma unroll
                        for (int e = 0; e < LB::kNP; ++e) xv[e] = xcs[lb.p0() + e];
                        lb.template encode<!kPre>(xv, enc_b, nrm_b, amx_b);
                    }
                }
                if (s + 1 < nsteps) {
                    load(s + 1);
                    if (ABFT && kPre) load_sums(s + 1);
                }
#pragma unroll
                for (int kk = 0; kk < E::NKK; ++kk) {
                    if (!FP8) {
                        bf8v fa[4], fb[NI];
#pragma unroll
                        for (int mi = 0; mi < 4; ++mi) {
                            const int r = wm * 64 + 16 * mi + c16;
                            fa[mi] = *(const bf8v *)&sm.u.st[stg].A[r][16 * swz(r, 4 * kk + q)];
                        }
#pragma unroll
                        for (int ni = 0; ni < NI; ++ni) {
                            const int r = wn * G::WC + 16 * ni + c16;
                            fb[ni] = *(const bf8v *)&sm.u.st[stg].B[r][16 * swz(r, 4 * kk + q)];
                        }
#pragma unroll
                        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                            for (int ni = 0; ni < NI; ++ni)
                                acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    fa[mi], fb[ni], acc[mi][ni], 0, 0, 0);
                        if (kInStep) {
                            // this wave's check blocks are among its own
                            // fragments: B block wm (columns WC wn + 16 wm)
                            // and A blocks NA wn + h; the wave index is
                            // uniform, so the choice is a scalar branch
                            const int wm_s = __builtin_amdgcn_readfirstlane(wm);
                            const int wn_s = __builtin_amdgcn_readfirstlane(wn);
                            const unsigned char(*sA)[SROW] = sm.u.st[stg].A;
                            const unsigned char(*sB)[SROW] = sm.u.st[stg].B;
                            const bf8v fyb =
                                *(const bf8v *)&sB[TN + c16][16 * swz(TN + c16, 4 * kk + q)];
                            if (!kOne) {
                                const bf8v fxa =
                                    *(const bf8v *)&sA[BM + c16][16 * swz(BM + c16, 4 * kk + q)];
#pragma unroll
                                for (int ni = 0; ni < NI; ++ni)
                                    if (ni == wm_s)
                                        acc_r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                            fxa, fb[ni], acc_r, 0, 0, 0);
                            }
#pragma unroll
                            for (int g2 = 0; g2 < G::WN; ++g2)
                                if (g2 == wn_s) {
#pragma unroll
                                    for (int h = 0; h < NA; ++h)
                                        acc_c[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                            fa[NA * g2 + h], fyb, acc_c[h], 0, 0, 0);
                                }
                        }
                        if (kLag) {
                            if (s > 0)
                                check_products(sm.u.st[stg ^ 1], kk, hold_b[kk], hold_a[kk], acc_r,
                                               acc_c);
                            const int rb = wn * G::WC + 16 * wm + c16;
                            if (!kOne)
                                hold_b[kk] =
                                    *(const bf8v *)&sm.u.st[stg].B[rb][16 * swz(rb, 4 * kk + q)];
#pragma unroll
                            for (int h = 0; h < NA; ++h) {
                                const int ra = 64 * wm + 16 * (NA * wn + h) + c16;
                                hold_a[kk][h] =
                                    *(const bf8v *)&sm.u.st[stg].A[ra][16 * swz(ra, 4 * kk + q)];
                            }
                        }
                    } else {
                        i8v fa[4], fb[NI];
#pragma unroll
                        for (int mi = 0; mi < 4; ++mi)
                        {
                            const int r = wm * 64 + 16 * mi + c16;
                            const i4v lo = *(const i4v *)&sm.u.st[stg].A[r][16 * swz(r, 2 * q)];
                            const i4v hi = *(const i4v *)&sm.u.st[stg].A[r][16 * swz(r, 2 * q + 1)];
                            fa[mi] = (i8v){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                        }
#pragma unroll
                        for (int ni = 0; ni < NI; ++ni)
                        {
                            const int r = wn * G::WC + 16 * ni + c16;
                            const i4v lo = *(const i4v *)&sm.u.st[stg].B[r][16 * swz(r, 2 * q)];
                            const i4v hi = *(const i4v *)&sm.u.st[stg].B[r][16 * swz(r, 2 * q + 1)];
                            fb[ni] = (i8v){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                        }
#pragma unroll
                        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                            for (int ni = 0; ni < NI; ++ni)
                                acc[mi][ni] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                                    fa[mi], fb[ni], acc[mi][ni], 0, 0, 0, 127, 0, 127);
                    }
                }
                if (ABFT && !kPre && s + 1 < nsteps) {
                    // operand checksums of step s + 1, published before its barrier
                    if (!kOne) la.template sum_to<kMma>(sm.xs[stg ^ 1], nrm_a);
                    lb.template sum_to<kMma>(sm.ys[stg ^ 1], nrm_b);
                }
            }
            if (ABFT && faults_on) {
                for (int f = 0; f < nf; ++f) {
                    const TileFault tf = sm.faults[f];
                    if (tf.target != FTGEMM_TGT_ACC || tf.kstep != stop) continue;
                    if (w != owner_wave<BM>(tf.row, tf.col)) continue;
                    const int ol = owner_lane(tf.row, tf.col), sel = owner_reg<BM>(tf.row, tf.col);
                    float before = 0.0f;
#pragma unroll
                    for (int e = 0; e < G::NREG; ++e)
                        if (sel == e) before = acc[e / (4 * NI)][(e >> 2) % NI][e & 3];
                    const float after = tf.mode == FTGEMM_INJ_ADD ? (float)((double)before + tf.delta)
                                                                  : flip_bit_f32(before, tf.bit & 31);
#pragma unroll
                    for (int e = 0; e < G::NREG; ++e)
                        if (sel == e && lane == ol) acc[e / (4 * NI)][(e >> 2) % NI][e & 3] = after;
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
        __syncthreads();
        if (kLag) {
            // the last step's checksum products (its parts are now visible);
            // the epilogue then reuses the stages' memory
#pragma unroll
            for (int kk = 0; kk < E::NKK; ++kk)
                check_products(sm.u.st[(nsteps - 1) & 1], kk, hold_b[kk], hold_a[kk], acc_r, acc_c);
            __syncthreads();
        }
        // From here on the lane-derived indices are formed again instead of
        // being carried across the main loop.
        const int t = fresh_tid(), lane = t & 63, w = t >> 6;
        const int wm = w % G::WM, wn = w / G::WM, q = lane >> 4, c16 = lane & 15;
        la.t = t;
        lb.t = t;

        const __amdgpu_buffer_rsrc_t crs = cin_rsrc(C, ldc, m, n, i0, j0);
        float cn[NI][4] = {}, cx[NI][4] = {};
        if (use_c) load_cin<BM>(crs, ldc, 0, wm, wn, q, c16, cn);
        if (!ABFT) {
            const bool vec = ((reinterpret_cast<uintptr_t>(C) | ((uintptr_t)ldc << 2)) & 15) == 0;
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
                if (use_c && mi + 1 < 4) load_cin<BM>(crs, ldc, mi + 1, wm, wn, q, c16, cx);
#pragma unroll
                for (int ni = 0; ni < NI; ++ni) {
                    f4 v;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double o = g.alpha * (double)acc[mi][ni][r];
                        v[r] = (float)(use_c ? o + g.beta * (double)cn[ni][r] : o);
                    }
                    store_rows4(C, ldc, i0, j0, wm * 64 + 16 * mi + 4 * q,
                                wn * G::WC + 16 * ni + c16, hrows, wcols, vec, v);
                }
#pragma unroll
                for (int ni = 0; ni < NI; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r) cn[ni][r] = cx[ni][r];
            }
            return;
        }

        if (kMma) {
            // encoded checksums from the matrix cores: row parts (lanes with
            // column 0..2 of the A . y block), column sums of the x-part rows
            if (c16 < 3)
#pragma unroll
                for (int h = 0; h < NA; ++h)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        sm.u.epi.enc_row[c16][64 * wm + 16 * (NA * wn + h) + 4 * q + r] =
                            (double)acc_c[h][r];
            if (!kOne && q == 0)
                sm.u.epi.enc_col[0][wn * G::WC + 16 * wm + c16] =
                    ((double)acc_r[0] + (double)acc_r[1]) + (double)acc_r[2];
        } else {
            la.partials_to(enc_a, sm.u.epi.enc_row);
            if (!kOne) lb.partials_to(enc_b, sm.u.epi.enc_col);
        }
        if (!kPre) {
            la.partials_to(nrm_a, sm.u.epi.nrm_row);
            lb.partials_to(nrm_b, sm.u.epi.nrm_col);
        }
        // |x|^2 and |y|^2: threads t < BK took one p each
        {
            const double sx = kOne ? 0.0 : sum64(t < E::BK ? (double)vx : 0.0);
            const double sy = sum64(t < E::BK ? (double)vy : 0.0);
            const double ma = FP8 && !kPre ? max64((double)amx_a) : 0.0;
            const double mb = FP8 && !kPre ? max64((double)amx_b) : 0.0;
            if (lane == 0) {
                sm.wsum[w][0] = sx; sm.wsum[w][1] = sy; sm.wsum[w][3] = ma; sm.wsum[w][4] = mb;
            }
        }

        // Beta pass fused with the C_in part of the encoding; the output is
        // rounded to FP32 and the reference sums are taken of what is stored.
        // (row group mi + 1 of C_in is fetched while group mi is summed)
        double col_o[NI] = {}, col_c[NI] = {}, col_c2[NI] = {};
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            if (use_c && mi + 1 < 4) load_cin<BM>(crs, ldc, mi + 1, wm, wn, q, c16, cx);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double row_o = 0, row_c = 0, row_c2 = 0;
                const int row = wm * 64 + 16 * mi + 4 * q + r;
#pragma unroll
                for (int ni = 0; ni < NI; ++ni) {
                    const int col = wn * G::WC + 16 * ni + c16;
                    const bool ok = row < hrows && col < wcols;
                    const double cin = (use_c && ok) ? (double)cn[ni][r] : 0.0;
                    double o = g.alpha * (double)acc[mi][ni][r];
                    if (use_c) o = o + g.beta * cin;
                    const float of = ok ? (float)o : 0.0f;
                    acc[mi][ni][r] = of;
                    row_o += (double)of; row_c += cin; row_c2 += cin * cin;
                    col_o[ni] += (double)of; col_c[ni] += cin; col_c2[ni] += cin * cin;
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
            for (int ni = 0; ni < NI; ++ni)
#pragma unroll
                for (int r = 0; r < 4; ++r) cn[ni][r] = cx[ni][r];
        }
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) {
            col_o[ni] = sum_rows(col_o[ni]);
            if (use_c) { col_c[ni] = sum_rows(col_c[ni]); col_c2[ni] = sum_rows(col_c2[ni]); }
            if (q == 0) {
                const int col = wn * G::WC + 16 * ni + c16;
                sm.u.epi.ref_col[wm][col] = col_o[ni];
                sm.u.epi.cin_col[wm][col] = col_c[ni];
                sm.u.epi.cin2_col[wm][col] = col_c2[ni];
            }
        }
        if (t == 0) { sm.nbad_r = 0; sm.nbad_c = 0; sm.ibad = BM; sm.jbad = TN; }
        __syncthreads();

        const bool is_row = t < BM, is_col = t >= BM && t < BM + TN;
        const int x = is_row ? t : t - BM;
        double nrm2 = 0.0;
        if (is_row) {
            double e = 0, nr = 0;
            if (kPre)
                nr = x < hrows ? g.row_nrm2[i0 + x] : 0.0;
            else
#pragma unroll
                for (int v = 0; v < LA::kOuterParts; ++v) nr += sm.u.epi.nrm_row[v][x];
            if (kMma) {
                e = (sm.u.epi.enc_row[0][x] + sm.u.epi.enc_row[1][x]) + sm.u.epi.enc_row[2][x];
            } else {
#pragma unroll
                for (int v = 0; v < LA::kOuterParts; ++v) e += sm.u.epi.enc_row[v][x];
            }
            nrm2 = nr;
            sm.u.epi.fin_row[x] = e;
        } else if (is_col && kOne) {
            nrm2 = x < wcols ? g.col_nrm2[j0 + x] : 0.0;
        } else if (is_col) {
            double e = 0, nr = 0;
            if (kPre)
                nr = x < wcols ? g.col_nrm2[j0 + x] : 0.0;
            else
#pragma unroll
                for (int v = 0; v < LB::kOuterParts; ++v) nr += sm.u.epi.nrm_col[v][x];
            if (kMma) {
                e = sm.u.epi.enc_col[0][x];
            } else {
#pragma unroll
                for (int v = 0; v < LB::kOuterParts; ++v) e += sm.u.epi.enc_col[v][x];
            }
            nrm2 = nr;
            sm.u.epi.fin_col[x] = e;
        }
        // Frobenius norms of the A and B tiles (the waves verifying rows,
        // then those verifying columns), |x|, |y|
        if (w < G::kVW) {
            const double f = sum64(nrm2);
            if (lane == 0) sm.wsum[w][2] = f;
            if (kPre && FP8) {
                // the tile's largest magnitudes, from the per-line maxima
                const double ra = is_row && x < hrows ? g.row_max[i0 + x] : 0.0;
                const double cb = is_col && x < wcols ? g.col_max[j0 + x] : 0.0;
                const double a = max64(ra), b = max64(cb);
                if (lane == 0) { sm.wsum[w][3] = a; sm.wsum[w][4] = b; }
            }
        }
        __syncthreads();
        if (t == 0) {
            double sx = 0, sy = 0, ma = 0, mb = 0;
#pragma unroll
            for (int v = 0; v < NW; ++v) {
                sx += sm.wsum[v][0]; sy += sm.wsum[v][1];
                ma = fmax(ma, sm.wsum[v][3]); mb = fmax(mb, sm.wsum[v][4]);
            }
            sm.scal[0] = sx;                                // |x|^2
            sm.scal[1] = sy;                                // |y|^2
            sm.scal[4] = ma;                                // max|A_I|
            sm.scal[5] = mb;                                // max|B_J|
            double fa = 0, fb = 0;
#pragma unroll
            for (int v = 0; v < G::kVW; ++v) (v < G::kRW ? fa : fb) += sm.wsum[v][2];
            sm.scal[2] = fa;                                // |A_I|_F^2
            sm.scal[3] = fb;                                // |B_J|_F^2
        }
        __syncthreads();

        {
            const double sqk = sqrt((double)k);
            double ratio = 0.0;
            if (is_row || (is_col && !kOne)) {
                double P = g.alpha * (is_row ? sm.u.epi.fin_row[x] : sm.u.epi.fin_col[x]);
                double R = 0.0, cs = 0.0, c2 = 0.0;
                if (is_row) {
#pragma unroll
                    for (int v = 0; v < G::WN; ++v) {
                        R += sm.u.epi.ref_row[v][x];
                        cs += sm.u.epi.cin_row[v][x];
                        c2 += sm.u.epi.cin2_row[v][x];
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < G::WM; ++v) {
                        R += sm.u.epi.ref_col[v][x];
                        cs += sm.u.epi.cin_col[v][x];
                        c2 += sm.u.epi.cin2_col[v][x];
                    }
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
                double tau = is_row
                    ? ft_threshold(kLambda, U, sqk, sqrt((double)wcols), g.alpha, sqrt(nrm2),
                                   sqrt(sm.scal[3]), sqrt(sm.scal[1]), g.beta, sqrt(c2))
                    : ft_threshold(kLambda, U, sqk, sqrt((double)hrows), g.alpha, sqrt(nrm2),
                                   sqrt(sm.scal[2]), sqrt(sm.scal[0]), g.beta, sqrt(c2));
                if (FP8)
                    tau += kLambda * fabs(g.alpha) * kTruncGrid * sqrt((double)kTruncGroup) *
                           sqrt((double)(is_row ? wcols : hrows)) *
                           (is_row ? sm.scal[5] : sm.scal[4]) * sqrt(nrm2);
                const double d = R - P;
                if (is_row) {
                    sm.u.epi.fin_row[x] = P; sm.u.epi.tau_row[x] = tau; sm.u.epi.d_row[x] = d;
                } else {
                    sm.u.epi.fin_col[x] = P; sm.u.epi.tau_col[x] = tau; sm.u.epi.d_col[x] = d;
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
            if (w < G::kVW) {
                ratio = max64(ratio);
                if (lane == 0) sm.wratio[w] = ratio;
            }
        }
        __syncthreads();
        if (t == 0) {
            double r = 0.0;
#pragma unroll
            for (int v = 0; v < G::kVW; ++v) r = fmax(r, sm.wratio[v]);
            atomic_max_nonneg(&g.counters->max_ratio_bits, r);
        }

        const int nr = sm.nbad_r, nc = sm.nbad_c;
        if (nr == 0 && nc == 0) {
            if (attempt == 1) kind = FTGEMM_KIND_RECOMPUTED;
            break;
        }
        if (attempt == 1) {
            kind = FTGEMM_KIND_UNCORRECTABLE;
            break;
        }
        first_nr = nr; first_nc = nc;
        first_i = nr ? sm.ibad : -1;
        first_j = nc ? sm.jbad : -1;

        if (kOne) {
            // one side: neither the column of a data fault nor a checksum
            // fault can be told apart -- the tile is computed again
        } else if (nr == 1 && nc == 1) {
            const int is = first_i, js = first_j;
            double s_col = 0.0, s_row = 0.0;
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < NI; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm * 64 + 16 * mi + 4 * q + r;
                        const int col = wn * G::WC + 16 * ni + c16;
                        const double o = (double)acc[mi][ni][r];
                        if (col == js && row != is) s_col += o;
                        if (row == is && col != js) s_row += o;
                    }
            s_col = sum64(s_col);
            s_row = sum64(s_row);
            __syncthreads();
            if (lane == 0) { sm.red[w][0] = s_col; sm.red[w][1] = s_row; }
            __syncthreads();
            double sc = 0.0, sr = 0.0;
#pragma unroll
            for (int v = 0; v < NW; ++v) { sc += sm.red[v][0]; sr += sm.red[v][1]; }
            const double fixed = sm.u.epi.fin_col[js] - sc;
            const float fixed_f = (float)fixed;
            if (fabs(sr + (double)fixed_f - sm.u.epi.fin_row[is]) <= sm.u.epi.tau_row[is]) {
                if (w == owner_wave<BM>(is, js)) {
                    const int ol = owner_lane(is, js), sel = owner_reg<BM>(is, js);
#pragma unroll
                    for (int e = 0; e < G::NREG; ++e)
                        if (sel == e && lane == ol) {
                            rec_before = (double)acc[e / (4 * NI)][(e >> 2) % NI][e & 3];
                            acc[e / (4 * NI)][(e >> 2) % NI][e & 3] = fixed_f;
                        }
                }
                rec_after = (double)fixed_f;
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
            if (fabs(dl - sumd) <= (by_row ? sm.u.epi.tau_row[line] : sm.u.epi.tau_col[line])) {
                // each crossing's residual at its position along the line
                // (the encoded-sum partials are no longer needed)
                double *lfix = sm.u.epi.enc_row[0];
                for (int x = t; x < (by_row ? TN : BM); x += NT) lfix[x] = 0.0;
                __syncthreads();
                if (t < nfix) {
                    const int cf = by_row ? sm.bad_c[t] : sm.bad_r[t];
                    lfix[cf] = by_row ? sm.u.epi.d_col[cf] : sm.u.epi.d_row[cf];
                }
                __syncthreads();
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = wm * 64 + 16 * mi + 4 * q + r;
                            const int col = wn * G::WC + 16 * ni + c16;
                            if ((by_row ? row : col) != line) continue;
                            const int at = by_row ? col : row;
                            const double d = lfix[at];
                            if (d == 0.0) continue;
                            const bool named = at == (by_row ? first_j : first_i);
                            if (named) rec_before = (double)acc[mi][ni][r];
                            acc[mi][ni][r] = (float)((double)acc[mi][ni][r] - d);
                            if (named) rec_after = (double)acc[mi][ni][r];
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
            if (t == 0) {
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
            // A lone disagreement is a checksum fault only beyond its own
            // threshold plus twice the other side's largest (a data error
            // shows on both sides); within that bound the tile is computed
            // again.  FP32 thresholds of the two sides differ by the
            // operands' norms, so a data error can pass one and not the other.
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
        __syncthreads();
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
        const int wm = w % G::WM, wn = w / G::WM, q = lane >> 4, c16 = lane & 15;
        if (kind == FTGEMM_KIND_CORRECTED && npairs == 0) {
            __syncthreads();
            if (w == owner_wave<BM>(first_i, first_j) && lane == owner_lane(first_i, first_j)) {
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
        const bool vec = ((reinterpret_cast<uintptr_t>(C) | ((uintptr_t)ldc << 2)) & 15) == 0;
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni)
                store_rows4(C, ldc, i0, j0, wm * 64 + 16 * mi + 4 * q,
                            wn * G::WC + 16 * ni + c16, hrows, wcols, vec, acc[mi][ni]);
        if (npairs > 0) {
            // Paired corrections: the lane that stored each element takes
            // the pair's residual off it in memory (its own store is ordered
            // before its atomics on the same address); the named element's
            // old and new values complete the record.
            const int *pcol = reinterpret_cast<const int *>(sm.u.epi.enc_row[1]);
            const double *pd = sm.u.epi.enc_row[0];
            for (int f = 0; f < npairs; ++f) {
                const int i = sm.bad_r[f], j = pcol[i];
                if (w != owner_wave<BM>(i, j) || lane != owner_lane(i, j)) continue;
                unsigned *a = reinterpret_cast<unsigned *>(C + (i0 + i) + (j0 + j) * ldc);
                unsigned cur = atomicOr(a, 0u);
                float before = __uint_as_float(cur);
                float after = (float)((double)before - pd[i]);
                for (int it = 0; it < 4; ++it) {
                    const unsigned prev = atomicCAS(a, cur, __float_as_uint(after));
                    if (prev == cur) break;
                    cur = prev;
                    before = __uint_as_float(cur);
                    after = (float)((double)before - pd[i]);
                }
                if (i == first_i) {
                    sm.red[2][0] = (double)before;
                    sm.red[2][1] = (double)after;
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

template <bool FP8, bool TA, bool TB, bool ABFT, int BM, bool ONE, bool PRE>
__global__ __launch_bounds__(NT, 2) void kernel(GemmArgs g)
{
    __shared__ Smem<BM> sm;
    int tm_, tn_;
    map_tile(blockIdx.x, g.tiles_m, g.tiles_n, tm_, tn_);
    tile<FP8, TA, TB, ABFT, BM, ONE, PRE>(g, tm_, tn_, sm);
}

// Default tile rows of the batched kernel (problems of mixed, often small,
// shapes); each problem may take 256-row tiles instead (GemmArgs::tile_rows,
// chosen per problem by the batch's tuning).
constexpr int kBatchBM = 128;

// Persistent batched kernel: workgroup w starts on queue w mod nqueues (with
// one queue per XCD, the XCD it runs on) and moves on to the others when it
// runs dry; every workgroup leaves once all queues are drained.  A work
// item runs the 128- or the 256-row tile as its problem says; the two share
// one LDS area.
// ROWS: 128 or 256 when every problem of the batch takes tiles of that
// many rows, 0 when they are mixed (the kernel then holds both tile codes,
// and the registers of the larger).
template <bool FP8, bool TA, bool TB, bool ABFT, int ROWS>
__global__ __launch_bounds__(NT, 2) void batched_kernel(BatchArgs b)
{
    constexpr size_t kBytes = ROWS == 128 ? sizeof(Smem<128>)
                              : ROWS == 256 ? sizeof(Smem<256>)
                              : sizeof(Smem<256>) > sizeof(Smem<128>) ? sizeof(Smem<256>)
                                                                      : sizeof(Smem<128>);
    __shared__ __align__(16) unsigned char smem[kBytes];
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
            if (ROWS == 256 || (ROWS == 0 && g.tile_rows == 256))
                tile<FP8, TA, TB, ABFT, 256>(g, w.tile_m, w.tile_n,
                                             *reinterpret_cast<Smem<256> *>(smem));
            else
                tile<FP8, TA, TB, ABFT, kBatchBM>(g, w.tile_m, w.tile_n,
                                                  *reinterpret_cast<Smem<kBatchBM> *>(smem));
            __syncthreads();
        }
    }
}

// Kernels built in a translation unit of their own, ftgemm_lp_ilp.hip, which
// includes this file with FTG_LP_OWN_UNIT defined and is compiled with the
// compiler's iterative ILP scheduling strategy: the BF16 two-sided kernels
// on 256-row tiles (norms from the pass before the product, or from the
// tiles), and the FP8 one-sided kernel on 256-row tiles (measured 4-5%
// faster with that strategy, where the others measured slower, FP8
// two-sided by 45%).
hipError_t launch_own_unit(const GemmArgs &g, bool fp8, bool ta, bool tb, int mode, bool pre,
                           hipStream_t stream);

#ifdef FTG_LP_OWN_UNIT
hipError_t launch_own_unit(const GemmArgs &g, bool fp8, bool ta, bool tb, int mode, bool pre,
                           hipStream_t stream)
{
    const unsigned grid = (unsigned)g.tiles_m * (unsigned)g.tiles_n;
    if (grid == 0) return hipSuccess;
#define FTG_LP_OWN(F, a, b, d, e) \
    hipLaunchKernelGGL((kernel<F, a, b, true, 256, d, e>), dim3(grid), dim3(NT), 0, stream, g)
#define FTG_LP_OWN_T(F, d, e)                                  \
    do {                                                       \
        if (!ta && !tb) FTG_LP_OWN(F, false, false, d, e);     \
        else if (!ta && tb) FTG_LP_OWN(F, false, true, d, e);  \
        else if (ta && !tb) FTG_LP_OWN(F, true, false, d, e);  \
        else FTG_LP_OWN(F, true, true, d, e);                  \
    } while (0)
    if (fp8 && mode == 2 && pre) FTG_LP_OWN_T(true, true, true);
    else if (!fp8 && mode == 1 && pre) FTG_LP_OWN_T(false, false, true);
    else if (!fp8 && mode == 1) FTG_LP_OWN_T(false, false, false);
    else return hipErrorInvalidValue;
#undef FTG_LP_OWN_T
#undef FTG_LP_OWN
    return hipGetLastError();
}
#else
template <bool FP8, int ROWS>
hipError_t launch_batched_rows(const BatchArgs &b, bool ta, bool tb, bool abft, int grid,
                               hipStream_t stream)
{
#define FTG_LP_BCASE(x, y, z) \
    hipLaunchKernelGGL((batched_kernel<FP8, x, y, z, ROWS>), dim3(grid), dim3(NT), 0, stream, b)
    if (abft) {
        if (!ta && !tb) FTG_LP_BCASE(false, false, true);
        else if (!ta && tb) FTG_LP_BCASE(false, true, true);
        else if (ta && !tb) FTG_LP_BCASE(true, false, true);
        else FTG_LP_BCASE(true, true, true);
    } else {
        if (!ta && !tb) FTG_LP_BCASE(false, false, false);
        else if (!ta && tb) FTG_LP_BCASE(false, true, false);
        else if (ta && !tb) FTG_LP_BCASE(true, false, false);
        else FTG_LP_BCASE(true, true, false);
    }
#undef FTG_LP_BCASE
    return hipGetLastError();
}

template <bool FP8>
hipError_t launch_batched(const BatchArgs &b, bool ta, bool tb, bool abft, int grid,
                          hipStream_t stream)
{
    if (b.rows == 128) return launch_batched_rows<FP8, 128>(b, ta, tb, abft, grid, stream);
    if (b.rows == 256) return launch_batched_rows<FP8, 256>(b, ta, tb, abft, grid, stream);
    return launch_batched_rows<FP8, 0>(b, ta, tb, abft, grid, stream);
}

template <bool FP8, int BM>
hipError_t launch(const GemmArgs &g, bool ta, bool tb, int mode, bool pre, hipStream_t stream)
{
    const unsigned grid = (unsigned)g.tiles_m * (unsigned)g.tiles_n;
    if (grid == 0) return hipSuccess;
#define FTG_LP_CASE(a, b, c, d, e) \
    hipLaunchKernelGGL((kernel<FP8, a, b, c, BM, d, e>), dim3(grid), dim3(NT), 0, stream, g)
#define FTG_LP_MODE(c, d, e)                                   \
    do {                                                       \
        if (!ta && !tb) FTG_LP_CASE(false, false, c, d, e);    \
        else if (!ta && tb) FTG_LP_CASE(false, true, c, d, e); \
        else if (ta && !tb) FTG_LP_CASE(true, false, c, d, e); \
        else FTG_LP_CASE(true, true, c, d, e);                 \
    } while (0)
    if (mode == 2) {
        if constexpr (FP8 && BM == 256) return launch_own_unit(g, FP8, ta, tb, mode, pre, stream);
        else FTG_LP_MODE(true, true, true);
    } else if (mode == 1 && pre) {
        if constexpr (!FP8 && BM == 256) return launch_own_unit(g, FP8, ta, tb, mode, pre, stream);
        else FTG_LP_MODE(true, false, true);
    } else if (mode == 1) {
        if constexpr (!FP8 && BM == 256) return launch_own_unit(g, FP8, ta, tb, mode, pre, stream);
        else FTG_LP_MODE(true, false, false);
    } else {
        FTG_LP_MODE(false, false, false);
    }
#undef FTG_LP_MODE
#undef FTG_LP_CASE
    return hipGetLastError();
}

#endif  // FTG_LP_OWN_UNIT

}  // namespace lp

#ifndef FTG_LP_OWN_UNIT
hipError_t launch_lp(const GemmArgs &g, bool fp8, bool ta, bool tb, int mode, bool pre, int tm,
                     hipStream_t stream)
{
    if (mode < 0 || mode > 2 || (mode == 2 && !pre)) return hipErrorInvalidValue;
    // the kernels that take their norms from g also take the operand
    // checksums from it (op(A)'s only in two-sided mode)
    if (pre && mode != 0 && (!g.ysum || (mode == 1 && !g.xsum) || g.ldxs < g.k))
        return hipErrorInvalidValue;
    if (tm == 256)
        return fp8 ? lp::launch<true, 256>(g, ta, tb, mode, pre, stream)
                   : lp::launch<false, 256>(g, ta, tb, mode, pre, stream);
    if (tm != 128) return hipErrorInvalidValue;
    return fp8 ? lp::launch<true, 128>(g, ta, tb, mode, pre, stream)
               : lp::launch<false, 128>(g, ta, tb, mode, pre, stream);
}

hipError_t launch_lp_batched(const BatchArgs &b, bool fp8, bool ta, bool tb, bool abft, int grid,
                             hipStream_t stream)
{
    return fp8 ? lp::launch_batched<true>(b, ta, tb, abft, grid, stream)
               : lp::launch_batched<false>(b, ta, tb, abft, grid, stream);
}

// 256-row tiles once they still give every compute unit a tile (they do
// twice the matrix work per staged byte of the 128-row tiles), 128 rows
// otherwise and in batches.  The two-sided fault-tolerant FP8 kernel that
// forms its operand checksums and norms in the tile (in_tile: the entry
// point that allocates nothing) keeps 128-row tiles: at 256 rows those
// registers no longer fit beside the accumulators.
void tiling_lp(bool fp8, int mode, int64_t m, int64_t n, bool batched, bool in_tile, int *tm,
               int *tn, int *bk)
{
    const int64_t tiles256 = ((m + 255) / 256) * ((n + lp::TN - 1) / lp::TN);
    const bool large =
        !batched && !(fp8 && mode == 1 && in_tile) && tiles256 >= kLargeTileMin;
    *tm = large ? 256 : lp::kBatchBM;
    *tn = lp::TN;
    *bk = fp8 ? lp::Elem<true>::BK : lp::Elem<false>::BK;
}
#endif  // FTG_LP_OWN_UNIT

}  // namespace ftg
