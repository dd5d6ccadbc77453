// ftgemm_host.cpp -- the C ABI of libftgemm: argument checks, quick returns,
// the per-GPU workspace (report area, fault plan), launches and report
// copy-back.  Declarations and the contract are in include/ftgemm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/ftgemm.h"
#include "ftgemm_kernels.h"

namespace {

using ftg::DevCounters;
using ftg::GemmArgs;

thread_local int32_t t_last_invalid = 0;

constexpr uint32_t kDevRecordCap = 4096;

std::mutex g_mu;
std::vector<ftgemm_injection> g_plan;
uint64_t g_plan_version = 1;

struct DeviceWs {
    DevCounters *counters = nullptr;         // device, kMaxCounters entries
    int counters_cap = 0;
    ftgemm_fault_record *records = nullptr;  // device
    ftgemm_injection *plan = nullptr;        // device
    ftgemm_injection_echo *echo = nullptr;   // device
    int plan_cap = 0;
    int nplan = 0;
    uint64_t plan_version = 0;
    // pinned host staging for report copy-back
    DevCounters *h_counters = nullptr;
    ftgemm_fault_record *h_records = nullptr;
    ftgemm_injection_echo *h_echo = nullptr;
    int h_echo_cap = 0;
    // split inner dimension (FP64): partial products, slice checksums; or
    // the line norms of the one-sided low-precision mode
    double *split = nullptr;
    size_t split_bytes = 0;
    // unfused mode: checksums, sums, norms and its checksum products' slices
    double *uf = nullptr;
    size_t uf_bytes = 0;
    // auxiliary counters: [0] record slots, [1 ..] batched work queues
    unsigned int *aux = nullptr;
    unsigned int *h_aux = nullptr;
    // batched launches: per-problem arguments, work items, captured graph
    ftg::GemmArgs *d_probs = nullptr, *h_probs = nullptr;
    int probs_cap = 0;
    ftg::WorkItem *d_items = nullptr, *h_items = nullptr;
    int items_cap = 0;
    hipEvent_t staged = nullptr;  // the last upload from the host staging
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> graph_key;
    int cus = 0;
};

constexpr int kAuxWords = 16;

std::unordered_map<int, DeviceWs> g_ws;

// The tuning table.  Its text form, one entry per line ('#' starts a
// comment):
//   tile <dtype> <abft> <rows>       single low-precision calls of that
//                                    dtype (1 BF16, 2 FP8) and mode take
//                                    tiles of 128 or 256 rows
//   batch_mstar <m>                  in low-precision batches, problems with
//                                    at least m rows take 256-row tiles (the
//                                    threshold is then not tuned; -1: tuned)
//   batch <signature> <schedule> <m> a batch tuned before: its signature
//                                    (hex), work order and threshold
// It is read from the file FTGEMM_TUNE_TABLE names (when set) at the first
// call that needs it, or from the file ftgemm_load_tune_table names; batches
// tuned afterwards are appended to that file.
constexpr int64_t kNoBigTiles = INT64_MAX;
struct TuneTable {
    bool loaded = false;
    std::string path;             // where tuned batches are appended ("": nowhere)
    int single_rows[3][3] = {};   // [dtype][abft], 0: the default choice
    int64_t batch_mstar = -1;     // forced threshold, -1: tuned
    std::unordered_map<uint64_t, std::pair<int, int64_t>> batches;
};
std::mutex g_tune_mu;
TuneTable g_tune;

// Parse a table file into t; false when the file cannot be read or a line
// is malformed.
bool parse_table(const char *path, TuneTable &t)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool ok = true;
    while (std::fgets(line, sizeof line, f)) {
        if (char *c = std::strchr(line, '#')) *c = 0;
        char key[32];
        if (std::sscanf(line, "%31s", key) != 1) continue;
        if (!std::strcmp(key, "tile")) {
            int dt, ab, rows;
            if (std::sscanf(line, "%*s %d %d %d", &dt, &ab, &rows) != 3 || dt < 1 || dt > 2 ||
                ab < 0 || ab > 2 || (rows != 128 && rows != 256)) {
                ok = false;
                break;
            }
            t.single_rows[dt][ab] = rows;
        } else if (!std::strcmp(key, "batch_mstar")) {
            long long v;
            if (std::sscanf(line, "%*s %lld", &v) != 1) { ok = false; break; }
            t.batch_mstar = v < 0 ? -1 : (int64_t)v;
        } else if (!std::strcmp(key, "batch")) {
            unsigned long long sig;
            int sched;
            long long mstar;
            if (std::sscanf(line, "%*s %llx %d %lld", &sig, &sched, &mstar) != 3 || sched < 0 ||
                sched > 2) {
                ok = false;
                break;
            }
            t.batches[(uint64_t)sig] = {sched, mstar < 0 ? kNoBigTiles : (int64_t)mstar};
        } else {
            ok = false;
            break;
        }
    }
    std::fclose(f);
    return ok;
}

// The table, read from FTGEMM_TUNE_TABLE on first use.  Called with
// g_tune_mu held.
TuneTable &tune_table()
{
    if (!g_tune.loaded) {
        g_tune.loaded = true;
        if (const char *e = std::getenv("FTGEMM_TUNE_TABLE")) {
            g_tune.path = e;
            TuneTable t;
            if (parse_table(e, t)) {
                t.loaded = true;
                t.path = e;
                g_tune = t;
            }
        }
    }
    return g_tune;
}

// Record a tuned batch in the table and append it to the table's file.
void remember_batch(uint64_t sig, int sched, int64_t mstar)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    TuneTable &t = tune_table();
    t.batches[sig] = {sched, mstar};
    if (t.path.empty()) return;
    if (FILE *f = std::fopen(t.path.c_str(), "a")) {
        std::fprintf(f, "batch %016llx %d %lld\n", (unsigned long long)sig, sched,
                     mstar == kNoBigTiles ? -1LL : (long long)mstar);
        std::fclose(f);
    }
}

ftgemm_status invalid(int pos)
{
    t_last_invalid = pos;
    return FTGEMM_ERR_INVALID_ARG;
}

// HIP failures become FTGEMM_ERR_HIP (or _NO_MEMORY); with FTGEMM_VERBOSE
// set in the environment the failing call and HIP's message go to stderr.
void report_hip_failure(const char *what, hipError_t e)
{
    static const bool verbose = std::getenv("FTGEMM_VERBOSE") != nullptr;
    if (verbose)
        std::fprintf(stderr, "libftgemm: %s failed: %s\n", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) {                        \
            report_hip_failure(#expr, e_);             \
            if (e_ == hipErrorOutOfMemory)             \
                return FTGEMM_ERR_NO_MEMORY;           \
            return FTGEMM_ERR_HIP;                     \
        }                                              \
    } while (0)

// Per-GPU workspace with room for `ncounters` report areas; uploads the
// current fault plan when it changed.  Called with g_mu held.
ftgemm_status workspace(DeviceWs **out, int ncounters)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    DeviceWs &ws = g_ws[dev];
    if (!ws.records) {
        HIP_TRY(hipMalloc((void **)&ws.records, sizeof(ftgemm_fault_record) * kDevRecordCap));
        HIP_TRY(hipHostMalloc((void **)&ws.h_records,
                              sizeof(ftgemm_fault_record) * kDevRecordCap, hipHostMallocDefault));
        HIP_TRY(hipMalloc((void **)&ws.aux, sizeof(unsigned int) * kAuxWords));
        HIP_TRY(hipMemset(ws.aux, 0, sizeof(unsigned int) * kAuxWords));
        HIP_TRY(hipHostMalloc((void **)&ws.h_aux, sizeof(unsigned int) * kAuxWords,
                              hipHostMallocDefault));
        HIP_TRY(hipDeviceGetAttribute(&ws.cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    if (ws.counters_cap < ncounters) {
        if (ws.counters) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ws.counters));
            HIP_TRY(hipHostFree(ws.h_counters));
        }
        const int cap = ncounters < 16 ? 16 : ncounters;
        HIP_TRY(hipMalloc((void **)&ws.counters, sizeof(DevCounters) * cap));
        HIP_TRY(hipHostMalloc((void **)&ws.h_counters, sizeof(DevCounters) * cap,
                              hipHostMallocDefault));
        HIP_TRY(hipMemset(ws.counters, 0, sizeof(DevCounters) * cap));
        ws.counters_cap = cap;
    }
    if (ws.plan_version != g_plan_version) {
        const int n = (int)g_plan.size();
        if (n > ws.plan_cap) {
            HIP_TRY(hipDeviceSynchronize());
            if (ws.plan) {
                HIP_TRY(hipFree(ws.plan));
                HIP_TRY(hipFree(ws.echo));
                HIP_TRY(hipHostFree(ws.h_echo));
            }
            HIP_TRY(hipMalloc((void **)&ws.plan, sizeof(ftgemm_injection) * n));
            HIP_TRY(hipMalloc((void **)&ws.echo, sizeof(ftgemm_injection_echo) * n));
            HIP_TRY(hipHostMalloc((void **)&ws.h_echo, sizeof(ftgemm_injection_echo) * n,
                                  hipHostMallocDefault));
            ws.plan_cap = n;
        }
        if (n > 0) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipMemcpy(ws.plan, g_plan.data(), sizeof(ftgemm_injection) * n,
                              hipMemcpyHostToDevice));
        }
        ws.nplan = n;
        ws.plan_version = g_plan_version;
    }
    *out = &ws;
    return FTGEMM_OK;
}

// Device scratch for a split inner dimension, grown on demand (the device is
// synchronised first: an earlier call may still be using it).
ftgemm_status split_space(DeviceWs &ws, size_t bytes)
{
    if (bytes <= ws.split_bytes) return FTGEMM_OK;
    if (ws.split) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(ws.split));
        ws.split = nullptr;
        ws.split_bytes = 0;
    }
    HIP_TRY(hipMalloc((void **)&ws.split, bytes));
    ws.split_bytes = bytes;
    return FTGEMM_OK;
}

// Number of inner-dimension slices for an FP64 problem: enough workgroups
// for two per compute unit when the output alone has fewer tiles than
// compute units and the inner dimension is at least 32 steps long, each
// slice at least 8 steps long and the partial products within 1 GiB.
// *slice_k is a multiple of bk.
constexpr int64_t kSplitTargetWgs = 512;
constexpr int64_t kSplitMaxSlices = 16;
constexpr int64_t kSplitMaxBytes = int64_t(1) << 30;

int choose_split(int64_t m, int64_t n, int64_t k, int tm, int tn, int bk, int64_t *slice_k)
{
    *slice_k = k;
    const int64_t tiles = ((m + tm - 1) / tm) * ((n + tn - 1) / tn);
    if (tiles == 0 || tiles >= 256 || k < 32 * bk) return 1;
    int64_t s = (kSplitTargetWgs + tiles - 1) / tiles;
    if (s > k / (8 * bk)) s = k / (8 * bk);
    if (s > kSplitMaxSlices) s = kSplitMaxSlices;
    while (s > 1 && s * m * n * 8 > kSplitMaxBytes) --s;
    if (s <= 1) return 1;
    const int64_t steps = (k + bk - 1) / bk;
    const int64_t per = (steps + s - 1) / s;
    *slice_k = per * bk;
    return (int)((k + *slice_k - 1) / *slice_k);
}

double unpack_ratio(unsigned long long bits)
{
    double v;
    std::memcpy(&v, &bits, sizeof v);
    return v;
}

// Host copies of a report area: counters per problem, the record-slot
// counter, the record slots and the echo slots of the plan's faults.
struct HostReport {
    const DevCounters *h_counters;
    const unsigned int *h_aux;
    const ftgemm_fault_record *h_records;
    const ftgemm_injection_echo *h_echo;
    int nplan;
    uint32_t rec_cap;
};

HostReport host_report(const DeviceWs &ws)
{
    return HostReport{ws.h_counters, ws.h_aux, ws.h_records, ws.h_echo, ws.nplan, kDevRecordCap};
}

// Copy the report area of problem `p` (and the echo slots of its faults)
// into the caller's report; the stream has been synchronised.
void fill_report(const HostReport &ws, int p, ftgemm_report *rep, int32_t problem)
{
    const uint32_t rec_cap = ws.rec_cap;
    const DevCounters &c = ws.h_counters[p];
    rep->tiles_verified = c.tiles_verified;
    rep->detected = c.detected;
    rep->corrected = c.corrected;
    rep->checksum_only = c.checksum_only;
    rep->recomputed = c.recomputed;
    rep->uncorrectable = c.uncorrectable;
    rep->max_ratio = unpack_ratio(c.max_ratio_bits);
    rep->record_count = 0;
    rep->echo_count = 0;
    // record slots are shared by the problems of a call (h_aux[0] taken)
    const uint32_t nslot = ws.h_aux[0] < rec_cap ? ws.h_aux[0] : rec_cap;
    uint32_t kept = 0;
    for (uint32_t r = 0; r < nslot; ++r) {
        const ftgemm_fault_record &src = ws.h_records[r];
        if (src.problem != problem) continue;
        if (rep->records && kept < rep->record_capacity) rep->records[kept] = src;
        kept++;
    }
    rep->record_count = c.record_count;  // also those that found no slot
    for (int q = 0; q < ws.nplan; ++q) {
        if (g_plan[q].problem != problem) continue;
        if (rep->echoes && rep->echo_count < rep->echo_capacity) {
            ftgemm_injection_echo e = ws.h_echo[q];
            if (!e.applied) {
                e.problem = problem;
                e.row = g_plan[q].row;
                e.col = g_plan[q].col;
                e.k_index = g_plan[q].k_index;
                e.before = e.after = 0.0;
            }
            rep->echoes[rep->echo_count] = e;
        }
        rep->echo_count++;
    }
}

size_t elem_size(ftgemm_dtype dt)
{
    return dt == FTGEMM_F64 ? 8 : dt == FTGEMM_BF16 ? 2 : 1;
}

// The loaders address one step of an operand through a buffer resource of at
// most 2^31 - 1 bytes with 32-bit byte offsets, and the norms pass reads one
// stored column per resource.  A call whose windows do not fit would read
// zeros or wrapped addresses without any sign, so it is refused: position 8
// or 10 when the leading dimension makes a step's window too wide, 3, 4 or 5
// when one stored column of an operand alone exceeds it.
int check_windows(const ftgemm_gemm_desc &d)
{
    const int64_t lim = INT32_MAX;
    const int64_t eb = (int64_t)elem_size(d.dtype);
    // largest outer extent of a tile, and the inner span of one step
    const int64_t outer = d.dtype == FTGEMM_F64 ? 128 : 256;
    const int64_t span = d.dtype == FTGEMM_F64 ? 32 : d.dtype == FTGEMM_BF16 ? 64 : 128;
    struct Op { bool outer_contig; int64_t rows, cols, ld; int pos_ld, pos_rows; };
    const Op ops[2] = {
        {d.transA == FTGEMM_OP_N, d.transA == FTGEMM_OP_N ? d.m : d.k,
         d.transA == FTGEMM_OP_N ? d.k : d.m, d.lda, 8, d.transA == FTGEMM_OP_N ? 3 : 5},
        {d.transB == FTGEMM_OP_T, d.transB == FTGEMM_OP_N ? d.k : d.n,
         d.transB == FTGEMM_OP_N ? d.n : d.k, d.ldb, 10, d.transB == FTGEMM_OP_N ? 5 : 4}};
    if (d.m == 0 || d.n == 0 || d.k == 0) return 0;
    for (const Op &o : ops) {
        if (o.rows * eb > lim) return o.pos_rows;
        const int64_t scols = o.outer_contig ? std::min(span, o.cols) : std::min(outer, o.cols);
        const int64_t srows = o.outer_contig ? std::min(outer, o.rows) : std::min(span, o.rows);
        // elements from the window's first element to the last one a step reads
        if (scols > 1 && o.ld > (lim / eb - srows) / (scols - 1)) return o.pos_ld;
    }
    // the beta pass reads C_in through one window per tile (its 128
    // columns of up to 128 FP64 or 256 FP32 rows), with 32-bit offsets
    const int64_t ceb = d.dtype == FTGEMM_F64 ? 8 : 4;
    if (d.n > 1 && d.ldc > (lim / ceb - outer) / (std::min<int64_t>(128, d.n) - 1)) return 13;
    return 0;
}

// Tile of a single low-precision call: the default choice, or the table's.
// in_tile: the call forms its operand checksums and norms in the tiles.
void lp_tiling(const ftgemm_gemm_desc &d, int *tm, int *tn, int *bk, bool in_tile = false)
{
    ftg::tiling_lp(d.dtype == FTGEMM_FP8_E4M3, d.abft, d.m, d.n, false, in_tile, tm, tn, bk);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const int rows = tune_table().single_rows[d.dtype][d.abft < 3 ? d.abft : 0];
    if (rows) *tm = rows;
}

// Argument checks in BLAS order; returns 0 or the 1-based position.
int check_args(const ftgemm_gemm_desc &d)
{
    if (d.transA != FTGEMM_OP_N && d.transA != FTGEMM_OP_T) return 1;
    if (d.transB != FTGEMM_OP_N && d.transB != FTGEMM_OP_T) return 2;
    if (d.m < 0) return 3;
    if (d.n < 0) return 4;
    if (d.k < 0) return 5;
    if (!std::isfinite(d.alpha)) return 6;
    const int64_t arows = d.transA == FTGEMM_OP_N ? d.m : d.k;
    const int64_t brows = d.transB == FTGEMM_OP_N ? d.k : d.n;
    const bool need_ab = d.m > 0 && d.n > 0 && d.k > 0 && d.alpha != 0.0;
    if (need_ab && !d.A) return 7;
    if (d.lda < (arows > 1 ? arows : 1)) return 8;
    if (need_ab && !d.B) return 9;
    if (d.ldb < (brows > 1 ? brows : 1)) return 10;
    if (!std::isfinite(d.beta)) return 11;
    if (d.m > 0 && d.n > 0 && !d.C) return 12;
    if (d.ldc < (d.m > 1 ? d.m : 1)) return 13;
    if (d.dtype != FTGEMM_F64 && d.dtype != FTGEMM_BF16 && d.dtype != FTGEMM_FP8_E4M3)
        return 14;
    if (d.dtype == FTGEMM_FP8_E4M3 &&
        !(std::isfinite(d.scaleA) && std::isfinite(d.scaleB) && d.scaleA > 0 && d.scaleB > 0))
        return 14;
    if (d.abft < 0 || d.abft > 4) return 14;
    if (d.m > INT32_MAX / 2 || d.n > INT32_MAX / 2) return d.m > INT32_MAX / 2 ? 3 : 4;
    return check_windows(d);
}

GemmArgs base_args(const ftgemm_gemm_desc &d, int tm, int tn)
{
    GemmArgs g{};
    g.A = d.A;
    g.B = d.B;
    g.C = d.C;
    g.m = d.m;
    g.n = d.n;
    g.k = d.k;
    g.lda = d.lda;
    g.ldb = d.ldb;
    g.ldc = d.ldc;
    g.alpha = d.dtype == FTGEMM_FP8_E4M3 ? d.alpha * d.scaleA * d.scaleB : d.alpha;
    g.beta = d.beta;
    g.problem = 0;
    g.tiles_m = (int32_t)((d.m + tm - 1) / tm);
    g.tiles_n = (int32_t)((d.n + tn - 1) / tn);
    g.tile_rows = tm;
    g.k_base = 0;
    return g;
}

// The device report of a single call into rep (waits for the stream).
ftgemm_status copy_report(DeviceWs &ws, ftgemm_report *rep, hipStream_t stream, int32_t problem)
{
    HIP_TRY(hipMemcpyAsync(ws.h_counters, ws.counters, sizeof(DevCounters),
                           hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(ws.h_aux, ws.aux, sizeof(unsigned int), hipMemcpyDeviceToHost,
                           stream));
    HIP_TRY(hipMemcpyAsync(ws.h_records, ws.records, sizeof(ftgemm_fault_record) * kDevRecordCap,
                           hipMemcpyDeviceToHost, stream));
    if (ws.nplan)
        HIP_TRY(hipMemcpyAsync(ws.h_echo, ws.echo, sizeof(ftgemm_injection_echo) * ws.nplan,
                               hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    fill_report(host_report(ws), 0, rep, problem);
    return FTGEMM_OK;
}

// C = alpha op(A) op(B) + beta C with the checksum-free FP64 kernel (its
// inner dimension split as for any call: the slices' partial products in
// wsp, room for their checksums in chk).
ftgemm_status plain_f64(const double *A, int64_t lda, bool ta, const double *B, int64_t ldb,
                        bool tb, int64_t m, int64_t n, int64_t k, double alpha, double beta,
                        double *C, int64_t ldc, double *wsp, double *chk, DeviceWs &ws,
                        hipStream_t stream)
{
    int tm, tn, bk;
    ftg::tiling_f64(&tm, &tn, &bk);
    GemmArgs g{};
    g.A = A; g.B = B; g.C = C;
    g.m = m; g.n = n; g.k = k; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta;
    g.tiles_m = (int32_t)((m + tm - 1) / tm);
    g.tiles_n = (int32_t)((n + tn - 1) / tn);
    g.counters = ws.counters; g.records = ws.records; g.rec_slot = ws.aux;
    g.plan = ws.plan; g.echo = ws.echo;
    int64_t slice_k = k;
    const int ns = choose_split(m, n, k, tm, tn, bk, &slice_k);
    if (ns > 1) {
        g.nslices = ns; g.slice_k = slice_k; g.wsp = wsp; g.chk = chk;
    }
    HIP_TRY(ftg::launch_f64(g, ta, tb, false, stream));
    if (ns > 1) {
        ftg::ReduceArgs r{};
        r.C = C; r.wsp = wsp; r.chk = chk; r.m = m; r.n = n; r.ldc = ldc;
        r.alpha = alpha; r.beta = beta; r.nslices = ns;
        r.tiles_m = g.tiles_m; r.tiles_n = g.tiles_n;
        r.counters = ws.counters; r.records = ws.records; r.record_cap = kDevRecordCap;
        r.rec_slot = ws.aux;
        HIP_TRY(ftg::launch_splitk_reduce(r, false, stream));
    }
    return FTGEMM_OK;
}

// Room for plain_f64's slices of an m x n product: (partials, checksums).
std::pair<int64_t, int64_t> plain_split_space(int64_t m, int64_t n, int64_t k)
{
    int tm, tn, bk;
    ftg::tiling_f64(&tm, &tn, &bk);
    int64_t slice_k = k;
    const int ns = choose_split(m, n, k, tm, tn, bk, &slice_k);
    if (ns <= 1) return {0, 0};
    const int64_t tiles = ((m + tm - 1) / tm) * ((n + tn - 1) / tn);
    return {ns * m * n, ns * tiles * 2 * (tm + tn)};
}

// The unfused FP64 fault tolerance (detection only): the same per-tile
// checksums and thresholds as the fused kernel, formed by separate passes
// around the checksum-free GEMM.
ftgemm_status run_unfused(const ftgemm_gemm_desc &d, DeviceWs &ws, bool report,
                          hipStream_t stream, int32_t problem)
{
    constexpr int64_t T = 128;
    const int64_t m = d.m, n = d.n, k = d.k;
    const int64_t tm_ = (m + T - 1) / T, tn_ = (n + T - 1) / T;
    const int64_t kseg = (k + T - 1) / T;
    const bool ta = d.transA == FTGEMM_OP_T, tb = d.transB == FTGEMM_OP_T;
    const bool use_c = d.beta != 0.0;
    const auto sr = plain_split_space(tm_, n, k), sc = plain_split_space(m, tn_, k);
    const int64_t part = std::max(std::max(m, n), tm_) * kseg;
    int64_t need = tm_ * k + k * tn_ + 2 * (tm_ * n + m * tn_) + m + n + tm_ + tn_ + part +
                   std::max(sr.first, sc.first) + std::max(sr.second, sc.second);
    if (use_c) need += 2 * (tm_ * n + m * tn_);
    const size_t bytes = sizeof(double) * (size_t)need;
    if (bytes > ws.uf_bytes) {
        if (ws.uf) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(ws.uf));
            ws.uf = nullptr;
            ws.uf_bytes = 0;
        }
        HIP_TRY(hipMalloc((void **)&ws.uf, bytes));
        ws.uf_bytes = bytes;
    }
    double *p = ws.uf;
    auto take = [&](int64_t cnt) { double *q = p; p += cnt; return q; };
    double *X = take(tm_ * k), *Y = take(k * tn_);
    double *Pr = take(tm_ * n), *Rr = take(tm_ * n), *Pc = take(m * tn_), *Rc = take(m * tn_);
    double *cr = nullptr, *cr2 = nullptr, *cc = nullptr, *cc2 = nullptr;
    if (use_c) { cr = take(tm_ * n); cr2 = take(tm_ * n); cc = take(m * tn_); cc2 = take(m * tn_); }
    double *rown2 = take(m), *coln2 = take(n), *xn2 = take(tm_), *yn2 = take(tn_);
    double *pw = take(part);
    double *wsp = take(std::max(sr.first, sc.first)), *chk = take(std::max(sr.second, sc.second));
    const double *A = (const double *)d.A, *B = (const double *)d.B;
    double *C = (double *)d.C;
    const int nplan = ws.nplan;
    auto seg = [stream](const double *Z, int64_t ld, int64_t R, int64_t Cn, int64_t L, bool down,
                        bool sq, double *out, double *out2, int64_t ldo, bool tr) {
        return ftg::launch_seg_sums(Z, ld, R, Cn, L, down, sq, out, out2, ldo, tr, stream);
    };
    if (report)
        HIP_TRY(ftg::launch_clear_report(ws.counters, 1, ws.echo, nplan, ws.aux, 1, stream));
    // C_in sums of every tile line (before C is overwritten)
    if (use_c) {
        HIP_TRY(seg(C, d.ldc, m, n, T, true, false, cr, cr2, tm_, false));
        HIP_TRY(seg(C, d.ldc, m, n, T, false, false, cc, cc2, m, false));
    }
    // operand checksums: X(I, p) = sum_{i in I} op(A)(i, p) (tiles_m x k),
    // Y(p, J) = sum_{j in J} op(B)(p, j) (k x tiles_n)
    if (!ta)
        HIP_TRY(seg(A, d.lda, m, k, T, true, false, X, nullptr, tm_, false));
    else
        HIP_TRY(seg(A, d.lda, k, m, T, false, false, X, nullptr, tm_, true));
    if (!tb)
        HIP_TRY(seg(B, d.ldb, k, n, T, false, false, Y, nullptr, k, false));
    else
        HIP_TRY(seg(B, d.ldb, n, k, T, true, false, Y, nullptr, k, true));
    // |x_I|^2 and |y_J|^2
    HIP_TRY(seg(X, tm_, tm_, k, T, false, true, pw, nullptr, tm_, false));
    HIP_TRY(seg(pw, tm_, tm_, kseg, kseg, false, false, xn2, nullptr, tm_, false));
    HIP_TRY(seg(Y, k, k, tn_, k, true, true, yn2, nullptr, 1, false));
    // squared norms of the rows of op(A) and the columns of op(B)
    if (!ta) {
        HIP_TRY(seg(A, d.lda, m, k, T, false, true, pw, nullptr, m, false));
        HIP_TRY(seg(pw, m, m, kseg, kseg, false, false, rown2, nullptr, m, false));
    } else {
        HIP_TRY(seg(A, d.lda, k, m, k, true, true, rown2, nullptr, 1, false));
    }
    if (!tb) {
        HIP_TRY(seg(B, d.ldb, k, n, k, true, true, coln2, nullptr, 1, false));
    } else {
        HIP_TRY(seg(B, d.ldb, n, k, T, false, true, pw, nullptr, n, false));
        HIP_TRY(seg(pw, n, n, kseg, kseg, false, false, coln2, nullptr, n, false));
    }
    // encoded product parts: Pr = X op(B) (tiles_m x n), Pc = op(A) Y (m x tiles_n)
    if (ftgemm_status st = plain_f64(X, tm_, false, B, d.ldb, tb, tm_, n, k, 1.0, 0.0, Pr, tm_,
                                     wsp, chk, ws, stream))
        return st;
    if (ftgemm_status st = plain_f64(A, d.lda, ta, Y, k, false, m, tn_, k, 1.0, 0.0, Pc, m, wsp,
                                     chk, ws, stream))
        return st;
    // the product itself, checksum-free (split as the plain call would be)
    {
        int tm, tn, bk;
        ftg::tiling_f64(&tm, &tn, &bk);
        int64_t slice_k = k;
        const int ns = choose_split(m, n, k, tm, tn, bk, &slice_k);
        double *mw = nullptr, *mc = nullptr;
        if (ns > 1) {
            const size_t wbytes = sizeof(double) * (size_t)ns * m * n;
            const size_t cbytes = sizeof(double) * (size_t)ns * tm_ * tn_ * 2 * (tm + tn);
            if (ftgemm_status st = split_space(ws, wbytes + cbytes)) return st;
            mw = ws.split;
            mc = ws.split + (size_t)ns * m * n;
        }
        if (ftgemm_status st = plain_f64(A, d.lda, ta, B, d.ldb, tb, m, n, k, d.alpha, d.beta, C,
                                         d.ldc, mw, mc, ws, stream))
            return st;
    }
    HIP_TRY(ftg::launch_uf_inject(C, m, n, d.ldc, d.alpha, ws.plan, nplan, ws.echo, problem,
                                  stream));
    // reference sums of the output, then the comparison per tile
    HIP_TRY(seg(C, d.ldc, m, n, T, true, false, Rr, nullptr, tm_, false));
    HIP_TRY(seg(C, d.ldc, m, n, T, false, false, Rc, nullptr, m, false));
    ftg::UfArgs a{};
    a.Pr = Pr; a.Pc = Pc; a.Rr = Rr; a.Rc = Rc; a.cr = cr; a.cc = cc; a.cr2 = cr2; a.cc2 = cc2;
    a.row_nrm2 = rown2; a.col_nrm2 = coln2; a.xn2 = xn2; a.yn2 = yn2;
    a.m = m; a.n = n; a.k = k;
    a.tiles_m = (int32_t)tm_; a.tiles_n = (int32_t)tn_; a.problem = problem; a.nplan = nplan;
    a.alpha = d.alpha; a.beta = d.beta;
    a.counters = ws.counters; a.records = ws.records; a.record_cap = kDevRecordCap;
    a.rec_slot = ws.aux; a.plan = ws.plan; a.echo = ws.echo;
    HIP_TRY(ftg::launch_uf_compare(a, stream));
    return FTGEMM_OK;
}

ftgemm_status run_one(const ftgemm_gemm_desc &d, ftgemm_report *rep, hipStream_t stream,
                      int32_t problem = 0)
{
    t_last_invalid = 0;
    if (int pos = check_args(d)) return invalid(pos);
    if (rep && ((rep->record_capacity && !rep->records) || (rep->echo_capacity && !rep->echoes)))
        return invalid(14);
    if (rep) {
        std::memset(rep, 0, offsetof(ftgemm_report, record_capacity));
    }
    if (d.m == 0 || d.n == 0) return FTGEMM_OK;
    const bool c_is_f64 = d.dtype == FTGEMM_F64;
    if (d.alpha == 0.0 || d.k == 0) {
        if (d.beta == 1.0) return FTGEMM_OK;
        HIP_TRY(ftg::launch_scale(d.C, c_is_f64, d.m, d.n, d.ldc, d.beta, stream));
        return FTGEMM_OK;
    }
    if (d.abft == 2 && d.dtype == FTGEMM_F64) return FTGEMM_ERR_UNSUPPORTED;
    if (d.abft >= 3 && d.dtype != FTGEMM_F64) return FTGEMM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (d.dtype != FTGEMM_F64 && d.abft)
        for (const ftgemm_injection &f : g_plan)  // FP32 accumulators have 32 bits
            if (f.mode == FTGEMM_INJ_BITFLIP && f.bit >= 32) return invalid(14);
    DeviceWs *ws = nullptr;
    if (ftgemm_status st = workspace(&ws, 1)) return st;
    if (d.abft == 3) {
        if (ftgemm_status st = run_unfused(d, *ws, rep != nullptr, stream, problem)) return st;
        return rep ? copy_report(*ws, rep, stream, problem) : FTGEMM_OK;
    }

    int tm, tn, bk;
    if (d.dtype == FTGEMM_F64)
        ftg::tiling_f64(&tm, &tn, &bk);
    else
        lp_tiling(d, &tm, &tn, &bk);
    GemmArgs g = base_args(d, tm, tn);
    const bool ta = d.transA == FTGEMM_OP_T, tb = d.transB == FTGEMM_OP_T;
    // Low precision: the threshold norms in one pass before the product for
    // the one-sided mode, and for outputs of at least kLargeTileMin tiles
    // (below that the extra launches cost more than the tiles' own norms).
    const bool pre = d.dtype != FTGEMM_F64 &&
                     (d.abft == 2 || (d.abft == 1 && (int64_t)g.tiles_m * g.tiles_n >=
                                                         ftg::kLargeTileMin));
    if (pre) {
        // line norms of op(A) (rows) and op(B) (columns) for the thresholds,
        // and in the same pass the operand checksums of every tile: of op(A)
        // over each tile's rows, of op(B) over each tile's columns (FP32,
        // tiles_m + tiles_n rows of k; the one-sided mode needs op(B)'s only)
        const bool fp8 = d.dtype == FTGEMM_FP8_E4M3;
        const int64_t part = std::max<int64_t>(int64_t(1) << 22, 2 * std::max(d.m, d.n));
        const int64_t nx = d.abft == 2 ? 0 : (int64_t)g.tiles_m * d.k;
        const int64_t nsum = nx + (int64_t)g.tiles_n * d.k;
        if (ftgemm_status st = split_space(
                *ws, sizeof(double) * (2 * (d.m + d.n) + part) + sizeof(float) * nsum))
            return st;
        double *nb = ws->split;
        g.row_nrm2 = nb;
        g.row_max = nb + d.m;
        g.col_nrm2 = nb + 2 * d.m;
        g.col_max = nb + 2 * d.m + d.n;
        double *pw = nb + 2 * (d.m + d.n);
        float *xs = (float *)(pw + part);
        g.xsum = nx ? xs : nullptr;
        g.ysum = xs + nx;
        g.ldxs = d.k;
        // op(A) row i is stored row i (N) or stored column i (T); op(B)
        // column j is stored column j (N) or stored row j (T)
        HIP_TRY(ftg::launch_line_norms(d.A, d.lda, ta ? d.k : d.m, ta ? d.m : d.k, fp8, !ta,
                                       nb, nb + d.m, pw, part, nx ? xs : nullptr, tm, d.k,
                                       stream));
        HIP_TRY(ftg::launch_line_norms(d.B, d.ldb, tb ? d.n : d.k, tb ? d.k : d.n, fp8, tb,
                                       nb + 2 * d.m, nb + 2 * d.m + d.n, pw, part, xs + nx, tn,
                                       d.k, stream));
    }
    // (the weighted mode never splits the inner dimension)
    int64_t slice_k = d.k;
    const int nslices = d.dtype == FTGEMM_F64 && d.abft != 4
                            ? choose_split(d.m, d.n, d.k, tm, tn, bk, &slice_k)
                            : 1;
    if (nslices > 1) {
        const int64_t ntiles = (int64_t)g.tiles_m * g.tiles_n;
        const size_t wbytes = sizeof(double) * (size_t)nslices * d.m * d.n;
        const size_t cbytes = sizeof(double) * (size_t)nslices * ntiles * 2 * (tm + tn);
        if (ftgemm_status st = split_space(*ws, wbytes + cbytes)) return st;
        g.nslices = nslices;
        g.slice_k = slice_k;
        g.wsp = ws->split;
        g.chk = ws->split + (size_t)nslices * d.m * d.n;
    }
    g.problem = problem;
    g.counters = ws->counters;
    g.records = ws->records;
    g.record_cap = kDevRecordCap;
    g.rec_slot = ws->aux;
    g.nplan = d.abft ? ws->nplan : 0;
    g.plan = ws->plan;
    g.echo = ws->echo;
    if (rep && d.abft)
        HIP_TRY(ftg::launch_clear_report(ws->counters, 1, ws->echo, ws->nplan, ws->aux, 1,
                                         stream));
    if (d.dtype == FTGEMM_F64) {
        HIP_TRY(ftg::launch_f64(g, ta, tb, d.abft != 0, stream, d.abft == 4));
        if (nslices > 1) {
            ftg::ReduceArgs r{};
            r.C = (double *)d.C;
            r.wsp = g.wsp;
            r.chk = g.chk;
            r.m = d.m;
            r.n = d.n;
            r.ldc = d.ldc;
            r.alpha = g.alpha;
            r.beta = d.beta;
            r.nslices = nslices;
            r.tiles_m = g.tiles_m;
            r.tiles_n = g.tiles_n;
            r.problem = problem;
            r.counters = ws->counters;
            r.records = ws->records;
            r.record_cap = kDevRecordCap;
            r.rec_slot = ws->aux;
            HIP_TRY(ftg::launch_splitk_reduce(r, d.abft != 0, stream));
        }
    } else
        HIP_TRY(ftg::launch_lp(g, d.dtype == FTGEMM_FP8_E4M3, ta, tb, d.abft, pre, tm, stream));
    if (rep && d.abft) return copy_report(*ws, rep, stream, problem);
    return FTGEMM_OK;
}

// ---------------------------------------------------------------------------
// Batched launches.
//
// All tiles of all problems become work items handed out by device work
// queues to a persistent grid of one workgroup per compute unit.  The
// schedule -- the order of the items and whether there is one queue or one
// per XCD (problems spread over the XCDs, so a problem's operand panels stay
// in one L2) -- is chosen by timing the candidates on the batch itself the
// first time a batch of that shape is seen (when its C is write-only, beta
// == 0 everywhere, so the trial runs change nothing), and remembered.  The
// clearing of the report area and the persistent launch are captured once
// into a HIP graph and replayed; a new batch only re-uploads the per-problem
// arguments and the work items.
// ---------------------------------------------------------------------------
enum Schedule { kLptOneQueue = 0, kGivenOneQueue = 1, kLptPerXcd = 2, kNumSchedules = 3 };

uint64_t fnv1a(uint64_t h, uint64_t v)
{
    for (int b = 0; b < 8; ++b) {
        h ^= (v >> (8 * b)) & 0xff;
        h *= 0x100000001b3ull;
    }
    return h;
}

struct BatchPlan {
    std::vector<ftg::WorkItem> items;
    int rows = 128;  // tile rows of every item's problem, 0 when mixed
    int nqueues = 1;
    int32_t qbegin[ftg::kMaxQueues + 1] = {};
};

// Work items of the live problems under a schedule.  A tile's cost is taken
// as its inner length (every tile computes a full TM x TN block).
void plan_items(const std::vector<ftg::GemmArgs> &probs, const std::vector<int> &live,
                int sched, BatchPlan *plan)
{
    std::vector<int> order(live);
    if (sched != kGivenOneQueue)
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return probs[a].k > probs[b].k; });
    auto emit = [&](int p) {
        const ftg::GemmArgs &g = probs[p];
        for (int tn = 0; tn < g.tiles_n; ++tn)
            for (int tm = 0; tm < g.tiles_m; ++tm)
                plan->items.push_back(ftg::WorkItem{p, tm, tn, 0});
    };
    plan->items.clear();
    plan->rows = live.empty() ? 128 : probs[live[0]].tile_rows;
    for (int p : live)
        if (probs[p].tile_rows != plan->rows) plan->rows = 0;
    if (sched != kLptPerXcd) {
        for (int p : order) emit(p);
        plan->nqueues = 1;
        plan->qbegin[0] = 0;
        plan->qbegin[1] = (int32_t)plan->items.size();
        return;
    }
    // largest problems first onto the least loaded of the XCDs
    const int nq = ftg::kMaxQueues;
    std::vector<double> load(nq, 0.0);
    std::vector<std::vector<int>> bins(nq);
    for (int p : order) {
        const ftg::GemmArgs &g = probs[p];
        const double cost = (double)g.tiles_m * g.tiles_n * (double)g.k;
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[b] += cost;
        bins[b].push_back(p);
    }
    plan->nqueues = nq;
    for (int q = 0; q < nq; ++q) {
        plan->qbegin[q] = (int32_t)plan->items.size();
        for (int p : bins[q]) emit(p);
    }
    plan->qbegin[nq] = (int32_t)plan->items.size();
}

// Upload the per-problem arguments and the work items (host staging is
// reused only after its previous upload has completed).
ftgemm_status upload_batch(DeviceWs &ws, const std::vector<ftg::GemmArgs> &probs,
                           const BatchPlan &plan, hipStream_t stream)
{
    const int np = (int)probs.size(), ni = (int)plan.items.size();
    if (!ws.staged) HIP_TRY(hipEventCreateWithFlags(&ws.staged, hipEventDisableTiming));
    if (!ws.capture) HIP_TRY(hipStreamCreateWithFlags(&ws.capture, hipStreamNonBlocking));
    HIP_TRY(hipEventSynchronize(ws.staged));
    if (np > ws.probs_cap || ni > ws.items_cap) {
        HIP_TRY(hipDeviceSynchronize());
        if (np > ws.probs_cap) {
            if (ws.d_probs) {
                HIP_TRY(hipFree(ws.d_probs));
                HIP_TRY(hipHostFree(ws.h_probs));
            }
            const int cap = np < 64 ? 64 : np;
            HIP_TRY(hipMalloc((void **)&ws.d_probs, sizeof(ftg::GemmArgs) * cap));
            HIP_TRY(hipHostMalloc((void **)&ws.h_probs, sizeof(ftg::GemmArgs) * cap,
                                  hipHostMallocDefault));
            ws.probs_cap = cap;
        }
        if (ni > ws.items_cap) {
            if (ws.d_items) {
                HIP_TRY(hipFree(ws.d_items));
                HIP_TRY(hipHostFree(ws.h_items));
            }
            const int cap = ni < 1024 ? 1024 : ni;
            HIP_TRY(hipMalloc((void **)&ws.d_items, sizeof(ftg::WorkItem) * cap));
            HIP_TRY(hipHostMalloc((void **)&ws.h_items, sizeof(ftg::WorkItem) * cap,
                                  hipHostMallocDefault));
            ws.items_cap = cap;
        }
    }
    std::memcpy(ws.h_probs, probs.data(), sizeof(ftg::GemmArgs) * np);
    if (ni) std::memcpy(ws.h_items, plan.items.data(), sizeof(ftg::WorkItem) * ni);
    HIP_TRY(hipMemcpyAsync(ws.d_probs, ws.h_probs, sizeof(ftg::GemmArgs) * np,
                           hipMemcpyHostToDevice, stream));
    if (ni)
        HIP_TRY(hipMemcpyAsync(ws.d_items, ws.h_items, sizeof(ftg::WorkItem) * ni,
                               hipMemcpyHostToDevice, stream));
    HIP_TRY(hipEventRecord(ws.staged, stream));
    return FTGEMM_OK;
}

ftg::BatchArgs batch_args(const DeviceWs &ws, const BatchPlan &plan)
{
    ftg::BatchArgs b{};
    b.rows = plan.rows;
    b.probs = ws.d_probs;
    b.items = ws.d_items;
    b.queue = ws.aux + 1;
    b.nqueues = plan.nqueues;
    for (int q = 0; q <= plan.nqueues; ++q) b.qbegin[q] = plan.qbegin[q];
    return b;
}

// Clear the report area and run the persistent kernel, on `stream`.
ftgemm_status launch_batch(DeviceWs &ws, const ftgemm_gemm_desc &d0, int count,
                           const BatchPlan &plan, hipStream_t stream)
{
    const ftg::BatchArgs b = batch_args(ws, plan);
    const bool ta = d0.transA == FTGEMM_OP_T, tb = d0.transB == FTGEMM_OP_T;
    HIP_TRY(ftg::launch_clear_report(ws.counters, count, ws.echo, d0.abft ? ws.nplan : 0,
                                     ws.aux, 1 + plan.nqueues, stream));
    if (plan.items.empty()) return FTGEMM_OK;
    if (d0.dtype == FTGEMM_F64)
        HIP_TRY(ftg::launch_f64_batched(b, ta, tb, d0.abft != 0, ws.cus, stream));
    else
        HIP_TRY(ftg::launch_lp_batched(b, d0.dtype == FTGEMM_FP8_E4M3, ta, tb, d0.abft != 0,
                                       ws.cus, stream));
    return FTGEMM_OK;
}

// Signature of a batch: its size, dtype, mode, transposes and every shape.
uint64_t batch_signature(int32_t count, const ftgemm_gemm_desc *descs)
{
    const ftgemm_gemm_desc &d0 = descs[0];
    uint64_t sig = 0xcbf29ce484222325ull;
    sig = fnv1a(sig, (uint64_t)count);
    sig = fnv1a(sig, (uint64_t)d0.dtype * 16 + (d0.abft ? 8 : 0) + d0.transA * 2 + d0.transB);
    for (int32_t p = 0; p < count; ++p)
        sig = fnv1a(fnv1a(fnv1a(sig, (uint64_t)descs[p].m), (uint64_t)descs[p].n),
                    (uint64_t)descs[p].k);
    return sig;
}

// Tile rows of each problem of a batch: low-precision problems with at least
// mstar rows take 256-row tiles, the others (and every FP64 problem) 128.
void set_tile_rows(std::vector<ftg::GemmArgs> &probs, const ftgemm_gemm_desc *descs, bool lp,
                   int64_t mstar)
{
    for (size_t p = 0; p < probs.size(); ++p) {
        const int rows = lp && descs[p].m >= mstar ? 256 : 128;
        probs[p].tile_rows = rows;
        probs[p].tiles_m = (int32_t)((descs[p].m + rows - 1) / rows);
    }
}

// The tile rows each problem of a batch takes now: the threshold the table
// fixes, else the one remembered for the batch, else 128 everywhere.
void batch_rows(int32_t count, const ftgemm_gemm_desc *descs, int32_t *rows)
{
    const bool lp = descs[0].dtype != FTGEMM_F64;
    int64_t mstar = kNoBigTiles;
    {
        std::lock_guard<std::mutex> tl(g_tune_mu);
        TuneTable &t = tune_table();
        auto it = t.batches.find(batch_signature(count, descs));
        if (it != t.batches.end()) mstar = it->second.second;
        if (t.batch_mstar >= 0) mstar = t.batch_mstar;
    }
    for (int32_t p = 0; p < count; ++p) rows[p] = lp && descs[p].m >= mstar ? 256 : 128;
}

ftgemm_status run_batched(int32_t count, const ftgemm_gemm_desc *descs, ftgemm_report *reps,
                          hipStream_t stream)
{
    t_last_invalid = 0;
    if (count < 0) return invalid(1);
    if (count > 0 && !descs) return invalid(2);
    for (int32_t p = 0; p < count; ++p) {
        if (int pos = check_args(descs[p])) return invalid(pos);
        const ftgemm_gemm_desc &d = descs[p];
        if (d.dtype != descs[0].dtype || (d.abft != 0) != (descs[0].abft != 0) ||
            d.transA != descs[0].transA || d.transB != descs[0].transB || d.abft >= 2)
            return FTGEMM_ERR_UNSUPPORTED;
        if (reps && ((reps[p].record_capacity && !reps[p].records) ||
                     (reps[p].echo_capacity && !reps[p].echoes)))
            return invalid(14);
    }
    for (int32_t p = 0; reps && p < count; ++p)
        std::memset(&reps[p], 0, offsetof(ftgemm_report, record_capacity));
    if (count == 0) return FTGEMM_OK;
    const ftgemm_gemm_desc &d0 = descs[0];

    std::lock_guard<std::mutex> lock(g_mu);
    if (d0.dtype != FTGEMM_F64 && d0.abft)
        for (const ftgemm_injection &f : g_plan)
            if (f.mode == FTGEMM_INJ_BITFLIP && f.bit >= 32) return invalid(14);
    DeviceWs *ws = nullptr;
    if (ftgemm_status st = workspace(&ws, count)) return st;

    int tm, tn, bk;
    if (d0.dtype == FTGEMM_F64)
        ftg::tiling_f64(&tm, &tn, &bk);
    else
        ftg::tiling_lp(d0.dtype == FTGEMM_FP8_E4M3, d0.abft, 0, 0, true, true, &tm, &tn, &bk);
    const bool lp = d0.dtype != FTGEMM_F64;
    std::vector<ftg::GemmArgs> probs(count);
    std::vector<int> live;
    const uint64_t sig = batch_signature(count, descs);
    bool write_only = true;
    for (int32_t p = 0; p < count; ++p) {
        const ftgemm_gemm_desc &d = descs[p];
        ftg::GemmArgs g = base_args(d, tm, tn);
        g.tile_rows = tm;
        g.problem = p;
        g.counters = ws->counters + p;
        g.records = ws->records;
        g.record_cap = kDevRecordCap;
        g.rec_slot = ws->aux;
        g.nplan = d.abft ? ws->nplan : 0;
        g.plan = ws->plan;
        g.echo = ws->echo;
        probs[p] = g;
        if (d.m == 0 || d.n == 0) continue;
        if (d.alpha == 0.0 || d.k == 0) {
            // no product: C <- beta C, outside the persistent launch
            if (d.beta != 1.0)
                HIP_TRY(ftg::launch_scale(d.C, d.dtype == FTGEMM_F64, d.m, d.n, d.ldc, d.beta,
                                          stream));
            continue;
        }
        if (d.beta != 0.0) write_only = false;
        live.push_back(p);
    }

    // tile rows and work order: remembered (or in the table), tuned now, or
    // the defaults (128-row tiles, cost-ordered single queue)
    int sched = kLptOneQueue;
    int64_t mstar = kNoBigTiles;
    bool known = false;
    int64_t forced = -1;
    {
        std::lock_guard<std::mutex> tl(g_tune_mu);
        TuneTable &t = tune_table();
        auto it = t.batches.find(sig);
        if (it != t.batches.end()) {
            sched = it->second.first;
            mstar = it->second.second;
            known = true;
        }
        forced = t.batch_mstar;
    }
    if (!lp) mstar = kNoBigTiles;
    else if (forced >= 0) mstar = forced;
    static const bool no_tune = std::getenv("FTGEMM_NO_TUNE") != nullptr;
    BatchPlan plan;
    if (!known && write_only && !no_tune && !live.empty()) {
        // Trials on the batch itself (C is write-only): one untimed launch,
        // then two timed ones.  First the threshold from which a
        // low-precision problem takes 256-row tiles (unless the table fixes
        // it), with the default order; then the order.
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        auto trial = [&](int c, int64_t ms_rows, float *out) -> ftgemm_status {
            set_tile_rows(probs, descs, lp, ms_rows);
            plan_items(probs, live, c, &plan);
            if (ftgemm_status st = upload_batch(*ws, probs, plan, stream)) return st;
            if (ftgemm_status st = launch_batch(*ws, d0, count, plan, stream)) return st;
            HIP_TRY(hipEventRecord(e0, stream));
            for (int r = 0; r < 2; ++r)
                if (ftgemm_status st = launch_batch(*ws, d0, count, plan, stream)) return st;
            HIP_TRY(hipEventRecord(e1, stream));
            HIP_TRY(hipEventSynchronize(e1));
            HIP_TRY(hipEventElapsedTime(out, e0, e1));
            return FTGEMM_OK;
        };
        if (lp && forced < 0) {
            const int64_t cand[4] = {kNoBigTiles, 1024, 512, 256};
            float best = 0.0f;
            for (int c = 0; c < 4; ++c) {
                float ms = 0.0f;
                if (ftgemm_status st = trial(kLptOneQueue, cand[c], &ms)) return st;
                if (c == 0 || ms < best) {
                    best = ms;
                    mstar = cand[c];
                }
            }
        }
        float best = 0.0f;
        for (int c = 0; c < kNumSchedules; ++c) {
            float ms = 0.0f;
            if (ftgemm_status st = trial(c, mstar, &ms)) return st;
            if (c == 0 || ms < best) {
                best = ms;
                sched = c;
            }
        }
        HIP_TRY(hipEventDestroy(e0));
        HIP_TRY(hipEventDestroy(e1));
        remember_batch(sig, sched, mstar);
    }
    set_tile_rows(probs, descs, lp, mstar);
    plan_items(probs, live, sched, &plan);
    if (ftgemm_status st = upload_batch(*ws, probs, plan, stream)) return st;

    // the captured graph is reused while everything baked into it holds
    std::vector<uint64_t> key = {
        (uint64_t)d0.dtype, (uint64_t)d0.abft, (uint64_t)d0.transA, (uint64_t)d0.transB,
        (uint64_t)count, (uint64_t)(d0.abft ? ws->nplan : 0), (uint64_t)(uintptr_t)ws->d_probs,
        (uint64_t)(uintptr_t)ws->d_items, (uint64_t)(uintptr_t)ws->counters,
        (uint64_t)(uintptr_t)ws->echo, (uint64_t)(uintptr_t)ws->aux, (uint64_t)plan.nqueues,
        (uint64_t)plan.rows,
        (uint64_t)ws->cus, (uint64_t)plan.items.size()};
    for (int q = 0; q <= plan.nqueues; ++q) key.push_back((uint64_t)plan.qbegin[q]);
    if (!ws->exec || key != ws->graph_key) {
        if (ws->exec) {
            HIP_TRY(hipGraphExecDestroy(ws->exec));
            HIP_TRY(hipGraphDestroy(ws->graph));
            ws->exec = nullptr;
            ws->graph = nullptr;
        }
        HIP_TRY(hipStreamBeginCapture(ws->capture, hipStreamCaptureModeThreadLocal));
        const ftgemm_status st = launch_batch(*ws, d0, count, plan, ws->capture);
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamEndCapture(ws->capture, &graph));
        if (st != FTGEMM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        HIP_TRY(hipGraphInstantiate(&ws->exec, graph, nullptr, nullptr, 0));
        ws->graph = graph;
        ws->graph_key = key;
    }
    HIP_TRY(hipGraphLaunch(ws->exec, stream));

    if (reps && d0.abft) {
        HIP_TRY(hipMemcpyAsync(ws->h_counters, ws->counters, sizeof(DevCounters) * count,
                               hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(ws->h_aux, ws->aux, sizeof(unsigned int),
                               hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(ws->h_records, ws->records,
                               sizeof(ftgemm_fault_record) * kDevRecordCap,
                               hipMemcpyDeviceToHost, stream));
        if (ws->nplan)
            HIP_TRY(hipMemcpyAsync(ws->h_echo, ws->echo,
                                   sizeof(ftgemm_injection_echo) * ws->nplan,
                                   hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        for (int32_t p = 0; p < count; ++p) fill_report(host_report(*ws), p, &reps[p], p);
    }
    return FTGEMM_OK;
}

// Host staging of the no-allocation path's report copy-back: file-scope
// arrays, so that path allocates nothing (used with g_mu held).
DevCounters g_na_counters[1];
unsigned int g_na_aux[kAuxWords];
ftgemm_fault_record g_na_records[ftg::kNoAllocRecords];
ftgemm_injection_echo g_na_echo[ftg::kNoAllocPlan];

}  // namespace

namespace ftg {

// ftgemm_gemm_ex with every piece of device memory the call needs taken
// from `scratch` (the caller's per-device array of kNoAllocBytes): the
// counters, the record slots (kNoAllocRecords), the fault plan and its
// echo slots (kNoAllocPlan).  Nothing grows with m, n or k: the FP64 inner
// dimension is never split, and low-precision tiles form their threshold
// norms and operand checksums themselves (no pass before the product).
ftgemm_status run_noalloc(const ftgemm_gemm_desc &d, ftgemm_report *rep, hipStream_t stream,
                          unsigned char *scratch, size_t bytes)
{
    t_last_invalid = 0;
    if (int pos = check_args(d)) return invalid(pos);
    if (rep && ((rep->record_capacity && !rep->records) || (rep->echo_capacity && !rep->echoes)))
        return invalid(14);
    if (rep) std::memset(rep, 0, offsetof(ftgemm_report, record_capacity));
    if (d.m == 0 || d.n == 0) return FTGEMM_OK;
    const bool c_is_f64 = d.dtype == FTGEMM_F64;
    if (d.alpha == 0.0 || d.k == 0) {
        if (d.beta == 1.0) return FTGEMM_OK;
        HIP_TRY(ftg::launch_scale(d.C, c_is_f64, d.m, d.n, d.ldc, d.beta, stream));
        return FTGEMM_OK;
    }
    // the one-sided and unfused modes need workspace that grows with the
    // problem; the weighted mode is for single calls
    if (d.abft >= 2) return FTGEMM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    const int nplan = d.abft ? (int)g_plan.size() : 0;
    if (nplan > kNoAllocPlan) {
        report_hip_failure("ftgemm_gemm_ex_noalloc: fault plan longer than its 256 slots",
                           hipErrorInvalidValue);
        return FTGEMM_ERR_UNSUPPORTED;
    }
    if (d.dtype != FTGEMM_F64 && d.abft)
        for (const ftgemm_injection &f : g_plan)  // FP32 accumulators have 32 bits
            if (f.mode == FTGEMM_INJ_BITFLIP && f.bit >= 32) return invalid(14);
    // carve the scratch array (256-byte aligned parts)
    size_t off = 0;
    auto take = [&](size_t nbytes) {
        unsigned char *q = scratch + off;
        off += (nbytes + 255) & ~size_t(255);
        return q;
    };
    DevCounters *counters = (DevCounters *)take(sizeof(DevCounters));
    unsigned int *aux = (unsigned int *)take(sizeof(unsigned int) * kAuxWords);
    ftgemm_fault_record *records =
        (ftgemm_fault_record *)take(sizeof(ftgemm_fault_record) * kNoAllocRecords);
    ftgemm_injection *plan = (ftgemm_injection *)take(sizeof(ftgemm_injection) * kNoAllocPlan);
    ftgemm_injection_echo *echo =
        (ftgemm_injection_echo *)take(sizeof(ftgemm_injection_echo) * kNoAllocPlan);
    if (off > bytes) return FTGEMM_ERR_HIP;

    int tm, tn, bk;
    if (d.dtype == FTGEMM_F64)
        ftg::tiling_f64(&tm, &tn, &bk);
    else
        lp_tiling(d, &tm, &tn, &bk, true);
    GemmArgs g = base_args(d, tm, tn);
    const bool ta = d.transA == FTGEMM_OP_T, tb = d.transB == FTGEMM_OP_T;
    g.counters = counters;
    g.records = records;
    g.record_cap = kNoAllocRecords;
    g.rec_slot = aux;
    g.nplan = nplan;
    g.plan = plan;
    g.echo = echo;
    if (nplan)
        HIP_TRY(hipMemcpyAsync(plan, g_plan.data(), sizeof(ftgemm_injection) * nplan,
                               hipMemcpyHostToDevice, stream));
    // the counters, record slots and echo slots start from zero every call
    // (the array keeps the last call's contents)
    if (d.abft) HIP_TRY(ftg::launch_clear_report(counters, 1, echo, nplan, aux, 1, stream));
    if (d.dtype == FTGEMM_F64)
        HIP_TRY(ftg::launch_f64(g, ta, tb, d.abft != 0, stream));
    else
        HIP_TRY(ftg::launch_lp(g, d.dtype == FTGEMM_FP8_E4M3, ta, tb, d.abft, false, tm, stream));
    if (!(rep && d.abft)) return FTGEMM_OK;
    HIP_TRY(hipMemcpyAsync(g_na_counters, counters, sizeof(DevCounters), hipMemcpyDeviceToHost,
                           stream));
    HIP_TRY(hipMemcpyAsync(g_na_aux, aux, sizeof(unsigned int), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(g_na_records, records, sizeof(ftgemm_fault_record) * kNoAllocRecords,
                           hipMemcpyDeviceToHost, stream));
    if (nplan)
        HIP_TRY(hipMemcpyAsync(g_na_echo, echo, sizeof(ftgemm_injection_echo) * nplan,
                               hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    fill_report(HostReport{g_na_counters, g_na_aux, g_na_records, g_na_echo, nplan,
                           (uint32_t)kNoAllocRecords},
                0, rep, 0);
    return FTGEMM_OK;
}

}  // namespace ftg

extern "C" {

ftgemm_status ftgemm_gemm(ftgemm_op transA, ftgemm_op transB, int64_t m, int64_t n, int64_t k,
                          double alpha, const double *A, int64_t lda, const double *B,
                          int64_t ldb, double beta, double *C, int64_t ldc,
                          ftgemm_report *report, void *stream)
{
    ftgemm_gemm_desc d{};
    d.dtype = FTGEMM_F64;
    d.transA = transA;
    d.transB = transB;
    d.abft = 1;
    d.m = m;
    d.n = n;
    d.k = k;
    d.lda = lda;
    d.ldb = ldb;
    d.ldc = ldc;
    d.alpha = alpha;
    d.beta = beta;
    d.scaleA = d.scaleB = 1.0;
    d.A = A;
    d.B = B;
    d.C = C;
    return run_one(d, report, (hipStream_t)stream);
}

ftgemm_status ftgemm_gemm_ex(const ftgemm_gemm_desc *desc, ftgemm_report *report, void *stream)
{
    t_last_invalid = 0;
    if (!desc) return invalid(14);
    return run_one(*desc, report, (hipStream_t)stream);
}

ftgemm_status ftgemm_gemm_batched(int32_t count, const ftgemm_gemm_desc *problems,
                                  ftgemm_report *reports, void *stream)
{
    return run_batched(count, problems, reports, (hipStream_t)stream);
}

ftgemm_status ftgemm_gemm_batched_loop(int32_t count, const ftgemm_gemm_desc *problems,
                                       ftgemm_report *reports, void *stream)
{
    t_last_invalid = 0;
    if (count < 0) return invalid(1);
    if (count > 0 && !problems) return invalid(2);
    for (int32_t p = 0; p < count; ++p)
        if (ftgemm_status st = run_one(problems[p], reports ? &reports[p] : nullptr,
                                       (hipStream_t)stream, p))
            return st;
    return FTGEMM_OK;
}

ftgemm_status ftgemm_set_fault_plan(const ftgemm_injection *plan, int32_t n)
{
    t_last_invalid = 0;
    if (n < 0) return invalid(2);
    if (n > 0 && !plan) return invalid(1);
    for (int32_t q = 0; q < n; ++q) {
        const ftgemm_injection &f = plan[q];
        const bool ok_mode = f.mode == FTGEMM_INJ_ADD || f.mode == FTGEMM_INJ_BITFLIP;
        const bool ok_tgt = f.target == FTGEMM_TGT_ACC || f.target == FTGEMM_TGT_ROW_CHECKSUM ||
                            f.target == FTGEMM_TGT_COL_CHECKSUM ||
                            f.target == FTGEMM_TGT_WEIGHTED_CHECKSUM;
        const bool ok_bit = f.mode != FTGEMM_INJ_BITFLIP || (f.bit >= 0 && f.bit < 64);
        const bool ok_ck = f.target == FTGEMM_TGT_ACC || f.mode == FTGEMM_INJ_ADD;
        if (!ok_mode || !ok_tgt || !ok_bit || !ok_ck || f.row < 0 || f.col < 0 ||
            f.k_index < 0 || f.problem < 0)
            return invalid(1);
    }
    std::lock_guard<std::mutex> lock(g_mu);
    g_plan.assign(plan, plan + n);
    ++g_plan_version;
    return FTGEMM_OK;
}

ftgemm_status ftgemm_query_tiling(ftgemm_dtype dtype, int64_t m, int64_t n, int64_t k,
                                  int32_t *tm, int32_t *tn, int32_t *bk, int32_t *split_k)
{
    t_last_invalid = 0;
    if (dtype != FTGEMM_F64 && dtype != FTGEMM_BF16 && dtype != FTGEMM_FP8_E4M3)
        return invalid(1);
    if (m < 0) return invalid(2);
    if (n < 0) return invalid(3);
    if (k < 0) return invalid(4);
    if (!tm || !tn || !bk || !split_k) return invalid(5);
    int a = 0, b = 0, c = 0;
    int64_t slice_k = k;
    int s = 1;
    if (dtype == FTGEMM_F64) {
        ftg::tiling_f64(&a, &b, &c);
        s = choose_split(m, n, k, a, b, c, &slice_k);
    } else {
        ftgemm_gemm_desc d{};
        d.dtype = dtype;
        d.abft = 1;
        d.m = m;
        d.n = n;
        d.k = k;
        lp_tiling(d, &a, &b, &c);
    }
    *tm = a;
    *tn = b;
    *bk = c;
    *split_k = s;
    return FTGEMM_OK;
}

ftgemm_status ftgemm_query_tiling_ex(const ftgemm_gemm_desc *desc, int32_t *tm, int32_t *tn,
                                     int32_t *bk, int32_t *split_k)
{
    t_last_invalid = 0;
    if (!desc) return invalid(1);
    const ftgemm_gemm_desc &d = *desc;
    if (d.dtype != FTGEMM_F64 && d.dtype != FTGEMM_BF16 && d.dtype != FTGEMM_FP8_E4M3)
        return invalid(1);
    if (d.abft < 0 || d.abft > 4) return invalid(1);
    if (d.m < 0 || d.n < 0 || d.k < 0) return invalid(1);
    if (!tm || !tn || !bk || !split_k) return invalid(2);
    if (d.abft == 2 && d.dtype == FTGEMM_F64) return FTGEMM_ERR_UNSUPPORTED;
    if (d.abft >= 3 && d.dtype != FTGEMM_F64) return FTGEMM_ERR_UNSUPPORTED;
    int a = 0, b = 0, c = 0;
    int64_t slice_k = d.k;
    int s = 1;
    if (d.dtype == FTGEMM_F64) {
        ftg::tiling_f64(&a, &b, &c);
        if (d.abft != 4) s = choose_split(d.m, d.n, d.k, a, b, c, &slice_k);
    } else {
        lp_tiling(d, &a, &b, &c);
    }
    *tm = a;
    *tn = b;
    *bk = c;
    *split_k = s;
    return FTGEMM_OK;
}

ftgemm_status ftgemm_load_tune_table(const char *path)
{
    t_last_invalid = 0;
    TuneTable t;
    t.loaded = true;
    if (path) {
        if (!parse_table(path, t)) return invalid(1);
        t.path = path;
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune = t;
    return FTGEMM_OK;
}

ftgemm_status ftgemm_batch_tiling(int32_t count, const ftgemm_gemm_desc *problems,
                                  int32_t *tile_rows)
{
    t_last_invalid = 0;
    if (count < 0) return invalid(1);
    if (count > 0 && !problems) return invalid(2);
    if (count > 0 && !tile_rows) return invalid(3);
    if (count == 0) return FTGEMM_OK;
    batch_rows(count, problems, tile_rows);
    return FTGEMM_OK;
}

int32_t ftgemm_last_invalid_arg(void) { return t_last_invalid; }

const char *ftgemm_status_string(ftgemm_status s)
{
    switch (s) {
    case FTGEMM_OK: return "FTGEMM_OK";
    case FTGEMM_ERR_INVALID_ARG: return "FTGEMM_ERR_INVALID_ARG: an argument is invalid";
    case FTGEMM_ERR_UNSUPPORTED: return "FTGEMM_ERR_UNSUPPORTED: combination not supported";
    case FTGEMM_ERR_HIP: return "FTGEMM_ERR_HIP: a HIP runtime call failed";
    case FTGEMM_ERR_NO_MEMORY: return "FTGEMM_ERR_NO_MEMORY: device memory exhausted";
    }
    return "FTGEMM: unknown status";
}

void ftgemm_finalize(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return;
    for (auto &kv : g_ws) {
        DeviceWs &ws = kv.second;
        if (hipSetDevice(kv.first) != hipSuccess) continue;
        (void)hipDeviceSynchronize();
        if (ws.counters) (void)hipFree(ws.counters);
        if (ws.records) (void)hipFree(ws.records);
        if (ws.plan) (void)hipFree(ws.plan);
        if (ws.echo) (void)hipFree(ws.echo);
        if (ws.h_counters) (void)hipHostFree(ws.h_counters);
        if (ws.h_records) (void)hipHostFree(ws.h_records);
        if (ws.h_echo) (void)hipHostFree(ws.h_echo);
        if (ws.split) (void)hipFree(ws.split);
        if (ws.uf) (void)hipFree(ws.uf);
        if (ws.aux) (void)hipFree(ws.aux);
        if (ws.h_aux) (void)hipHostFree(ws.h_aux);
        if (ws.exec) (void)hipGraphExecDestroy(ws.exec);
        if (ws.graph) (void)hipGraphDestroy(ws.graph);
        if (ws.d_probs) (void)hipFree(ws.d_probs);
        if (ws.h_probs) (void)hipHostFree(ws.h_probs);
        if (ws.d_items) (void)hipFree(ws.d_items);
        if (ws.h_items) (void)hipHostFree(ws.h_items);
        if (ws.staged) (void)hipEventDestroy(ws.staged);
        if (ws.capture) (void)hipStreamDestroy(ws.capture);
    }
    g_ws.clear();
    g_plan_version++;
    (void)hipSetDevice(cur);
}

}  // extern "C"
