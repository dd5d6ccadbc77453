// ftgemm_host.cpp -- the C ABI of libftgemm: argument checks, quick returns,
// the per-GPU workspace (report area, fault plan), launches and report
// copy-back.  Declarations and the contract are in include/ftgemm.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_map>
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
    // split inner dimension: partial products, slice checksums
    double *split = nullptr;
    size_t split_bytes = 0;
};

std::unordered_map<int, DeviceWs> g_ws;

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

// Copy the report area of problem `p` (and the echo slots of its faults)
// into the caller's report; the stream has been synchronised.
void fill_report(const DeviceWs &ws, int p, ftgemm_report *rep, int32_t problem)
{
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
    const uint32_t nrec = c.record_count < kDevRecordCap ? c.record_count : kDevRecordCap;
    for (uint32_t r = 0; r < nrec; ++r) {
        const ftgemm_fault_record &src = ws.h_records[r];
        if (src.problem != problem) continue;
        if (rep->records && rep->record_count < rep->record_capacity)
            rep->records[rep->record_count] = src;
        rep->record_count++;
    }
    if (c.record_count > kDevRecordCap) rep->record_count += c.record_count - kDevRecordCap;
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
    if (d.m > INT32_MAX / 2 || d.n > INT32_MAX / 2) return d.m > INT32_MAX / 2 ? 3 : 4;
    return 0;
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
    g.k_base = 0;
    return g;
}

ftgemm_status run_one(const ftgemm_gemm_desc &d, ftgemm_report *rep, hipStream_t stream)
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
    std::lock_guard<std::mutex> lock(g_mu);
    if (d.dtype != FTGEMM_F64 && d.abft)
        for (const ftgemm_injection &f : g_plan)  // FP32 accumulators have 32 bits
            if (f.mode == FTGEMM_INJ_BITFLIP && f.bit >= 32) return invalid(14);
    DeviceWs *ws = nullptr;
    if (ftgemm_status st = workspace(&ws, 1)) return st;

    int tm, tn, bk;
    if (d.dtype == FTGEMM_F64)
        ftg::tiling_f64(&tm, &tn, &bk);
    else
        ftg::tiling_lp(d.dtype == FTGEMM_FP8_E4M3, &tm, &tn, &bk);
    GemmArgs g = base_args(d, tm, tn);
    int64_t slice_k = d.k;
    const int nslices =
        d.dtype == FTGEMM_F64 ? choose_split(d.m, d.n, d.k, tm, tn, bk, &slice_k) : 1;
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
    g.counters = ws->counters;
    g.records = ws->records;
    g.record_cap = kDevRecordCap;
    g.nplan = d.abft ? ws->nplan : 0;
    g.plan = ws->plan;
    g.echo = ws->echo;
    if (rep && d.abft) HIP_TRY(ftg::launch_clear_report(ws->counters, 1, ws->echo, ws->nplan, stream));
    const bool ta = d.transA == FTGEMM_OP_T, tb = d.transB == FTGEMM_OP_T;
    if (d.dtype == FTGEMM_F64) {
        HIP_TRY(ftg::launch_f64(g, ta, tb, d.abft != 0, stream));
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
            r.problem = 0;
            r.counters = ws->counters;
            r.records = ws->records;
            r.record_cap = kDevRecordCap;
            HIP_TRY(ftg::launch_splitk_reduce(r, d.abft != 0, stream));
        }
    } else
        HIP_TRY(ftg::launch_lp(g, d.dtype == FTGEMM_FP8_E4M3, ta, tb, d.abft != 0, stream));
    if (rep && d.abft) {
        HIP_TRY(hipMemcpyAsync(ws->h_counters, ws->counters, sizeof(DevCounters),
                               hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(ws->h_records, ws->records,
                               sizeof(ftgemm_fault_record) * kDevRecordCap,
                               hipMemcpyDeviceToHost, stream));
        if (ws->nplan)
            HIP_TRY(hipMemcpyAsync(ws->h_echo, ws->echo,
                                   sizeof(ftgemm_injection_echo) * ws->nplan,
                                   hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        fill_report(*ws, 0, rep, 0);
    }
    return FTGEMM_OK;
}

}  // namespace

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
    (void)count; (void)problems; (void)reports; (void)stream;
    return FTGEMM_ERR_UNSUPPORTED;
}

ftgemm_status ftgemm_gemm_batched_loop(int32_t count, const ftgemm_gemm_desc *problems,
                                       ftgemm_report *reports, void *stream)
{
    (void)count; (void)problems; (void)reports; (void)stream;
    return FTGEMM_ERR_UNSUPPORTED;
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
                            f.target == FTGEMM_TGT_COL_CHECKSUM;
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
        ftg::tiling_lp(dtype == FTGEMM_FP8_E4M3, &a, &b, &c);
    }
    *tm = a;
    *tn = b;
    *bk = c;
    *split_k = s;
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
    }
    g_ws.clear();
    g_plan_version++;
    (void)hipSetDevice(cur);
}

}  // extern "C"
