// ftgemm_kernels.h -- launchers of the libftgemm kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "ftgemm_device.h"

namespace ftg {

// FP64 tile kernel (one 128 x 128 output tile per workgroup).
hipError_t launch_f64(const GemmArgs &g, bool ta, bool tb, bool abft, hipStream_t stream);
void tiling_f64(int *tm, int *tn, int *bk);

// BF16 / FP8 E4M3 tile kernel (FP32 accumulation and output, one 128 x 128
// output tile per workgroup).
hipError_t launch_lp(const GemmArgs &g, bool fp8, bool ta, bool tb, bool abft,
                     hipStream_t stream);
void tiling_lp(bool fp8, int *tm, int *tn, int *bk);

// Verified reduction of a split inner dimension (FP64): C = alpha * sum_s
// W_s + beta * C, checked against the slices' encoded checksums.
struct ReduceArgs {
    double *C;
    const double *wsp;   // nslices partial products, each m x n, leading dimension m
    const double *chk;   // the slices' encoded checksums and thresholds
    int64_t m, n, ldc;
    double alpha, beta;
    int32_t nslices, tiles_m, tiles_n, problem;
    DevCounters *counters;
    ftgemm_fault_record *records;
    uint32_t record_cap;
};
hipError_t launch_splitk_reduce(const ReduceArgs &r, bool abft, hipStream_t stream);

// C = beta * C over an m x n column-major matrix of double (f64) or float.
hipError_t launch_scale(void *C, bool f64, int64_t m, int64_t n, int64_t ldc, double beta,
                        hipStream_t stream);

// Clear a report area: counters and the first n echo slots.
hipError_t launch_clear_report(DevCounters *ct, int ncounters, ftgemm_injection_echo *echo,
                               int nech, hipStream_t stream);

}  // namespace ftg
