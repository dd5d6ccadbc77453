// ftgemm_util.hip -- small helper kernels of libftgemm: the beta-only scaling
// of C (alpha == 0 or k == 0) and the clearing of a report area.  The report
// is cleared by a kernel rather than hipMemsetAsync so the same sequence can
// be recorded into a HIP graph.
#include "ftgemm_kernels.h"

namespace ftg {

template <typename T>
__global__ void scale_kernel(T *C, int64_t m, int64_t n, int64_t ldc, double beta)
{
    const int64_t total = m * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % m, j = e / m;
        T *p = C + i + j * ldc;
        *p = beta == 0.0 ? (T)0 : (T)(beta * (double)*p);
    }
}

hipError_t launch_scale(void *C, bool f64, int64_t m, int64_t n, int64_t ldc, double beta,
                        hipStream_t stream)
{
    const int64_t total = m * n;
    if (total == 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (f64)
        hipLaunchKernelGGL(scale_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (double *)C, m, n, ldc, beta);
    else
        hipLaunchKernelGGL(scale_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (float *)C, m, n, ldc, beta);
    return hipGetLastError();
}

__global__ void clear_report_kernel(DevCounters *ct, int nct, ftgemm_injection_echo *echo,
                                    int nech, unsigned int *aux, int naux)
{
    for (int i = threadIdx.x; i < naux; i += blockDim.x) aux[i] = 0u;
    for (int i = threadIdx.x; i < nct; i += blockDim.x) {
        DevCounters z{};
        ct[i] = z;
    }
    for (int i = threadIdx.x; i < nech; i += blockDim.x) {
        ftgemm_injection_echo z{};
        echo[i] = z;
    }
}

hipError_t launch_clear_report(DevCounters *ct, int nct, ftgemm_injection_echo *echo, int nech,
                               unsigned int *aux, int naux, hipStream_t stream)
{
    hipLaunchKernelGGL(clear_report_kernel, dim3(1), dim3(256), 0, stream, ct, nct, echo, nech,
                       aux, naux);
    return hipGetLastError();
}

}  // namespace ftg
