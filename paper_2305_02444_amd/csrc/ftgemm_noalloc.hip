// ftgemm_noalloc.hip -- the entry point that allocates nothing.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid it): the device
// memory a call needs beyond its operands (report counters, record slots,
// the fault plan and its echo slots) lives in one file-scope array per GPU,
// `scratch`, of ftg::kNoAllocBytes (128 KiB), which each GPU the library
// runs on keeps until the process ends.  Its device address is looked up
// once per device (hipGetSymbolAddress) and used from then on; the name
// itself is only a host-side stand-in.  Every call on a GPU shares that
// GPU's array, so calls that overlap on one GPU race.
#include <mutex>

#include "ftgemm_device.h"
#include "ftgemm_kernels.h"

static __device__ __align__(256) unsigned char scratch[ftg::kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the
// first call there).
hipError_t scratch_address(unsigned char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = (unsigned char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" ftgemm_status ftgemm_gemm_ex_noalloc(const ftgemm_gemm_desc *desc,
                                                ftgemm_report *report, void *stream)
{
    if (!desc) return ftgemm_gemm_ex(nullptr, report, stream);  // the argument error
    unsigned char *ptr = nullptr;
    if (scratch_address(&ptr) != hipSuccess) return FTGEMM_ERR_HIP;
    return ftg::run_noalloc(*desc, report, (hipStream_t)stream, ptr, ftg::kNoAllocBytes);
}
