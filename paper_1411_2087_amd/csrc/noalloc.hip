// The deterministic dot product without any allocation, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// Its scratch is a file-scope device array: one copy per GPU, held until the
// process ends, shared by every call on that GPU (calls that overlap on one
// GPU race on it).  In host code the array's name is only a host-side
// stand-in, so kernels and copies receive the per-device address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current.  The two reduction stages write every partial and the result
// before reading them, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cg_internal.hpp"

namespace hisq {

// per-workgroup partials (at most BLAS_MAX_BLOCKS pairs) and the result: 16.25 KB
static __device__ __align__(256) char scratch[DOT_WS_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static void *scratch_addr[NOALLOC_MAX_DEVICES];
static std::mutex scratch_mu;

// The device address of `scratch` on the current device.
static int scratch_on_current_device(void **ptr)
{
    int dev = 0;
    HISQ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(HISQ_EINVAL, "hisq_dot_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hisq_dot_noalloc: hipGetSymbolAddress(scratch)");
        if (!p) return fail(HISQ_EHIP, "hisq_dot_noalloc: no device address for the scratch array");
        scratch_addr[dev] = p;
    }
    *ptr = scratch_addr[dev];
    return HISQ_OK;
}

// n beyond this would describe vectors larger than any GPU memory
constexpr long long NOALLOC_MAX_N = 1LL << 37;

}  // namespace hisq

using namespace hisq;

extern "C" int hisq_dot_noalloc(const void *x, const void *y, long long n, int prec, double out_host[2], void *stream)
{
    if (!x || !y || !out_host || n < 0) return fail(HISQ_EINVAL, "hisq_dot_noalloc: bad argument");
    if (!aligned16({x, y}))
        return fail(HISQ_EINVAL, "hisq_dot_noalloc: device pointers must be 16-byte aligned");
    if (n > NOALLOC_MAX_N) return fail(HISQ_EINVAL, "hisq_dot_noalloc: n exceeds 2^37 complex entries");
    if (prec < HISQ_F64 || prec > HISQ_I16SC) return fail(HISQ_EINVAL, "hisq_dot_noalloc: bad precision");
    void *ws = nullptr;
    const int rc = scratch_on_current_device(&ws);
    if (rc) return rc;
    return dot_on(x, y, n, prec, out_host, (char *)ws, (hipStream_t)stream);
}
