// Achievable HBM read rate on this device, for the context of the Dslash
// roofline: a grid-stride stream of nontemporal 16-byte loads (the load
// style of the Dslash's link stream), 8 loads in flight per thread.
#include "hisq_common.hpp"

namespace hisq {

typedef double pd2 __attribute__((ext_vector_type(2)));

constexpr int RP_NT = 256;
constexpr int RP_U = 8;

__global__ __launch_bounds__(RP_NT) void k_read_probe(const pd2 *__restrict__ p, long long n, double *__restrict__ sink)
{
    double s = 0.0;
    const long long stride = (long long)gridDim.x * RP_NT * RP_U;
    for (long long base = (long long)blockIdx.x * RP_NT * RP_U + threadIdx.x; base < n; base += stride) {
        pd2 v[RP_U];
#pragma unroll
        for (int u = 0; u < RP_U; ++u) {
            const long long i = base + (long long)u * RP_NT;
            v[u] = i < n ? __builtin_nontemporal_load(p + i) : pd2{ 0.0, 0.0 };
        }
#pragma unroll
        for (int u = 0; u < RP_U; ++u) s += v[u].x + v[u].y;
    }
    // one sum per block, so the loads cannot be dropped
    __shared__ double lds[RP_NT / 64];
    s = block_sum<RP_NT>(s, lds);
    if (threadIdx.x == 0) sink[blockIdx.x] = s;
}

}  // namespace hisq

using namespace hisq;

extern "C" int hisq_read_probe(const void *buf, size_t bytes, void *sink, size_t sink_bytes, int reps, double *us,
                               void *stream)
{
    constexpr int GRID = 8192;
    if (!buf || !sink || !us) return fail(HISQ_EINVAL, "hisq_read_probe: NULL pointer");
    if (!aligned16({buf, sink}))
        return fail(HISQ_EINVAL, "hisq_read_probe: device pointers must be 16-byte aligned");
    if (bytes < 16 || sink_bytes < GRID * sizeof(double))
        return fail(HISQ_EINVAL, "hisq_read_probe: need bytes >= 16 and sink_bytes >= 65536");
    if (reps <= 0) reps = 5;
    hipStream_t s = (hipStream_t)stream;
    const long long n = (long long)(bytes / 16);
    hipEvent_t a, b;
    HISQ_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        hipEventDestroy(a);
        return fail(HISQ_EHIP, "hisq_read_probe: event");
    }
    hipLaunchKernelGGL(k_read_probe, dim3(GRID), dim3(RP_NT), 0, s, (const pd2 *)buf, n, (double *)sink);
    hipEventRecord(a, s);
    for (int i = 0; i < reps; ++i)
        hipLaunchKernelGGL(k_read_probe, dim3(GRID), dim3(RP_NT), 0, s, (const pd2 *)buf, n, (double *)sink);
    hipEventRecord(b, s);
    hipError_t e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "hisq_read_probe");
    *us = 1e3 * ms / reps;
    return HISQ_OK;
}
