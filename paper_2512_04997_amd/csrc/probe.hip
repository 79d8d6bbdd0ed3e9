// probe.hip -- libpsmprobe.so (include/psmprobe.h): attainable streaming
// bandwidth of the device, a measurement utility beside the roofline figures
// and kept out of the method's library: plain grid-stride copy, read and write
// kernels over 16-byte elements, four independent accesses per lane per
// iteration.
#include <hip/hip_runtime.h>

#include "psmprobe.h"

namespace {

constexpr int PU = 4;

__global__ __launch_bounds__(256) void k_probe_copy(const float4* __restrict__ a, float4* __restrict__ b, long long n) {
    const long long stride = (long long)gridDim.x * 256 * PU;
    for (long long i = (long long)blockIdx.x * 256 * PU + threadIdx.x; i < n; i += stride) {
        float4 v[PU];
#pragma unroll
        for (int u = 0; u < PU; ++u) v[u] = i + u * 256 < n ? a[i + u * 256] : float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < PU; ++u)
            if (i + u * 256 < n) b[i + u * 256] = v[u];
    }
}

__global__ __launch_bounds__(256) void k_probe_read(const float4* __restrict__ a, float* __restrict__ sink, long long n) {
    const long long stride = (long long)gridDim.x * 256 * PU;
    float s = 0.f;
    for (long long i = (long long)blockIdx.x * 256 * PU + threadIdx.x; i < n; i += stride)
#pragma unroll
        for (int u = 0; u < PU; ++u)
            if (i + u * 256 < n) {
                const float4 v = a[i + u * 256];
                s += (v.x + v.y) + (v.z + v.w);
            }
    // the compare keeps the loads live: sink[0] is written only by a lane
    // whose sum is exactly this value
    if (s == 1234.5f) sink[0] = s;
}

__global__ __launch_bounds__(256) void k_probe_write(float4* __restrict__ b, long long n) {
    const long long stride = (long long)gridDim.x * 256 * PU;
    for (long long i = (long long)blockIdx.x * 256 * PU + threadIdx.x; i < n; i += stride)
#pragma unroll
        for (int u = 0; u < PU; ++u)
            if (i + u * 256 < n) b[i + u * 256] = float4{1.f, 2.f, 3.f, 4.f};
}

}  // namespace

#define PROBE_CHECK(call)                      \
    do {                                       \
        if ((call) != hipSuccess) return -5;   \
    } while (0)

extern "C" int32_t psmprobe_stream(int32_t kind, const void* src, void* dst, int64_t bytes, int32_t grid,
                                   int32_t reps, double* ms_per_launch) {
    if (!ms_per_launch || bytes < 16 || grid < 1 || reps < 1 || kind < 0 || kind > 2 || !dst || (kind != 2 && !src))
        return -1;
    const long long n = bytes / 16;
    const float4* a = (const float4*)src;
    float4* b = (float4*)dst;
    auto launch = [&]() {
        if (kind == 0) k_probe_copy<<<grid, 256>>>(a, b, n);
        else if (kind == 1) k_probe_read<<<grid, 256>>>(a, (float*)dst, n);
        else k_probe_write<<<grid, 256>>>(b, n);
    };
    hipEvent_t e0, e1;
    PROBE_CHECK(hipEventCreate(&e0));
    PROBE_CHECK(hipEventCreate(&e1));
    for (int w = 0; w < 2; ++w) launch();
    PROBE_CHECK(hipGetLastError());
    PROBE_CHECK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r) launch();
    PROBE_CHECK(hipEventRecord(e1, 0));
    PROBE_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    PROBE_CHECK(hipEventElapsedTime(&ms, e0, e1));
    PROBE_CHECK(hipEventDestroy(e0));
    PROBE_CHECK(hipEventDestroy(e1));
    *ms_per_launch = (double)ms / reps;
    return 0;
}
