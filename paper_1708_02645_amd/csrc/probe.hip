// Attainable-bandwidth probe: a plain streaming read of a device buffer,
// used to report the rate that a simple coalesced read achieves beside the
// published peak.  Each workgroup reads contiguous 32 KB chunks (eight
// 16-byte loads per lane in flight, non-temporal), chunks grid-strided.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace qs {

constexpr int kProbeUnroll = 8;
typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_read_kernel(const float4* __restrict__ x, int64_t n4, float* out)
{
    constexpr int64_t chunk = kProbeUnroll * 256;  // float4 per workgroup chunk
    float s[kProbeUnroll] = {};
    int64_t c = blockIdx.x;
    for (; (c + 1) * chunk <= n4; c += gridDim.x) {
        const f4* p = reinterpret_cast<const f4*>(x + c * chunk + threadIdx.x);
        f4 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(p + u * 256);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) s[u] += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    if (c * chunk < n4) {  // the partial last chunk, if this workgroup owns it
        for (int64_t i = c * chunk + threadIdx.x; i < n4; i += 256) {
            const float4 v = x[i];
            s[0] += (v.x + v.y) + (v.z + v.w);
        }
    }
    float t = 0.f;
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) t += s[u];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = t;  // keeps the loads live
}

}  // namespace qs

extern "C" int spline_probe_stream_read(const void* buf, size_t bytes, float* out, int32_t grid, void* stream)
{
    if (!buf || !out) return qs::fail(SPL_EINVAL, "NULL argument");
    if (grid < 1 || grid > (1 << 20)) return qs::fail(SPL_EINVAL, "grid must be in [1, 2^20]");
    if ((reinterpret_cast<uintptr_t>(buf) & 15) != 0) return qs::fail(SPL_EINVAL, "buffer not 16-byte aligned");
    hipLaunchKernelGGL(qs::stream_read_kernel, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const float4*>(buf), (int64_t)(bytes / 16), out);
    QS_HIP(hipGetLastError());
    return SPL_OK;
}
