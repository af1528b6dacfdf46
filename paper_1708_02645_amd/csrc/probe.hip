// Attainable-bandwidth probe: a plain streaming read of a device buffer
// (16 bytes per lane, grid-stride), used to report the HBM rate that a
// simple read achieves beside the published peak.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace qs {

__global__ __launch_bounds__(256) void stream_read_kernel(const float4* __restrict__ x, int64_t n4, float* out)
{
    float s = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256) {
        const float4 v = x[i];
        s += v.x + v.y + v.z + v.w;
    }
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;  // keeps the loads live
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
