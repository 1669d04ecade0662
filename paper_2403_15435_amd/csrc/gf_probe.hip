// Achievable HBM bandwidth probe: a grid-stride triad over 16-byte vectors,
// launched with enough workgroups to fill every CU several times over.  Not a
// step of the method; it measures the roofline's denominator on the device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/geoflood.h"

namespace {

__global__ void __launch_bounds__(256) triad_kernel(const float4 *__restrict__ a, const float4 *__restrict__ b,
                                                    float4 *__restrict__ c, int64_t n4, float s)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 x = a[i], y = b[i];
        c[i] = make_float4(x.x + s * y.x, x.y + s * y.y, x.z + s * y.z, x.w + s * y.w);
    }
}

}  // namespace

extern "C" int gf_probe_triad(const float *a, const float *b, float *c, int64_t n, float s, void *hip_stream)
{
    if (!a || !b || !c || n <= 0 || (n & 3)) return GF_E_INVALID;
    if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) return GF_E_INVALID;
    const int64_t n4 = n / 4;
    // 8 workgroups of 256 threads per CU on 256 CUs, fewer for small arrays
    const int64_t want = (n4 + 255) / 256;
    const unsigned grid = (unsigned)(want < 2048 ? want : 2048);
    hipLaunchKernelGGL(triad_kernel, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream, (const float4 *)a,
                       (const float4 *)b, (float4 *)c, n4, s);
    return hipGetLastError() == hipSuccess ? GF_OK : GF_E_HIP;
}
