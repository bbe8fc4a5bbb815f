// Read-bandwidth probe: the ceiling a cache level offers to streaming reads,
// beside which the fused kernel's measured traffic is judged.  Workgroup b
// runs on XCD b % 8 (the hardware deals workgroups round-robin over the 8
// XCDs), so giving XCD x its own eighth of the buffer keeps each L2's working
// set at bytes / 8: a buffer of up to ~32 MB stays in the eight 4 MB L2s, up
// to ~256 MB in the Infinity Cache, larger ones stream from HBM.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pxm {

__global__ void __launch_bounds__(256) k_probe_read(const float4* __restrict__ buf, int64_t n4, int passes,
                                                    float* __restrict__ sink) {
    const int64_t per_xcd = n4 / 8;
    const int64_t base = (int64_t)(blockIdx.x % 8) * per_xcd;
    const int64_t wg = blockIdx.x / 8, n_wg = gridDim.x / 8;
    float acc = 0.f;
    for (int p = 0; p < passes; ++p)
        for (int64_t i = wg * blockDim.x + threadIdx.x; i < per_xcd; i += n_wg * blockDim.x) {
            const float4 v = buf[base + i];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

hipError_t launch_probe_read(const float4* buf, int64_t n4, int passes, float* sink, int n_wg,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_probe_read, dim3(n_wg), dim3(256), 0, st, buf, n4, passes, sink);
    return hipGetLastError();
}

}  // namespace pxm
