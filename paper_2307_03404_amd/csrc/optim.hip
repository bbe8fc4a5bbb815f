// Mapping update: one sparse RMSProp step over the vertex records (Sec. 5.4
// names RMSProp for the mapping).  A record is touched when any of its 28
// gradient entries is non-zero; only touched records change (values and
// running averages), so vertices no ray reached keep their state, as in the
// Plenoxel optimiser this method builds on.  The gradient is zeroed after it
// is read, so one call ends a mapping iteration.
//
// Eight lanes per record, seven of them holding one float4 of it: the
// record's "touched" bit comes from a wave ballot over its group of eight,
// and every load and store is a contiguous 112-byte run.  Bound by HBM:
// 112 B read per record, plus 112 B written (gradient zeroed) and 2 x 224 B
// read-modify-write (values, averages) per touched record.
#include "internal.hpp"

namespace pxm {

__global__ void __launch_bounds__(256) k_rmsprop(int64_t n, float4* __restrict__ data,
                                                 float4* __restrict__ grad,
                                                 float4* __restrict__ avg, float lr_d, float lr_sh,
                                                 float alpha, float eps) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t rec = t >> 3;
    const int q = (int)(t & 7);
    const bool act = rec < n && q < 7;
    const int64_t i = rec * 7 + q;
    const float4 g = act ? grad[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const bool nz = g.x != 0.f || g.y != 0.f || g.z != 0.f || g.w != 0.f;
    const unsigned long long m = __ballot(nz);
    const bool touched = ((m >> (lane_id() & ~7)) & 0xffull) != 0ull;
    if (!act || !touched) return;
    float4 v = avg[i];
    float4 x = data[i];
    const float a1 = 1.f - alpha;
    v.x = alpha * v.x + a1 * g.x * g.x;
    v.y = alpha * v.y + a1 * g.y * g.y;
    v.z = alpha * v.z + a1 * g.z * g.z;
    v.w = alpha * v.w + a1 * g.w * g.w;
    x.x -= (q == 0 ? lr_d : lr_sh) * g.x / (sqrtf(v.x) + eps);   // entry 0 is the density
    x.y -= lr_sh * g.y / (sqrtf(v.y) + eps);
    x.z -= lr_sh * g.z / (sqrtf(v.z) + eps);
    x.w -= lr_sh * g.w / (sqrtf(v.w) + eps);
    avg[i] = v;
    data[i] = x;
    grad[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_rmsprop(int64_t n, float* data, float* grad, float* avg, float lr_d, float lr_sh,
                          float alpha, float eps, hipStream_t st) {
    const int64_t threads = n * 8;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    hipLaunchKernelGGL(k_rmsprop, dim3(blocks), dim3(256), 0, st, n,
                       reinterpret_cast<float4*>(data), reinterpret_cast<float4*>(grad),
                       reinterpret_cast<float4*>(avg), lr_d, lr_sh, alpha, eps);
    return hipGetLastError();
}

}  // namespace pxm
