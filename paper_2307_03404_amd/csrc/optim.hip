// Mapping update: one sparse RMSProp step over the vertex records (Sec. 5.4
// names RMSProp for the mapping).  A record is touched when any of its
// gradient entries is non-zero; only touched records change (values and
// running averages), so vertices no ray reached keep their state, as in the
// Plenoxel optimiser this method builds on.  The gradient is zeroed after it
// is read, so one call ends a mapping iteration.
//
// A group of L lanes per record (L = 8, 4, 1 for records of 7, 4, 1 float4:
// SH degree 2, 1, 0), lane q < Q holding float4 q of it: the record's
// "touched" bit comes from a wave ballot over its group, and every load and
// store is a contiguous run.  Bound by HBM: at degree 2, 112 B read per
// record, plus 112 B written (gradient zeroed) and 2 x 224 B
// read-modify-write (values, averages) per touched record.
#include "internal.hpp"

namespace pxm {

template <int Q, int L>
__global__ void __launch_bounds__(256) k_rmsprop(int64_t n, float4* __restrict__ data,
                                                 float4* __restrict__ grad,
                                                 float4* __restrict__ avg, float lr_d, float lr_sh,
                                                 float alpha, float eps) {
    static_assert(Q <= L && (L & (L - 1)) == 0 && L <= 8, "a record's lanes form one ballot group");
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t rec = t / L;
    const int q = (int)(t % L);
    const bool act = rec < n && q < Q;
    const int64_t i = rec * Q + q;
    const float4 g = act ? grad[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const bool nz = g.x != 0.f || g.y != 0.f || g.z != 0.f || g.w != 0.f;
    const unsigned long long m = __ballot(nz);
    const bool touched = ((m >> (lane_id() & ~(L - 1))) & ((1ull << L) - 1ull)) != 0ull;
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

template <int Q, int L>
static void rmsprop_go(int64_t n, float* data, float* grad, float* avg, float lr_d, float lr_sh,
                       float alpha, float eps, hipStream_t st) {
    const int64_t threads = n * L;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    hipLaunchKernelGGL((k_rmsprop<Q, L>), dim3(blocks), dim3(256), 0, st, n,
                       reinterpret_cast<float4*>(data), reinterpret_cast<float4*>(grad),
                       reinterpret_cast<float4*>(avg), lr_d, lr_sh, alpha, eps);
}

hipError_t launch_rmsprop(int64_t n, int deg, float* data, float* grad, float* avg, float lr_d,
                          float lr_sh, float alpha, float eps, hipStream_t st) {
    if (deg == 0) rmsprop_go<1, 1>(n, data, grad, avg, lr_d, lr_sh, alpha, eps, st);
    else if (deg == 1) rmsprop_go<4, 4>(n, data, grad, avg, lr_d, lr_sh, alpha, eps, st);
    else rmsprop_go<7, 8>(n, data, grad, avg, lr_d, lr_sh, alpha, eps, st);
    return hipGetLastError();
}

}  // namespace pxm
