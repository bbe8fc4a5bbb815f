// Total-variation gradient in gather form: one lane per lattice vertex writes
// the full dTV/d(record) of its own vertex, reading the 12 lattice neighbours
// whose difference terms involve it.  No atomics, one writer per record.
//
//   TV = sum_m lambda_m sum_{u allocated, not on an upper face}
//            sqrt(dx_m(u)^2 + dy_m(u)^2 + dz_m(u)^2 + eps),
//   dx_m(u) = val_m(u + x) - val_m(u)  (empty vertices read as 0).
// dTV/d val_m(v) = lambda_m [ -(dx+dy+dz)(v)/root(v)           if v has a term
//                           + dx(v-x)/root(v-x)                  if v-x has a term
//                           + dy(v-y)/root(v-y) + dz(v-z)/root(v-z) (likewise) ]
#include "internal.hpp"

namespace pxm {

__device__ __forceinline__ float4 rec4(const float* __restrict__ data, int id, int q) {
    if (id < 0) return make_float4(0.f, 0.f, 0.f, 0.f);
    return reinterpret_cast<const float4*>(data + (int64_t)id * REC)[q];
}

__device__ __forceinline__ float comp(const float4& v, int c) {
    return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}

__global__ void __launch_bounds__(256) k_tv(KGrid g, float lam_d, float lam_sh, float eps,
                                            float* __restrict__ grad) {
    const int64_t total = (int64_t)g.R[0] * g.R[1] * g.R[2];
    const int64_t lin = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lin >= total) return;
    const int id = g.link[lin];
    if (id < 0 || (int64_t)id >= g.n_alloc) return;
    const int x = (int)(lin / g.sx);
    const int y = (int)((lin / g.sy) % g.R[1]);
    const int z = (int)(lin % g.R[2]);
    const int X = g.R[0] - 1, Yt = g.R[1] - 1, Z = g.R[2] - 1;
    const bool own = x < X && y < Yt && z < Z;
    auto L = [&](int64_t l) -> int {
        const int v = g.link[l];
        return ((uint32_t)v < (uint64_t)g.n_alloc) ? v : -1;
    };
    // neighbours of v itself
    const int nx = own ? L(lin + g.sx) : -1;
    const int ny = own ? L(lin + g.sy) : -1;
    const int nz = own ? L(lin + 1) : -1;
    // lower neighbours whose own term reads v, and their other two upper neighbours
    const int mx = (x >= 1 && y < Yt && z < Z) ? L(lin - g.sx) : -1;
    const int my = (y >= 1 && x < X && z < Z) ? L(lin - g.sy) : -1;
    const int mz = (z >= 1 && x < X && y < Yt) ? L(lin - 1) : -1;
    const int mx_y = mx >= 0 ? L(lin - g.sx + g.sy) : -1;
    const int mx_z = mx >= 0 ? L(lin - g.sx + 1) : -1;
    const int my_x = my >= 0 ? L(lin - g.sy + g.sx) : -1;
    const int my_z = my >= 0 ? L(lin - g.sy + 1) : -1;
    const int mz_x = mz >= 0 ? L(lin - 1 + g.sx) : -1;
    const int mz_y = mz >= 0 ? L(lin - 1 + g.sy) : -1;
    float* __restrict__ out = grad + (int64_t)id * REC;
#pragma unroll 1
    for (int q = 0; q < 7; ++q) {
        const float4 v = rec4(g.data, id, q);
        const float4 vx = rec4(g.data, nx, q), vy = rec4(g.data, ny, q), vz = rec4(g.data, nz, q);
        const float4 a = rec4(g.data, mx, q), ay = rec4(g.data, mx_y, q), az = rec4(g.data, mx_z, q);
        const float4 b = rec4(g.data, my, q), bx = rec4(g.data, my_x, q), bz = rec4(g.data, my_z, q);
        const float4 c = rec4(g.data, mz, q), cx = rec4(g.data, mz_x, q), cy = rec4(g.data, mz_y, q);
        float4 o = reinterpret_cast<float4*>(out)[q];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const int m = 4 * q + cc;
            const float lam = m == 0 ? lam_d : lam_sh;
            const float v0 = comp(v, cc);
            float acc = 0.f;
            if (own) {
                const float dx = comp(vx, cc) - v0, dy = comp(vy, cc) - v0, dz = comp(vz, cc) - v0;
                acc -= (dx + dy + dz) * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (mx >= 0) {
                const float a0 = comp(a, cc);
                const float dx = v0 - a0, dy = comp(ay, cc) - a0, dz = comp(az, cc) - a0;
                acc += dx * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (my >= 0) {
                const float b0 = comp(b, cc);
                const float dx = comp(bx, cc) - b0, dy = v0 - b0, dz = comp(bz, cc) - b0;
                acc += dy * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (mz >= 0) {
                const float c0 = comp(c, cc);
                const float dx = comp(cx, cc) - c0, dy = comp(cy, cc) - c0, dz = v0 - c0;
                acc += dz * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            const float add = lam * acc;
            if (cc == 0) o.x += add; else if (cc == 1) o.y += add; else if (cc == 2) o.z += add; else o.w += add;
        }
        reinterpret_cast<float4*>(out)[q] = o;
    }
}

hipError_t launch_tv(const KGrid& g, float lambda_density, float lambda_sh, float eps,
                     float* grad_data, hipStream_t st) {
    const int64_t total = (int64_t)g.R[0] * g.R[1] * g.R[2];
    const unsigned nb = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_tv, dim3(nb), dim3(256), 0, st, g, lambda_density, lambda_sh, eps, grad_data);
    return hipGetLastError();
}

}  // namespace pxm
