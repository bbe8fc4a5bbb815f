// Total-variation gradient in gather form: every allocated vertex's record
// is written by exactly one lane per field, no atomics.
//
//   TV = sum_m lambda_m sum_{u allocated, not on an upper face}
//            sqrt(dx_m(u)^2 + dy_m(u)^2 + dz_m(u)^2 + eps),
//   dx_m(u) = val_m(u + x) - val_m(u)  (empty vertices read as 0).
// dTV/d val_m(v) = lambda_m [ -(dx+dy+dz)(v)/root(v)             if v has a term
//                           + dx(v-x)/root(v-x)                    if v-x has a term
//                           + dy(v-y)/root(v-y) + dz(v-z)/root(v-z)  (likewise) ]
//
// Mapping: a wave scans 64 consecutive lattice positions (one link load per
// lane), ballots the allocated ones and then processes them two at a time:
// lanes 0-27 take field m = lane of the first vertex, lanes 32-59 field
// m = lane - 32 of the second, so every record read is one contiguous
// 112-byte row across 28 lanes.
#include "internal.hpp"

namespace pxm {

__device__ __forceinline__ int link_at(const KGrid& g, int64_t l) {
    const int v = g.link[l];
    return ((uint32_t)v < (uint64_t)g.n_alloc) ? v : -1;
}

__device__ __forceinline__ float field(const float* __restrict__ data, int id, int m) {
    return id >= 0 ? data[(int64_t)id * REC + m] : 0.f;
}

__global__ void __launch_bounds__(256) k_tv(KGrid g, float lam_d, float lam_sh, float eps,
                                            float* __restrict__ grad) {
    const int64_t total = (int64_t)g.R[0] * g.R[1] * g.R[2];
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t lin0 = wave * WAVE;
    if (lin0 >= total) return;                       // whole wave leaves together
    const int64_t my = lin0 + lane;
    const int myid = my < total ? link_at(g, my) : -1;
    unsigned long long todo = __ballot(myid >= 0);
    const int half = lane >> 5;                      // which of the two vertices
    const int m = lane & 31;                         // field handled by this lane
    const int X = g.R[0] - 1, Yt = g.R[1] - 1, Z = g.R[2] - 1;
    while (todo) {
        // take up to two allocated positions from the ballot
        const int p0 = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        int p1 = -1;
        if (todo) {
            p1 = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
        }
        // every lane takes part in the shuffles (the ballot loop is wave-uniform)
        const int id0 = __shfl(myid, p0, WAVE);
        const int id1 = p1 >= 0 ? __shfl(myid, p1, WAVE) : -1;
        const int p = half ? p1 : p0;
        if (p < 0 || m >= REC) continue;             // lanes without work idle this round
        const int64_t lin = lin0 + p;
        const int id = half ? id1 : id0;
        const int x = (int)(lin / g.sx);
        const int y = (int)((lin / g.sy) % g.R[1]);
        const int z = (int)(lin % g.R[2]);
        const float lam = m == 0 ? lam_d : lam_sh;
        const float v0 = field(g.data, id, m);
        float acc = 0.f;
        if (x < X && y < Yt && z < Z) {
            const float dx = field(g.data, link_at(g, lin + g.sx), m) - v0;
            const float dy = field(g.data, link_at(g, lin + g.sy), m) - v0;
            const float dz = field(g.data, link_at(g, lin + 1), m) - v0;
            acc -= (dx + dy + dz) * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
        }
        if (x >= 1 && y < Yt && z < Z) {
            const int a = link_at(g, lin - g.sx);
            if (a >= 0) {
                const float a0 = field(g.data, a, m);
                const float dx = v0 - a0;
                const float dy = field(g.data, link_at(g, lin - g.sx + g.sy), m) - a0;
                const float dz = field(g.data, link_at(g, lin - g.sx + 1), m) - a0;
                acc += dx * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
        }
        if (y >= 1 && x < X && z < Z) {
            const int b = link_at(g, lin - g.sy);
            if (b >= 0) {
                const float b0 = field(g.data, b, m);
                const float dx = field(g.data, link_at(g, lin - g.sy + g.sx), m) - b0;
                const float dy = v0 - b0;
                const float dz = field(g.data, link_at(g, lin - g.sy + 1), m) - b0;
                acc += dy * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
        }
        if (z >= 1 && x < X && y < Yt) {
            const int c = link_at(g, lin - 1);
            if (c >= 0) {
                const float c0 = field(g.data, c, m);
                const float dx = field(g.data, link_at(g, lin - 1 + g.sx), m) - c0;
                const float dy = field(g.data, link_at(g, lin - 1 + g.sy), m) - c0;
                const float dz = v0 - c0;
                acc += dz * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
        }
        float* __restrict__ out = grad + (int64_t)id * REC + m;
        *out += lam * acc;
    }
}

hipError_t launch_tv(const KGrid& g, float lambda_density, float lambda_sh, float eps,
                     float* grad_data, hipStream_t st) {
    const int64_t total = (int64_t)g.R[0] * g.R[1] * g.R[2];
    const int64_t waves = (total + WAVE - 1) / WAVE;
    const unsigned nb = (unsigned)((waves * WAVE + 255) / 256);
    hipLaunchKernelGGL(k_tv, dim3(nb), dim3(256), 0, st, g, lambda_density, lambda_sh, eps, grad_data);
    return hipGetLastError();
}

}  // namespace pxm
