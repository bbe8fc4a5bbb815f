// Total-variation gradient in gather form: every allocated vertex's record
// is written by exactly one thread per field, no atomics.
//
//   TV = sum_m lambda_m sum_{u allocated, not on an upper face}
//            sqrt(dx_m(u)^2 + dy_m(u)^2 + dz_m(u)^2 + eps),
//   dx_m(u) = val_m(u + x) - val_m(u)  (empty vertices read as 0).
// dTV/d val_m(v) = lambda_m [ -(dx+dy+dz)(v)/root(v)             if v has a term
//                           + dx(v-x)/root(v-x)                    if v-x has a term
//                           + dy(v-y)/root(v-y) + dz(v-z)/root(v-z)  (likewise) ]
//
// One workgroup per brick of 8^3 lattice vertices.  It stages the brick and a
// one-vertex halo (10^3 positions) in LDS four fields at a time, so each
// allocated record is fetched about twice instead of once per neighbour that
// reads it.  Bricks are dealt to XCDs in contiguous runs so that the halo a
// brick shares with its neighbours is read through the same L2.  A brick is
// left at once when the occupancy bitfield says its cells have no allocated
// corner, else after its link loads if none of its vertices is allocated; the
// arithmetic runs over a compacted list of the allocated vertices only.
#include "internal.hpp"

namespace pxm {

constexpr int TB = 8;                 // brick edge (vertices)
constexpr int TH = TB + 2;            // with halo
constexpr int TH3 = TH * TH * TH;     // 1000 staged positions
constexpr int TV_THREADS = 256;

__device__ __forceinline__ int hidx(int x, int y, int z) { return (x * TH + y) * TH + z; }

__global__ void __launch_bounds__(TV_THREADS) k_tv(KGrid g, float lam_d, float lam_sh, float eps,
                                                   float* __restrict__ grad, int nbx, int nby,
                                                   int nbz) {
    __shared__ int s_id[TH3];
    __shared__ float s_v[4][TH3];          // four field planes of the current chunk
    __shared__ int s_list[TB * TB * TB];   // halo positions of allocated brick vertices
    __shared__ int s_n;
    const int t = threadIdx.x;
    const int64_t brick = xcd_tile(blockIdx.x, gridDim.x);
    const int bz = (int)(brick % nbz), by = (int)((brick / nbz) % nby);
    const int bx = (int)(brick / ((int64_t)nbz * nby));
    const int x0 = bx * TB, y0 = by * TB, z0 = bz * TB;
    const int X = g.R[0], Y = g.R[1], Z = g.R[2];
    // An allocated vertex v of this brick is a corner of cell min(v, R-2) per
    // axis, which lies in cell brick (bx, by, bz) whenever that brick exists.
    if (g.occ1 && bx < g.B[0] && by < g.B[1] && bz < g.B[2]) {
        const int c[3] = {x0, y0, z0};
        if (brick_empty(g, c)) return;                      // workgroup-uniform
    }
    if (t == 0) s_n = 0;
    // link ids of the halo box (-1 outside the lattice or empty)
    for (int p = t; p < TH3; p += TV_THREADS) {
        const int hx = p / (TH * TH), hy = (p / TH) % TH, hz = p % TH;
        const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        int id = -1;
        if (x >= 0 && x < X && y >= 0 && y < Y && z >= 0 && z < Z) {
            id = g.link[((int64_t)x * Y + y) * Z + z];
            id = ((uint32_t)id < (uint64_t)g.n_alloc) ? id : -1;
        }
        s_id[p] = id;
    }
    __syncthreads();
    // compact the allocated vertices of the brick (the order is irrelevant:
    // every vertex is computed and written by one thread)
    for (int v = t; v < TB * TB * TB; v += TV_THREADS) {
        const int c = hidx(v / (TB * TB) + 1, (v / TB) % TB + 1, v % TB + 1);
        const bool a = s_id[c] >= 0;                        // outside the lattice reads -1
        const unsigned long long m = __ballot(a);
        int base = 0;
        if (lane_id() == 0 && m) base = atomicAdd(&s_n, __popcll(m));
        base = __shfl(base, 0);
        if (a) s_list[base + __popcll(m & ((1ull << lane_id()) - 1))] = c;
    }
    __syncthreads();
    const int n = s_n;
    if (n == 0) return;                                     // workgroup-uniform
#pragma unroll 1
    for (int q = 0; q < 7; ++q) {
        for (int p = t; p < TH3; p += TV_THREADS) {
            const int id = s_id[p];
            const float4 w = id >= 0 ? reinterpret_cast<const float4*>(g.data + (int64_t)id * REC)[q]
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
            s_v[0][p] = w.x;
            s_v[1][p] = w.y;
            s_v[2][p] = w.z;
            s_v[3][p] = w.w;
        }
        __syncthreads();
        for (int it = t; it < 4 * n; it += TV_THREADS) {
            const int f = it & 3;
            const int c = s_list[it >> 2];
            const int ix = c / (TH * TH), iy = (c / TH) % TH, iz = c % TH;
            const int x = x0 + ix - 1, y = y0 + iy - 1, z = z0 + iz - 1;
            const int id = s_id[c];
            const float* plane = s_v[f];
            auto val = [&](int p) -> float { return plane[p]; };
            const int m = 4 * q + f;
            const float lam = m == 0 ? lam_d : lam_sh;
            const float v0 = val(c);
            float acc = 0.f;
            if (x < X - 1 && y < Y - 1 && z < Z - 1) {
                const float dx = val(c + TH * TH) - v0;
                const float dy = val(c + TH) - v0;
                const float dz = val(c + 1) - v0;
                acc -= (dx + dy + dz) * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (x >= 1 && y < Y - 1 && z < Z - 1 && s_id[c - TH * TH] >= 0) {
                const float a0 = val(c - TH * TH);
                const float dx = v0 - a0;
                const float dy = val(c - TH * TH + TH) - a0;
                const float dz = val(c - TH * TH + 1) - a0;
                acc += dx * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (y >= 1 && x < X - 1 && z < Z - 1 && s_id[c - TH] >= 0) {
                const float b0 = val(c - TH);
                const float dx = val(c - TH + TH * TH) - b0;
                const float dy = v0 - b0;
                const float dz = val(c - TH + 1) - b0;
                acc += dy * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (z >= 1 && x < X - 1 && y < Y - 1 && s_id[c - 1] >= 0) {
                const float c0 = val(c - 1);
                const float dx = val(c - 1 + TH * TH) - c0;
                const float dy = val(c - 1 + TH) - c0;
                const float dz = v0 - c0;
                acc += dz * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            grad[(int64_t)id * REC + m] += lam * acc;
        }
        __syncthreads();
    }
}

hipError_t launch_tv(const KGrid& g, float lambda_density, float lambda_sh, float eps,
                     float* grad_data, hipStream_t st) {
    const int nbx = (g.R[0] + TB - 1) / TB, nby = (g.R[1] + TB - 1) / TB;
    const int nbz = (g.R[2] + TB - 1) / TB;
    const int64_t nb = (int64_t)nbx * nby * nbz;
    hipLaunchKernelGGL(k_tv, dim3((unsigned)nb), dim3(TV_THREADS), 0, st, g, lambda_density, lambda_sh,
                       eps, grad_data, nbx, nby, nbz);
    return hipGetLastError();
}

}  // namespace pxm
