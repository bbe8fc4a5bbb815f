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
// reads it; bricks without an allocated vertex leave after their link loads.
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
    __shared__ int s_any;
    const int t = threadIdx.x;
    const int64_t brick = blockIdx.x;
    const int bz = (int)(brick % nbz), by = (int)((brick / nbz) % nby);
    const int bx = (int)(brick / ((int64_t)nbz * nby));
    const int x0 = bx * TB, y0 = by * TB, z0 = bz * TB;
    const int X = g.R[0], Y = g.R[1], Z = g.R[2];
    if (t == 0) s_any = 0;
    __syncthreads();
    // link ids of the halo box (-1 outside the lattice or empty)
    bool any = false;
    for (int p = t; p < TH3; p += TV_THREADS) {
        const int hx = p / (TH * TH), hy = (p / TH) % TH, hz = p % TH;
        const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        int id = -1;
        if (x >= 0 && x < X && y >= 0 && y < Y && z >= 0 && z < Z) {
            id = g.link[((int64_t)x * Y + y) * Z + z];
            id = ((uint32_t)id < (uint64_t)g.n_alloc) ? id : -1;
        }
        s_id[p] = id;
        if (id >= 0 && hx >= 1 && hx <= TB && hy >= 1 && hy <= TB && hz >= 1 && hz <= TB) any = true;
    }
    if (any) s_any = 1;
    __syncthreads();
    if (!s_any) return;                                     // workgroup-uniform
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
        // 512 interior vertices x 4 fields, 8 items per thread
        for (int it = t; it < TB * TB * TB * 4; it += TV_THREADS) {
            const int f = it & 3, v = it >> 2;
            const int ix = v / (TB * TB) + 1, iy = (v / TB) % TB + 1, iz = v % TB + 1;
            const int x = x0 + ix - 1, y = y0 + iy - 1, z = z0 + iz - 1;
            if (x >= X || y >= Y || z >= Z) continue;
            const int c = hidx(ix, iy, iz);
            const int id = s_id[c];
            if (id < 0) continue;
            const float* plane = s_v[f];
            auto val = [&](int p) -> float { return plane[p]; };
            const int m = 4 * q + f;
            const float lam = m == 0 ? lam_d : lam_sh;
            const float v0 = val(c);
            float acc = 0.f;
            if (x < X - 1 && y < Y - 1 && z < Z - 1) {
                const float dx = val(hidx(ix + 1, iy, iz)) - v0;
                const float dy = val(hidx(ix, iy + 1, iz)) - v0;
                const float dz = val(hidx(ix, iy, iz + 1)) - v0;
                acc -= (dx + dy + dz) * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (x >= 1 && y < Y - 1 && z < Z - 1 && s_id[hidx(ix - 1, iy, iz)] >= 0) {
                const float a0 = val(hidx(ix - 1, iy, iz));
                const float dx = v0 - a0;
                const float dy = val(hidx(ix - 1, iy + 1, iz)) - a0;
                const float dz = val(hidx(ix - 1, iy, iz + 1)) - a0;
                acc += dx * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (y >= 1 && x < X - 1 && z < Z - 1 && s_id[hidx(ix, iy - 1, iz)] >= 0) {
                const float b0 = val(hidx(ix, iy - 1, iz));
                const float dx = val(hidx(ix + 1, iy - 1, iz)) - b0;
                const float dy = v0 - b0;
                const float dz = val(hidx(ix, iy - 1, iz + 1)) - b0;
                acc += dy * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (z >= 1 && x < X - 1 && y < Y - 1 && s_id[hidx(ix, iy, iz - 1)] >= 0) {
                const float c0 = val(hidx(ix, iy, iz - 1));
                const float dx = val(hidx(ix + 1, iy, iz - 1)) - c0;
                const float dy = val(hidx(ix, iy + 1, iz - 1)) - c0;
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
