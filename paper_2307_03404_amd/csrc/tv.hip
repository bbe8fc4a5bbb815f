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
// Bricks of 4^3 lattice vertices.  A workgroup stages a brick and a
// one-vertex halo (6^3 positions) in LDS with all 28 fields at once: every
// record is read as one contiguous 112-byte run, and every gradient record is
// written by 28 consecutive lanes, so no cache line is fetched or written back
// twice by one brick.  (Staging four fields at a time over 8^3 bricks fetched
// each record line once per chunk: with ~200 bricks in flight per XCD their
// lines did not survive in L2 between chunks.)  Bricks are dealt to XCDs in
// contiguous runs so that halos shared with neighbours are read through the
// same L2.  A brick is left at once when the occupancy bitfield says its
// cells have no allocated corner, else after its link loads if none of its
// vertices is allocated; the arithmetic runs over the allocated vertices only.
#include "internal.hpp"

namespace pxm {

constexpr int TB = 4;                 // brick edge (vertices)
constexpr int TH = TB + 2;            // with halo
constexpr int TH3 = TH * TH * TH;     // 216 staged positions
constexpr int PLANE = TH3 + 1;        // padded field plane: lanes over fields hit distinct banks
constexpr int TV_THREADS = 256;

__device__ __forceinline__ int hidx(int x, int y, int z) { return (x * TH + y) * TH + z; }

// One brick: stage, compact, compute.  Reached by the whole workgroup.
__device__ __forceinline__ void tv_brick(const KGrid& g, float lam_d, float lam_sh, float eps,
                                         float* __restrict__ grad, int64_t brick, int nby, int nbz,
                                         int* s_id, float (*s_v)[PLANE], int* s_list, int& s_n) {
    const int t = threadIdx.x;
    const int bz = (int)(brick % nbz), by = (int)((brick / nbz) % nby);
    const int bx = (int)(brick / ((int64_t)nbz * nby));
    const int x0 = bx * TB, y0 = by * TB, z0 = bz * TB;
    const int X = g.R[0], Y = g.R[1], Z = g.R[2];
    // An allocated vertex v of this brick is a corner of cell min(v, R-2) per
    // axis; with x0 <= R-2 that cell lies in the 8^3 cell brick of x0.
    if (g.occ1 && x0 <= X - 2 && y0 <= Y - 2 && z0 <= Z - 2) {
        const int c[3] = {x0, y0, z0};
        if (brick_empty(g, c)) return;                      // workgroup-uniform
    }
    // link ids of the halo box (-1 outside the lattice or empty)
    if (t < TH3) {
        const int hx = t / (TH * TH), hy = (t / TH) % TH, hz = t % TH;
        const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        int id = -1;
        if (x >= 0 && x < X && y >= 0 && y < Y && z >= 0 && z < Z) {
            id = g.link[((int64_t)x * Y + y) * Z + z];
            id = ((uint32_t)id < (uint64_t)g.n_alloc) ? id : -1;
        }
        s_id[t] = id;
    }
    __syncthreads();
    // compact the allocated brick vertices (one wave covers the 64 of them)
    if (t < TB * TB * TB) {
        const int c = hidx(t / (TB * TB) + 1, (t / TB) % TB + 1, t % TB + 1);
        const bool a = s_id[c] >= 0;                        // outside the lattice reads -1
        const unsigned long long m = __ballot(a);
        if (a) s_list[__popcll(m & ((1ull << t) - 1))] = c;
        if (t == 0) s_n = __popcll(m);
    }
    __syncthreads();
    const int n = s_n;
    if (n == 0) return;                                     // workgroup-uniform
    // stage the halo records: 7 lanes per position, one float4 each
    for (int i = t; i < TH3 * 7; i += TV_THREADS) {
        const int p = i / 7, q = i - 7 * p;
        const int id = s_id[p];
        const float4 w = id >= 0 ? reinterpret_cast<const float4*>(g.data + (int64_t)id * REC)[q]
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
        s_v[4 * q][p] = w.x;
        s_v[4 * q + 1][p] = w.y;
        s_v[4 * q + 2][p] = w.z;
        s_v[4 * q + 3][p] = w.w;
    }
    __syncthreads();
    // 32 lanes per allocated vertex, lane m < 28 takes field m
    for (int it = t; it < n * 32; it += TV_THREADS) {
        const int m = it & 31;
        if (m >= REC) continue;
        const int c = s_list[it >> 5];
        const int ix = c / (TH * TH), iy = (c / TH) % TH, iz = c % TH;
        const int x = x0 + ix - 1, y = y0 + iy - 1, z = z0 + iz - 1;
        const int id = s_id[c];
        const float* plane = s_v[m];
        auto val = [&](int p) -> float { return plane[p]; };
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
}

// One workgroup per brick (the hardware's dispatch keeps the bricks in flight
// balanced; a resident grid walking bricks serially was 2.3x slower).
__global__ void __launch_bounds__(TV_THREADS) k_tv(KGrid g, float lam_d, float lam_sh, float eps,
                                                   float* __restrict__ grad, int nby, int nbz) {
    __shared__ int s_id[TH3];
    __shared__ float s_v[REC][PLANE];      // field m of halo position p at s_v[m][p]
    __shared__ int s_list[TB * TB * TB];   // halo positions of allocated brick vertices
    __shared__ int s_n;
    tv_brick(g, lam_d, lam_sh, eps, grad, xcd_tile(blockIdx.x, gridDim.x), nby, nbz, s_id, s_v,
             s_list, s_n);
}

hipError_t launch_tv(const KGrid& g, float lambda_density, float lambda_sh, float eps,
                     float* grad_data, hipStream_t st) {
    const int nbx = (g.R[0] + TB - 1) / TB, nby = (g.R[1] + TB - 1) / TB;
    const int nbz = (g.R[2] + TB - 1) / TB;
    const int64_t nb = (int64_t)nbx * nby * nbz;
    hipLaunchKernelGGL(k_tv, dim3((unsigned)nb), dim3(TV_THREADS), 0, st, g, lambda_density, lambda_sh,
                       eps, grad_data, nby, nbz);
    return hipGetLastError();
}

}  // namespace pxm
