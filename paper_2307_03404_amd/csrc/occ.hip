// Occupancy bitfield used to skip empty space exactly.
//
// Level 0: one bit per cell (x, y, z), z fastest: word ((x * (Ry-1) + y) * W0
//          + z / 32), bit z % 32, W0 = ceil((Rz-1) / 32).  A cell is occupied
//          iff one of its 8 corner links is a valid record id.
// Level 1: one bit per brick of 8^3 cells, brick (bx, by, bz) at linear index
//          (bx * By + by) * Bz + bz, stored after level 0.
// Both levels are rebuilt from the link table on the caller's stream; a
// bitfield that does not match the link table gives wrong renders.
#include "internal.hpp"

namespace pxm {

void occ_layout(const int R[3], int64_t& w0_words, int& W0, int B[3], int64_t& w1_words) {
    W0 = (R[2] - 1 + 31) / 32;
    w0_words = (int64_t)(R[0] - 1) * (R[1] - 1) * W0;
    for (int a = 0; a < 3; ++a) B[a] = (R[a] - 1 + 7) / 8;
    w1_words = ((int64_t)B[0] * B[1] * B[2] + 31) / 32;
}

__device__ __forceinline__ bool valid_link(const KGrid& g, int64_t l) {
    return (uint32_t)g.link[l] < (uint64_t)g.n_alloc;
}

// One lane per level-0 word: 32 cells of one (x, y) row.
__global__ void k_occ0(KGrid g, uint32_t* __restrict__ occ0, int64_t nwords, int W0) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    const int64_t row = w / W0;
    const int z0 = (int)(w % W0) * 32;
    const int cx = (int)(row / (g.R[1] - 1)), cy = (int)(row % (g.R[1] - 1));
    const int64_t c00 = (int64_t)cx * g.sx + (int64_t)cy * g.sy;
    // column (z) occupancy of the four corner lines, then cells = any(z, z+1)
    auto column = [&](int z) -> bool {
        return valid_link(g, c00 + z) || valid_link(g, c00 + g.sy + z) || valid_link(g, c00 + g.sx + z)
            || valid_link(g, c00 + g.sx + g.sy + z);
    };
    uint32_t bits = 0;
    bool prev = column(z0);
    const int zend = min(z0 + 32, g.R[2] - 1);
    for (int z = z0; z < zend; ++z) {
        const bool next = column(z + 1);
        if (prev || next) bits |= 1u << (z - z0);
        prev = next;
    }
    occ0[w] = bits;
}

// One lane per brick; the wave's 64 bricks fill two level-1 words.
__global__ void k_occ1(KGrid g, const uint32_t* __restrict__ occ0, uint32_t* __restrict__ occ1,
                       int W0, int B0, int B1, int B2, int64_t nwords1) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = (int64_t)B0 * B1 * B2;
    bool any = false;
    if (b < nb) {
        const int bx = (int)(b / ((int64_t)B1 * B2)), by = (int)((b / B2) % B1), bz = (int)(b % B2);
        const int z0 = 8 * bz;
        const uint32_t mask = 0xFFu << (z0 & 31);
        const int xe = min(8 * bx + 8, g.R[0] - 1), ye = min(8 * by + 8, g.R[1] - 1);
        for (int cx = 8 * bx; cx < xe && !any; ++cx)
            for (int cy = 8 * by; cy < ye; ++cy)
                if (occ0[((int64_t)cx * (g.R[1] - 1) + cy) * W0 + (z0 >> 5)] & mask) {
                    any = true;
                    break;
                }
    }
    const unsigned long long m = __ballot(any);
    const int lane = lane_id();
    const int64_t word = b >> 5;
    if ((lane == 0 || lane == 32) && word < nwords1)
        occ1[word] = lane == 0 ? (uint32_t)m : (uint32_t)(m >> 32);
}

hipError_t launch_occupancy(const KGrid& g, uint32_t* occ, hipStream_t st) {
    int64_t w0, w1;
    int W0, B[3];
    occ_layout(g.R, w0, W0, B, w1);
    hipLaunchKernelGGL(k_occ0, dim3((unsigned)((w0 + 255) / 256)), dim3(256), 0, st, g, occ, w0, W0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = (int64_t)B[0] * B[1] * B[2];
    hipLaunchKernelGGL(k_occ1, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, g, occ, occ + w0,
                       W0, B[0], B[1], B[2], w1);
    return hipGetLastError();
}

}  // namespace pxm
