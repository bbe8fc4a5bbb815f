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

// One lane per cell, z fastest along each (x, y) row of cells padded to W0
// words; each lane requests its 8 corner links at once (neighbouring lanes
// read neighbouring links), and a ballot per 64 cells writes two level-0
// words.  The loop runs over a multiple of 64 cells so every wave reaches the
// ballot whole.
__global__ void k_occ0(KGrid g, uint32_t* __restrict__ occ0, int64_t nwords, int W0) {
    const int64_t n_cells = nwords * 32;                    // including the row padding
    const int64_t padded = (n_cells + WAVE - 1) / WAVE * WAVE;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = lane_id();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < padded; i += stride) {
        bool occ = false;
        if (i < n_cells) {
            const int64_t w = i >> 5;
            const int64_t row = w / W0;
            const int cz = (int)(w - row * W0) * 32 + (int)(i & 31);
            if (cz < g.R[2] - 1) {
                const int cx = (int)(row / (g.R[1] - 1)), cy = (int)(row % (g.R[1] - 1));
                const int64_t c = (int64_t)cx * g.sx + (int64_t)cy * g.sy + cz;
                int32_t l[8];
#pragma unroll
                for (int b = 0; b < 8; ++b)
                    l[b] = g.link[c + ((b >> 2) & 1) * g.sx + ((b >> 1) & 1) * g.sy + (b & 1)];
#pragma unroll
                for (int b = 0; b < 8; ++b) occ |= (uint32_t)l[b] < (uint64_t)g.n_alloc;
            }
        }
        const unsigned long long m = __ballot(occ);
        const int64_t w0 = (i - lane) >> 5;
        if (lane == 0 && w0 < nwords) occ0[w0] = (uint32_t)m;
        if (lane == 32 && w0 + 1 < nwords) occ0[w0 + 1] = (uint32_t)(m >> 32);
    }
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
    const int64_t cells = w0 * 32;
    const int64_t blocks0 = (cells + 255) / 256;
    hipLaunchKernelGGL(k_occ0, dim3((unsigned)(blocks0 < (1 << 20) ? blocks0 : (1 << 20))), dim3(256), 0, st, g, occ,
                       w0, W0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = (int64_t)B[0] * B[1] * B[2];
    hipLaunchKernelGGL(k_occ1, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, g, occ, occ + w0,
                       W0, B[0], B[1], B[2], w1);
    return hipGetLastError();
}

}  // namespace pxm
