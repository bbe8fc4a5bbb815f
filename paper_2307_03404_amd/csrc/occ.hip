// Occupancy bitfield used to skip empty space exactly.
//
// Level 0: one 64-bit word per block of 4^3 cells, block (qx, qy, qz) at
//          linear index (qx * Qy + qy) * Qz + qz, Q = ceil((R - 1) / 4); cell
//          (x, y, z) is bit (x & 3) * 16 + (y & 3) * 4 + (z & 3) of its block's
//          word.  A cell is occupied iff one of its 8 corner links is a valid
//          record id; cells beyond R - 2 are empty.
// Level 1: one bit per brick of 8^3 cells, brick (bx, by, bz) at linear index
//          (bx * By + by) * Bz + bz, stored after level 0 (32-bit words).
// Both levels are rebuilt from the link table on the caller's stream; a
// bitfield that does not match the link table gives wrong renders.  The
// 4^3 blocks let a march keep the word of the block it is in and load the
// next only when it crosses into another block.
#include "internal.hpp"

namespace pxm {

void occ_layout(const int R[3], int64_t& w0_words, int Q[3], int B[3], int64_t& w1_words) {
    for (int a = 0; a < 3; ++a) {
        Q[a] = (R[a] - 1 + 3) / 4;
        B[a] = (R[a] - 1 + 7) / 8;
    }
    w0_words = 2 * (int64_t)Q[0] * Q[1] * Q[2];
    w1_words = ((int64_t)B[0] * B[1] * B[2] + 31) / 32;
}

// One wave per 4^3 block, one lane per cell (lane = bit); each lane requests
// its 8 corner links at once, and the wave's ballot is the block's word.
__global__ void k_occ0(KGrid g, uint64_t* __restrict__ occ0, int64_t n_blocks) {
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int cx0 = lane >> 4, cy0 = (lane >> 2) & 3, cz0 = lane & 3;
    for (int64_t q = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; q < n_blocks;
         q += waves) {
        const int qz = (int)(q % g.Q[2]);
        const int qy = (int)((q / g.Q[2]) % g.Q[1]);
        const int qx = (int)(q / ((int64_t)g.Q[2] * g.Q[1]));
        const int cx = 4 * qx + cx0, cy = 4 * qy + cy0, cz = 4 * qz + cz0;
        bool occ = false;
        if (cx < g.R[0] - 1 && cy < g.R[1] - 1 && cz < g.R[2] - 1) {
            const int64_t c = (int64_t)cx * g.sx + (int64_t)cy * g.sy + cz;
            int32_t l[8];
#pragma unroll
            for (int b = 0; b < 8; ++b)
                l[b] = g.link[c + ((b >> 2) & 1) * g.sx + ((b >> 1) & 1) * g.sy + (b & 1)];
#pragma unroll
            for (int b = 0; b < 8; ++b) occ |= (uint32_t)l[b] < (uint64_t)g.n_alloc;
        }
        const unsigned long long m = __ballot(occ);
        if (lane == 0) occ0[q] = (uint64_t)m;
    }
}

// One lane per brick: the OR of its (up to) 2 x 2 x 2 level-0 words; the
// wave's 64 bricks fill two level-1 words.
__global__ void k_occ1(KGrid g, const uint64_t* __restrict__ occ0, uint32_t* __restrict__ occ1,
                       int64_t nwords1) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = (int64_t)g.B[0] * g.B[1] * g.B[2];
    bool any = false;
    if (b < nb) {
        const int bx = (int)(b / ((int64_t)g.B[1] * g.B[2])), by = (int)((b / g.B[2]) % g.B[1]);
        const int bz = (int)(b % g.B[2]);
        for (int i = 0; i < 8; ++i) {
            const int qx = 2 * bx + ((i >> 2) & 1), qy = 2 * by + ((i >> 1) & 1), qz = 2 * bz + (i & 1);
            if (qx < g.Q[0] && qy < g.Q[1] && qz < g.Q[2])
                any |= occ0[((int64_t)qx * g.Q[1] + qy) * g.Q[2] + qz] != 0ull;
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
    int Q[3], B[3];
    occ_layout(g.R, w0, Q, B, w1);
    KGrid k = g;
    for (int a = 0; a < 3; ++a) {
        k.Q[a] = Q[a];
        k.B[a] = B[a];
    }
    const int64_t n_blocks = w0 / 2;
    const int64_t wgs = (n_blocks + 3) / 4;               // four waves per workgroup
    hipLaunchKernelGGL(k_occ0, dim3((unsigned)(wgs < (1 << 20) ? wgs : (1 << 20))), dim3(256), 0, st, k,
                       reinterpret_cast<uint64_t*>(occ), n_blocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = (int64_t)B[0] * B[1] * B[2];
    hipLaunchKernelGGL(k_occ1, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, k,
                       reinterpret_cast<const uint64_t*>(occ), occ + w0, w1);
    return hipGetLastError();
}

}  // namespace pxm
