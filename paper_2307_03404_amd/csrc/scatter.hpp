// Wave-aggregated scatter of grid gradients.
//
// Rays of one wave come from one 8x8 pixel tile, so at the same sample step
// most lanes sit in the same lattice cell and add into the same 8 vertex
// records.  Issuing those adds as per-lane float atomics serialises them on
// identical addresses.  Instead, at every step the lanes that have a gradient
// are grouped by cell; each group's 8 x 28 contributions are summed across
// the wave with a reduce-scatter (DPP row permutations plus two cross-row
// shuffles), after which lane l < 28 owns field l of one corner and issues a
// single add: 28 distinct, contiguous addresses per corner per group.
#pragma once

#include "kcommon.hpp"

namespace pxm {

// Lane-permutation controls of DPP used below (GFX9 encoding).
constexpr int DPP_XOR1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int DPP_XOR3 = 0x1B;        // quad_perm [3,2,1,0]
constexpr int DPP_HALF_MIRROR = 0x141; // lane i <-> 7 - i within 8 (= xor 7)
constexpr int DPP_MIRROR = 0x140;      // lane i <-> 15 - i within 16 (= xor 15)

template <int CTRL>
__device__ __forceinline__ float dpp_from(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Recursive-halving reduce-scatter of 32 slots over the 64 lanes.  In each
// round a lane pairs with a partner that differs in one lane bit (and agrees
// on the bits already used); it keeps the half of its slots whose slot bit
// matches that lane bit and adds the partner's copy of them.  Each round
// writes a half-size array indexed by the undecided slot bits only, so every
// index is a compile-time constant after unrolling.
//   round 1: slot bit 3, partner lane ^ 15 (row mirror)
//   round 2: slot bit 2, partner lane ^ 7  (half-row mirror)
//   round 3: slot bit 1, partner lane ^ 3  (quad permutation)
//   round 4: slot bit 0, partner lane ^ 1  (quad permutation)
//   round 5: slot bit 4, partner lane ^ 16 (cross-row shuffle)
//   then add lane ^ 32.
__device__ __forceinline__ float pair_keep(float lo, float hi, bool up, float recv) {
    return (up ? hi : lo) + recv;
}

__device__ __forceinline__ float reduce_scatter32(const float v[32], int lane) {
    const bool u3 = (lane >> 3) & 1, u2 = (lane >> 2) & 1, u1 = (lane >> 1) & 1, u0 = lane & 1;
    const bool u4 = (lane >> 4) & 1;
    float r1[16];   // index j: slot bits 0-2 = j bits 0-2, slot bit 4 = j bit 3
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int lo = (j & 7) | ((j & 8) << 1), hi = lo | 8;
        r1[j] = pair_keep(v[lo], v[hi], u3, dpp_from<DPP_MIRROR>(u3 ? v[lo] : v[hi]));
    }
    float r2[8];    // index i: slot bits 0-1 = i bits 0-1, slot bit 4 = i bit 2
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int lo = (i & 3) | ((i & 4) << 1), hi = lo | 4;
        r2[i] = pair_keep(r1[lo], r1[hi], u2, dpp_from<DPP_HALF_MIRROR>(u2 ? r1[lo] : r1[hi]));
    }
    float r3[4];    // index h: slot bit 0 = h bit 0, slot bit 4 = h bit 1
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const int lo = (h & 1) | ((h & 2) << 1), hi = lo | 2;
        r3[h] = pair_keep(r2[lo], r2[hi], u1, dpp_from<DPP_XOR3>(u1 ? r2[lo] : r2[hi]));
    }
    float r4[2];    // index q: slot bit 4
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int lo = q << 1, hi = lo | 1;
        r4[q] = pair_keep(r3[lo], r3[hi], u0, dpp_from<DPP_XOR1>(u0 ? r3[lo] : r3[hi]));
    }
    const float r5 = pair_keep(r4[0], r4[1], u4, __shfl_xor(u4 ? r4[0] : r4[1], 16, WAVE));
    return r5 + __shfl_xor(r5, 32, WAVE);
}

// Per-wave write-combining cache of vertex gradients in LDS: CACHE_SLOTS
// direct-mapped slots of (vertex id, 28 partial sums).  Merged sums are added
// into it with LDS arithmetic; a slot is written back to HBM with 28 atomics
// only when another vertex claims it, and once more when the wave ends.  Lane
// l only ever touches column l of the data, and every lane writes the
// (wave-uniform) key, so no cross-lane ordering is needed after set-up.
constexpr int CACHE_SLOTS = 128;
constexpr int CACHE_FLOATS = CACHE_SLOTS * (REC + 1);   // per wave

struct WaveCache {
    int* key;       // [CACHE_SLOTS], -1 = free
    float* data;    // [CACHE_SLOTS][REC]
};

__device__ __forceinline__ WaveCache wave_cache(float* smem) {
    const int w = threadIdx.x / WAVE;
    float* base = smem + (size_t)w * CACHE_FLOATS;
    return WaveCache{reinterpret_cast<int*>(base), base + CACHE_SLOTS};
}

// Mark every slot free; the caller synchronises the workgroup afterwards.
__device__ __forceinline__ void cache_init(const WaveCache& wc) {
    for (int s = lane_id(); s < CACHE_SLOTS; s += WAVE) wc.key[s] = -1;
}

__device__ __forceinline__ int cache_slot(int id) {
    return (int)(((uint32_t)id * 2654435761u) >> (32 - 7)) & (CACHE_SLOTS - 1);
}

// Add lane l's value `tot` (l < 28) to field l of vertex `id` (wave-uniform).
__device__ __forceinline__ void cache_add(const WaveCache& wc, int id, float tot, int lane,
                                          float* __restrict__ grad) {
    const int slot = cache_slot(id);
    const int cur = wc.key[slot];
    float* cell = wc.data + slot * REC;
    if (cur == id) {
        if (lane < REC) cell[lane] += tot;
    } else {
        if (lane < REC) {
            if (cur >= 0) unsafeAtomicAdd(grad + (int64_t)cur * REC + lane, cell[lane]);
            cell[lane] = tot;
        }
        wc.key[slot] = id;
    }
}

// Write every occupied slot back to HBM and free it.
__device__ __forceinline__ void cache_flush(const WaveCache& wc, float* __restrict__ grad) {
    const int lane = lane_id();
#pragma unroll 1
    for (int s = 0; s < CACHE_SLOTS; ++s) {
        const int cur = wc.key[s];
        if (cur < 0) continue;
        if (lane < REC) unsafeAtomicAdd(grad + (int64_t)cur * REC + lane, wc.data[s * REC + lane]);
        wc.key[s] = -1;
    }
}

// Gradient of one sample: dL/d sigma_raw (gsig) and dL/ds_c (gs[c]) to be
// spread over the cell's corners with weights w[b]; field m of corner b
// receives w[b] * G_m with G_0 = gsig and G_{1+9c+k} = gs[c] * Y[k].
// Lanes are grouped by cell; each group is reduced across the wave and its
// totals go through the wave's cache.  Must be reached by every lane.
__device__ __forceinline__ void scatter_merged(bool have, int64_t key, const int idx[8],
                                               const float w[8], float gsig, const float gs[3],
                                               const float Y[9], const WaveCache& wc,
                                               float* __restrict__ grad) {
    const int lane = lane_id();
    unsigned long long pending = __ballot(have);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int klo = __builtin_amdgcn_readlane((int)(uint32_t)key, leader);
        const int khi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)key >> 32), leader);
        const int64_t k0 = (int64_t)(((uint64_t)(uint32_t)khi << 32) | (uint32_t)klo);
        const bool mine = have && key == k0;
        pending &= ~__ballot(mine);
#pragma unroll 1
        for (int b = 0; b < 8; ++b) {
            const int id = __builtin_amdgcn_readlane(idx[b], leader);
            if (id < 0) continue;
            const float wb = mine ? w[b] : 0.f;
            float v[32];
            v[0] = wb * gsig;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float a = wb * gs[c];
#pragma unroll
                for (int k = 0; k < 9; ++k) v[1 + 9 * c + k] = a * Y[k];
            }
            v[28] = v[29] = v[30] = v[31] = 0.f;
            const float tot = reduce_scatter32(v, lane);
            cache_add(wc, id, tot, lane, grad);
        }
    }
}

}  // namespace pxm
