// Wave-aggregated scatter of grid gradients.
//
// Rays of one wave come from one 8x8 pixel tile, so at one sample step most
// lanes sit in the same lattice cell and add into the same 8 vertex records;
// per-lane float atomics would serialise on identical addresses.  At every
// step the lanes that carry a gradient are grouped by cell.  For a group g,
// field m of its corner b receives
//     C[g*8 + b][m] = sum over lanes l of W[l][g*8 + b] * G[l][m],
//     W[l][g*8 + b] = w_b(l) if lane l is in group g, else 0,
//     G[l][0] = dL/d sigma_raw,  G[l][1 + 9c + k] = dL/ds_c * Y_k(d_l),
// a small dense contraction over the 64 lanes.  Up to four groups (32 rows)
// are contracted per pass on the matrix cores with 32 FP32 MFMA 32x32x2
// instructions (K = 2 lanes each); W and G are staged in LDS in the operand
// order the instruction reads.  The 32 x 28 totals are added into a per-wave
// write-combining cache of vertex records in LDS, which writes back to HBM
// with atomics only on eviction and when the wave ends.
#pragma once

#include "kcommon.hpp"

namespace pxm {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// per-wave LDS: write-combining cache + MFMA operand staging
// ---------------------------------------------------------------------------

constexpr int CACHE_SLOTS = 64;
constexpr int STAGE_LD = 33;                              // padded row: conflict-free reads
constexpr int STAGE_FLOATS = 64 * STAGE_LD;               // one operand: 64 rows (h*32 + i)
constexpr int WAVE_LDS_FLOATS = CACHE_SLOTS * (REC + 1) + 2 * STAGE_FLOATS + WAVE * 8;

struct WaveCache {
    int* key;       // [CACHE_SLOTS], -1 = free
    float* data;    // [CACHE_SLOTS][REC]
    float* sa;      // staged W operand
    float* sb;      // staged G operand
    float* sw;      // [WAVE][8] each lane's trilinear weights (16-byte aligned)
};

__device__ __forceinline__ WaveCache wave_cache(float* smem) {
    const int w = threadIdx.x / WAVE;
    float* base = smem + (size_t)w * WAVE_LDS_FLOATS;
    float* data = base + CACHE_SLOTS;
    float* sa = data + CACHE_SLOTS * REC;
    return WaveCache{reinterpret_cast<int*>(base), data, sa, sa + STAGE_FLOATS, sa + 2 * STAGE_FLOATS};
}

// Mark every slot free; the caller synchronises the workgroup afterwards.
__device__ __forceinline__ void cache_init(const WaveCache& wc) {
    for (int s = lane_id(); s < CACHE_SLOTS; s += WAVE) wc.key[s] = -1;
}

// Slot of lattice vertex (x, y, z): its parity bits select 3 of the 6 slot bits,
// so the 8 corners of any cell land in 8 different slots.
__device__ __forceinline__ int vertex_slot(int x, int y, int z) {
    const uint32_t h = ((uint32_t)(x >> 1) * 73856093u) ^ ((uint32_t)(y >> 1) * 19349663u)
                     ^ ((uint32_t)(z >> 1) * 83492791u);
    return (int)(((x & 1) << 5) | ((y & 1) << 4) | ((z & 1) << 3) | ((h >> 13) & 7));
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

// Staging addresses.  Operand element for MFMA step c (lanes 2c and 2c+1) and
// row i (0..31) sits at ((h * 32 + i) * STAGE_LD + c) with h = ray lane & 1.
__device__ __forceinline__ int stage_at(int i, int ray_lane) {
    return (((ray_lane & 1) << 5) + i) * STAGE_LD + (ray_lane >> 1);
}

// ---------------------------------------------------------------------------
// the scatter
// ---------------------------------------------------------------------------

// A pass whose groups cover at most this many lanes is summed lane by lane
// (scalar broadcast of each member's weights) instead of on the matrix cores,
// and written out without the cache: rays of a sparse pixel subset rarely
// share a cell, and one MFMA pass plus its cache update costs as much as
// about this many broadcast members.
constexpr int SMALL_PASS_LANES = 16;

// Gradient of one sample: dL/d sigma_raw (gsig) and dL/ds_c (gs[c]) to be
// spread over the corners of cell `cell` (link base `key`, corner ids idx[],
// trilinear weights w[]).  Must be reached by every lane of the wave.
__device__ __forceinline__ void scatter_merged(bool have, int64_t key, const int cell[3],
                                               const int idx[8], const float w[8], float gsig,
                                               const float gs[3], const float Y[9],
                                               const WaveCache& wc, float* __restrict__ grad) {
    unsigned long long pending = __ballot(have);
    if (!pending) return;
    const int lane = lane_id();
    const int j = lane & 31;            // output column (field) and operand row
    const int h = lane >> 5;
    // G rows, once per step (lanes without a gradient stage zeros)
    {
        float G[REC];
        G[0] = have ? gsig : 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float a = have ? gs[c] : 0.f;
#pragma unroll
            for (int k = 0; k < 9; ++k) G[1 + 9 * c + k] = a * Y[k];
        }
#pragma unroll
        for (int m = 0; m < REC; ++m) wc.sb[stage_at(m, lane)] = G[m];
        float4* sw = reinterpret_cast<float4*>(wc.sw + lane * 8);
        sw[0] = make_float4(w[0], w[1], w[2], w[3]);
        sw[1] = make_float4(w[4], w[5], w[6], w[7]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    while (pending) {
        // discover up to four groups (distinct cells) for this pass
        int grp = -1, ng = 0;
        int leader[4] = {0, 0, 0, 0};
        unsigned long long members[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            if (pending) {
                const int ld = __ffsll((long long)pending) - 1;
                const int klo = __builtin_amdgcn_readlane((int)(uint32_t)key, ld);
                const int khi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)key >> 32), ld);
                const int64_t k0 = (int64_t)(((uint64_t)(uint32_t)khi << 32) | (uint32_t)klo);
                const bool mine = have && key == k0 && grp < 0;
                if (mine) grp = g;
                members[g] = __ballot(mine);
                pending &= ~members[g];
                leader[g] = ld;
                ng = g + 1;
            }
        }
        f32x16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        const int covered = __popcll(members[0] | members[1] | members[2] | members[3]);
        if (covered > SMALL_PASS_LANES) {
            // W rows of this pass
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int b = 0; b < 8; ++b) wc.sa[stage_at(g * 8 + b, lane)] = (grp == g) ? w[b] : 0.f;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // C = W^T G over the 64 lanes, two lanes per instruction
            const float* pa = wc.sa + ((h << 5) + j) * STAGE_LD;
            const float* pb = wc.sb + ((h << 5) + j) * STAGE_LD;
#pragma unroll
            for (int c = 0; c < 32; ++c) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[c], pb[c], acc, 0, 0, 0);
        } else {
            // the same totals in the same register layout, member by member:
            // lane (h, j) adds w_{4h+r}(s) * G[s][j] into row 4h + r of group g;
            // then straight to HBM (each atomic instruction covers the two
            // 112-byte records of corners r and 4 + r), bypassing the cache
            // that small groups would mostly evict from
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                if (g >= ng) continue;                      // wave-uniform
                unsigned long long mb = members[g];
                while (mb) {
                    const int src = __ffsll((long long)mb) - 1;
                    mb &= mb - 1;
                    const float gv = wc.sb[stage_at(j, src)];
                    const float4 wv = *reinterpret_cast<const float4*>(wc.sw + src * 8 + 4 * h);
                    acc[4 * g + 0] = fmaf(wv.x, gv, acc[4 * g + 0]);
                    acc[4 * g + 1] = fmaf(wv.y, gv, acc[4 * g + 1]);
                    acc[4 * g + 2] = fmaf(wv.z, gv, acc[4 * g + 2]);
                    acc[4 * g + 3] = fmaf(wv.w, gv, acc[4 * g + 3]);
                }
                const int ld = leader[g];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int id0 = __builtin_amdgcn_readlane(idx[r], ld);
                    const int id1 = __builtin_amdgcn_readlane(idx[4 + r], ld);
                    const int vid = h ? id1 : id0;
                    if (vid >= 0 && j < REC) unsafeAtomicAdd(grad + (int64_t)vid * REC + j, acc[4 * g + r]);
                }
            }
            continue;
        }
        // accumulator r holds row 8*(r/4) + 4*h + r%4 = group r/4, corner 4*h + r%4, column j
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int g = r >> 2;
            if (g >= ng) continue;                          // wave-uniform
            const int ld = leader[g];
            const int b0 = r & 3, b1 = 4 + (r & 3);
            const int id0 = __builtin_amdgcn_readlane(idx[b0], ld);
            const int id1 = __builtin_amdgcn_readlane(idx[b1], ld);
            const int cx = __builtin_amdgcn_readlane(cell[0], ld);
            const int cy = __builtin_amdgcn_readlane(cell[1], ld);
            const int cz = __builtin_amdgcn_readlane(cell[2], ld);
            const int b = h ? b1 : b0;
            const int vid = h ? id1 : id0;
            const int slot = vertex_slot(cx + ((b >> 2) & 1), cy + ((b >> 1) & 1), cz + (b & 1));
            const int cur = wc.key[slot];
            if (vid >= 0) {
                if (j < REC) {
                    float* p = wc.data + slot * REC + j;
                    const float old = *p;
                    if (cur == vid) {
                        *p = old + acc[r];
                    } else {
                        if (cur >= 0) unsafeAtomicAdd(grad + (int64_t)cur * REC + j, old);
                        *p = acc[r];
                    }
                }
                wc.key[slot] = vid;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

}  // namespace pxm
