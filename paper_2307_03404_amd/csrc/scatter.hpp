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
// instructions (K = 2 lanes each).  G is staged in LDS in the operand order
// the instruction reads; W is formed on the fly from the lanes' staged
// trilinear weights and the groups' member masks.  The 32 x 28 totals go to HBM with atomics,
// each instruction covering the two contiguous 112-byte records of corners r
// and 4 + r of a group.  (A per-wave LDS write-combining cache in front of
// the atomics saved HBM writes but its 7 KB per wave lowered occupancy from
// 8 to 6 waves per CU, which cost more than it saved.)
#pragma once

#include "kcommon.hpp"

namespace pxm {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// per-wave LDS: the G operand, the lanes' trilinear weights and work masks
// ---------------------------------------------------------------------------

constexpr int STAGE_LD = 33;                              // padded row: conflict-free reads
constexpr int STAGE_FLOATS = 64 * STAGE_LD;               // G: 64 rows (h*32 + i)
constexpr int MARK_WORDS = 32;                            // work-position mask: 1024 bits per lane
constexpr int WAVE_LDS_FLOATS = STAGE_FLOATS + WAVE * 8 + MARK_WORDS * WAVE;

struct WaveStage {
    float* sb;          // staged G operand
    float* sw;          // [WAVE][8] each lane's trilinear weights (16-byte aligned)
    uint32_t* marks;    // [MARK_WORDS][WAVE] each lane's work-position mask (fused kernel)
    unsigned long long* gfix;   // deterministic mode: fixed-point gradient, else nullptr
};

// Must be reached by every lane of the wave, before its first scatter.  The
// MFMA B operand reads rows 0..31 of each half of the staging block, but a
// gradient row has only REC = 28 fields: rows 28..31 are never staged, so
// they are zeroed here once (their products land in output columns that
// are discarded, and the matrix cores then never see undefined LDS).
__device__ __forceinline__ WaveStage wave_stage(float* smem) {
    const int w = threadIdx.x / WAVE;
    float* sb = smem + (size_t)w * WAVE_LDS_FLOATS;
    float* sw = sb + STAGE_FLOATS;                        // 2112 floats in: 16-byte aligned
    const int lane = (int)(threadIdx.x % WAVE);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = lane * 4 + q;                       // 2 halves x 4 rows x 32 columns
        const int h = i >> 7, row = REC + ((i >> 5) & 3), c = i & 31;
        sb[((h << 5) + row) * STAGE_LD + c] = 0.f;
    }
    return WaveStage{sb, sw, reinterpret_cast<uint32_t*>(sw + WAVE * 8), nullptr};
}

// Staging addresses.  Operand element for MFMA step c (lanes 2c and 2c+1) and
// row i (0..31) sits at ((h * 32 + i) * STAGE_LD + c) with h = ray lane & 1.
__device__ __forceinline__ int stage_at(int i, int ray_lane) {
    return (((ray_lane & 1) << 5) + i) * STAGE_LD + (ray_lane >> 1);
}

// ---------------------------------------------------------------------------
// the scatter
// ---------------------------------------------------------------------------

static_assert(REC + 4 == 32, "the staging rows beyond the record are the last four of 32");

// A pass whose groups cover at most this many lanes is summed lane by lane
// (broadcast of each member's weights and gradient row from LDS) instead of
// on the matrix cores: rays of a sparse pixel subset rarely share a cell, and
// one MFMA pass costs about as much as this many broadcast members.
constexpr int SMALL_PASS_LANES = 16;

// Gradient of one sample: dL/d sigma_raw (gsig) and dL/ds_c (gs[c]) to be
// spread over the corners of the cell with link base `key` (corner ids
// idx[], trilinear weights w[]) in records of SH degree DEG (fields beyond
// the record's used ones are staged as zeros and never written).  Must be
// reached by every lane of the wave.
template <int DEG, bool FIX = false>
__device__ __forceinline__ void scatter_merged(bool have, int64_t key, const int idx[8],
                                               const float w[8], float gsig, const float gs[3],
                                               const float Y[9], const WaveStage& wc,
                                               float* __restrict__ grad) {
    constexpr int NSH = RecL<DEG>::NSH, USED = RecL<DEG>::USED, S = RecL<DEG>::S;
    unsigned long long pending = __ballot(have);
    if (!pending) return;
    const int lane = lane_id();
    const int j = lane & 31;            // output column (field) and operand row
    const int h = lane >> 5;
    // G rows, once per step (lanes without a gradient stage zeros)
    {
        float G[REC];
#pragma unroll
        for (int m = USED; m < REC; ++m) G[m] = 0.f;
        G[0] = have ? gsig : 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float a = have ? gs[c] : 0.f;
#pragma unroll
            for (int k = 0; k < NSH; ++k) G[1 + NSH * c + k] = a * Y[k];
        }
#pragma unroll
        for (int m = 0; m < REC; ++m) wc.sb[stage_at(m, lane)] = G[m];
        float4* sw = reinterpret_cast<float4*>(wc.sw + lane * 8);
        sw[0] = have ? make_float4(w[0], w[1], w[2], w[3]) : make_float4(0.f, 0.f, 0.f, 0.f);
        sw[1] = have ? make_float4(w[4], w[5], w[6], w[7]) : make_float4(0.f, 0.f, 0.f, 0.f);
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
            // C = W^T G over the 64 lanes, two lanes per instruction: step c
            // takes rays 2c (h = 0) and 2c + 1 (h = 1); lane (h, j) supplies
            // W[ray][row j] = w_{j%8}(ray) if the ray is in group j/8 (a bit of
            // that group's member mask), and G[ray][j]
            const float* pb = wc.sb + ((h << 5) + j) * STAGE_LD;
            const int jg = j >> 3, jb = j & 7;
            const unsigned long long mine_mask =
                jg == 0 ? members[0] : jg == 1 ? members[1] : jg == 2 ? members[2] : members[3];
            const unsigned long long rows = mine_mask >> h;
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                const float a = ((rows >> (2 * c)) & 1ull) ? wc.sw[(2 * c + h) * 8 + jb] : 0.f;
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, pb[c], acc, 0, 0, 0);
            }
        } else {
            // the same totals in the same register layout, member by member:
            // lane (h, j) adds w_{4h+r}(s) * G[s][j] into row 4h + r of group g
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
            }
        }
        // accumulator r holds row 8*(r/4) + 4*h + r%4 = group r/4, corner 4*h + r%4,
        // field j: one atomic instruction per r covers corners r%4 and 4 + r%4
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int g = r >> 2;
            if (g >= ng) continue;                          // wave-uniform
            const int ld = leader[g];
            const int id0 = __builtin_amdgcn_readlane(idx[r & 3], ld);
            const int id1 = __builtin_amdgcn_readlane(idx[4 + (r & 3)], ld);
            const int vid = h ? id1 : id0;
            if (vid >= 0 && j < USED) {
                if (FIX)              // the deterministic (fixed-point) mode
                    atomicAdd(wc.gfix + (int64_t)vid * S + j,
                              (unsigned long long)__double2ll_rn((double)acc[r] * FIX_SCALE));
                else
                    unsafeAtomicAdd(grad + (int64_t)vid * S + j, acc[r]);
            }
        }
    }
}

}  // namespace pxm
