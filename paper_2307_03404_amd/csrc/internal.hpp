// Host-side launchers shared by the C ABI translation unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kcommon.hpp"

namespace pxm {

// Fused-kernel workspace: tile counter and finished-workgroup counter of the
// persistent variants (the kernel leaves both at zero when it completes),
// then the per-ray state the two-launch variant hands from its forward
// launch to its backward launch (arrays of n_pad entries, n_pad = n_rays
// rounded up to 64): work-mask words [MARK_WORDS][n_pad] u32, FP64 colour
// and range sums [4][n_pad], upstream gradients [4][n_pad] f32, samples to
// replay [n_pad] i32 and mask extent [n_pad] i32.
constexpr size_t FUSED_WS_BYTES = 256;
constexpr size_t SPLIT_BYTES_PER_RAY = 32 * 4 + 4 * 8 + 4 * 4 + 4 + 4;

struct KSplit {
    uint32_t* marks;
    double* sums;
    float* up;
    int32_t* nb;
    int32_t* minfo;
    int64_t n_pad;
    unsigned long long* gfix;   // deterministic scatter: fixed-point grid gradient, or nullptr
};

// Bytes of the fixed-point gradient buffer of the deterministic scatter
// (FIX_SHIFT in kcommon.hpp), rounded up to 256.
inline size_t fix_bytes(int64_t n_alloc, int record_floats) {
    const size_t b = (size_t)n_alloc * (size_t)record_floats * sizeof(unsigned long long);
    return (b + 255) & ~size_t(255);
}

inline int64_t split_pad(int64_t n_rays) { return (n_rays + 63) / 64 * 64; }
inline size_t fused_workspace_bytes(int64_t n_rays) {
    return FUSED_WS_BYTES + (size_t)split_pad(n_rays) * SPLIT_BYTES_PER_RAY;
}
inline KSplit split_state(void* ws, int64_t n_rays) {
    KSplit k;
    k.gfix = nullptr;
    k.n_pad = split_pad(n_rays);
    char* p = static_cast<char*>(ws) + FUSED_WS_BYTES;
    k.sums = reinterpret_cast<double*>(p);
    p += (size_t)k.n_pad * 4 * sizeof(double);
    k.marks = reinterpret_cast<uint32_t*>(p);
    p += (size_t)k.n_pad * 32 * sizeof(uint32_t);
    k.up = reinterpret_cast<float*>(p);
    p += (size_t)k.n_pad * 4 * sizeof(float);
    k.nb = reinterpret_cast<int32_t*>(p);
    p += (size_t)k.n_pad * sizeof(int32_t);
    k.minfo = reinterpret_cast<int32_t*>(p);
    return k;
}

hipError_t launch_forward(const KGrid& g, const KRays& rs, const KOpts& op, float* rgb,
                          float* depth, int32_t* nsamp, hipStream_t st);

hipError_t launch_backward(const KGrid& g, const KRays& rs, const KOpts& op, const float* rgb,
                           const float* depth, const int32_t* nsamp, const float* g_rgb,
                           const float* g_depth, float* grad_data, double* grad_pose,
                           hipStream_t st);

// gfix: the zeroed fixed-point buffer of the deterministic scatter ([n_alloc][S] int64,
// left zeroed), or nullptr for float atomics.
hipError_t launch_fused(const KGrid& g, const KRays& rs, const KOpts& op, const float* tgt_rgb,
                        const float* tgt_depth, const float* frame_weight, int want, float* rgb,
                        float* depth, double* loss, float* grad_data, double* grad_pose,
                        int64_t* stats, unsigned* ws, int block, int variant,
                        unsigned long long* gfix, hipStream_t st);

// set: grad_data = dTV for the visited records' used fields, else += dTV
hipError_t launch_tv(const KGrid& g, float lambda_density, float lambda_sh, float eps,
                     float* grad_data, bool set, hipStream_t st);

// Occupancy bitfield: level-0 32-bit words (two per 4^3-cell block), 4^3
// blocks per axis, 8^3 bricks per axis, level-1 words for a lattice of R
// vertices per axis.
void occ_layout(const int R[3], int64_t& w0_words, int Q[3], int B[3], int64_t& w1_words);
hipError_t launch_occupancy(const KGrid& g, uint32_t* occ, hipStream_t st);

hipError_t launch_adam(int F, float* c2w, double* grad_pose, double* state, float lr, float b1,
                       float b2, float eps, hipStream_t st);

// Gauss-Newton slots per frame: H upper triangle (21), g (6), E (1).
constexpr int GN_VALUES = 28;

hipError_t launch_gn(const KGrid& g, const KRays& rs, const KOpts& op, const float* tgt_rgb,
                     const float* tgt_depth, const float* frame_weight, double* gn, hipStream_t st);
hipError_t launch_pose_gn(int F, float* c2w, double* gn, float mu, hipStream_t st);

hipError_t launch_rmsprop(int64_t n, int deg, float* data, float* grad, float* avg, float lr_d,
                          float lr_sh, float alpha, float eps, hipStream_t st);

// Dynamic-grid edits: flags are compacted in chunks of EDIT_CHUNK items
// (one workgroup).  Workspace bytes of a prune of n_alloc records and of the
// growth of an R[0] x R[1] x R[2] lattice.
constexpr int EDIT_CHUNK = 8192;
size_t prune_workspace_bytes(int64_t n_alloc);
size_t grow_workspace_bytes(const int R[3]);
hipError_t launch_upsample_link(const KGrid& g, int32_t* link_fine, int64_t* n_fine, void* ws, hipStream_t st);
hipError_t launch_upsample_data(const KGrid& g, const int32_t* link_fine, int64_t n_fine, float* data_fine,
                                hipStream_t st);
hipError_t launch_prune(const KGrid& g, float tau, int32_t* link_out, float* data_out, int64_t* n_out, void* ws,
                        hipStream_t st);

}  // namespace pxm
