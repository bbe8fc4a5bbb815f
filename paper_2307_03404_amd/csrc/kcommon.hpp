// Device-side building blocks of the sparse-voxel volume renderer (gfx950).
//
// Layout in HBM
//   link  int32 [Rx*Ry*Rz]    vertex (x,y,z) -> record id, -1 = empty
//   data  f32   [n][S]        density, then SH[c][k] for c = 0..2, k < (d+1)^2
//   grad  f32   [n][S]        same layout as data
// At the paper's SH degree d = 2 a record is 28 floats (112 bytes, 7 float4
// loads); degree 1 keeps 13 of a 16-float record, degree 0 is 4 floats.
// Records are 16-byte aligned.
//
// Precision plan
//   * ray direction and sample positions in FP64: a voxel coordinate near 512
//     has an FP32 ulp of 6e-5, above the forward tolerance, so the lattice
//     cell and the in-cell fraction are taken from an FP64 position; the
//     fraction itself is then FP32;
//   * the optical depth sum_j sigma_j delta is accumulated in FP64 and the
//     transmittance is exp of it, so T does not drift multiplicatively;
//   * alpha = 1 - exp(-sigma delta) via expm1 (no cancellation for small x);
//   * everything else (interpolation, SH, compositing, gradients) in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace pxm {

constexpr int REC = 28;          // floats per record at SH degree 2 (the largest)
constexpr int WAVE = 64;

// Record layout of SH degree DEG: the first (DEG+1)^2 functions of the
// degree-2 basis per channel (the real SH of degree <= DEG are a prefix of
// it), padded to whole float4s.
template <int DEG>
struct RecL {
    static constexpr int NSH = (DEG + 1) * (DEG + 1);   // coefficients per channel
    static constexpr int USED = 1 + 3 * NSH;            // density + SH fields
    static constexpr int S = DEG == 0 ? 4 : DEG == 1 ? 16 : 28;   // floats per record
    static constexpr int Q = S / 4;                     // float4 per record
};

enum { ACT_RELU_SHIFT = 0, ACT_SIGMOID = 1, ACT_IDENTITY = 2 };
enum { LOSS_L1 = 0, LOSS_L2 = 1 };

// Deterministic grid scatter: every merged contribution is rounded to a
// fixed-point integer in units of 2^-FIX_SHIFT and added with 64-bit integer
// atomics, which commute exactly, so the sum does not depend on the order in
// which waves arrive; a last pass adds each integer sum, converted once, into
// the float gradient.  Range +-2^(63 - FIX_SHIFT) = +-32768 per entry,
// resolution 2^-48 = 3.6e-15.
constexpr int FIX_SHIFT = 48;
constexpr double FIX_SCALE = (double)(1ull << FIX_SHIFT);

// Floats per record of SH degree deg (RecL<deg>::S at run time).
__host__ __device__ __forceinline__ int record_floats(int deg) {
    return deg == 0 ? 4 : deg == 1 ? 16 : 28;
}

struct KGrid {
    int R[3];
    int deg;                    // SH degree of the records (0, 1 or 2)
    int64_t sx, sy;             // link strides of +x and +y (the +z stride is 1)
    double lo[3];               // aabb_min
    double inv_vs;              // 1 / voxel_size
    float vs;
    int64_t n_alloc;
    const int32_t* __restrict__ link;
    const float* __restrict__ data;
    // optional occupancy bitfield (see occ.hip); occ0 == nullptr disables skipping
    const uint64_t* __restrict__ occ0;   // one 64-bit word per 4^3-cell block, a bit per cell
    const uint32_t* __restrict__ occ1;   // one bit per 8^3-cell brick
    int Q[3];                            // 4^3 blocks per axis
    int B[3];                            // bricks per axis
};

struct KRays {
    int F;
    int64_t n;
    const float* __restrict__ c2w;
    const float* __restrict__ intr;
    const int32_t* __restrict__ off;
    const int32_t* __restrict__ pix;
};

struct KOpts {
    float step_vox;             // delta, in voxels
    int max_samples;
    float t_near;
    float t_stop;
    int act;
    int depth_loss;
    float lambda_d;
    int flags;
};

// ---------------------------------------------------------------------------
// small math
// ---------------------------------------------------------------------------

__device__ __forceinline__ float act_fwd(int act, float s) {
    if (act == ACT_SIGMOID) return 1.0f / (1.0f + expf(-s));
    if (act == ACT_IDENTITY) return s;
    return fmaxf(s + 0.5f, 0.0f);
}

__device__ __forceinline__ float act_bwd(int act, float s) {
    if (act == ACT_SIGMOID) {
        float g = 1.0f / (1.0f + expf(-s));
        return g * (1.0f - g);
    }
    if (act == ACT_IDENTITY) return 1.0f;
    return (s + 0.5f > 0.0f) ? 1.0f : 0.0f;
}

// exp(-L) for an FP64 optical depth L, accurate to ~1 ulp of FP32: split L
// into its FP32 rounding and the remainder, exp(-hi) * (1 - lo).
__device__ __forceinline__ float trans_of(double L) {
    float hi = (float)L;
    float lo = (float)(L - (double)hi);
    return expf(-hi) * (1.0f - lo);
}

// Real SH basis of degree 2 at a unit direction.
__device__ __forceinline__ void sh9(float x, float y, float z, float Y[9]) {
    const float c0 = 0.28209479177387814f;
    const float c1 = 0.4886025119029199f;
    const float c2 = 1.0925484305920792f;
    const float c3 = 0.31539156525252005f;
    const float c4 = 0.5462742152960396f;
    Y[0] = c0;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    Y[4] = c2 * x * y;
    Y[5] = -c2 * y * z;
    Y[6] = c3 * (2.0f * z * z - x * x - y * y);
    Y[7] = -c2 * x * z;
    Y[8] = c4 * (x * x - y * y);
}

// d Y_k / d(x,y,z) for the exact view-direction pose term.
__device__ __forceinline__ void sh9_grad(float x, float y, float z, float G[9][3]) {
    const float c1 = 0.4886025119029199f;
    const float c2 = 1.0925484305920792f;
    const float c3 = 0.31539156525252005f;
    const float c4 = 0.5462742152960396f;
#pragma unroll
    for (int k = 0; k < 9; ++k) G[k][0] = G[k][1] = G[k][2] = 0.0f;
    G[1][1] = -c1;
    G[2][2] = c1;
    G[3][0] = -c1;
    G[4][0] = c2 * y;  G[4][1] = c2 * x;
    G[5][1] = -c2 * z; G[5][2] = -c2 * y;
    G[6][0] = -2.0f * c3 * x; G[6][1] = -2.0f * c3 * y; G[6][2] = 4.0f * c3 * z;
    G[7][0] = -c2 * z; G[7][2] = -c2 * x;
    G[8][0] = 2.0f * c4 * x; G[8][1] = -2.0f * c4 * y;
}

// ---------------------------------------------------------------------------
// wave-level reductions (64 lanes)
// ---------------------------------------------------------------------------

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}

// Sum over the 64 lanes (every lane active), returned to all of them:
// data-parallel-primitive moves within rows of 16 lanes (shift right by 1,
// 2, 4, 8), then the last lane of each row broadcast into the next rows,
// leave the total in lane 63 (a lane with no source lane reads 0).
__device__ __forceinline__ double wave_sum(double v) {
    auto step = [&](auto ctrl, auto row_mask) {
        const uint64_t u = (uint64_t)__double_as_longlong(v);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, decltype(ctrl)::value,
                                                   decltype(row_mask)::value, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), decltype(ctrl)::value,
                                                   decltype(row_mask)::value, 0xf, false);
        v += __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
    };
    step(std::integral_constant<int, 0x111>{}, std::integral_constant<int, 0xf>{});   // row_shr:1
    step(std::integral_constant<int, 0x112>{}, std::integral_constant<int, 0xf>{});   // row_shr:2
    step(std::integral_constant<int, 0x114>{}, std::integral_constant<int, 0xf>{});   // row_shr:4
    step(std::integral_constant<int, 0x118>{}, std::integral_constant<int, 0xf>{});   // row_shr:8
    step(std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xa>{});   // row_bcast:15
    step(std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xc>{});   // row_bcast:31
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Segmented sum over the lanes of a wave keyed by `key` (rays of one frame
// are contiguous, so a wave spans few keys): one leader lane per distinct key
// adds the key's N partial sums into out[key*N + n] with FP64 atomics.  Must be
// reached by every lane of the wave.
template <int N>
__device__ __forceinline__ void seg_sum_atomic(int key, bool active, const double* vals,
                                               double* out) {
    unsigned long long pending = __ballot(active);
    while (pending) {
        int leader = __ffsll((long long)pending) - 1;
        const int k0 = __builtin_amdgcn_readlane(key, leader);
        bool mine = active && (key == k0);
        unsigned long long mask = __ballot(mine);
#pragma unroll
        for (int n = 0; n < N; ++n) {
            double s = wave_sum(mine ? vals[n] : 0.0);
            if (lane_id() == leader) atomicAdd(out + (int64_t)k0 * N + n, s);
        }
        pending &= ~mask;
    }
}

__device__ __forceinline__ void add_stats(bool active, const long long* v, int64_t* out) {
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        long long s = wave_sum(active ? v[n] : 0LL);
        if (lane_id() == 0 && s != 0)
            atomicAdd(reinterpret_cast<unsigned long long*>(out + n), (unsigned long long)s);
    }
}

// ---------------------------------------------------------------------------
// rays
// ---------------------------------------------------------------------------

// Frame of ray r by binary search of the CSR offsets; always in [0, F-1].
__device__ __forceinline__ int frame_of(const int32_t* __restrict__ off, int F, int64_t r) {
    int lo = 0, hi = F;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if ((int64_t)off[mid] <= r) lo = mid; else hi = mid;
    }
    return lo;
}

struct Ray {
    double b[3];        // voxel-space position of sample k = 0
    double st[3];       // voxel-space step between samples
    float d[3];         // unit world direction
    float o[3];         // camera centre (world)
    float s;            // |d_cam|: z-depth = range / s
    float dw;           // world spacing of samples
    float t0;           // t_near
    int64_t k_first;    // first kept sample index (valid if n_inbox > 0)
    bool empty;         // no sample position inside the box
};

__device__ __forceinline__ bool in_box(const KGrid& g, double q0, double q1, double q2) {
    return q0 >= 0.0 && q0 <= (double)(g.R[0] - 1) && q1 >= 0.0 && q1 <= (double)(g.R[1] - 1)
        && q2 >= 0.0 && q2 <= (double)(g.R[2] - 1);
}

__device__ __forceinline__ void setup_ray(const KGrid& g, const KRays& rs, const KOpts& op,
                                          int64_t r, int f, Ray& ray) {
    const float* __restrict__ M = rs.c2w + 12 * (int64_t)f;
    const float* __restrict__ K = rs.intr + 4 * (int64_t)f;
    const int u = rs.pix[2 * r], v = rs.pix[2 * r + 1];
    const double dcx = ((double)u + 0.5 - (double)K[2]) / (double)K[0];
    const double dcy = ((double)v + 0.5 - (double)K[3]) / (double)K[1];
    const double s = sqrt(dcx * dcx + dcy * dcy + 1.0);
    const double inv = 1.0 / s;
    double d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d[a] = ((double)M[4 * a] * dcx + (double)M[4 * a + 1] * dcy + (double)M[4 * a + 2]) * inv;
        ray.d[a] = (float)d[a];
        ray.o[a] = M[4 * a + 3];
    }
    ray.s = (float)s;
    ray.t0 = op.t_near;
    ray.dw = op.step_vox * g.vs;
    const double tn = (double)op.t_near * g.inv_vs;
    const double sv = (double)op.step_vox;
    double klo = 0.0, khi = 1.0e300;
    bool empty = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ray.b[a] = ((double)M[4 * a + 3] - g.lo[a]) * g.inv_vs + tn * d[a];
        ray.st[a] = sv * d[a];
        const double top = (double)(g.R[a] - 1);
        if (ray.st[a] > 0.0) {
            klo = fmax(klo, (0.0 - ray.b[a]) / ray.st[a]);
            khi = fmin(khi, (top - ray.b[a]) / ray.st[a]);
        } else if (ray.st[a] < 0.0) {
            klo = fmax(klo, (top - ray.b[a]) / ray.st[a]);
            khi = fmin(khi, (0.0 - ray.b[a]) / ray.st[a]);
        } else if (!(ray.b[a] >= 0.0 && ray.b[a] <= top)) {
            empty = true;
        }
    }
    if (!(khi >= klo) || khi < 0.0 || klo > 4.0e18) empty = true;
    int64_t k = 0;
    if (!empty) {
        // one step early, then advance with the exact predicate the march uses
        k = (int64_t)ceil(klo) - 1;
        if (k < 0) k = 0;
        int guard = 0;
        while (guard < 4 && !in_box(g, fma((double)k, ray.st[0], ray.b[0]),
                                    fma((double)k, ray.st[1], ray.b[1]),
                                    fma((double)k, ray.st[2], ray.b[2]))) {
            ++k;
            ++guard;
        }
        if (guard == 4) empty = true;
    }
    ray.k_first = k;
    ray.empty = empty;
}

// ---------------------------------------------------------------------------
// one sample: cell, fractions, corner gather
// ---------------------------------------------------------------------------

struct Sample {
    int64_t base;       // link index of the cell's (0,0,0) corner
    int c[3];           // cell coordinates
    float f[3];         // in-cell fractions
    float t;            // distance from the camera centre (world)
};

// Returns false when sample k has left the box.
__device__ __forceinline__ bool sample_at(const KGrid& g, const Ray& ray, int64_t k, Sample& s) {
    const double q0 = fma((double)k, ray.st[0], ray.b[0]);
    const double q1 = fma((double)k, ray.st[1], ray.b[1]);
    const double q2 = fma((double)k, ray.st[2], ray.b[2]);
    if (!in_box(g, q0, q1, q2)) return false;
    int c0 = min(max((int)floor(q0), 0), g.R[0] - 2);
    int c1 = min(max((int)floor(q1), 0), g.R[1] - 2);
    int c2 = min(max((int)floor(q2), 0), g.R[2] - 2);
    s.f[0] = (float)(q0 - (double)c0);
    s.f[1] = (float)(q1 - (double)c1);
    s.f[2] = (float)(q2 - (double)c2);
    s.base = (int64_t)c0 * g.sx + (int64_t)c1 * g.sy + c2;
    s.c[0] = c0; s.c[1] = c1; s.c[2] = c2;
    s.t = ray.t0 + (float)k * ray.dw;
    return true;
}

// Workgroup b of G -> work item, grouping consecutive items on one XCD: the
// hardware deals workgroups round-robin over the 8 XCDs, each with its own
// L2, and neighbouring items (ray tiles, grid bricks) read the same vertices.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G) {
    const int64_t q = G / 8, rem = G % 8;
    const int64_t x = b % 8, j = b / 8;
    const int64_t start = x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;
    return start + j;
}

// ---------------------------------------------------------------------------
// empty-space skipping with the occupancy bitfield
// ---------------------------------------------------------------------------

// A cell is occupied iff one of its 8 corners is allocated.  Level 1 holds a
// bit per 8^3-cell brick; level 0 a 64-bit word per 4^3-cell block, bit
// (x & 3) * 16 + (y & 3) * 4 + (z & 3) for cell (x, y, z).
__device__ __forceinline__ bool brick_empty(const KGrid& g, const int c[3]) {
    const int64_t b = ((int64_t)(c[0] >> 3) * g.B[1] + (c[1] >> 3)) * g.B[2] + (c[2] >> 3);
    return !((g.occ1[b >> 5] >> (b & 31)) & 1u);
}

// For sample k lying in an empty block of E^3 cells (E = 8: a brick, E = 4:
// a level-0 block): the first sample index after k that is not guaranteed
// to lie inside the block.  Every index in (k, result) has its position
// inside [E b, min(E b + E, R - 1)) shrunk by 1e-6 voxel on each axis, hence
// in one of the block's (empty) cells and inside the box.
template <int E>
__device__ __forceinline__ int64_t block_exit(const KGrid& g, const Ray& ray, int64_t k,
                                              const int c[3]) {
    double kx = 1.0e300;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double lo = (double)(E * (c[a] / E));
        const double hi = fmin(lo + (double)E, (double)(g.R[a] - 1));
        if (ray.st[a] > 0.0) kx = fmin(kx, (hi - 1e-6 - ray.b[a]) / ray.st[a]);
        else if (ray.st[a] < 0.0) kx = fmin(kx, (lo + 1e-6 - ray.b[a]) / ray.st[a]);
    }
    if (!(kx < 4.0e18)) return k + 1;
    const int64_t nxt = (int64_t)floor(kx) + 1;
    return nxt > k + 1 ? nxt : k + 1;
}

// The brick and level-0 block a march is in, and their occupancy: a sample
// loads a word only when it enters another brick or block (a ray crosses
// ~13 blocks of 4^3 cells in the ~70 samples it takes through non-empty
// bricks of the room frame).
struct OccCache {
    int brick;          // linear brick id, -1 = none yet
    int blk;            // linear level-0 block id, -1 = none yet
    bool brick_empty;
    uint64_t word;
};

__device__ __forceinline__ void occ_cache_init(OccCache& oc) {
    oc.brick = -1;
    oc.blk = -1;
    oc.brick_empty = false;
    oc.word = 0ull;
}

enum { OCC_CELL = 0, OCC_EMPTY_CELL = 1, OCC_JUMP = 2 };

// What the march does at sample k (inside the box, cell s.c): work at an
// occupied cell, step over one empty cell, or jump to *nxt over an empty
// brick or level-0 block.  Needs g.occ0 != nullptr.
__device__ __forceinline__ int occ_classify(const KGrid& g, const Ray& ray, int64_t k,
                                            const int c[3], OccCache& oc, int64_t& nxt) {
    const int bid = ((c[0] >> 3) * g.B[1] + (c[1] >> 3)) * g.B[2] + (c[2] >> 3);
    if (bid != oc.brick) {
        oc.brick = bid;
        oc.brick_empty = !((g.occ1[bid >> 5] >> (bid & 31)) & 1u);
    }
    if (oc.brick_empty) {
        nxt = block_exit<8>(g, ray, k, c);
        return OCC_JUMP;
    }
    const int qid = ((c[0] >> 2) * g.Q[1] + (c[1] >> 2)) * g.Q[2] + (c[2] >> 2);
    if (qid != oc.blk) {
        oc.blk = qid;
        oc.word = g.occ0[qid];
    }
    if (oc.word == 0ull) {
        nxt = block_exit<4>(g, ray, k, c);
        return OCC_JUMP;
    }
    const int bit = ((c[0] & 3) << 4) | ((c[1] & 3) << 2) | (c[2] & 3);
    return ((oc.word >> bit) & 1ull) ? OCC_CELL : OCC_EMPTY_CELL;
}

// Corner b = 4*i + 2*j + k  (x, y, z offsets in {0,1}).
__device__ __forceinline__ int64_t corner_off(const KGrid& g, int b) {
    return ((b >> 2) & 1) * g.sx + ((b >> 1) & 1) * g.sy + (b & 1);
}

__device__ __forceinline__ void trilinear_weights(const float f[3], float w[8]) {
    const float x1 = f[0], x0 = 1.0f - f[0];
    const float y1 = f[1], y0 = 1.0f - f[1];
    const float z1 = f[2], z0 = 1.0f - f[2];
    const float a00 = x0 * y0, a01 = x0 * y1, a10 = x1 * y0, a11 = x1 * y1;
    w[0] = a00 * z0; w[1] = a00 * z1; w[2] = a01 * z0; w[3] = a01 * z1;
    w[4] = a10 * z0; w[5] = a10 * z1; w[6] = a11 * z0; w[7] = a11 * z1;
}

// Link ids of the 8 corners; returns the number allocated.  An id outside
// [0, n_alloc) reads as empty, so a corrupt link table cannot send a gather
// out of bounds.
__device__ __forceinline__ int load_links(const KGrid& g, int64_t base, int idx[8]) {
    int n = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        int id = g.link[base + corner_off(g, b)];
        id = ((uint32_t)id < (uint64_t)g.n_alloc) ? id : -1;
        idx[b] = id;
        n += id >= 0;
    }
    return n;
}

template <int DEG>
__device__ __forceinline__ void load_record(const float* __restrict__ data, int id, float rec[REC]) {
    const float4* p = reinterpret_cast<const float4*>(data + (int64_t)id * RecL<DEG>::S);
#pragma unroll
    for (int q = 0; q < RecL<DEG>::Q; ++q) {
        float4 v = p[q];
        rec[4 * q] = v.x; rec[4 * q + 1] = v.y; rec[4 * q + 2] = v.z; rec[4 * q + 3] = v.w;
    }
}

// The fields of one sample, interpolated (and, for the pose, differentiated
// in space: Eq. 16 / Appendix A) corner by corner as the records arrive, so
// no per-corner values stay live.  Colour entries are the SH expansions
// s_c = sum_k Y_k SH_{c,k} of the ray's basis.
struct Interp {
    float sig;          // raw density
    float s[3];         // colour pre-activations
    float dsig[3];      // d sig / dq_a (voxel units)           GRAD only
    float ds[3][3];     // d s_c / dq_a                          GRAD only
    float ev[3][3];     // sum_b w_b sum_k dY_k/dd_a SH_{b,c,k}  VIEW only
};

template <bool GRAD, bool VIEW, int DEG>
__device__ __forceinline__ void gather_interp(const KGrid& g, const int idx[8], const float Y[9],
                                              const float GY[9][3], const float f[3], Interp& v) {
    constexpr int NSH = RecL<DEG>::NSH;
    v.sig = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v.s[c] = 0.f;
        v.dsig[c] = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) v.ds[c][a] = v.ev[c][a] = 0.f;
    }
    const float x1 = f[0], x0 = 1.0f - f[0];
    const float y1 = f[1], y0 = 1.0f - f[1];
    const float z1 = f[2], z0 = 1.0f - f[2];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        if (idx[b] < 0) continue;
        const int bx = (b >> 2) & 1, by = (b >> 1) & 1, bz = b & 1;
        const float wx = bx ? x1 : x0, wy = by ? y1 : y0, wz = bz ? z1 : z0;
        const float w = (wx * wy) * wz;
        float rec[REC];
        load_record<DEG>(g.data, idx[b], rec);
        float e[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < NSH; ++k) acc = fmaf(Y[k], rec[1 + NSH * c + k], acc);
            e[c] = acc;
        }
        v.sig = fmaf(w, rec[0], v.sig);
#pragma unroll
        for (int c = 0; c < 3; ++c) v.s[c] = fmaf(w, e[c], v.s[c]);
        if (GRAD) {
            // d w_b / dq = (+-wy wz, wx +-wz... ) with the sign of each offset
            const float dw[3] = {(bx ? 1.f : -1.f) * wy * wz, wx * (by ? 1.f : -1.f) * wz,
                                 wx * wy * (bz ? 1.f : -1.f)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                v.dsig[a] = fmaf(dw[a], rec[0], v.dsig[a]);
#pragma unroll
                for (int c = 0; c < 3; ++c) v.ds[c][a] = fmaf(dw[a], e[c], v.ds[c][a]);
            }
        }
        if (VIEW) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    float acc = 0.f;
#pragma unroll
                    for (int k = 0; k < NSH; ++k) acc = fmaf(GY[k][a], rec[1 + NSH * c + k], acc);
                    v.ev[c][a] = fmaf(w, acc, v.ev[c][a]);
                }
        }
    }
}

}  // namespace pxm
