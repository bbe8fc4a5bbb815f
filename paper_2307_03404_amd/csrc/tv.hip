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
// Blocks of 8^3 lattice vertices, one workgroup each, split into eight 4^3
// sub-bricks.  The workgroup tests the block against the occupancy bitfield
// once, loads the links of the block and its one-vertex halo (10^3) in one
// pass, and then, for each sub-brick with an allocated vertex, stages the
// sub-brick's 6^3 halo records with all their fields at once (each record
// read as one contiguous run: 112 bytes at SH degree 2, and kept in LDS
// position-major, as it arrived) and computes its
// vertices' fields (28 at degree 2, 13 at degree 1, 4 at degree 0) with
// consecutive lanes, so each gradient record is written as one run.
// (Staging four fields at a time over 8^3 blocks fetched every record line
// once per chunk, as the lines of ~200 blocks in flight per XCD do not
// survive in L2 between chunks; one workgroup per 4^3 brick made the launch
// dispatch-bound on sparse 512^3 grids.)  Blocks are dealt to XCDs in
// contiguous runs so that halos shared with neighbours are read through the
// same L2.  Each phase issues all of a thread's global loads before it uses
// any (links, staged records, gradient entries), so a phase costs one memory
// round trip: the gradient read-modify-writes, one per item in turn, were the
// longest chain.  The allocated vertices of all eight sub-bricks are listed
// first, so that the records of the next non-empty sub-brick are requested
// before the current one is computed and arrive while it is.
//
// SET writes the gradient (grad = dTV) instead of adding to it, which saves
// the read of the gradient: a step that zeroes its gradient can run the TV
// term first and let the rendering backward add onto it.
#include "internal.hpp"

namespace pxm {

constexpr int TB8 = 8;                  // block edge (vertices)
constexpr int TH8 = TB8 + 2;            // with halo
constexpr int TH83 = TH8 * TH8 * TH8;   // 1000 link positions
constexpr int TB = 4;                   // sub-brick edge
constexpr int TH = TB + 2;
constexpr int TH3 = TH * TH * TH;       // 216 staged positions
constexpr int TV_THREADS = 256;
// a listed vertex: its sub-halo position and the TV terms that touch it
// (its own, and those of its -x, -y, -z neighbours)
constexpr int TERM_POS = 0xff, TERM_OWN = 0x100, TERM_X = 0x200, TERM_Y = 0x400, TERM_Z = 0x800;
static_assert(TH3 <= TERM_POS + 1, "sub-halo positions fit in the low byte");
constexpr int TV_ITEMS = TB * TB * TB * 32 / TV_THREADS;   // vertex-field items per thread, at most

__device__ __forceinline__ int hidx8(int x, int y, int z) { return (x * TH8 + y) * TH8 + z; }
__device__ __forceinline__ int hidx(int x, int y, int z) { return (x * TH + y) * TH + z; }

template <int DEG, bool SET>
__global__ void __launch_bounds__(TV_THREADS) k_tv(KGrid g, float lam_d, float lam_sh, float eps,
                                                   float* __restrict__ grad, int nby, int nbz) {
    constexpr int S = RecL<DEG>::S, Q = RecL<DEG>::Q, USED = RecL<DEG>::USED;
    constexpr int STAGE_ITERS = (TH3 * Q + TV_THREADS - 1) / TV_THREADS;   // staged float4 per thread
    static_assert(TV_THREADS == 4 * WAVE, "one wave lists two sub-bricks");
    __shared__ int s_id8[TH83];             // links of the block halo (-1 empty or outside)
    __shared__ int s_id[TH3];               // links of the current sub-brick halo
    __shared__ float4 s_v4[TH3 * Q];        // the sub-halo records, position-major: field m of
                                            // position p at float p * S + m
    __shared__ int s_list[8][TB * TB * TB]; // per sub-brick: sub-halo positions of its allocated vertices
    __shared__ int s_n[8];
    const int t = threadIdx.x;
    const int64_t block = xcd_tile(blockIdx.x, gridDim.x);
    const int bz = (int)(block % nbz), by = (int)((block / nbz) % nby);
    const int bx = (int)(block / ((int64_t)nbz * nby));
    const int x0 = bx * TB8, y0 = by * TB8, z0 = bz * TB8;
    const int X = g.R[0], Y = g.R[1], Z = g.R[2];
    // An allocated vertex v of this block is a corner of cell min(v, R-2) per
    // axis, which lies in cell brick (bx, by, bz) whenever that brick exists.
    if (g.occ1 && bx < g.B[0] && by < g.B[1] && bz < g.B[2]) {
        const int c[3] = {x0, y0, z0};
        if (brick_empty(g, c)) return;                      // workgroup-uniform
    }
    {
        // all of a thread's link loads are issued before the first LDS write
        constexpr int LINK_ITERS = (TH83 + TV_THREADS - 1) / TV_THREADS;
        int ids[LINK_ITERS];
#pragma unroll
        for (int k = 0; k < LINK_ITERS; ++k) {
            const int p = t + k * TV_THREADS;
            const int hx = p / (TH8 * TH8), hy = (p / TH8) % TH8, hz = p % TH8;
            const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
            ids[k] = -1;
            if (p < TH83 && x >= 0 && x < X && y >= 0 && y < Y && z >= 0 && z < Z)
                ids[k] = g.link[((int64_t)x * Y + y) * Z + z];
        }
#pragma unroll
        for (int k = 0; k < LINK_ITERS; ++k) {
            const int p = t + k * TV_THREADS;
            if (p < TH83) s_id8[p] = ((uint32_t)ids[k] < (uint64_t)g.n_alloc) ? ids[k] : -1;
        }
    }
    __syncthreads();
    // sub-brick sb: origin 4 * (bit 2, bit 1, bit 0 of sb) in block-halo
    // coordinates (its halo starts one lower).  Wave w lists sub-bricks w
    // and w + 4 (64 vertices each, one per lane).  An entry holds the
    // vertex's sub-halo position and which of the four terms touching it
    // exist (TERM_*), decided once per vertex here rather than per field.
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int sb = t / WAVE + 4 * j, l = t % WAVE;
        const int ox = 4 * ((sb >> 2) & 1), oy = 4 * ((sb >> 1) & 1), oz = 4 * (sb & 1);
        const int ix = l / (TB * TB) + 1, iy = (l / TB) % TB + 1, iz = l % TB + 1;
        const int h = hidx8(ox + ix, oy + iy, oz + iz);
        const bool a = s_id8[h] >= 0;
        const unsigned long long m = __ballot(a);
        if (a) {
            const int x = x0 + ox + ix - 1, y = y0 + oy + iy - 1, z = z0 + oz + iz - 1;
            const bool ix_ = x < X - 1, iy_ = y < Y - 1, iz_ = z < Z - 1;
            int e = hidx(ix, iy, iz);
            if (ix_ && iy_ && iz_) e |= TERM_OWN;
            if (x >= 1 && iy_ && iz_ && s_id8[h - TH8 * TH8] >= 0) e |= TERM_X;
            if (y >= 1 && ix_ && iz_ && s_id8[h - TH8] >= 0) e |= TERM_Y;
            if (z >= 1 && ix_ && iy_ && s_id8[h - 1] >= 0) e |= TERM_Z;
            s_list[sb][__popcll(m & ((1ull << l) - 1))] = e;
        }
        if (l == 0) s_n[sb] = __popcll(m);
    }
    __syncthreads();
    auto next_nonempty = [&](int sb) {
        while (sb < 8 && s_n[sb] == 0) ++sb;                // workgroup-uniform
        return sb;
    };
    // the sub-halo records of sub-brick sb: Q lanes per position, one float4 each
    float4 wv[STAGE_ITERS];
    auto request = [&](int sb) {
        const int ox = 4 * ((sb >> 2) & 1), oy = 4 * ((sb >> 1) & 1), oz = 4 * (sb & 1);
#pragma unroll
        for (int k = 0; k < STAGE_ITERS; ++k) {
            const int i = t + k * TV_THREADS;
            wv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (i < TH3 * Q) {
                const int p = i / Q, q = i - Q * p;
                const int hx = p / (TH * TH), hy = (p / TH) % TH, hz = p % TH;
                const int id = s_id8[hidx8(ox + hx, oy + hy, oz + hz)];
                if (id >= 0) wv[k] = reinterpret_cast<const float4*>(g.data + (int64_t)id * S)[q];
            }
        }
    };
    // halo offset of sub-halo position t (positions of every sub-brick
    // differ from it by the sub-brick's origin)
    const int my_h8 = t < TH3 ? hidx8(t / (TH * TH), (t / TH) % TH, t % TH) : 0;
    int sb = next_nonempty(0);
    if (sb < 8) request(sb);
#pragma unroll 1
    while (sb < 8) {
        const int ox = 4 * ((sb >> 2) & 1), oy = 4 * ((sb >> 1) & 1), oz = 4 * (sb & 1);
        // records as they arrived (float4 i of the sub-halo is float4 i of
        // the position-major block), and the sub-halo links, position t
#pragma unroll
        for (int k = 0; k < STAGE_ITERS; ++k) {
            const int i = t + k * TV_THREADS;
            if (i < TH3 * Q) s_v4[i] = wv[k];
        }
        if (t < TH3) s_id[t] = s_id8[hidx8(ox, oy, oz) + my_h8];
        __syncthreads();
        const int nx = next_nonempty(sb + 1);
        if (nx < 8) request(nx);                            // in flight while sb is computed
        const int n = s_n[sb];
        const int* list = s_list[sb];
        // 32 lanes per allocated vertex, lane m < USED takes field m; a thread
        // has at most TV_ITEMS items (n <= 64)
        auto dtv = [&](int e, int m) -> float {
            const int c = e & TERM_POS;
            const float* field = reinterpret_cast<const float*>(s_v4) + m;
            auto val = [&](int p) -> float { return field[p * S]; };
            const float v0 = val(c);
            float acc = 0.f;
            if (e & TERM_OWN) {
                const float dx = val(c + TH * TH) - v0;
                const float dy = val(c + TH) - v0;
                const float dz = val(c + 1) - v0;
                acc -= (dx + dy + dz) * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (e & TERM_X) {
                const float a0 = val(c - TH * TH);
                const float dx = v0 - a0;
                const float dy = val(c - TH * TH + TH) - a0;
                const float dz = val(c - TH * TH + 1) - a0;
                acc += dx * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (e & TERM_Y) {
                const float b0 = val(c - TH);
                const float dx = val(c - TH + TH * TH) - b0;
                const float dy = v0 - b0;
                const float dz = val(c - TH + 1) - b0;
                acc += dy * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            if (e & TERM_Z) {
                const float c0 = val(c - 1);
                const float dx = val(c - 1 + TH * TH) - c0;
                const float dy = val(c - 1 + TH) - c0;
                const float dz = v0 - c0;
                acc += dz * rsqrtf(dx * dx + dy * dy + dz * dz + eps);
            }
            return (m == 0 ? lam_d : lam_sh) * acc;
        };
        if constexpr (SET) {
#pragma unroll
            for (int k = 0; k < TV_ITEMS; ++k) {
                const int it = t + k * TV_THREADS;
                const int m = it & 31;
                if (it < n * 32 && m < USED) {
                    const int e = list[it >> 5];
                    grad[(int64_t)s_id[e & TERM_POS] * S + m] = dtv(e, m);
                }
            }
        } else {
            // the items' gradient entries are read first, so the
            // read-modify-writes cost one round trip, not one each
            float gv[TV_ITEMS];
            int64_t ga[TV_ITEMS];
#pragma unroll
            for (int k = 0; k < TV_ITEMS; ++k) {
                const int it = t + k * TV_THREADS;
                const int m = it & 31;
                ga[k] = -1;
                gv[k] = 0.f;
                if (it < n * 32 && m < USED) {
                    ga[k] = (int64_t)s_id[list[it >> 5] & TERM_POS] * S + m;
                    gv[k] = grad[ga[k]];
                }
            }
#pragma unroll
            for (int k = 0; k < TV_ITEMS; ++k) {
                if (ga[k] < 0) continue;
                const int it = t + k * TV_THREADS;
                grad[ga[k]] = gv[k] + dtv(list[it >> 5], it & 31);
            }
        }
        __syncthreads();                                    // LDS reused by the next sub-brick
        sb = nx;
    }
}

template <bool SET>
static void tv_go(const KGrid& g, float lambda_density, float lambda_sh, float eps, float* grad_data,
                  hipStream_t st) {
    const int nbx = (g.R[0] + TB8 - 1) / TB8, nby = (g.R[1] + TB8 - 1) / TB8;
    const int nbz = (g.R[2] + TB8 - 1) / TB8;
    const int64_t nb = (int64_t)nbx * nby * nbz;
    if (g.deg == 0)
        hipLaunchKernelGGL((k_tv<0, SET>), dim3((unsigned)nb), dim3(TV_THREADS), 0, st, g, lambda_density,
                           lambda_sh, eps, grad_data, nby, nbz);
    else if (g.deg == 1)
        hipLaunchKernelGGL((k_tv<1, SET>), dim3((unsigned)nb), dim3(TV_THREADS), 0, st, g, lambda_density,
                           lambda_sh, eps, grad_data, nby, nbz);
    else
        hipLaunchKernelGGL((k_tv<2, SET>), dim3((unsigned)nb), dim3(TV_THREADS), 0, st, g, lambda_density,
                           lambda_sh, eps, grad_data, nby, nbz);
}

hipError_t launch_tv(const KGrid& g, float lambda_density, float lambda_sh, float eps,
                     float* grad_data, bool set, hipStream_t st) {
    if (set) tv_go<true>(g, lambda_density, lambda_sh, eps, grad_data, st);
    else tv_go<false>(g, lambda_density, lambda_sh, eps, grad_data, st);
    return hipGetLastError();
}

}  // namespace pxm
