// Forward, backward, fused and Gauss-Newton kernels of the sparse-voxel volume
// renderer.
//
// One lane per ray.  A wave holds 64 rays of one pixel tile (the ray packer
// orders full frames in 8x8 tiles), so the lanes gather nearly the same
// vertices at the same sample index and share cache lines.
//
// Forward (Eq. 1-3): march the kept sample positions, skip empty bricks and
// cells (exact: they interpolate to zero density) and composite colour and
// range.  Backward (Eq. 6-14): replay exactly the
// forward's nsamp positions, re-deriving sigma, c, w and T_{i+1} (nothing is
// stored per sample), and scatter or reduce the gradients.  Gauss-Newton
// (Sec. 5.3): per-ray pose Jacobians of the four outputs from the same march,
// reduced to per-frame normal equations.
#include <atomic>
#include <type_traits>

#include "internal.hpp"
#include "scatter.hpp"

namespace pxm {

struct FwdResult {
    float C[3];
    float D;            // expected range (world units), Eq. 3
    double Cd[3];       // the same sums in FP64, for the backward of the same kernel
    double Dd;
    int n;              // kept sample positions
    int mark_last;      // last word of the work-position mask written
    bool mark_overflow; // a work position lay beyond the mask
    long long occ;      // samples in cells with an allocated corner
    long long occ_corners;
    long long grad_corners;   // allocated corners of samples with sigma_raw > 0
};

// Forward march of one ray (Eq. 1-3).  With the occupancy bitfield, samples
// in empty bricks are stepped over in one jump and empty cells cost one bit
// test; both are exact (such samples interpolate to zero density) and still
// count as kept positions.
//
// With a non-null `marks` the march also records, for the backward of the
// same kernel, which of its positions passed the occupancy tests (the only
// ones the backward has work at): bit o of the lane's mask is set for
// position k_first + o, in words marks[w * WAVE] (w < MARK_WORDS) written
// in order from a register; out.mark_last is the last word written and
// out.mark_overflow is set if a marked position lay beyond the mask.
template <int DEG>
__device__ __forceinline__ void ray_forward(const KGrid& g, const KOpts& op, const Ray& ray,
                                            const float Y[9], FwdResult& out,
                                            uint32_t* marks = nullptr, int64_t mstride = WAVE) {
    // colour and range are summed in FP64: the backward differences them
    // with its own prefix sums (Eq. 9, 10), and in FP32 that difference
    // would carry rounding that grows with the number of samples
    double C0 = 0.0, C1 = 0.0, C2 = 0.0, D = 0.0;
    float T = 1.f;
    double L = 0.0;
    int n = 0;
    long long occ = 0, occc = 0, gradc = 0;
    int mw = 0;                     // current mark word
    uint32_t mbits = 0;
    bool movf = false;
    if (!ray.empty) {
        const float delta = op.step_vox;
        int64_t k = ray.k_first;
        OccCache oc;
        occ_cache_init(oc);
        while (n < op.max_samples) {
            Sample s;
            if (!sample_at(g, ray, k, s)) break;
            if (g.occ0) {
                int64_t nxt;
                const int cls = occ_classify(g, ray, k, s.c, oc, nxt);
                if (cls == OCC_JUMP) {
                    if (nxt - k >= (int64_t)(op.max_samples - n)) {
                        n = op.max_samples;
                        break;
                    }
                    n += (int)(nxt - k);
                    k = nxt;
                    continue;
                }
                if (cls == OCC_EMPTY_CELL) {
                    ++n;
                    ++k;
                    continue;
                }
            }
            if (marks) {
                const int64_t o = k - ray.k_first;
                if (o >= (int64_t)MARK_WORDS * 32) {
                    movf = true;
                } else {
                    const int w = (int)(o >> 5);
                    while (mw < w) {
                        marks[mw * mstride] = mbits;
                        mbits = 0u;
                        ++mw;
                    }
                    mbits |= 1u << (int)(o & 31);
                }
            }
            ++n;
            ++k;
            int idx[8];
            const int na = load_links(g, s.base, idx);
            if (na == 0) continue;
            Interp v;
            gather_interp<false, false, DEG>(g, idx, Y, nullptr, s.f, v);
            const float sr = v.sig, s0 = v.s[0], s1 = v.s[1], s2 = v.s[2];
            ++occ;
            occc += na;
            if (!(sr > 0.f)) continue;
            gradc += na;
            const float x = sr * delta;
            const float wt = T * (-expm1f(-x));
            C0 = fma((double)wt, (double)act_fwd(op.act, s0), C0);
            C1 = fma((double)wt, (double)act_fwd(op.act, s1), C1);
            C2 = fma((double)wt, (double)act_fwd(op.act, s2), C2);
            D = fma((double)wt, (double)s.t, D);
            L += (double)x;
            T = trans_of(L);
            if (T < op.t_stop) break;
        }
    }
    if (marks) marks[mw * mstride] = mbits;
    out.mark_last = mw;
    out.mark_overflow = movf;
    out.Cd[0] = C0; out.Cd[1] = C1; out.Cd[2] = C2;
    out.Dd = D;
    out.C[0] = (float)C0; out.C[1] = (float)C1; out.C[2] = (float)C2;
    out.D = (float)D;
    out.n = n;
    out.occ = occ;
    out.occ_corners = occc;
    out.grad_corners = gradc;
}

struct PoseAcc {
    float go[3];        // dL/do summed over samples (Eq. 14: dp/do = 1)
    float gd[3];        // dL/dd through positions (dp/dd = t_i)
    float gv[3];        // dL/dd through the SH basis (optional exact term)
};

// Running state of a backward march.
struct BwdState {
    double A[3];        // sum_{j<=i} c_j w_j
    double AD;          // sum_{j<=i} t_j w_j
    float T;            // T_i
    double L;           // sum_{j<i} sigma_j delta
};

// Backward work of one occupied sample (Eq. 6-14): updates the running state
// and the pose accumulators; returns true with the sample's grid-gradient
// factors (gsig = dL/d sigma_raw, gs = dL/ds_c) when it carries light.
template <bool POSE, bool VIEW, int DEG>
__device__ __forceinline__ bool backward_sample(const KGrid& g, const KOpts& op, const Ray& ray,
                                                const float Y[9], const float GY[9][3],
                                                const Sample& s, const double Chat[3], double Dhat,
                                                const float gC[3], float gDr, BwdState& st,
                                                PoseAcc& pa, int idx[8], float w[8], float& gsig,
                                                float gs[3]) {
    if (load_links(g, s.base, idx) == 0) return false;
    Interp v;
    gather_interp<POSE, POSE && VIEW, DEG>(g, idx, Y, GY, s.f, v);
    trilinear_weights(s.f, w);
    const float sr = v.sig;
    if (!(sr > 0.f)) return false;      // sigma = 0: no light, zero gradient (ReLU)
    const float delta = op.step_vox;
    const float x = sr * delta;
    const float wt = st.T * (-expm1f(-x));
    st.L += (double)x;
    const float Tn = trans_of(st.L);
    float c[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        c[ch] = act_fwd(op.act, v.s[ch]);
        gs[ch] = act_bwd(op.act, v.s[ch]) * wt * gC[ch];      // Eq. 8 through act
        st.A[ch] = fma((double)wt, (double)c[ch], st.A[ch]);
    }
    st.AD = fma((double)wt, (double)s.t, st.AD);
    // Eq. 9 and Eq. 10 with inclusive prefixes A = sum_{j<=i} c_j w_j; the
    // suffix A - C-hat is formed in FP64
    gsig = delta * (gC[0] * (c[0] * Tn + (float)(st.A[0] - Chat[0]))
                  + gC[1] * (c[1] * Tn + (float)(st.A[1] - Chat[1]))
                  + gC[2] * (c[2] * Tn + (float)(st.A[2] - Chat[2]))
                  + gDr * (s.t * Tn + (float)(st.AD - Dhat)));
    if (POSE) {
        // Appendix A: the spatial gradient of the interpolant, dL/dp =
        // gsig grad(sigma) + sum_c gs_c grad(s_c), in world units
        const float inv_vs = (float)g.inv_vs;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float gp = (gsig * v.dsig[a] + gs[0] * v.ds[0][a] + gs[1] * v.ds[1][a]
                              + gs[2] * v.ds[2][a]) * inv_vs;
            pa.go[a] += gp;
            pa.gd[a] = fmaf(s.t, gp, pa.gd[a]);
            if (VIEW) pa.gv[a] += gs[0] * v.ev[0][a] + gs[1] * v.ev[1][a] + gs[2] * v.ev[2][a];
        }
    }
    st.T = Tn;
    return true;
}

// Minimum over the 64 lanes (every lane active), returned to all of them.
// Data-parallel-primitive moves within rows of 16 lanes (shift right by 1,
// 2, 4, 8), then the last lane of each row broadcast into the next rows,
// leave the wave's minimum in lane 63; a lane with no source lane reads the
// identity INT64_MAX.  No LDS round trip, unlike a butterfly of shuffles.
__device__ __forceinline__ int64_t wave_min(int64_t v) {
    constexpr int ID_LO = -1, ID_HI = 0x7fffffff;            // INT64_MAX
    auto step = [&](auto ctrl, auto row_mask) {
        const int lo = __builtin_amdgcn_update_dpp(ID_LO, (int)(uint32_t)v, decltype(ctrl)::value,
                                                   decltype(row_mask)::value, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(ID_HI, (int)((uint64_t)v >> 32), decltype(ctrl)::value,
                                                   decltype(row_mask)::value, 0xf, false);
        const int64_t o = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
        v = o < v ? o : v;
    };
    using std::integral_constant;
    step(integral_constant<int, 0x111>{}, integral_constant<int, 0xf>{});   // row_shr:1
    step(integral_constant<int, 0x112>{}, integral_constant<int, 0xf>{});   // row_shr:2
    step(integral_constant<int, 0x114>{}, integral_constant<int, 0xf>{});   // row_shr:4
    step(integral_constant<int, 0x118>{}, integral_constant<int, 0xf>{});   // row_shr:8
    step(integral_constant<int, 0x142>{}, integral_constant<int, 0xa>{});   // row_bcast:15 -> rows 1, 3
    step(integral_constant<int, 0x143>{}, integral_constant<int, 0xc>{});   // row_bcast:31 -> rows 2, 3
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const int hi = __builtin_amdgcn_readlane((int)((uint64_t)v >> 32), 63);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// The smallest marked position offset >= o in a lane's work mask (words
// marks[w * WAVE], w <= last), or -1.
__device__ __forceinline__ int next_mark(const uint32_t* marks, int last, int o) {
    int w = o >> 5;
    if (w > last) return -1;
    uint32_t b = marks[w * WAVE] & (0xffffffffu << (o & 31));
    while (b == 0u) {
        if (++w > last) return -1;
        b = marks[w * WAVE];
    }
    return w * 32 + __ffs(b) - 1;
}

// Backward march of one ray over its first n kept positions (Eq. 6-14).
//   Chat, Dhat: the forward's colour and expected range
//   gC, gDr:    dL/dC-hat and dL/d(range)
// With GRID the lanes of a wave march in lockstep on the absolute sample
// index (so that lanes of one tile share cells and their scatters merge):
// every lane must call this (lanes without a ray pass n = 0); steps where no
// lane has an occupied cell are jumped over together.  Without GRID every
// lane marches on its own.
template <bool GRID, bool POSE, bool VIEW, int DEG, bool FIX = false>
__device__ __forceinline__ void ray_backward(const KGrid& g, const KOpts& op, const Ray& ray,
                                             const float Y[9], int n, const double Chat[3],
                                             double Dhat, const float gC[3], float gDr,
                                             float* __restrict__ grad, const WaveStage& wc,
                                             PoseAcc& pa, const uint32_t* marks = nullptr,
                                             int mark_last = 0, bool mark_overflow = true) {
    float GY[9][3];
    if (VIEW) sh9_grad(ray.d[0], ray.d[1], ray.d[2], GY);
    BwdState st = {{0.0, 0.0, 0.0}, 0.0, 1.f, 0.0};
    const int64_t ks = ray.k_first, ke = ray.k_first + (n > 0 ? n : 0);
    bool has = n > 0;
    if (GRID && marks && __ballot(mark_overflow && n > 0) == 0) {
        // the forward of this kernel marked every work position: visit only
        // those, the wave at the smallest pending one
        int off = has ? next_mark(marks, mark_last, 0) : -1;
        for (;;) {
            const int64_t mine = off >= 0 ? ks + off : INT64_MAX;
            const int64_t k = wave_min(mine);
            if (k == INT64_MAX) break;
            const bool work = mine == k;
            bool have = false;
            int idx[8];
            float w[8];
            float gsig = 0.f, gs[3] = {0.f, 0.f, 0.f};
            Sample s;
            if (work && sample_at(g, ray, k, s))
                have = backward_sample<POSE, VIEW, DEG>(g, op, ray, Y, GY, s, Chat, Dhat, gC, gDr, st,
                                                   pa, idx, w, gsig, gs);
            scatter_merged<DEG, FIX>(have, s.base, idx, w, gsig, gs, Y, wc, grad);
            if (work) off = next_mark(marks, mark_last, off + 1);
        }
    } else if (GRID) {
        int64_t k = wave_min(has ? ks : INT64_MAX);
        OccCache oc;
        occ_cache_init(oc);
        for (;;) {
            const bool live = has && k < ke;
            if (__ballot(live) == 0) break;
            const bool run = live && k >= ks;
            int64_t adv = live ? (run ? 1 : ks - k) : INT64_MAX;
            bool work = false;
            Sample s;
            if (run) {
                if (!sample_at(g, ray, k, s)) {
                    has = false;            // left the box: nothing further on this ray
                    adv = INT64_MAX;
                } else if (!g.occ0) {
                    work = true;
                } else {
                    int64_t nxt;
                    const int cls = occ_classify(g, ray, k, s.c, oc, nxt);
                    if (cls == OCC_JUMP) adv = (nxt < ke ? nxt : ke) - k;
                    else work = cls == OCC_CELL;
                }
            }
            if (__ballot(work) == 0) {
                const int64_t step = wave_min(adv);
                if (step == INT64_MAX) break;       // every live lane has just left the box
                k += step;
                continue;
            }
            bool have = false;
            int idx[8];
            float w[8];
            float gsig = 0.f, gs[3] = {0.f, 0.f, 0.f};
            if (work)
                have = backward_sample<POSE, VIEW, DEG>(g, op, ray, Y, GY, s, Chat, Dhat, gC, gDr, st,
                                                   pa, idx, w, gsig, gs);
            scatter_merged<DEG, FIX>(have, s.base, idx, w, gsig, gs, Y, wc, grad);
            ++k;
        }
    } else if (marks && !mark_overflow) {
        // per lane: straight from one marked position to the next
        for (int off = has ? next_mark(marks, mark_last, 0) : -1; off >= 0;
             off = next_mark(marks, mark_last, off + 1)) {
            Sample s;
            if (!sample_at(g, ray, ks + off, s)) break;
            int idx[8];
            float w[8];
            float gsig, gs[3];
            backward_sample<POSE, VIEW, DEG>(g, op, ray, Y, GY, s, Chat, Dhat, gC, gDr, st, pa, idx, w,
                                        gsig, gs);
        }
    } else {
        int64_t k = ks;
        OccCache oc;
        occ_cache_init(oc);
        while (k < ke) {
            Sample s;
            if (!sample_at(g, ray, k, s)) break;
            if (g.occ0) {
                int64_t nxt;
                const int cls = occ_classify(g, ray, k, s.c, oc, nxt);
                if (cls == OCC_JUMP) {
                    k = nxt < ke ? nxt : ke;
                    continue;
                }
                if (cls == OCC_EMPTY_CELL) {
                    ++k;
                    continue;
                }
            }
            int idx[8];
            float w[8];
            float gsig, gs[3];
            backward_sample<POSE, VIEW, DEG>(g, op, ray, Y, GY, s, Chat, Dhat, gC, gDr, st, pa, idx, w,
                                        gsig, gs);
            ++k;
        }
    }
}

// (g_rho, g_phi) of one ray: rho = g_o, phi = o x g_o + d x g_d (+ d x g_view).
template <bool VIEW>
__device__ __forceinline__ void pose_six(const Ray& ray, const PoseAcc& pa, double out[6]) {
    const float* o = ray.o;
    const float* d = ray.d;
    float gd[3] = {pa.gd[0], pa.gd[1], pa.gd[2]};
    if (VIEW) { gd[0] += pa.gv[0]; gd[1] += pa.gv[1]; gd[2] += pa.gv[2]; }
    out[0] = pa.go[0];
    out[1] = pa.go[1];
    out[2] = pa.go[2];
    out[3] = (double)(o[1] * pa.go[2] - o[2] * pa.go[1]) + (double)(d[1] * gd[2] - d[2] * gd[1]);
    out[4] = (double)(o[2] * pa.go[0] - o[0] * pa.go[2]) + (double)(d[2] * gd[0] - d[0] * gd[2]);
    out[5] = (double)(o[0] * pa.go[1] - o[1] * pa.go[0]) + (double)(d[0] * gd[1] - d[1] * gd[0]);
}

// ---------------------------------------------------------------------------
// Gauss-Newton tracking: per-ray pose Jacobian of (R, G, B, z-depth)
// ---------------------------------------------------------------------------

// Pose accumulators of the four outputs (colour channels, then z-depth).
struct JacAcc {
    float go[4][3];
    float gd[4][3];
    float gv[4][3];
};

// One occupied sample of the Jacobian march: row k is the pose gradient of
// output k alone (unit upstream on it), so the sample's factors are those of
// Eq. 8-10 with gC = e_k (colour rows) or dL/d range = 1/s (depth row).
template <bool VIEW, int DEG>
__device__ __forceinline__ void jacobian_sample(const KGrid& g, const KOpts& op, const Ray& ray,
                                                const float Y[9], const float GY[9][3],
                                                const Sample& s, const double Chat[3], double Dhat,
                                                BwdState& st, JacAcc& ja) {
    int idx[8];
    if (load_links(g, s.base, idx) == 0) return;
    Interp v;
    gather_interp<true, VIEW, DEG>(g, idx, Y, GY, s.f, v);
    const float sr = v.sig;
    if (!(sr > 0.f)) return;
    const float delta = op.step_vox;
    const float x = sr * delta;
    const float wt = st.T * (-expm1f(-x));
    st.L += (double)x;
    const float Tn = trans_of(st.L);
    float c[3], dact[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        c[ch] = act_fwd(op.act, v.s[ch]);
        dact[ch] = act_bwd(op.act, v.s[ch]) * wt;
        st.A[ch] = fma((double)wt, (double)c[ch], st.A[ch]);
    }
    st.AD = fma((double)wt, (double)s.t, st.AD);
    // per-output density factor (Eq. 9 / Eq. 10) and colour factor (Eq. 8)
    float gsig[4];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) gsig[ch] = delta * (c[ch] * Tn + (float)(st.A[ch] - Chat[ch]));
    gsig[3] = delta * (s.t * Tn + (float)(st.AD - Dhat)) / ray.s;
    const float inv_vs = (float)g.inv_vs;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float gp = gsig[k] * v.dsig[a];
            if (k < 3) gp = fmaf(dact[k < 3 ? k : 0], v.ds[k < 3 ? k : 0][a], gp);
            gp *= inv_vs;
            ja.go[k][a] += gp;
            ja.gd[k][a] = fmaf(s.t, gp, ja.gd[k][a]);
            if (VIEW && k < 3) ja.gv[k][a] = fmaf(dact[k < 3 ? k : 0], v.ev[k < 3 ? k : 0][a], ja.gv[k][a]);
        }
    }
    st.T = Tn;
}

// Jacobian rows J[k] = (g_o, o x g_o + d x g_d (+ d x g_view)) of one ray.
template <bool VIEW, int DEG>
__device__ __forceinline__ void ray_jacobian(const KGrid& g, const KOpts& op, const Ray& ray,
                                             const float Y[9], int n, const double Chat[3],
                                             double Dhat, float J[4][6],
                                             const uint32_t* marks = nullptr, int mark_last = 0,
                                             bool mark_overflow = true) {
    float GY[9][3];
    if (VIEW) sh9_grad(ray.d[0], ray.d[1], ray.d[2], GY);
    BwdState st = {{0.0, 0.0, 0.0}, 0.0, 1.f, 0.0};
    JacAcc ja;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) ja.go[k][a] = ja.gd[k][a] = ja.gv[k][a] = 0.f;
    const int64_t ke = ray.k_first + (n > 0 ? n : 0);
    if (marks && !mark_overflow) {
        for (int off = n > 0 ? next_mark(marks, mark_last, 0) : -1; off >= 0;
             off = next_mark(marks, mark_last, off + 1)) {
            Sample s;
            if (!sample_at(g, ray, ray.k_first + off, s)) break;
            jacobian_sample<VIEW, DEG>(g, op, ray, Y, GY, s, Chat, Dhat, st, ja);
        }
    } else {
        int64_t k = ray.k_first;
        OccCache oc;
        occ_cache_init(oc);
        while (k < ke) {
            Sample s;
            if (!sample_at(g, ray, k, s)) break;
            if (g.occ0) {
                int64_t nxt;
                const int cls = occ_classify(g, ray, k, s.c, oc, nxt);
                if (cls == OCC_JUMP) {
                    k = nxt < ke ? nxt : ke;
                    continue;
                }
                if (cls == OCC_EMPTY_CELL) {
                    ++k;
                    continue;
                }
            }
            jacobian_sample<VIEW, DEG>(g, op, ray, Y, GY, s, Chat, Dhat, st, ja);
            ++k;
        }
    }
    const float* o = ray.o;
    const float* d = ray.d;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float gd[3] = {ja.gd[q][0], ja.gd[q][1], ja.gd[q][2]};
        if (VIEW) { gd[0] += ja.gv[q][0]; gd[1] += ja.gv[q][1]; gd[2] += ja.gv[q][2]; }
        const float* go = ja.go[q];
        J[q][0] = go[0];
        J[q][1] = go[1];
        J[q][2] = go[2];
        J[q][3] = (o[1] * go[2] - o[2] * go[1]) + (d[1] * gd[2] - d[2] * gd[1]);
        J[q][4] = (o[2] * go[0] - o[0] * go[2]) + (d[2] * gd[0] - d[0] * gd[2]);
        J[q][5] = (o[0] * go[1] - o[1] * go[0]) + (d[0] * gd[1] - d[1] * gd[0]);
    }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <int DEG>
__global__ void __launch_bounds__(256) k_forward(KGrid g, KRays rs, KOpts op, float* __restrict__ rgb,
                                                 float* __restrict__ depth, int32_t* __restrict__ nsamp) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rs.n) return;
    const int f = frame_of(rs.off, rs.F, r);
    Ray ray;
    setup_ray(g, rs, op, r, f, ray);
    float Y[9];
    sh9(ray.d[0], ray.d[1], ray.d[2], Y);
    FwdResult fr;
    ray_forward<DEG>(g, op, ray, Y, fr);
    rgb[3 * r] = fr.C[0];
    rgb[3 * r + 1] = fr.C[1];
    rgb[3 * r + 2] = fr.C[2];
    depth[r] = fr.D / ray.s;
    nsamp[r] = fr.n;
}

template <bool GRID, bool POSE, bool VIEW, int DEG>
__global__ void __launch_bounds__(256) k_backward(KGrid g, KRays rs, KOpts op,
                                                  const float* __restrict__ rgb,
                                                  const float* __restrict__ depth,
                                                  const int32_t* __restrict__ nsamp,
                                                  const float* __restrict__ g_rgb,
                                                  const float* __restrict__ g_depth,
                                                  float* __restrict__ grad,
                                                  double* __restrict__ grad_pose) {
    extern __shared__ float smem[];
    WaveStage wc{nullptr, nullptr, nullptr, nullptr};
    if (GRID) wc = wave_stage(smem);
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool active = r < rs.n;
    int f = 0;
    Ray ray;
    PoseAcc pa = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    float Y[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float gC[3] = {0.f, 0.f, 0.f};
    double Chat[3] = {0.0, 0.0, 0.0};
    float gDr = 0.f;
    double Dhat = 0.0;
    int n = 0;
    ray.empty = true;
    if (active) {
        gC[0] = g_rgb[3 * r];
        gC[1] = g_rgb[3 * r + 1];
        gC[2] = g_rgb[3 * r + 2];
        const float gD = g_depth[r];
        active = gC[0] != 0.f || gC[1] != 0.f || gC[2] != 0.f || gD != 0.f;
        if (active) {
            f = frame_of(rs.off, rs.F, r);
            setup_ray(g, rs, op, r, f, ray);
            sh9(ray.d[0], ray.d[1], ray.d[2], Y);
            Chat[0] = rgb[3 * r];
            Chat[1] = rgb[3 * r + 1];
            Chat[2] = rgb[3 * r + 2];
            Dhat = (double)depth[r] * (double)ray.s;
            gDr = gD / ray.s;
            n = ray.empty ? 0 : nsamp[r];
        }
    }
    ray_backward<GRID, POSE, VIEW, DEG>(g, op, ray, Y, n, Chat, Dhat, gC, gDr, grad, wc, pa);
    if (POSE) {
        double six[6] = {0, 0, 0, 0, 0, 0};
        if (active) pose_six<VIEW>(ray, pa, six);
        seg_sum_atomic<6>(f, active, six, grad_pose);
    }
}

// Fused step, in one launch (PH 0) or split in two (PH 1: forward and loss,
// PH 2: backward).  The forward launch needs no LDS and few registers, so it
// runs at the occupancy of a forward-only kernel; it leaves each ray's work
// mask and backward inputs in `sp`, from which the backward launch resumes.
template <bool GRID, bool POSE, bool VIEW, int PH, int DEG, bool FIX>
__global__ void __launch_bounds__(256, (PH == 1 ? 4 : 1)) k_fused(KGrid g, KRays rs, KOpts op,
                                               const float* __restrict__ tgt_rgb,
                                               const float* __restrict__ tgt_depth,
                                               const float* __restrict__ fw,
                                               float* __restrict__ rgb_out,
                                               float* __restrict__ depth_out,
                                               double* __restrict__ loss,
                                               float* __restrict__ grad,
                                               double* __restrict__ grad_pose,
                                               int64_t* __restrict__ stats,
                                               unsigned* __restrict__ ws, int persistent,
                                               KSplit sp) {
    __shared__ int64_t s_tile;
    extern __shared__ float smem[];
    WaveStage wc{nullptr, nullptr, nullptr, nullptr};
    if (GRID && PH != 1) {
        wc = wave_stage(smem);
        wc.gfix = sp.gfix;
    }
    const int64_t n_tiles = (rs.n + blockDim.x - 1) / blockDim.x;
    // Persistent form: workgroups take tiles in order from one queue counter
    // (ws[0]), so the tiles in flight at any time are neighbours in the
    // image and gather from one compact region of the grid.
    for (;;) {
        int64_t tile;
        if (persistent) {
            if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(ws, 1u);
            __syncthreads();
            tile = s_tile;
            __syncthreads();
            if (tile >= n_tiles) break;
        } else {
            tile = xcd_tile(blockIdx.x, gridDim.x);
        }
        const int64_t r = tile * blockDim.x + threadIdx.x;
        const bool inr = r < rs.n;
        int f = 0;
        Ray ray;
        ray.empty = true;
        FwdResult fr;
        bool valid = false;
        double lval = 0.0;
        PoseAcc pa = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
        float Y[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float gC[3] = {0.f, 0.f, 0.f};
        float gDr = 0.f;
        int nb = 0;
        fr.mark_last = 0;
        fr.mark_overflow = false;
        uint32_t* marks = PH == 1 ? ((GRID || POSE) && inr ? sp.marks + r : nullptr)
                        : GRID ? wc.marks + lane_id()
                        : POSE ? reinterpret_cast<uint32_t*>(smem) + (threadIdx.x / WAVE) * (MARK_WORDS * WAVE)
                                     + lane_id()
                               : nullptr;
        if (PH == 2) {
            // resume from the forward launch: backward inputs and work mask
            if (inr) {
                f = frame_of(rs.off, rs.F, r);
                setup_ray(g, rs, op, r, f, ray);
                sh9(ray.d[0], ray.d[1], ray.d[2], Y);
                const float Dt = tgt_depth[r];
                valid = isfinite(Dt) && Dt > 0.f;
                nb = sp.nb[r];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    fr.Cd[c] = sp.sums[c * sp.n_pad + r];
                    gC[c] = sp.up[c * sp.n_pad + r];
                }
                fr.Dd = sp.sums[3 * sp.n_pad + r];
                gDr = sp.up[3 * sp.n_pad + r];
                const int mi = sp.minfo[r];
                fr.mark_last = mi & 0xff;
                fr.mark_overflow = (mi >> 8) != 0;
                if (marks && !fr.mark_overflow)
                    for (int w = 0; w <= fr.mark_last; ++w) marks[w * WAVE] = sp.marks[w * sp.n_pad + r];
            } else {
                fr.Cd[0] = fr.Cd[1] = fr.Cd[2] = fr.Dd = 0.0;
            }
        } else if (inr) {
            f = frame_of(rs.off, rs.F, r);
            setup_ray(g, rs, op, r, f, ray);
            sh9(ray.d[0], ray.d[1], ray.d[2], Y);
            ray_forward<DEG>(g, op, ray, Y, fr, marks, PH == 1 ? sp.n_pad : (int64_t)WAVE);
            const float z = fr.D / ray.s;
            if (rgb_out) {
                rgb_out[3 * r] = fr.C[0];
                rgb_out[3 * r + 1] = fr.C[1];
                rgb_out[3 * r + 2] = fr.C[2];
            }
            if (depth_out) depth_out[r] = z;
            // Eq. 4, 5, 11; invalid depth drops the ray (Sec. 6.1)
            const float Dt = tgt_depth[r];
            valid = isfinite(Dt) && Dt > 0.f;
            if (valid) {
                const float wf = fw[f];
                const float e0 = fr.C[0] - tgt_rgb[3 * r];
                const float e1 = fr.C[1] - tgt_rgb[3 * r + 1];
                const float e2 = fr.C[2] - tgt_rgb[3 * r + 2];
                const float ed = z - Dt;
                float rho, drho;
                if (op.depth_loss == LOSS_L2) { rho = ed * ed; drho = 2.f * ed; }
                else { rho = fabsf(ed); drho = ed > 0.f ? 1.f : (ed < 0.f ? -1.f : 0.f); }
                lval = (double)wf * ((double)e0 * e0 + (double)e1 * e1 + (double)e2 * e2)
                     + (double)op.lambda_d * wf * rho;
                gC[0] = 2.f * wf * e0;
                gC[1] = 2.f * wf * e1;
                gC[2] = 2.f * wf * e2;
                gDr = op.lambda_d * wf * drho / ray.s;
                nb = fr.n;
            }
            if (PH == 1) {
                // hand the backward inputs to the backward launch
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    sp.sums[c * sp.n_pad + r] = fr.Cd[c];
                    sp.up[c * sp.n_pad + r] = gC[c];
                }
                sp.sums[3 * sp.n_pad + r] = fr.Dd;
                sp.up[3 * sp.n_pad + r] = gDr;
                sp.nb[r] = nb;
                sp.minfo[r] = fr.mark_last | (fr.mark_overflow ? 0x100 : 0);
            }
        } else {
            fr.C[0] = fr.C[1] = fr.C[2] = fr.D = 0.f;
            fr.Cd[0] = fr.Cd[1] = fr.Cd[2] = fr.Dd = 0.0;
        }
        if ((GRID || POSE) && PH != 1)
            ray_backward<GRID, POSE, VIEW, DEG, FIX>(g, op, ray, Y, nb, fr.Cd, fr.Dd, gC, gDr, grad, wc, pa, marks,
                                           fr.mark_last, fr.mark_overflow);
        if (loss && PH != 2) {
            double lv[1] = {lval};
            seg_sum_atomic<1>(f, valid, lv, loss);
        }
        if (POSE && PH != 1) {
            double six[6] = {0, 0, 0, 0, 0, 0};
            if (valid) pose_six<VIEW>(ray, pa, six);
            seg_sum_atomic<6>(f, valid, six, grad_pose);
        }
        if (stats && PH != 2) {
            long long sv[4] = {inr ? fr.occ : 0, inr ? fr.occ_corners : 0,
                               valid ? fr.grad_corners : 0, valid ? 1 : 0};
            add_stats(inr, sv, stats);
        }
        if (!persistent) break;
    }
    if (persistent && threadIdx.x == 0) {
        // the last workgroup to finish re-arms the queue for the next launch
        __threadfence();
        const unsigned prev = atomicAdd(ws + 1, 1u);
        if (prev == gridDim.x - 1) {
            atomicExch(ws, 0u);
            atomicExch(ws + 1, 0u);
        }
    }
}

// Gauss-Newton normal equations: per ray, forward, 4-residual and Jacobian;
// per frame, H = sum w J^T W J (upper triangle), g = sum w J^T W e and the
// error E, with W = diag(1, 1, 1, lambda_depth) over rays with a valid depth.
template <bool VIEW, int DEG>
__global__ void __launch_bounds__(256) k_gn(KGrid g, KRays rs, KOpts op,
                                            const float* __restrict__ tgt_rgb,
                                            const float* __restrict__ tgt_depth,
                                            const float* __restrict__ fw,
                                            double* __restrict__ gn) {
    extern __shared__ uint32_t gn_marks[];
    uint32_t* marks = gn_marks + (threadIdx.x / WAVE) * (MARK_WORDS * WAVE) + lane_id();
    const int64_t r = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const bool inr = r < rs.n;
    int f = 0;
    bool valid = false;
    double vals[GN_VALUES];
#pragma unroll
    for (int i = 0; i < GN_VALUES; ++i) vals[i] = 0.0;
    if (inr) {
        f = frame_of(rs.off, rs.F, r);
        Ray ray;
        setup_ray(g, rs, op, r, f, ray);
        float Y[9];
        sh9(ray.d[0], ray.d[1], ray.d[2], Y);
        FwdResult fr;
        ray_forward<DEG>(g, op, ray, Y, fr, marks);
        const float Dt = tgt_depth[r];
        valid = isfinite(Dt) && Dt > 0.f;
        if (valid) {
            const float e[4] = {fr.C[0] - tgt_rgb[3 * r], fr.C[1] - tgt_rgb[3 * r + 1],
                                fr.C[2] - tgt_rgb[3 * r + 2], fr.D / ray.s - Dt};
            float J[4][6];
            ray_jacobian<VIEW, DEG>(g, op, ray, Y, fr.n, fr.Cd, fr.Dd, J, marks, fr.mark_last,
                               fr.mark_overflow);
            const double wf = (double)fw[f];
            const double Wk[4] = {wf, wf, wf, wf * (double)op.lambda_d};
            int q = 0;
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int j = i; j < 6; ++j) {
                    double acc = 0.0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) acc += Wk[k] * (double)J[k][i] * (double)J[k][j];
                    vals[q++] = acc;
                }
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < 4; ++k) acc += Wk[k] * (double)J[k][i] * (double)e[k];
                vals[21 + i] = acc;
            }
            double E = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) E += Wk[k] * (double)e[k] * (double)e[k];
            vals[27] = E;
        }
    }
    seg_sum_atomic<GN_VALUES>(f, valid, vals, gn);
}

// Deterministic scatter, last step: grad += fixed-point sum x 2^-FIX_SHIFT
// (one conversion of an exact integer sum), and the buffer is zeroed for the
// next call.  Padding fields of a record are left alone.
__global__ void __launch_bounds__(256) k_fix_finalize(unsigned long long* __restrict__ gfix,
                                                      float* __restrict__ grad, int64_t n, int S,
                                                      int used) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const long long v = (long long)gfix[i];
        if (v != 0 && (int)(i % S) < used) grad[i] += (float)((double)v / FIX_SCALE);
        gfix[i] = 0ull;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t n, int block) {
    return (unsigned)((n + block - 1) / block);
}

// Calls f(std::integral_constant<int, DEG>) for the grid's SH degree.
template <class F>
static void by_degree(int deg, F&& f) {
    if (deg == 0) f(std::integral_constant<int, 0>{});
    else if (deg == 1) f(std::integral_constant<int, 1>{});
    else f(std::integral_constant<int, 2>{});
}

hipError_t launch_forward(const KGrid& g, const KRays& rs, const KOpts& op, float* rgb,
                          float* depth, int32_t* nsamp, hipStream_t st) {
    by_degree(g.deg, [&](auto D) {
        hipLaunchKernelGGL(k_forward<decltype(D)::value>, dim3(blocks_for(rs.n, 256)), dim3(256), 0, st,
                           g, rs, op, rgb, depth, nsamp);
    });
    return hipGetLastError();
}

hipError_t launch_backward(const KGrid& g, const KRays& rs, const KOpts& op, const float* rgb,
                           const float* depth, const int32_t* nsamp, const float* g_rgb,
                           const float* g_depth, float* grad_data, double* grad_pose,
                           hipStream_t st) {
    const dim3 grid(blocks_for(rs.n, 256)), block(256);
    const bool view = (op.flags & 1) != 0;
    if (!((grad_data != nullptr) ^ (grad_pose != nullptr))) return hipErrorInvalidValue;
    by_degree(g.deg, [&](auto D) {
        constexpr int DEG = decltype(D)::value;
        if (grad_data) {
            // one wave per workgroup: each wave stages its MFMA operands in ~19 KB of LDS
            const size_t lds = WAVE_LDS_FLOATS * sizeof(float);
            hipLaunchKernelGGL((k_backward<true, false, false, DEG>), dim3(blocks_for(rs.n, WAVE)),
                               dim3(WAVE), lds, st, g, rs, op, rgb, depth, nsamp, g_rgb, g_depth,
                               grad_data, grad_pose);
        } else if (view) {
            hipLaunchKernelGGL((k_backward<false, true, true, DEG>), grid, block, 0, st, g, rs, op, rgb,
                               depth, nsamp, g_rgb, g_depth, grad_data, grad_pose);
        } else {
            hipLaunchKernelGGL((k_backward<false, true, false, DEG>), grid, block, 0, st, g, rs, op, rgb,
                               depth, nsamp, g_rgb, g_depth, grad_data, grad_pose);
        }
    });
    return hipGetLastError();
}

static size_t device_lds() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 65536;
    return (size_t)v;
}

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

// Persistent grid: as many workgroups as the device holds at once (from the
// kernel's register and LDS use), never more than there are tiles.
// The per-CU figure is cached per kernel and block size; concurrent callers
// may both compute it, and they store the same value.
template <bool GRID, bool POSE, bool VIEW, int PH, int DEG, bool FIX>
static unsigned resident_blocks(int block, size_t lds, int64_t tiles) {
    static std::atomic<int> per_cu[4];                    // by block 64/128/256/512, 0 = unknown
    const int slot = block == 64 ? 0 : block == 128 ? 1 : block == 256 ? 2 : 3;
    int n = per_cu[slot].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fused<GRID, POSE, VIEW, PH, DEG, FIX>, block,
                                                         lds) != hipSuccess || n <= 0)
            n = 1;
        per_cu[slot].store(n, std::memory_order_relaxed);
    }
    static const int cus = device_cus();
    const int64_t cap = (int64_t)cus * n;
    return (unsigned)(tiles < cap ? tiles : cap);
}

template <bool GRID, bool POSE, bool VIEW, int PH, int DEG, bool FIX>
static void fused_phase(int64_t tiles, dim3 block, hipStream_t st, const KGrid& g, const KRays& rs,
                        const KOpts& op, const float* tgt_rgb, const float* tgt_depth,
                        const float* fw, float* rgb, float* depth, double* loss, float* grad,
                        double* gp, int64_t* stats, unsigned* ws, int persistent, const KSplit& sp) {
    const size_t lds = PH == 1 ? 0
                     : GRID ? (block.x / WAVE) * WAVE_LDS_FLOATS * sizeof(float)
                     : POSE ? (block.x / WAVE) * MARK_WORDS * WAVE * sizeof(uint32_t) : 0;
    const dim3 grid(persistent ? resident_blocks<GRID, POSE, VIEW, PH, DEG, FIX>(block.x, lds, tiles)
                               : (unsigned)tiles);
    hipLaunchKernelGGL((k_fused<GRID, POSE, VIEW, PH, DEG, FIX>), grid, block, lds, st, g, rs, op, tgt_rgb,
                       tgt_depth, fw, rgb, depth, loss, grad, gp, stats, ws, persistent, sp);
}

// variant 0: one workgroup per tile; 1: persistent workgroups on the tile
// queue; 2: a forward launch then a backward launch, both persistent, with
// the per-ray state in the workspace
template <bool GRID, bool POSE, bool VIEW, int DEG, bool FIX>
static void fused_go(int64_t tiles, dim3 block, hipStream_t st, const KGrid& g, const KRays& rs,
                     const KOpts& op, const float* tgt_rgb, const float* tgt_depth,
                     const float* fw, float* rgb, float* depth, double* loss, float* grad,
                     double* gp, int64_t* stats, unsigned* ws, int variant,
                     unsigned long long* gfix) {
    if (variant == 2) {
        KSplit sp = split_state(ws, rs.n);
        sp.gfix = gfix;
        fused_phase<GRID, POSE, VIEW, 1, DEG, false>(tiles, block, st, g, rs, op, tgt_rgb, tgt_depth, fw,
                                                     rgb, depth, loss, grad, gp, stats, ws, 1, sp);
        fused_phase<GRID, POSE, VIEW, 2, DEG, FIX>(tiles, block, st, g, rs, op, tgt_rgb, tgt_depth, fw,
                                                   rgb, depth, loss, grad, gp, stats, ws, 1, sp);
    } else {
        KSplit sp{};
        sp.gfix = gfix;
        fused_phase<GRID, POSE, VIEW, 0, DEG, FIX>(tiles, block, st, g, rs, op, tgt_rgb, tgt_depth, fw,
                                                   rgb, depth, loss, grad, gp, stats, ws, variant, sp);
    }
}

hipError_t launch_fused(const KGrid& g, const KRays& rs, const KOpts& op, const float* tgt_rgb,
                        const float* tgt_depth, const float* frame_weight, int want, float* rgb,
                        float* depth, double* loss, float* grad_data, double* grad_pose,
                        int64_t* stats, unsigned* ws, int block, int variant,
                        unsigned long long* gfix, hipStream_t st) {
    if (want & 1) {
        // the grid scatter needs WAVE_LDS_FLOATS of LDS per wave: shrink the
        // workgroup if the device cannot give this many waves' worth
        static const size_t max_lds = device_lds();
        while (block > WAVE && (size_t)(block / WAVE) * WAVE_LDS_FLOATS * sizeof(float) > max_lds)
            block /= 2;
    }
    const int64_t tiles = (rs.n + block - 1) / block;
    if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;  // 32-bit grid and queue counters
    const dim3 blk(block);
    const bool G = want & 1, P = want & 2, V = (op.flags & 1) != 0;
    int64_t* sp = (want & 4) ? stats : nullptr;
    by_degree(g.deg, [&](auto D) {
        constexpr int DEG = decltype(D)::value;
        if (G && P) {
            if (V) {
                if (gfix) fused_go<true, true, true, DEG, true>(tiles, blk, st, g, rs, op, tgt_rgb, tgt_depth, frame_weight, rgb, depth, loss, grad_data, grad_pose, sp, ws, variant, gfix);
                else fused_go<true, true, true, DEG, false>(tiles, blk, st, g, rs, op, tgt_rgb, tgt_depth, frame_weight, rgb, depth, loss, grad_data, grad_pose, sp, ws, variant, gfix);
            } else {
                if (gfix) fused_go<true, true, false, DEG, true>(tiles, blk, st, g, rs, op, tgt_rgb, tgt_depth, frame_weight, rgb, depth, loss, grad_data, grad_pose, sp, ws, variant, gfix);
                else fused_go<true, true, false, DEG, false>(tiles, blk, st, g, rs, op, tgt_rgb, tgt_depth, frame_weight, rgb, depth, loss, grad_data, grad_pose, sp, ws, variant, gfix);
            }
        } else if (G) {
            if (gfix) fused_go<true, false, false, DEG, true>(tiles, blk, st, g, rs, op, tgt_rgb, tgt_depth, frame_weight, rgb, depth, loss, grad_data, grad_pose, sp, ws, variant, gfix);
            else fused_go<true, false, false, DEG, false>(tiles, blk, st, g, rs, op, tgt_rgb, tgt_depth, frame_weight, rgb, depth, loss, grad_data, grad_pose, sp, ws, variant, gfix);
        } else if (P) {
            if (V) fused_go<false, true, true, DEG, false>(tiles, blk, st, g, rs, op, tgt_rgb, tgt_depth, frame_weight, rgb, depth, loss, grad_data, grad_pose, sp, ws, variant, nullptr);
            else fused_go<false, true, false, DEG, false>(tiles, blk, st, g, rs, op, tgt_rgb, tgt_depth, frame_weight, rgb, depth, loss, grad_data, grad_pose, sp, ws, variant, nullptr);
        } else {
            fused_go<false, false, false, DEG, false>(tiles, blk, st, g, rs, op, tgt_rgb, tgt_depth, frame_weight, rgb, depth, loss, grad_data, grad_pose, sp, ws, variant, nullptr);
        }
    });
    if (G && gfix) {
        // fold the exact integer sums into the float gradient, once per entry
        const int S = record_floats(g.deg);
        const int64_t n = g.n_alloc * S;
        const int64_t wgs = (n + 255) / 256;
        hipLaunchKernelGGL(k_fix_finalize, dim3((unsigned)(wgs < (1 << 20) ? wgs : (1 << 20))), dim3(256), 0,
                           st, gfix, grad_data, n, S, 1 + 3 * (g.deg + 1) * (g.deg + 1));
    }
    return hipGetLastError();
}

hipError_t launch_gn(const KGrid& g, const KRays& rs, const KOpts& op, const float* tgt_rgb,
                     const float* tgt_depth, const float* frame_weight, double* gn, hipStream_t st) {
    const dim3 grid(blocks_for(rs.n, 256)), block(256);
    const size_t lds = (256 / WAVE) * MARK_WORDS * WAVE * sizeof(uint32_t);
    by_degree(g.deg, [&](auto D) {
        constexpr int DEG = decltype(D)::value;
        if (op.flags & 1)
            hipLaunchKernelGGL((k_gn<true, DEG>), grid, block, lds, st, g, rs, op, tgt_rgb, tgt_depth,
                               frame_weight, gn);
        else
            hipLaunchKernelGGL((k_gn<false, DEG>), grid, block, lds, st, g, rs, op, tgt_rgb, tgt_depth,
                               frame_weight, gn);
    });
    return hipGetLastError();
}

}  // namespace pxm
