// C ABI of libpxm: host-side argument checks, then one launch per call.
// Nothing here allocates device memory or synchronises a stream.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "../../include/pxm.h"
#include "internal.hpp"

namespace {

thread_local char g_err[512] = "";
// Launch tuning of pxm_render_fused: rays per workgroup in the low 16 bits,
// variant above them, in ONE atomic word so that a reader never sees the
// block of one pxm_set_tuning call with the variant of another.
constexpr int32_t TUNE_DEFAULT = 256;
std::atomic<int32_t> g_tuning{TUNE_DEFAULT};
inline int32_t tune_block(int32_t t) { return t & 0xffff; }
inline int32_t tune_variant(int32_t t) { return t >> 16; }

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

bool finite(float v) { return std::isfinite(v); }

int check_grid(const pxm_grid* g, bool need_payload = true) {
    if (!g) return fail(PXM_INVALID_ARGUMENT, "grid is NULL");
    for (int a = 0; a < 3; ++a) {
        if (g->reso[a] < 2) return fail(PXM_UNSUPPORTED, "grid reso[%d] = %d < 2", a, g->reso[a]);
        if (!finite(g->aabb_min[a])) return fail(PXM_INVALID_ARGUMENT, "aabb_min[%d] not finite", a);
    }
    const long double cells = (long double)g->reso[0] * g->reso[1] * g->reso[2];
    if (cells > 9.0e18L) return fail(PXM_UNSUPPORTED, "lattice too large");
    if (!(g->voxel_size > 0.f) || !finite(g->voxel_size))
        return fail(PXM_INVALID_ARGUMENT, "voxel_size must be finite and > 0");
    if (!g->link) return fail(PXM_INVALID_ARGUMENT, "grid.link is NULL");
    if (g->sh_degree < 0 || g->sh_degree > 2)
        return fail(PXM_INVALID_ARGUMENT, "sh_degree = %d not in {0, 1, 2}", g->sh_degree);
    if (g->n_alloc < 0 || g->n_alloc > 2147483647LL)
        return fail(PXM_INVALID_ARGUMENT, "n_alloc = %lld outside [0, 2^31)", (long long)g->n_alloc);
    if (need_payload && g->n_alloc > 0 && !g->data)
        return fail(PXM_INVALID_ARGUMENT, "grid.data is NULL");
    if (g->data && (reinterpret_cast<uintptr_t>(g->data) & 15))
        return fail(PXM_INVALID_ARGUMENT, "grid.data must be 16-byte aligned");
    if (g->occ && (reinterpret_cast<uintptr_t>(g->occ) & 7))
        return fail(PXM_INVALID_ARGUMENT, "grid.occ must be 8-byte aligned");
    return PXM_OK;
}

int check_rays(const pxm_rays* r) {
    if (!r) return fail(PXM_INVALID_ARGUMENT, "rays is NULL");
    if (r->n_frames < 1) return fail(PXM_INVALID_ARGUMENT, "n_frames = %d < 1", r->n_frames);
    if (r->n_rays < 0) return fail(PXM_INVALID_ARGUMENT, "n_rays < 0");
    if (r->n_rays > 2147483647LL) return fail(PXM_UNSUPPORTED, "n_rays beyond int32 offsets");
    if (!r->c2w || !r->intr || !r->frame_offsets)
        return fail(PXM_INVALID_ARGUMENT, "rays.c2w / intr / frame_offsets is NULL");
    if (r->n_rays > 0 && !r->pix) return fail(PXM_INVALID_ARGUMENT, "rays.pix is NULL");
    return PXM_OK;
}

int check_opts(const pxm_opts* o) {
    if (!o) return fail(PXM_INVALID_ARGUMENT, "opts is NULL");
    if (!(o->step_vox > 0.f) || !finite(o->step_vox))
        return fail(PXM_INVALID_ARGUMENT, "step_vox must be finite and > 0");
    if (o->max_samples < 1) return fail(PXM_INVALID_ARGUMENT, "max_samples < 1");
    if (!(o->t_near >= 0.f) || !finite(o->t_near)) return fail(PXM_INVALID_ARGUMENT, "t_near must be finite and >= 0");
    if (!(o->t_stop >= 0.f && o->t_stop < 1.f)) return fail(PXM_INVALID_ARGUMENT, "t_stop outside [0, 1)");
    if (o->color_act < 0 || o->color_act > 2) return fail(PXM_INVALID_ARGUMENT, "color_act = %d", o->color_act);
    if (o->depth_loss < 0 || o->depth_loss > 1) return fail(PXM_INVALID_ARGUMENT, "depth_loss = %d", o->depth_loss);
    if (!finite(o->lambda_depth)) return fail(PXM_INVALID_ARGUMENT, "lambda_depth not finite");
    if (o->flags & ~PXM_FLAG_POSE_VIEWDIR) return fail(PXM_INVALID_ARGUMENT, "unknown flags 0x%x", o->flags);
    return PXM_OK;
}

pxm::KGrid kgrid(const pxm_grid* g) {
    pxm::KGrid k;
    k.deg = g->sh_degree;
    for (int a = 0; a < 3; ++a) {
        k.R[a] = g->reso[a];
        k.lo[a] = (double)g->aabb_min[a];
    }
    k.sy = g->reso[2];
    k.sx = (int64_t)g->reso[1] * g->reso[2];
    k.vs = g->voxel_size;
    k.inv_vs = 1.0 / (double)g->voxel_size;
    k.n_alloc = g->n_alloc;
    k.link = g->link;
    k.data = g->data;
    int64_t w0, w1;
    pxm::occ_layout(g->reso, w0, k.Q, k.B, w1);
    k.occ0 = reinterpret_cast<const uint64_t*>(g->occ);
    k.occ1 = g->occ ? g->occ + w0 : nullptr;
    return k;
}

pxm::KRays krays(const pxm_rays* r) {
    pxm::KRays k;
    k.F = r->n_frames;
    k.n = r->n_rays;
    k.c2w = r->c2w;
    k.intr = r->intr;
    k.off = r->frame_offsets;
    k.pix = r->pix;
    return k;
}

pxm::KOpts kopts(const pxm_opts* o) {
    pxm::KOpts k;
    k.step_vox = o->step_vox;
    k.max_samples = o->max_samples;
    k.t_near = o->t_near;
    k.t_stop = o->t_stop;
    k.act = o->color_act;
    k.depth_loss = o->depth_loss;
    k.lambda_d = o->lambda_depth;
    k.flags = o->flags;
    return k;
}

int launched(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(PXM_DEVICE_ERROR, "%s: %s", what, hipGetErrorString(e));
    g_err[0] = 0;
    return PXM_OK;
}

#define PXM_TRY(x)                 \
    do {                           \
        int _s = (x);              \
        if (_s != PXM_OK) return _s; \
    } while (0)

}  // namespace

extern "C" {

int pxm_abi_version(void) { return PXM_ABI_VERSION; }

const char* pxm_last_error(void) { return g_err; }

const char* pxm_status_string(int s) {
    switch (s) {
        case PXM_OK: return "ok";
        case PXM_INVALID_ARGUMENT: return "invalid argument";
        case PXM_UNSUPPORTED: return "unsupported";
        case PXM_DEVICE_ERROR: return "device error";
        case PXM_WORKSPACE_TOO_SMALL: return "workspace too small";
        default: return "unknown status";
    }
}

int pxm_set_tuning(int32_t block, int32_t variant) {
    if (block == 0) block = 256;
    if (block != 64 && block != 128 && block != 256)
        return fail(PXM_INVALID_ARGUMENT, "block = %d not in {64,128,256}", block);
    if (variant < 0 || variant > 2) return fail(PXM_INVALID_ARGUMENT, "variant = %d not in {0,1,2}", variant);
    g_tuning.store(block | (variant << 16));
    return PXM_OK;
}

void pxm_get_tuning(int32_t* block, int32_t* variant) {
    const int32_t t = g_tuning.load();
    if (block) *block = tune_block(t);
    if (variant) *variant = tune_variant(t);
}

int pxm_render_forward(const pxm_grid* grid, const pxm_rays* rays, const pxm_opts* opts,
                       float* rgb, float* depth, int32_t* nsamp, void* stream) {
    PXM_TRY(check_grid(grid));
    PXM_TRY(check_rays(rays));
    PXM_TRY(check_opts(opts));
    if (rays->n_rays == 0) return PXM_OK;
    if (!rgb || !depth || !nsamp) return fail(PXM_INVALID_ARGUMENT, "rgb / depth / nsamp is NULL");
    return launched(pxm::launch_forward(kgrid(grid), krays(rays), kopts(opts), rgb, depth, nsamp,
                                        (hipStream_t)stream), "render_forward");
}

int pxm_render_backward_grid(const pxm_grid* grid, const pxm_rays* rays, const pxm_opts* opts,
                             const float* rgb, const float* depth, const int32_t* nsamp,
                             const float* g_rgb, const float* g_depth, float* grad_data,
                             void* stream) {
    PXM_TRY(check_grid(grid));
    PXM_TRY(check_rays(rays));
    PXM_TRY(check_opts(opts));
    if (!grad_data && grid->n_alloc > 0) return fail(PXM_INVALID_ARGUMENT, "grad_data is NULL");
    if (rays->n_rays == 0 || grid->n_alloc == 0) return PXM_OK;   // no record can receive a gradient
    if (!rgb || !depth || !nsamp || !g_rgb || !g_depth)
        return fail(PXM_INVALID_ARGUMENT, "a required array is NULL");
    return launched(pxm::launch_backward(kgrid(grid), krays(rays), kopts(opts), rgb, depth, nsamp,
                                         g_rgb, g_depth, grad_data, nullptr, (hipStream_t)stream),
                    "render_backward_grid");
}

int pxm_render_backward_pose(const pxm_grid* grid, const pxm_rays* rays, const pxm_opts* opts,
                             const float* rgb, const float* depth, const int32_t* nsamp,
                             const float* g_rgb, const float* g_depth, double* grad_pose,
                             void* stream) {
    PXM_TRY(check_grid(grid));
    PXM_TRY(check_rays(rays));
    PXM_TRY(check_opts(opts));
    if (!grad_pose) return fail(PXM_INVALID_ARGUMENT, "grad_pose is NULL");
    if (rays->n_rays == 0) return PXM_OK;
    if (!rgb || !depth || !nsamp || !g_rgb || !g_depth)
        return fail(PXM_INVALID_ARGUMENT, "a required array is NULL");
    return launched(pxm::launch_backward(kgrid(grid), krays(rays), kopts(opts), rgb, depth, nsamp,
                                         g_rgb, g_depth, nullptr, grad_pose, (hipStream_t)stream),
                    "render_backward_pose");
}

static int tv_grad(const pxm_grid* grid, float lambda_density, float lambda_sh, float eps,
                   float* grad_data, bool set, void* stream) {
    PXM_TRY(check_grid(grid));
    if (!grad_data && grid->n_alloc > 0) return fail(PXM_INVALID_ARGUMENT, "grad_data is NULL");
    if (!finite(lambda_density) || !finite(lambda_sh))
        return fail(PXM_INVALID_ARGUMENT, "lambda not finite");
    if (!(eps > 0.f) || !finite(eps)) return fail(PXM_INVALID_ARGUMENT, "eps must be finite and > 0");
    if (grid->n_alloc == 0) return PXM_OK;                          // no vertex has a term
    if (reinterpret_cast<uintptr_t>(grad_data) & 15)
        return fail(PXM_INVALID_ARGUMENT, "grad_data must be 16-byte aligned");
    return launched(pxm::launch_tv(kgrid(grid), lambda_density, lambda_sh, eps, grad_data, set,
                                   (hipStream_t)stream), set ? "tv_grad_set" : "tv_grad");
}

int pxm_tv_grad(const pxm_grid* grid, float lambda_density, float lambda_sh, float eps,
                float* grad_data, void* stream) {
    return tv_grad(grid, lambda_density, lambda_sh, eps, grad_data, false, stream);
}

int pxm_tv_grad_set(const pxm_grid* grid, float lambda_density, float lambda_sh, float eps,
                    float* grad_data, void* stream) {
    return tv_grad(grid, lambda_density, lambda_sh, eps, grad_data, true, stream);
}

size_t pxm_occupancy_words(const pxm_grid* grid) {
    if (check_grid(grid, false) != PXM_OK) return 0;
    int64_t w0, w1;
    int Q[3], B[3];
    pxm::occ_layout(grid->reso, w0, Q, B, w1);
    return (size_t)(w0 + w1);
}

int pxm_build_occupancy(const pxm_grid* grid, uint32_t* occ, size_t n_words, void* stream) {
    PXM_TRY(check_grid(grid, false));
    if (!occ) return fail(PXM_INVALID_ARGUMENT, "occ is NULL");
    if (reinterpret_cast<uintptr_t>(occ) & 7) return fail(PXM_INVALID_ARGUMENT, "occ must be 8-byte aligned");
    const size_t need = pxm_occupancy_words(grid);
    if (n_words < need) return fail(PXM_WORKSPACE_TOO_SMALL, "occ has %zu < %zu words", n_words, need);
    pxm::KGrid k = kgrid(grid);
    k.occ0 = nullptr;
    k.occ1 = nullptr;
    return launched(pxm::launch_occupancy(k, occ, (hipStream_t)stream), "build_occupancy");
}

size_t pxm_workspace_bytes(const pxm_grid* grid, const pxm_rays* rays, const pxm_opts* opts,
                           int32_t want) {
    (void)opts;
    size_t b = pxm::fused_workspace_bytes(rays && rays->n_rays > 0 ? rays->n_rays : 0);
    if ((want & PXM_WANT_DETERMINISTIC) && (want & PXM_WANT_GRID) && grid && grid->n_alloc > 0 &&
        grid->sh_degree >= 0 && grid->sh_degree <= 2)
        b += pxm::fix_bytes(grid->n_alloc, PXM_RECORD_FLOATS(grid->sh_degree));
    return b;
}

int pxm_render_fused(const pxm_grid* grid, const pxm_rays* rays, const pxm_opts* opts,
                     const float* tgt_rgb, const float* tgt_depth, const float* frame_weight,
                     int32_t want, float* rgb, float* depth, double* loss, float* grad_data,
                     double* grad_pose, int64_t* stats, void* ws, size_t ws_bytes, void* stream) {
    PXM_TRY(check_grid(grid));
    PXM_TRY(check_rays(rays));
    PXM_TRY(check_opts(opts));
    if (want & ~(PXM_WANT_GRID | PXM_WANT_POSE | PXM_WANT_STATS | PXM_WANT_DETERMINISTIC))
        return fail(PXM_INVALID_ARGUMENT, "unknown want bits 0x%x", want);
    if (rays->n_rays > 0 && (!tgt_rgb || !tgt_depth || !frame_weight))
        return fail(PXM_INVALID_ARGUMENT, "targets / frame_weight is NULL");
    if ((want & PXM_WANT_GRID) && !grad_data && grid->n_alloc > 0)
        return fail(PXM_INVALID_ARGUMENT, "grad_data is NULL");
    if ((want & PXM_WANT_POSE) && !grad_pose) return fail(PXM_INVALID_ARGUMENT, "grad_pose is NULL");
    if ((want & PXM_WANT_STATS) && !stats) return fail(PXM_INVALID_ARGUMENT, "stats is NULL");
    const size_t need = pxm_workspace_bytes(grid, rays, opts, want);
    if (!ws) return fail(PXM_INVALID_ARGUMENT, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(PXM_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(PXM_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, need);
    if (rays->n_rays == 0) return PXM_OK;
    const int32_t tune = g_tuning.load();
    const int block = tune_block(tune), variant = tune_variant(tune);
    unsigned long long* gfix = nullptr;
    if ((want & PXM_WANT_DETERMINISTIC) && (want & PXM_WANT_GRID) && grid->n_alloc > 0)
        gfix = reinterpret_cast<unsigned long long*>(static_cast<char*>(ws) +
                                                     pxm::fused_workspace_bytes(rays->n_rays));
    return launched(pxm::launch_fused(kgrid(grid), krays(rays), kopts(opts), tgt_rgb, tgt_depth,
                                      frame_weight, want, rgb, depth, loss, grad_data, grad_pose,
                                      stats, reinterpret_cast<unsigned*>(ws), block, variant, gfix,
                                      (hipStream_t)stream), "render_fused");
}

int pxm_pose_adam(int32_t n_frames, float* c2w, double* grad_pose, double* state, float lr,
                  float beta1, float beta2, float eps, void* stream) {
    if (n_frames < 1) return fail(PXM_INVALID_ARGUMENT, "n_frames < 1");
    if (!c2w || !grad_pose || !state) return fail(PXM_INVALID_ARGUMENT, "a required array is NULL");
    if (!(lr >= 0.f) || !finite(lr)) return fail(PXM_INVALID_ARGUMENT, "lr must be finite and >= 0");
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
        return fail(PXM_INVALID_ARGUMENT, "betas outside [0, 1)");
    if (!(eps > 0.f) || !finite(eps)) return fail(PXM_INVALID_ARGUMENT, "eps must be finite and > 0");
    return launched(pxm::launch_adam(n_frames, c2w, grad_pose, state, lr, beta1, beta2, eps,
                                     (hipStream_t)stream), "pose_adam");
}

int pxm_render_gn(const pxm_grid* grid, const pxm_rays* rays, const pxm_opts* opts,
                  const float* tgt_rgb, const float* tgt_depth, const float* frame_weight,
                  double* gn, void* stream) {
    PXM_TRY(check_grid(grid));
    PXM_TRY(check_rays(rays));
    PXM_TRY(check_opts(opts));
    if (!gn) return fail(PXM_INVALID_ARGUMENT, "gn is NULL");
    if (rays->n_rays > 0 && (!tgt_rgb || !tgt_depth || !frame_weight))
        return fail(PXM_INVALID_ARGUMENT, "targets / frame_weight is NULL");
    if (rays->n_rays == 0) return PXM_OK;
    return launched(pxm::launch_gn(kgrid(grid), krays(rays), kopts(opts), tgt_rgb, tgt_depth,
                                   frame_weight, gn, (hipStream_t)stream), "render_gn");
}

int pxm_pose_gn(int32_t n_frames, float* c2w, double* gn, float damping, void* stream) {
    if (n_frames < 1) return fail(PXM_INVALID_ARGUMENT, "n_frames < 1");
    if (!c2w || !gn) return fail(PXM_INVALID_ARGUMENT, "a required array is NULL");
    if (!(damping >= 0.f) || !finite(damping))
        return fail(PXM_INVALID_ARGUMENT, "damping must be finite and >= 0");
    return launched(pxm::launch_pose_gn(n_frames, c2w, gn, damping, (hipStream_t)stream), "pose_gn");
}

int pxm_grid_rmsprop(int64_t n_alloc, int32_t sh_degree, float* data, float* grad_data, float* state,
                     float lr_density, float lr_sh, float alpha, float eps, void* stream) {
    if (n_alloc < 0 || n_alloc > INT32_MAX) return fail(PXM_INVALID_ARGUMENT, "n_alloc outside [0, 2^31)");
    if (sh_degree < 0 || sh_degree > 2)
        return fail(PXM_INVALID_ARGUMENT, "sh_degree = %d not in {0, 1, 2}", sh_degree);
    if (!finite(lr_density) || !finite(lr_sh) || !(lr_density >= 0.f) || !(lr_sh >= 0.f))
        return fail(PXM_INVALID_ARGUMENT, "learning rates must be finite and >= 0");
    if (!(alpha >= 0.f && alpha < 1.f)) return fail(PXM_INVALID_ARGUMENT, "alpha outside [0, 1)");
    if (!(eps > 0.f) || !finite(eps)) return fail(PXM_INVALID_ARGUMENT, "eps must be finite and > 0");
    if (n_alloc == 0) return PXM_OK;
    if (!data || !grad_data || !state) return fail(PXM_INVALID_ARGUMENT, "a required array is NULL");
    if (((uintptr_t)data | (uintptr_t)grad_data | (uintptr_t)state) & 15u)
        return fail(PXM_INVALID_ARGUMENT, "data, grad_data and state must be 16-byte aligned");
    return launched(pxm::launch_rmsprop(n_alloc, sh_degree, data, grad_data, state, lr_density, lr_sh,
                                        alpha, eps, (hipStream_t)stream), "grid_rmsprop");
}

size_t pxm_grid_edit_workspace_bytes(const pxm_grid* grid) {
    if (check_grid(grid, false) != PXM_OK) return 0;
    const size_t up = pxm::grow_workspace_bytes(grid->reso);
    const size_t pr = pxm::prune_workspace_bytes(grid->n_alloc);
    return up > pr ? up : pr;
}

namespace {

int check_edit_ws(const pxm_grid* grid, void* ws, size_t ws_bytes) {
    const size_t need = pxm_grid_edit_workspace_bytes(grid);
    if (ws_bytes < need) return fail(PXM_WORKSPACE_TOO_SMALL, "ws_bytes = %zu < %zu", ws_bytes, need);
    if (!ws) return fail(PXM_INVALID_ARGUMENT, "ws is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(PXM_INVALID_ARGUMENT, "ws must be 256-byte aligned");
    return PXM_OK;
}

int64_t fine_vertices(const pxm_grid* grid) {
    return (int64_t)(2 * grid->reso[0] - 1) * (2 * grid->reso[1] - 1) * (2 * grid->reso[2] - 1);
}

}  // namespace

int pxm_grid_upsample_link(const pxm_grid* grid, int32_t* link_fine, int64_t* n_fine, void* ws, size_t ws_bytes,
                           void* stream) {
    PXM_TRY(check_grid(grid, false));
    for (int a = 0; a < 3; ++a)
        if (grid->reso[a] > 1073741823) return fail(PXM_UNSUPPORTED, "reso[%d] too large to double", a);
    if (fine_vertices(grid) > 2147483647LL)
        return fail(PXM_UNSUPPORTED, "doubled lattice has more than 2^31 - 1 vertices");
    if (!link_fine || !n_fine) return fail(PXM_INVALID_ARGUMENT, "link_fine / n_fine is NULL");
    PXM_TRY(check_edit_ws(grid, ws, ws_bytes));
    return launched(pxm::launch_upsample_link(kgrid(grid), link_fine, n_fine, ws, (hipStream_t)stream),
                    "grid_upsample_link");
}

int pxm_grid_upsample_data(const pxm_grid* grid, const int32_t* link_fine, int64_t n_fine, float* data_fine,
                           void* stream) {
    PXM_TRY(check_grid(grid, true));
    for (int a = 0; a < 3; ++a)
        if (grid->reso[a] > 1073741823) return fail(PXM_UNSUPPORTED, "reso[%d] too large to double", a);
    if (fine_vertices(grid) > 2147483647LL)
        return fail(PXM_UNSUPPORTED, "doubled lattice has more than 2^31 - 1 vertices");
    if (!link_fine) return fail(PXM_INVALID_ARGUMENT, "link_fine is NULL");
    if (n_fine < 0 || n_fine > fine_vertices(grid))
        return fail(PXM_INVALID_ARGUMENT, "n_fine = %lld outside [0, fine vertices]", (long long)n_fine);
    if (n_fine == 0) return PXM_OK;
    if (!data_fine) return fail(PXM_INVALID_ARGUMENT, "data_fine is NULL");
    if (reinterpret_cast<uintptr_t>(data_fine) & 15)
        return fail(PXM_INVALID_ARGUMENT, "data_fine must be 16-byte aligned");
    return launched(pxm::launch_upsample_data(kgrid(grid), link_fine, n_fine, data_fine, (hipStream_t)stream),
                    "grid_upsample_data");
}

int pxm_grid_prune(const pxm_grid* grid, float tau, int32_t* link_out, float* data_out, int64_t* n_out, void* ws,
                   size_t ws_bytes, void* stream) {
    PXM_TRY(check_grid(grid, true));
    if (std::isnan(tau)) return fail(PXM_INVALID_ARGUMENT, "tau is NaN");
    if (!link_out || !n_out) return fail(PXM_INVALID_ARGUMENT, "link_out / n_out is NULL");
    const int64_t nv = (int64_t)grid->reso[0] * grid->reso[1] * grid->reso[2];
    if (link_out != grid->link) {
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(link_out), a1 = a0 + 4 * (uintptr_t)nv;
        const uintptr_t b0 = reinterpret_cast<uintptr_t>(grid->link), b1 = b0 + 4 * (uintptr_t)nv;
        if (a0 < b1 && b0 < a1) return fail(PXM_INVALID_ARGUMENT, "link_out partly overlaps grid.link");
    }
    if (grid->n_alloc > 0) {
        if (!data_out) return fail(PXM_INVALID_ARGUMENT, "data_out is NULL");
        if (reinterpret_cast<uintptr_t>(data_out) & 15)
            return fail(PXM_INVALID_ARGUMENT, "data_out must be 16-byte aligned");
        const uintptr_t bytes = (uintptr_t)grid->n_alloc * PXM_RECORD_FLOATS(grid->sh_degree) * 4;
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(data_out), b0 = reinterpret_cast<uintptr_t>(grid->data);
        if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(PXM_INVALID_ARGUMENT, "data_out overlaps grid.data");
    }
    PXM_TRY(check_edit_ws(grid, ws, ws_bytes));
    return launched(pxm::launch_prune(kgrid(grid), tau, link_out, data_out, n_out, ws, (hipStream_t)stream),
                    "grid_prune");
}

}  // extern "C"

namespace pxm {
// probe.hip: n_wg workgroups of 256 (a multiple of 8), `passes` reads of the
// n4 float4s, XCD x reading its own eighth
hipError_t launch_probe_read(const float4* buf, int64_t n4, int passes, float* sink, int n_wg,
                             hipStream_t st);
}  // namespace pxm

extern "C" {

int pxm_probe_read_bandwidth(const void* buf, size_t bytes, int32_t passes, float* sink,
                             size_t sink_floats, void* stream) {
    if (!buf || !sink) return fail(PXM_INVALID_ARGUMENT, "buf / sink is NULL");
    if (reinterpret_cast<uintptr_t>(buf) & 15) return fail(PXM_INVALID_ARGUMENT, "buf must be 16-byte aligned");
    if (bytes < 128 || (bytes % 128) != 0) return fail(PXM_INVALID_ARGUMENT, "bytes must be a positive multiple of 128");
    if (passes < 1) return fail(PXM_INVALID_ARGUMENT, "passes < 1");
    const int n_wg = 2048;                                  // a multiple of the 8 XCDs
    if (sink_floats < (size_t)n_wg * 256)
        return fail(PXM_WORKSPACE_TOO_SMALL, "sink needs %d floats", n_wg * 256);
    return launched(pxm::launch_probe_read(static_cast<const float4*>(buf), (int64_t)(bytes / 16), passes, sink,
                                           n_wg, (hipStream_t)stream), "probe_read_bandwidth");
}

// ---------------------------------------------------------------------------
// Allocation-free fused step: the workspace is a file-scope device array.
// ---------------------------------------------------------------------------

// One copy per GPU, alive until the process ends.  Host code must never pass
// `scratch` itself to a kernel (in host code it names a host-side stand-in):
// its device address is looked up once per device and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[PXM_NOALLOC_SCRATCH_BYTES];

static_assert(pxm::FUSED_WS_BYTES + (size_t)PXM_NOALLOC_MAX_SPLIT_RAYS * pxm::SPLIT_BYTES_PER_RAY
                  <= (size_t)PXM_NOALLOC_SCRATCH_BYTES
              && PXM_NOALLOC_MAX_SPLIT_RAYS % 64 == 0
              && pxm::FUSED_WS_BYTES + ((size_t)PXM_NOALLOC_MAX_SPLIT_RAYS + 64) * pxm::SPLIT_BYTES_PER_RAY
                  > (size_t)PXM_NOALLOC_SCRATCH_BYTES,
              "PXM_NOALLOC_MAX_SPLIT_RAYS is the largest ray count whose split state fits the scratch");

namespace {

constexpr int MAX_DEVICES = 64;
std::atomic<void*> g_scratch[MAX_DEVICES];
std::mutex g_scratch_mu;

// Device address of this device's scratch array, looked up on first use with
// the device current.
int scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PXM_DEVICE_ERROR, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(PXM_UNSUPPORTED, "device %d beyond %d", dev, MAX_DEVICES);
    void* p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        p = g_scratch[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(PXM_DEVICE_ERROR, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            g_scratch[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return PXM_OK;
}

// Clears the tile-queue counters with a kernel (not a memset node, so the
// call stays capturable).
__global__ void k_clear_counters(unsigned* w, int n) {
    const int i = (int)threadIdx.x;
    if (i < n) w[i] = 0u;
}

}  // namespace

int pxm_render_fused_noalloc(const pxm_grid* grid, const pxm_rays* rays, const pxm_opts* opts,
                             const float* tgt_rgb, const float* tgt_depth, const float* frame_weight,
                             int32_t want, float* rgb, float* depth, double* loss, float* grad_data,
                             double* grad_pose, int64_t* stats, void* stream) {
    PXM_TRY(check_grid(grid));
    PXM_TRY(check_rays(rays));
    PXM_TRY(check_opts(opts));
    if (want & PXM_WANT_DETERMINISTIC)
        return fail(PXM_UNSUPPORTED, "the deterministic scatter needs a workspace: use pxm_render_fused");
    if (want & ~(PXM_WANT_GRID | PXM_WANT_POSE | PXM_WANT_STATS))
        return fail(PXM_INVALID_ARGUMENT, "unknown want bits 0x%x", want);
    if (rays->n_rays > 0 && (!tgt_rgb || !tgt_depth || !frame_weight))
        return fail(PXM_INVALID_ARGUMENT, "targets / frame_weight is NULL");
    if ((want & PXM_WANT_GRID) && !grad_data && grid->n_alloc > 0)
        return fail(PXM_INVALID_ARGUMENT, "grad_data is NULL");
    if ((want & PXM_WANT_POSE) && !grad_pose) return fail(PXM_INVALID_ARGUMENT, "grad_pose is NULL");
    if ((want & PXM_WANT_STATS) && !stats) return fail(PXM_INVALID_ARGUMENT, "stats is NULL");
    const int32_t tune = g_tuning.load();
    const int block = tune_block(tune), variant = tune_variant(tune);
    // the two-launch form keeps per-ray state in the scratch; the others only
    // the queue counters
    const size_t need = variant == 2 ? pxm::fused_workspace_bytes(rays->n_rays) : pxm::FUSED_WS_BYTES;
    if (need > (size_t)PXM_NOALLOC_SCRATCH_BYTES)
        return fail(PXM_UNSUPPORTED,
                    "%lld rays need %zu bytes of scratch in the two-launch form, above the %zu-byte "
                    "static scratch (at most %lld rays; use pxm_render_fused with a workspace, or "
                    "launch variant 0 or 1)",
                    (long long)rays->n_rays, need, (size_t)PXM_NOALLOC_SCRATCH_BYTES,
                    (long long)PXM_NOALLOC_MAX_SPLIT_RAYS);
    if (rays->n_rays == 0) return PXM_OK;
    void* ws = nullptr;
    PXM_TRY(scratch_ptr(&ws));
    const hipStream_t st = (hipStream_t)stream;
    unsigned* counters = reinterpret_cast<unsigned*>(ws);
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(64), 0, st, counters,
                       (int)(pxm::FUSED_WS_BYTES / sizeof(unsigned)));
    PXM_TRY(launched(hipGetLastError(), "render_fused_noalloc (clear)"));
    return launched(pxm::launch_fused(kgrid(grid), krays(rays), kopts(opts), tgt_rgb, tgt_depth,
                                      frame_weight, want, rgb, depth, loss, grad_data, grad_pose,
                                      stats, counters, block, variant, nullptr, st),
                    "render_fused_noalloc");
}

}  // extern "C"
