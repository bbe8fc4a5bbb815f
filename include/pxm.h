/*
 * pxm.h -- C ABI of the MI355X (gfx950) kernels for differentiable volume
 * rendering of a sparse voxel grid, the hot path of "RGB-D Mapping and
 * Tracking in a Plenoxel Radiance Field" (Teigen et al., WACV 2024).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.   Every array pointer is DEVICE memory owned by the caller; the
 *           library never allocates, frees or retains it.  Descriptors
 *           (pxm_grid, pxm_rays, pxm_opts) are HOST structs read during the
 *           call only.  Scratch space, where an entry point needs any, comes
 *           from a caller-provided workspace sized by pxm_workspace_bytes.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *           stream).  Calls only enqueue work and return; results are ready
 *           when the stream is synchronised.  Nothing inside allocates or
 *           synchronises, so every call may be captured into a HIP graph.
 * Outputs.  rgb / depth / nsamp / loss are overwritten.  Every gradient
 *           output ACCUMULATES (+=): zero it before the first contribution.
 * Errors.   Each call returns PXM_OK (0) or a positive pxm_status.  All
 *           argument checks run on the host before anything is enqueued, so
 *           a rejected call has no effect.  With n_rays == 0 a render call
 *           is a no-op and its per-ray arrays may be NULL.  pxm_last_error() returns a
 *           thread-local description of the last failure.  A fault in a
 *           kernel surfaces at the caller's next stream synchronisation.
 *           Device-resident metadata (frame_offsets) cannot be checked on the
 *           host; kernels clamp every index they derive from it so a
 *           malformed CSR yields wrong numbers, never an out-of-bounds access.
 *
 * Grid (Sec. 5.2, model representation).  A lattice of Rx x Ry x Rz
 * vertices; vertex (i,j,k) sits at aabb_min + voxel_size * (i,j,k).  Each
 * allocated vertex holds the density followed by the spherical-harmonic
 * coefficients of each colour channel: at the paper's degree 2, nine per
 * channel in a record of 28 floats (record[1+9c+k]).  Lower degrees d = 0, 1
 * keep the first (d+1)^2 functions of the same basis per channel
 * (record[1+(d+1)^2 c+k]) in records of PXM_RECORD_FLOATS(d) = 4 or 16 floats
 * (at d = 1 the last three floats are padding: never read as SH, never given
 * a gradient).  Samples are trilinearly interpolated from the 8 closest
 * vertices (Fig. 4, Appendix A); an empty vertex (link -1) reads as zero.
 *
 * Ray model (Sec. 4).  Pixel (u,v) of frame f defines
 *   d_cam = ((u + 0.5 - cx) / fx, (v + 0.5 - cy) / fy, 1)  (OpenCV axes),
 *   d = R d_cam / |d_cam|,  o = t,  with c2w[f] = [R | t] row-major 3x4.
 * Samples sit at distances t_k = t_near + k * step_vox * voxel_size from o,
 * k = 0, 1, ...; a sample is kept while its position lies inside the vertex
 * box [0, R-1]^3 (voxel units), at most max_samples positions counted from
 * the first kept one.  delta = step_vox is the sample spacing in the
 * exponent, with density in per-voxel units.
 */
#ifndef PXM_H
#define PXM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PXM_ABI_VERSION 7   /* 7: pxm_tv_grad_set; 6: SH degree 0/1 records (pxm_grid.sh_degree) */
#define PXM_RECORD 28          /* floats per vertex at SH degree 2: density + 3 x 9 SH */
#define PXM_RECORD_FLOATS(d) ((d) == 0 ? 4 : (d) == 1 ? 16 : 28)   /* per SH degree */

typedef enum {
    PXM_OK = 0,
    PXM_INVALID_ARGUMENT = 1,    /* null pointer, bad enum, non-finite or out-of-range scalar */
    PXM_UNSUPPORTED = 2,         /* valid but outside what the kernels handle (e.g. R < 2) */
    PXM_DEVICE_ERROR = 3,        /* the HIP runtime refused a launch */
    PXM_WORKSPACE_TOO_SMALL = 4  /* ws_bytes below pxm_workspace_bytes() */
} pxm_status;

/* Colour activation c = act(s) applied to the SH sum s (the paper leaves it open). */
enum { PXM_COLOR_RELU_SHIFT = 0,   /* max(s + 0.5, 0) */
       PXM_COLOR_SIGMOID = 1,      /* 1 / (1 + exp(-s)) */
       PXM_COLOR_IDENTITY = 2 };   /* s */

/* Penalty rho on the z-depth residual: Eq. 5 is squared; L1 is the metric of Sec. 6.1. */
enum { PXM_DEPTH_L1 = 0, PXM_DEPTH_L2 = 1 };

/* pxm_opts.flags */
enum { PXM_FLAG_POSE_VIEWDIR = 1 };  /* add the exact d(colour)/d(view direction) term to the
                                        rotation gradient; Eq. 12 omits it (default off) */

/* pxm_render_fused `want` bits */
enum { PXM_WANT_GRID = 1,    /* accumulate grad_data */
       PXM_WANT_POSE = 2,    /* accumulate grad_pose */
       PXM_WANT_STATS = 4,   /* accumulate the traffic counters into `stats` */
       PXM_WANT_DETERMINISTIC = 8 };  /* with PXM_WANT_GRID: order-independent grid gradient
                                         (a debug and race-detection mode; see pxm_render_fused) */

typedef struct {
    int32_t reso[3];        /* vertices per axis, each >= 2 */
    float aabb_min[3];      /* world position of vertex (0,0,0) */
    float voxel_size;       /* world edge length of one voxel, > 0 */
    const int32_t *link;    /* [Rx*Ry*Rz], index (x*Ry + y)*Rz + z -> record id or -1 */
    int64_t n_alloc;        /* number of records (0: an empty map, every link -1) */
    const float *data;      /* [n_alloc][PXM_RECORD_FLOATS(sh_degree)], 16-byte aligned; may be
                               NULL when n_alloc == 0, as may every grad_data argument (grad_data
                               arrays have the same layout as data) */
    const uint32_t *occ;    /* optional occupancy bitfield from pxm_build_occupancy for THIS
                               link table (8-byte aligned), or NULL.  Lets the march step over
                               empty cells, 4^3-cell blocks and 8^3-cell bricks; results are
                               identical with or without it. */
    int32_t sh_degree;      /* SH degree of the records: 2 (the paper's), 1 or 0 */
} pxm_grid;

typedef struct {
    int32_t n_frames;              /* F >= 1 */
    const float *c2w;              /* [F][3][4] camera-to-world, row-major */
    const float *intr;             /* [F][4] fx, fy, cx, cy (pixels) */
    int64_t n_rays;                /* total rays, >= 0 */
    const int32_t *frame_offsets;  /* [F+1] CSR: rays of frame f are [off[f], off[f+1]),
                                      off[0] = 0, non-decreasing, off[F] = n_rays */
    const int32_t *pix;            /* [n_rays][2] pixel (u, v) */
} pxm_rays;

typedef struct {
    float step_vox;         /* sample spacing in voxels, > 0 (0.5 in every workload here) */
    int32_t max_samples;    /* cap on kept sample positions per ray, >= 1 */
    float t_near;           /* distance of sample k = 0 from the camera centre, >= 0 */
    float t_stop;           /* stop after sample i once T_{i+1} < t_stop; 0 <= t_stop < 1 */
    int32_t color_act;      /* PXM_COLOR_* */
    int32_t depth_loss;     /* PXM_DEPTH_* (used by pxm_render_fused) */
    float lambda_depth;     /* lambda_d of Eq. 11 (used by pxm_render_fused) */
    int32_t flags;          /* PXM_FLAG_* */
} pxm_opts;

/*
 * Forward render, Eq. 1-3 (Sec. 4).  For every ray: the composited colour
 * C-hat = sum_i T_i (1 - exp(-sigma_i delta)) c_i, the expected depth
 * D-hat = sum_i T_i (1 - exp(-sigma_i delta)) t_i reported as z-depth
 * D-hat / |d_cam|, and the number of sample positions kept (nsamp), which
 * the backward passes replay.  sigma_i = max(interpolated density, 0),
 * c_i = act(sum_k Y_k(d) * interpolated SH_k) per channel.
 *   rgb   [n_rays][3] f32 out,   depth [n_rays] f32 out,   nsamp [n_rays] i32 out
 */
int pxm_render_forward(const pxm_grid *grid, const pxm_rays *rays, const pxm_opts *opts,
                       float *rgb, float *depth, int32_t *nsamp, void *stream);

/*
 * Mapping backward, Eq. 6-10 (Sec. 5.2).  Given the forward outputs and the
 * upstream gradients g_rgb = dL/dC-hat [n_rays][3] and g_depth = dL/d(z-depth)
 * [n_rays], recomputes each ray's samples and adds
 *   dL/d sigma_raw,i = 1[sigma_raw,i > 0] delta [g_C.(c_i T_{i+1} - C-hat + sum_{j<=i} c_j w_j)
 *                                                + g_D (t_i T_{i+1} - D-hat + sum_{j<=i} t_j w_j)]
 *   dL/d SH_k,c,i    = act'(s_c,i) w_i g_C,c Y_k(d)
 * through the trilinear weights into grad_data [n_alloc][S] (accumulated;
 * empty vertices receive nothing).  Rays with all-zero upstream gradients are skipped.
 */
int pxm_render_backward_grid(const pxm_grid *grid, const pxm_rays *rays, const pxm_opts *opts,
                             const float *rgb, const float *depth, const int32_t *nsamp,
                             const float *g_rgb, const float *g_depth, float *grad_data,
                             void *stream);

/*
 * Tracking backward, Eq. 12-14 (Sec. 5.3) with the Appendix A spatial
 * gradients of the trilinear interpolant.  For each ray,
 *   g_p,i = dL/d sigma_raw,i * grad sigma_raw(p_i) + sum_c dL/ds_c,i * grad s_c(p_i),
 *   g_o = sum_i g_p,i,  g_d = sum_i t_i g_p,i   (dp/do = 1, dp/dd = t_i),
 * and the gradient with respect to a left, world-frame perturbation
 * exp(xi^) c2w, xi = (rho, phi), is (g_o, o x g_o + d x g_d); these are summed
 * over each frame's rays into grad_pose [F][6] (float64, accumulated).  With
 * PXM_FLAG_POSE_VIEWDIR the exact term d x (dL/dd through the SH basis) is
 * added to phi.
 */
int pxm_render_backward_pose(const pxm_grid *grid, const pxm_rays *rays, const pxm_opts *opts,
                             const float *rgb, const float *depth, const int32_t *nsamp,
                             const float *g_rgb, const float *g_depth, double *grad_pose,
                             void *stream);

/*
 * Total-variation gradient over the allocated vertices (the Plenoxel-style
 * regulariser; the paper does not define one):
 *   TV = sum_m lambda_m sum_v sqrt(dx_m(v)^2 + dy_m(v)^2 + dz_m(v)^2 + eps),
 * forward differences to the +x/+y/+z neighbours (empty reads as 0), v
 * allocated and not on an upper face, lambda_0 = lambda_density for the
 * density field and lambda_sh for each SH field (27 at degree 2).  dTV/d
 * record is added into grad_data [n_alloc][S] (accumulated, gather form: one writer
 * per vertex, no atomics).  With grid->occ set, 8^3 bricks whose cells have
 * no allocated corner are skipped.
 */
int pxm_tv_grad(const pxm_grid *grid, float lambda_density, float lambda_sh, float eps,
                float *grad_data, void *stream);

/*
 * The same TV gradient written instead of added: for every allocated vertex
 * the link table reaches, grad_data[v][m] = dTV/d val_m(v) for its used
 * fields m < 1 + 3 (d+1)^2; the padding fields of a record, and records no
 * link reaches, are left as they are.  Arguments and errors as
 * pxm_tv_grad.  It saves reading grad_data: a step that zeroes the gradient
 * can call this first and then let pxm_render_fused add the rendering
 * gradient onto it.
 */
int pxm_tv_grad_set(const pxm_grid *grid, float lambda_density, float lambda_sh, float eps,
                    float *grad_data, void *stream);

/*
 * Fused batched step: forward (Eq. 1-3), the loss of Eq. 4, 5 and 11, and the
 * mapping and/or tracking backward for every ray of every frame in ONE
 * launch.  A ray whose target depth is non-finite or <= 0 is dropped from
 * the loss (Sec. 6.1).  Per frame f, with w_f = frame_weight[f] (1/M):
 *   L_f = w_f sum_r |C-hat_r - C_r|^2 + lambda_depth w_f sum_r rho(z_r - D_r).
 *   tgt_rgb [n_rays][3], tgt_depth [n_rays], frame_weight [F]      (in)
 *   rgb, depth   [n_rays][3], [n_rays]       (out, may be NULL)
 *   loss         [F] float64                 (accumulated, may be NULL)
 *   grad_data    [n_alloc][S]                (accumulated; required with PXM_WANT_GRID)
 *   grad_pose    [F][6] float64              (accumulated; required with PXM_WANT_POSE)
 *   stats        [4] int64                   (accumulated with PXM_WANT_STATS:
 *                 occupied samples, allocated corners of those, allocated
 *                 corners that received a gradient, rays with a valid target)
 * ws / ws_bytes: device workspace of at least pxm_workspace_bytes(..., want)
 *   bytes, 256-byte aligned: the tile-queue counters of the persistent launch
 *   forms (first 256 bytes), then the per-ray state that the two-launch form
 *   hands from its forward launch to its backward launch (184 bytes per ray).
 *   The counters must be zeroed before the first use; every call leaves them
 *   zeroed again (the per-ray state needs no initialisation).  Calls that
 *   share one workspace must not run concurrently.
 * PXM_WANT_DETERMINISTIC (with PXM_WANT_GRID): each merged grid-gradient
 *   contribution is rounded to a fixed-point integer (units of 2^-48) and
 *   summed with 64-bit integer atomics, which commute exactly; a last pass
 *   adds every integer sum, converted once, into grad_data.  The result is
 *   bit-for-bit the same whatever the order in which waves run, the launch
 *   tuning or the run; it differs from the float-atomic result by rounding
 *   only (each contribution within 2^-49, each entry within +-32768).  The
 *   workspace then also holds the [n_alloc][S] int64 fixed-point buffer
 *   (pxm_workspace_bytes with the same `want`), which must be zeroed before
 *   the first use and is left zeroed.
 */
int pxm_render_fused(const pxm_grid *grid, const pxm_rays *rays, const pxm_opts *opts,
                     const float *tgt_rgb, const float *tgt_depth, const float *frame_weight,
                     int32_t want, float *rgb, float *depth, double *loss, float *grad_data,
                     double *grad_pose, int64_t *stats, void *ws, size_t ws_bytes, void *stream);

/*
 * Tracking update (Sec. 5.4: Adam for tracking): per frame, one Adam step
 * (beta1, beta2, eps; bias-corrected with the frame's own step counter) on
 * the se(3) tangent xi = -lr m_hat / (sqrt(v_hat) + eps), then the left
 * retraction c2w <- exp(xi^) c2w.  grad_pose is read and then zeroed, so a
 * captured graph needs no separate clearing node.
 *   c2w [F][3][4] f32 (in/out), grad_pose [F][6] f64 (in, zeroed),
 *   state [F][16] f64 (in/out: m[6], v[6], step count, 3 unused; start zeroed)
 */
int pxm_pose_adam(int32_t n_frames, float *c2w, double *grad_pose, double *state, float lr,
                  float beta1, float beta2, float eps, void *stream);

/*
 * Gauss-Newton tracking, normal equations (Sec. 5.3, Eq. 12-14 and App. A;
 * the squared form of Eq. 4, 5 and 11).  Per ray with a valid depth target:
 * the forward (Eq. 1-3), the residual e = (C-hat - C, z - D) and the pose
 * Jacobian J [4][6] of (R, G, B, z-depth) with respect to the left se(3)
 * perturbation (rho, phi), whose row k is the pose gradient of output k
 * alone.  Per frame f, with w_f = frame_weight[f] and
 * W = w_f diag(1, 1, 1, lambda_depth):
 *   gn[f][0..20]  += sum_r (J^T W J)_ij, upper triangle row by row
 *                    (i <= j: (0,0), (0,1), .., (0,5), (1,1), .., (5,5)),
 *   gn[f][21..26] += sum_r (J^T W e)_i,
 *   gn[f][27]     += sum_r e^T W e.
 * gn is [F][28] float64, accumulated.  opts->depth_loss is not used (the
 * Gauss-Newton energy is the squared one); PXM_FLAG_POSE_VIEWDIR adds the
 * exact view-direction term to the rotation columns.
 */
int pxm_render_gn(const pxm_grid *grid, const pxm_rays *rays, const pxm_opts *opts,
                  const float *tgt_rgb, const float *tgt_depth, const float *frame_weight,
                  double *gn, void *stream);

/*
 * Gauss-Newton pose update: per frame, xi = -(H + damping I)^-1 g from the
 * gn slots of pxm_render_gn (Cholesky in float64), then the left retraction
 * c2w <- exp(xi^) c2w.  The frame's gn slots are zeroed after they are read;
 * a frame whose damped H is not positive definite keeps its pose.
 *   c2w [F][3][4] f32 (in/out), gn [F][28] f64 (in, zeroed).
 */
int pxm_pose_gn(int32_t n_frames, float *c2w, double *gn, float damping, void *stream);

/*
 * Mapping update (Sec. 5.4: RMSProp for mapping): one sparse RMSProp step
 * over the vertex records of SH degree sh_degree (S = PXM_RECORD_FLOATS(
 * sh_degree) floats each).  A record is touched when any of its S entries of
 * grad_data is non-zero; for touched records, entry by entry,
 *   state <- alpha state + (1 - alpha) g^2,
 *   data  <- data - lr g / (sqrt(state) + eps),
 * with lr = lr_density for entry 0 and lr_sh for the SH entries (padding
 * entries have a zero gradient and do not move).
 * Untouched records keep their values and running averages (the rule of the
 * Plenoxel optimiser the method builds on; the paper states none).
 * grad_data is read and then zeroed, so one call ends a mapping iteration.
 *   data, grad_data, state [n_alloc][S] f32, 16-byte aligned (in/out;
 *   state starts zeroed).  n_alloc == 0 is a no-op.
 */
int pxm_grid_rmsprop(int64_t n_alloc, int32_t sh_degree, float *data, float *grad_data,
                     float *state, float lr_density, float lr_sh, float alpha, float eps,
                     void *stream);

/*
 * Occupancy bitfield for empty-space skipping (an exact acceleration: a cell
 * whose 8 corners are all empty interpolates to zero density and carries no
 * light or gradient).  Level 0 holds one 64-bit word per block of 4^3 cells,
 * block (qx, qy, qz) at (qx*Qy + qy)*Qz + qz with Q = ceil((R-1)/4) per axis,
 * cell (x, y, z) at bit (x&3)*16 + (y&3)*4 + (z&3) of its block's word
 * (little-endian: the low half is the first of two uint32 words).  Level 1,
 * after level 0, holds one bit per brick of 8^3 cells.  Build it on `stream`
 * from grid->link / grid->n_alloc (grid->data and grid->occ are not read) into
 * `occ` (8-byte aligned) of n_words >= pxm_occupancy_words(grid) uint32 words,
 * and rebuild it whenever the link table changes.
 */
size_t pxm_occupancy_words(const pxm_grid *grid);
int pxm_build_occupancy(const pxm_grid *grid, uint32_t *occ, size_t n_words, void *stream);

/*
 * Dynamic grid (Sec. 6.1: a dynamic voxel grid with a peak resolution of
 * 512^3; the paper gives no growth or pruning policy, so the schedule is the
 * caller's).  Both edits write a new link table and a new payload; the
 * caller then rebuilds the occupancy bitfield of the new grid.
 *
 * Workspace.  `ws` is device scratch of at least
 * pxm_grid_edit_workspace_bytes(grid) bytes, 256-byte aligned.  Its contents
 * on entry do not matter and are left undefined: a buffer shared with
 * pxm_render_fused must be zeroed again before that call.
 *
 * Counts.  n_fine / n_out are DEVICE int64 written on `stream`; synchronise
 * before reading them.
 */
size_t pxm_grid_edit_workspace_bytes(const pxm_grid *grid);

/*
 * Coarse-to-fine growth, step 1 of 2: the link table of the doubled lattice.
 * The fine grid has 2R - 1 vertices per axis, voxel_size / 2 and the same
 * aabb_min, so fine vertex 2v sits on coarse vertex v.  A fine vertex is
 * allocated when some coarse cell whose closed box holds it has an allocated
 * corner; allocated fine vertices are numbered 0 .. n_fine-1 in lattice order.
 *   link_fine  [(2Rx-1)(2Ry-1)(2Rz-1)] int32, written (-1 = empty)
 *   n_fine     device int64, written
 * grid->data is not read.  PXM_UNSUPPORTED when the doubled lattice exceeds
 * 2^31 - 1 vertices.
 */
int pxm_grid_upsample_link(const pxm_grid *grid, int32_t *link_fine, int64_t *n_fine, void *ws,
                           size_t ws_bytes, void *stream);

/*
 * Coarse-to-fine growth, step 2 of 2: the fine records.  Each is the coarse
 * trilinear interpolant at the fine vertex (empty coarse vertices read 0),
 * summed in FP64 and rounded once to FP32, with the density halved: density
 * is per voxel, so the optical depth of a world-length step is unchanged and
 * rendering the fine grid at twice the step_vox reproduces the coarse render.
 *   link_fine  the table step 1 wrote for this grid
 *   n_fine     its count (host value, read back by the caller)
 *   data_fine  [n_fine][S] f32 (the grid's record layout), 16-byte aligned, written
 */
int pxm_grid_upsample_data(const pxm_grid *grid, const int32_t *link_fine, int64_t n_fine,
                           float *data_fine, void *stream);

/*
 * Pruning: records whose density is <= tau are dropped; the others keep their
 * order and are renumbered 0 .. n_out-1, and the link table is rewritten
 * (dropped or invalid links -> -1).
 *   link_out  [Rx*Ry*Rz] int32, written; may be grid->link itself (in place)
 *   data_out  [n_alloc][S] f32 capacity, 16-byte aligned, must not overlap
 *             grid->data; rows [0, n_out) are written
 *   n_out     device int64, written
 * tau = -inf keeps every record.  NaN tau is PXM_INVALID_ARGUMENT.
 */
int pxm_grid_prune(const pxm_grid *grid, float tau, int32_t *link_out, float *data_out,
                   int64_t *n_out, void *ws, size_t ws_bytes, void *stream);

/*
 * Allocation-free form of pxm_render_fused, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, semantics and results as
 * pxm_render_fused without the workspace: its scratch (the tile-queue
 * counters, and in the two-launch form the per-ray state) lives in a static
 * device array of PXM_NOALLOC_SCRATCH_BYTES that every GPU the library runs on
 * holds until the process ends.  The call allocates nothing: it clears the
 * counters with a kernel on `stream`, then launches as pxm_render_fused.
 *   Limit: under launch variant 2 (see pxm_set_tuning) at most
 *   PXM_NOALLOC_MAX_SPLIT_RAYS rays, else PXM_UNSUPPORTED; variants 0 and 1
 *   take any ray count.
 *   Concurrency: every call on one GPU shares that GPU's array, so calls that
 *   overlap on one GPU (two streams, two threads) race and give wrong
 *   results; serialise them on one stream.
 */
#define PXM_NOALLOC_SCRATCH_BYTES (32u << 20)
#define PXM_NOALLOC_MAX_SPLIT_RAYS 182336
int pxm_render_fused_noalloc(const pxm_grid *grid, const pxm_rays *rays, const pxm_opts *opts,
                             const float *tgt_rgb, const float *tgt_depth,
                             const float *frame_weight, int32_t want, float *rgb, float *depth,
                             double *loss, float *grad_data, double *grad_pose, int64_t *stats,
                             void *stream);

/*
 * Measurement aid (not part of the method): streaming-read bandwidth of
 * `bytes` (a multiple of 128) of device memory at `buf` (16-byte aligned),
 * read `passes` times by 2048 workgroups of 256 lanes with float4 loads,
 * workgroup b reading only the (b % 8)-th eighth of the buffer (the XCD
 * workgroup b runs on), so the per-XCD working set is bytes / 8: ~32 MB in
 * total stays in the L2s, ~256 MB in the Infinity Cache.  Time it with events
 * on `stream`.  sink: >= 2048 * 256 floats of device memory, overwritten.
 */
int pxm_probe_read_bandwidth(const void *buf, size_t bytes, int32_t passes, float *sink,
                             size_t sink_floats, void *stream);

/* Workspace bytes pxm_render_fused needs for these arguments and `want`, under
 * any launch tuning: 256 + 184 * (n_rays rounded up to 64), plus, with
 * PXM_WANT_GRID | PXM_WANT_DETERMINISTIC, 8 * n_alloc * S rounded up to 256. */
size_t pxm_workspace_bytes(const pxm_grid *grid, const pxm_rays *rays, const pxm_opts *opts,
                           int32_t want);

/*
 * Launch tuning for pxm_render_fused (process-wide; read at each call):
 *   block    rays per workgroup (64, 128 or 256; 0 = default 256)
 *   variant  0 = one workgroup per ray tile, 1 = persistent workgroups
 *            pulling ray tiles from a device counter in the workspace,
 *            2 = two persistent launches: the forward and loss (few
 *            registers, higher occupancy), then the backward resuming
 *            from the per-ray state the first left in the workspace
 * Returns PXM_INVALID_ARGUMENT for values outside these sets.
 */
int pxm_set_tuning(int32_t block, int32_t variant);
void pxm_get_tuning(int32_t *block, int32_t *variant);

const char *pxm_status_string(int status);
const char *pxm_last_error(void);
int pxm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PXM_H */
