/*
 * FP64 reference ("oracle") for differentiable volume rendering of a sparse
 * voxel grid, after Teigen, Park, Stahl and Mester, "RGB-D Mapping and
 * Tracking in a Plenoxel Radiance Field" (WACV 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or constant table
 * with the HIP kernels.
 *
 * It is deliberately plain: one ray at a time, every sample stored, the grid
 * read densely through the link table (an empty link reads as zero), sums
 * taken in the order the equations write them, double precision throughout.
 * OpenMP only splits independent rays across host threads.
 *
 * Readings of points the paper leaves open (each one is listed, with its
 * reason, in the design notes of the repository):
 *   - samples t_k = t_near + k * step_vox * voxel_size, k = 0, 1, ..., kept
 *     while the position lies in the vertex box [0, R-1]^3 (voxel units);
 *     at most max_samples kept positions, counted from the first in-box one;
 *   - delta = step_vox (density in per-voxel units), the same for every
 *     sample including the last;
 *   - density sigma = max(sigma_raw, 0) of the interpolated raw value;
 *   - colour c = act(sum_k Y_k(d) * sh_k), act selectable;
 *   - real SH of degree 2 with the Condon-Shortley phase at the unit world
 *     ray direction;
 *   - no background colour, expected depth not normalised;
 *   - after sample i the march stops when T_{i+1} < t_stop;
 *   - output depth is z-depth = expected range / |d_cam| with
 *     d_cam = ((u+.5-cx)/fx, (v+.5-cy)/fy, 1);
 *   - pose gradient w.r.t. a left (world-frame) perturbation
 *     exp(xi^) T, xi = (rho, phi); by default only the sample-position chain
 *     of Eq. 12-13 (optional exact view-direction term behind a flag).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NREC 28            /* 1 density + 3 channels x 9 SH coefficients (Sec. 5.2) */
#define NSH 9              /* SH coefficients per channel at degree 2 */

enum { ACT_RELU_SHIFT = 0, ACT_SIGMOID = 1, ACT_IDENTITY = 2 };
enum { LOSS_L1 = 0, LOSS_L2 = 1 };
enum { FLAG_POSE_VIEWDIR = 1 };

/*
 * Record layout.  The paper's records hold nine SH coefficients per channel
 * (degree 2).  Records of a lower degree d keep the first (d+1)^2 functions
 * of the same basis (the real SH of degree <= d are a prefix of it):
 * density, then sh[ch][k] for k < nsh at record[1 + ch*nsh + k], in a record
 * of `stride` floats (4, 16 or 28; the unused tail of a degree-1 record is
 * ignored and receives no gradient).
 */
typedef struct {
    int32_t R[3];
    double lo[3];
    double vs;
    const int32_t *link;
    const float *data;
    int nsh;              /* SH coefficients per channel: 1, 4 or 9 */
    int nrec;             /* used fields: 1 + 3 nsh */
    int stride;           /* floats per record */
} ogrid;

typedef struct {
    double step_vox;
    int32_t max_samples;
    double t_near;
    double t_stop;
    int32_t act;
} oopts;

/* ------------------------------------------------------------------------- */
/* Camera ray through a pixel (Sec. 4: r = o + t d, o = camera centre).      */
/* ------------------------------------------------------------------------- */
static void ray_through_pixel(const double *c2w, const double *intr, int u, int v,
                              double o[3], double d[3], double *s_out)
{
    double dc[3];
    dc[0] = ((double)u + 0.5 - intr[2]) / intr[0];
    dc[1] = ((double)v + 0.5 - intr[3]) / intr[1];
    dc[2] = 1.0;
    double s = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
    for (int a = 0; a < 3; ++a) {
        double acc = 0.0;
        for (int b = 0; b < 3; ++b)
            acc += c2w[a * 4 + b] * dc[b];
        d[a] = acc / s;
        o[a] = c2w[a * 4 + 3];
    }
    *s_out = s;
}

/* ------------------------------------------------------------------------- */
/* Real spherical harmonics up to degree 2 (nine per channel, Sec. 5.2).     */
/* ------------------------------------------------------------------------- */
static void sh_basis(const double d[3], double Y[NSH])
{
    const double x = d[0], y = d[1], z = d[2];
    const double pi = 3.14159265358979323846;
    const double k00 = 0.5 * sqrt(1.0 / pi);
    const double k1 = sqrt(3.0 / (4.0 * pi));
    const double k2a = 0.5 * sqrt(15.0 / pi);
    const double k20 = 0.25 * sqrt(5.0 / pi);
    const double k22 = 0.25 * sqrt(15.0 / pi);
    Y[0] = k00;
    Y[1] = -k1 * y;
    Y[2] = k1 * z;
    Y[3] = -k1 * x;
    Y[4] = k2a * x * y;
    Y[5] = -k2a * y * z;
    Y[6] = k20 * (2.0 * z * z - x * x - y * y);
    Y[7] = -k2a * x * z;
    Y[8] = k22 * (x * x - y * y);
}

/* d Y_k / d(x,y,z) of the polynomial above, for the optional view term. */
static void sh_basis_grad(const double d[3], double G[NSH][3])
{
    const double x = d[0], y = d[1], z = d[2];
    const double pi = 3.14159265358979323846;
    const double k1 = sqrt(3.0 / (4.0 * pi));
    const double k2a = 0.5 * sqrt(15.0 / pi);
    const double k20 = 0.25 * sqrt(5.0 / pi);
    const double k22 = 0.25 * sqrt(15.0 / pi);
    memset(G, 0, sizeof(double) * NSH * 3);
    G[1][1] = -k1;
    G[2][2] = k1;
    G[3][0] = -k1;
    G[4][0] = k2a * y;  G[4][1] = k2a * x;
    G[5][1] = -k2a * z; G[5][2] = -k2a * y;
    G[6][0] = -2.0 * k20 * x; G[6][1] = -2.0 * k20 * y; G[6][2] = 4.0 * k20 * z;
    G[7][0] = -k2a * z; G[7][2] = -k2a * x;
    G[8][0] = 2.0 * k22 * x; G[8][1] = -2.0 * k22 * y;
}

static double act_f(int act, double s)
{
    if (act == ACT_SIGMOID) return 1.0 / (1.0 + exp(-s));
    if (act == ACT_IDENTITY) return s;
    return s + 0.5 > 0.0 ? s + 0.5 : 0.0;
}

static double act_df(int act, double s)
{
    if (act == ACT_SIGMOID) { double g = 1.0 / (1.0 + exp(-s)); return g * (1.0 - g); }
    if (act == ACT_IDENTITY) return 1.0;
    return s + 0.5 > 0.0 ? 1.0 : 0.0;
}

/* ------------------------------------------------------------------------- */
/* Trilinear interpolation of the 8 closest vertices (Sec. 5.2, Fig. 4).     */
/* ------------------------------------------------------------------------- */
typedef struct {
    int cell[3];
    double f[3];          /* position inside the cell, [0,1]^3 */
    int64_t idx[8];       /* corner b = 4*i + 2*j + k (x, y, z offsets); -1 empty */
    double v[8][NREC];    /* corner values (first nrec fields), zero for empty links */
    double w[8];          /* trilinear weights */
    int n_alloc_corners;
    int nrec;             /* fields in use */
} ocorners;

static void gather_cell(const ogrid *g, const double q[3], ocorners *c)
{
    for (int a = 0; a < 3; ++a) {
        int fl = (int)floor(q[a]);
        if (fl < 0) fl = 0;
        if (fl > g->R[a] - 2) fl = g->R[a] - 2;
        c->cell[a] = fl;
        c->f[a] = q[a] - (double)fl;
    }
    c->n_alloc_corners = 0;
    c->nrec = g->nrec;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) {
                int b = 4 * i + 2 * j + k;
                int64_t lin = ((int64_t)(c->cell[0] + i) * g->R[1] + (c->cell[1] + j)) * g->R[2]
                              + (c->cell[2] + k);
                int32_t id = g->link[lin];
                c->idx[b] = id;
                for (int m = 0; m < g->nrec; ++m)
                    c->v[b][m] = id >= 0 ? (double)g->data[(int64_t)id * g->stride + m] : 0.0;
                if (id >= 0) c->n_alloc_corners++;
                double wx = i ? c->f[0] : 1.0 - c->f[0];
                double wy = j ? c->f[1] : 1.0 - c->f[1];
                double wz = k ? c->f[2] : 1.0 - c->f[2];
                c->w[b] = wx * wy * wz;
            }
}

static void interp(const ocorners *c, double out[NREC])
{
    for (int m = 0; m < c->nrec; ++m) {
        double acc = 0.0;
        for (int b = 0; b < 8; ++b) acc += c->w[b] * c->v[b][m];
        out[m] = acc;
    }
}

/*
 * Appendix A: with the lower lattice point moved to the origin, the
 * interpolant is a0 + a1 x + a2 y + a3 z + a4 xy + a5 xz + a6 yz + a7 xyz,
 * whose coefficients solve an 8x8 linear system over the cell corners.
 * The matrix only depends on corner coordinates in {0,1}, so it is inverted
 * once by Gauss-Jordan elimination.  Row order follows the corner numbering
 * b = 4*i + 2*j + k used above.
 */
static double g_Minv[8][8];
static int g_Minv_ready = 0;

static void build_minv(void)
{
    double A[8][16];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) {
                int r = 4 * i + 2 * j + k;
                double x = i, y = j, z = k;
                double row[8] = {1.0, x, y, z, x * y, x * z, y * z, x * y * z};
                for (int cidx = 0; cidx < 8; ++cidx) {
                    A[r][cidx] = row[cidx];
                    A[r][8 + cidx] = (r == cidx) ? 1.0 : 0.0;
                }
            }
    for (int col = 0; col < 8; ++col) {
        int piv = col;
        for (int r = col + 1; r < 8; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (piv != col)
            for (int cidx = 0; cidx < 16; ++cidx) {
                double t = A[col][cidx]; A[col][cidx] = A[piv][cidx]; A[piv][cidx] = t;
            }
        double p = A[col][col];
        for (int cidx = 0; cidx < 16; ++cidx) A[col][cidx] /= p;
        for (int r = 0; r < 8; ++r) {
            if (r == col) continue;
            double fct = A[r][col];
            for (int cidx = 0; cidx < 16; ++cidx) A[r][cidx] -= fct * A[col][cidx];
        }
    }
    for (int r = 0; r < 8; ++r)
        for (int cidx = 0; cidx < 8; ++cidx) g_Minv[r][cidx] = A[r][8 + cidx];
    g_Minv_ready = 1;
}

/* Eq. 16: spatial gradient (voxel units) of every interpolated field. */
static void interp_grad(const ocorners *c, double out[NREC][3])
{
    const double x = c->f[0], y = c->f[1], z = c->f[2];
    for (int m = 0; m < c->nrec; ++m) {
        double a[8];
        for (int r = 0; r < 8; ++r) {
            double acc = 0.0;
            for (int b = 0; b < 8; ++b) acc += g_Minv[r][b] * c->v[b][m];
            a[r] = acc;
        }
        out[m][0] = a[1] + a[4] * y + a[5] * z + a[7] * y * z;
        out[m][1] = a[2] + a[4] * x + a[6] * z + a[7] * x * z;
        out[m][2] = a[3] + a[5] * x + a[6] * y + a[7] * x * y;
    }
}

/* ------------------------------------------------------------------------- */
/* One ray: samples, compositing (Eq. 1-3).                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n;                 /* samples kept (nsamp) */
    int cap;
    double *t;             /* distance from the camera centre */
    double (*q)[3];        /* position in voxel units */
    double *sigma_raw, *sigma;
    double (*s)[3], (*c)[3];
    double *T;             /* T_i, transmittance before sample i */
    double *w;             /* w_i = T_i (1 - exp(-sigma_i delta)) */
    double rgb[3], D;      /* C-hat and expected range D-hat */
    double T_end;
    long n_occ;            /* samples whose cell has an allocated corner */
    long n_occ_corners;    /* allocated corners summed over those samples */
    long n_grad_corners;   /* allocated corners of samples with sigma_raw > 0 */
} otrace;

static void trace_alloc(otrace *tr, int cap)
{
    tr->cap = cap;
    tr->t = malloc(sizeof(double) * cap);
    tr->q = malloc(sizeof(double) * 3 * cap);
    tr->sigma_raw = malloc(sizeof(double) * cap);
    tr->sigma = malloc(sizeof(double) * cap);
    tr->s = malloc(sizeof(double) * 3 * cap);
    tr->c = malloc(sizeof(double) * 3 * cap);
    tr->T = malloc(sizeof(double) * (cap + 1));
    tr->w = malloc(sizeof(double) * cap);
}

static void trace_grow(otrace *tr)
{
    int cap = tr->cap * 2;
    tr->t = realloc(tr->t, sizeof(double) * cap);
    tr->q = realloc(tr->q, sizeof(double) * 3 * cap);
    tr->sigma_raw = realloc(tr->sigma_raw, sizeof(double) * cap);
    tr->sigma = realloc(tr->sigma, sizeof(double) * cap);
    tr->s = realloc(tr->s, sizeof(double) * 3 * cap);
    tr->c = realloc(tr->c, sizeof(double) * 3 * cap);
    tr->T = realloc(tr->T, sizeof(double) * (cap + 1));
    tr->w = realloc(tr->w, sizeof(double) * cap);
    tr->cap = cap;
}

static void trace_free(otrace *tr)
{
    free(tr->t); free(tr->q); free(tr->sigma_raw); free(tr->sigma);
    free(tr->s); free(tr->c); free(tr->T); free(tr->w);
}

static int in_box(const ogrid *g, const double q[3])
{
    for (int a = 0; a < 3; ++a)
        if (!(q[a] >= 0.0 && q[a] <= (double)(g->R[a] - 1))) return 0;
    return 1;
}

static void march(const ogrid *g, const oopts *op, const double o[3], const double d[3],
                  otrace *tr)
{
    const double dw = op->step_vox * g->vs;          /* spacing in world units */
    const double delta = op->step_vox;               /* spacing in voxel units */
    double Y[NSH];
    sh_basis(d, Y);

    /* far bound: beyond it the ray has certainly left the box */
    double cen[3], hd = 0.0, dist = 0.0;
    for (int a = 0; a < 3; ++a) {
        double ext = (g->R[a] - 1) * g->vs;
        cen[a] = g->lo[a] + 0.5 * ext;
        hd += 0.25 * ext * ext;
        dist += (o[a] - cen[a]) * (o[a] - cen[a]);
    }
    double t_far = sqrt(dist) + sqrt(hd) + 2.0 * dw;
    long k_far = (long)ceil((t_far - op->t_near) / dw) + 2;

    tr->n = 0;
    tr->rgb[0] = tr->rgb[1] = tr->rgb[2] = 0.0;
    tr->D = 0.0;
    tr->n_occ = tr->n_occ_corners = tr->n_grad_corners = 0;
    double optical = 0.0;      /* sum_{j<i} sigma_j delta_j (Eq. 2) */
    int entered = 0;
    tr->T[0] = 1.0;
    for (long k = 0; k <= k_far; ++k) {
        double t = op->t_near + (double)k * dw;
        double q[3];
        for (int a = 0; a < 3; ++a) q[a] = (o[a] - g->lo[a]) / g->vs + (t / g->vs) * d[a];
        if (!in_box(g, q)) {
            if (entered) break;
            continue;
        }
        entered = 1;
        if (tr->n >= op->max_samples) break;
        if (tr->n + 1 >= tr->cap) trace_grow(tr);
        int i = tr->n;
        ocorners cc;
        gather_cell(g, q, &cc);
        double val[NREC];
        interp(&cc, val);
        tr->t[i] = t;
        tr->q[i][0] = q[0]; tr->q[i][1] = q[1]; tr->q[i][2] = q[2];
        tr->sigma_raw[i] = val[0];
        tr->sigma[i] = val[0] > 0.0 ? val[0] : 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.0;
            for (int kk = 0; kk < g->nsh; ++kk) acc += Y[kk] * val[1 + ch * g->nsh + kk];
            tr->s[i][ch] = acc;
            tr->c[i][ch] = act_f(op->act, acc);
        }
        if (cc.n_alloc_corners > 0) {
            tr->n_occ++;
            tr->n_occ_corners += cc.n_alloc_corners;
            if (val[0] > 0.0) tr->n_grad_corners += cc.n_alloc_corners;
        }
        /* Eq. 2 and Eq. 1/3 */
        double Ti = exp(-optical);
        double alpha = 1.0 - exp(-tr->sigma[i] * delta);
        tr->T[i] = Ti;
        tr->w[i] = Ti * alpha;
        for (int ch = 0; ch < 3; ++ch) tr->rgb[ch] += tr->w[i] * tr->c[i][ch];
        tr->D += tr->w[i] * t;
        optical += tr->sigma[i] * delta;
        tr->n = i + 1;
        tr->T[i + 1] = exp(-optical);
        if (tr->T[i + 1] < op->t_stop) break;
    }
    tr->T_end = tr->T[tr->n];
}

static void load_grid(ogrid *g, const int32_t *R, const float *lo, double vs,
                      const int32_t *link, const float *data, int32_t deg)
{
    for (int a = 0; a < 3; ++a) { g->R[a] = R[a]; g->lo[a] = lo[a]; }
    g->vs = vs;
    g->link = link;
    g->data = data;
    g->nsh = (deg + 1) * (deg + 1);
    g->nrec = 1 + 3 * g->nsh;
    g->stride = deg == 0 ? 4 : deg == 1 ? 16 : NREC;
    if (!g_Minv_ready) build_minv();
}

/* floats per record of SH degree deg (0, 1 or 2) */
int orc_record_floats(int32_t deg) { return deg == 0 ? 4 : deg == 1 ? 16 : NREC; }

static int frame_of(const int32_t *off, int32_t F, int64_t r)
{
    int lo = 0, hi = F;          /* find f with off[f] <= r < off[f+1] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (off[mid] <= r) lo = mid; else hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------------------- */
/* Public entry points (called from Python through ctypes).                  */
/* ------------------------------------------------------------------------- */

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void orc_sh_basis(const double *d, double *Y) { sh_basis(d, Y); }

void orc_sh_basis_grad(const double *d, double *G) { sh_basis_grad(d, (double (*)[3])G); }

void orc_ray(const double *c2w, const double *intr, int u, int v, double *o, double *d, double *s)
{
    ray_through_pixel(c2w, intr, u, v, o, d, s);
}

/* Interpolated 28 values and their Eq. 16 gradients at a voxel-unit point. */
void orc_interp(const int32_t *R, const float *lo, double vs, const int32_t *link,
                const float *data, int32_t deg, const double *q, double *val, double *grad)
{
    ogrid g;
    load_grid(&g, R, lo, vs, link, data, deg);
    ocorners cc;
    gather_cell(&g, q, &cc);
    interp(&cc, val);
    if (grad) interp_grad(&cc, (double (*)[3])grad);
}

/* The per-sample record of one ray (for the tests' brute-force sums). */
int orc_trace(const int32_t *R, const float *lo, double vs, const int32_t *link,
              const float *data, int32_t deg, const double *o, const double *d,
              double step_vox, int32_t max_samples, double t_near, double t_stop, int32_t act,
              int32_t cap, double *t, double *sigma_raw, double *rgb_s, double *T, double *w,
              double *out_rgb_D)
{
    ogrid g;
    load_grid(&g, R, lo, vs, link, data, deg);
    oopts op = {step_vox, max_samples, t_near, t_stop, act};
    otrace tr;
    trace_alloc(&tr, 64);
    march(&g, &op, o, d, &tr);
    int n = tr.n < cap ? tr.n : cap;
    for (int i = 0; i < n; ++i) {
        t[i] = tr.t[i];
        sigma_raw[i] = tr.sigma_raw[i];
        for (int ch = 0; ch < 3; ++ch) rgb_s[3 * i + ch] = tr.c[i][ch];
        T[i] = tr.T[i];
        w[i] = tr.w[i];
    }
    if (n < cap) T[n] = tr.T[tr.n];
    out_rgb_D[0] = tr.rgb[0]; out_rgb_D[1] = tr.rgb[1]; out_rgb_D[2] = tr.rgb[2];
    out_rgb_D[3] = tr.D;
    int total = tr.n;
    trace_free(&tr);
    return total;
}

/*
 * Forward render of every ray: colour (Eq. 1), z-depth from Eq. 3, number of
 * samples kept.  stats (optional, [n_rays][3]): occupied samples, allocated
 * corners of those, allocated corners of samples with positive raw density.
 */
void orc_render(const int32_t *R, const float *lo, double vs, const int32_t *link,
                const float *data, int32_t deg, int32_t F, const double *c2w, const double *intr,
                const int32_t *off, const int32_t *pix, int64_t n_rays,
                double step_vox, int32_t max_samples, double t_near, double t_stop, int32_t act,
                double *rgb, double *depth, int32_t *nsamp, int64_t *stats)
{
    ogrid g;
    load_grid(&g, R, lo, vs, link, data, deg);
    oopts op = {step_vox, max_samples, t_near, t_stop, act};
#pragma omp parallel
    {
        otrace tr;
        trace_alloc(&tr, 256);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n_rays; ++r) {
            int f = frame_of(off, F, r);
            double o[3], d[3], s;
            ray_through_pixel(c2w + 12 * f, intr + 4 * f, pix[2 * r], pix[2 * r + 1], o, d, &s);
            march(&g, &op, o, d, &tr);
            for (int ch = 0; ch < 3; ++ch) rgb[3 * r + ch] = tr.rgb[ch];
            depth[r] = tr.D / s;
            nsamp[r] = tr.n;
            if (stats) {
                stats[3 * r] = tr.n_occ;
                stats[3 * r + 1] = tr.n_occ_corners;
                stats[3 * r + 2] = tr.n_grad_corners;
            }
        }
        trace_free(&tr);
    }
}

/*
 * Loss of Eq. 4, 5 and 11 per frame, and its gradient with respect to the
 * rendered colour and z-depth.  A ray with a non-finite or non-positive
 * target depth is dropped entirely (Sec. 6.1).
 */
void orc_loss(int32_t F, const int32_t *off, const double *rgb, const double *depth,
              const float *tgt_rgb, const float *tgt_depth, const float *frame_weight,
              int32_t depth_loss, double lambda_d, double *loss, double *g_rgb, double *g_depth)
{
    for (int f = 0; f < F; ++f) {
        double om = frame_weight[f];
        double acc = 0.0;
        for (int64_t r = off[f]; r < off[f + 1]; ++r) {
            double D = tgt_depth[r];
            int valid = isfinite(D) && D > 0.0;
            if (!valid) {
                g_rgb[3 * r] = g_rgb[3 * r + 1] = g_rgb[3 * r + 2] = 0.0;
                g_depth[r] = 0.0;
                continue;
            }
            double sq = 0.0;
            for (int ch = 0; ch < 3; ++ch) {
                double e = rgb[3 * r + ch] - (double)tgt_rgb[3 * r + ch];
                sq += e * e;
                g_rgb[3 * r + ch] = 2.0 * om * e;
            }
            double e = depth[r] - D;
            double rho, drho;
            if (depth_loss == LOSS_L2) { rho = e * e; drho = 2.0 * e; }
            else { rho = fabs(e); drho = e > 0.0 ? 1.0 : (e < 0.0 ? -1.0 : 0.0); }
            acc += om * sq + lambda_d * om * rho;
            g_depth[r] = lambda_d * om * drho;
        }
        loss[f] = acc;
    }
}

/* Backward of one ray (Eq. 6-14 and Appendix A) for upstream gradients gC
 * (dL/dC-hat) and gDz (dL/d z-depth): scatters into grad_data when it is not
 * NULL and writes the ray's (rho, phi) pose gradient into out6 when that is
 * not NULL. */
static void ray_backward(const ogrid *g, const oopts *op, int32_t flags, const double *c2w_f,
                         const double *intr_f, int u, int v, const double gC[3], double gDz,
                         otrace *tr, double *grad_data, double out6[6])
{
    const double delta = op->step_vox;
    const int act = op->act;
    double o[3], d[3], s;
    ray_through_pixel(c2w_f, intr_f, u, v, o, d, &s);
    march(g, op, o, d, tr);
    /* the loss sees z-depth = D-hat / s, so dL/dD-hat = g_depth / s */
    const double gD = gDz / s;
    double Y[NSH], GY[NSH][3];
    sh_basis(d, Y);
    sh_basis_grad(d, GY);
    double prefC[3] = {0.0, 0.0, 0.0}, prefD = 0.0;
    double go[3] = {0, 0, 0}, gd[3] = {0, 0, 0}, gview[3] = {0, 0, 0};
    for (int i = 0; i < tr->n; ++i) {
        /* inclusive prefixes sum_{j<=i} c_j w_j and sum_{j<=i} t_j w_j */
        for (int ch = 0; ch < 3; ++ch) prefC[ch] += tr->c[i][ch] * tr->w[i];
        prefD += tr->t[i] * tr->w[i];
        const double Tn = tr->T[i + 1];
        /* Eq. 9 and Eq. 10 */
        double dL_dsigma = 0.0;
        for (int ch = 0; ch < 3; ++ch)
            dL_dsigma += gC[ch] * delta * (tr->c[i][ch] * Tn - tr->rgb[ch] + prefC[ch]);
        dL_dsigma += gD * delta * (tr->t[i] * Tn - tr->D + prefD);
        const double dL_dsraw = tr->sigma_raw[i] > 0.0 ? dL_dsigma : 0.0;
        /* Eq. 8 through the colour activation */
        double dL_ds[3];
        for (int ch = 0; ch < 3; ++ch)
            dL_ds[ch] = gC[ch] * tr->w[i] * act_df(act, tr->s[i][ch]);
        if (dL_dsraw == 0.0 && dL_ds[0] == 0.0 && dL_ds[1] == 0.0 && dL_ds[2] == 0.0)
            continue;
        ocorners cc;
        gather_cell(g, tr->q[i], &cc);
        if (grad_data) {
            double gval[NREC];
            gval[0] = dL_dsraw;
            for (int ch = 0; ch < 3; ++ch)
                for (int k = 0; k < g->nsh; ++k) gval[1 + ch * g->nsh + k] = dL_ds[ch] * Y[k];
            for (int b = 0; b < 8; ++b) {
                if (cc.idx[b] < 0) continue;
                double *dst = grad_data + cc.idx[b] * g->stride;
                for (int m = 0; m < g->nrec; ++m) {
                    double add = cc.w[b] * gval[m];
#pragma omp atomic
                    dst[m] += add;
                }
            }
        }
        if (out6) {
            double G[NREC][3];
            interp_grad(&cc, G);
            double gp[3];
            for (int a = 0; a < 3; ++a) {
                double acc = dL_dsraw * G[0][a];
                for (int ch = 0; ch < 3; ++ch) {
                    double dsa = 0.0;
                    for (int k = 0; k < g->nsh; ++k) dsa += Y[k] * G[1 + ch * g->nsh + k][a];
                    acc += dL_ds[ch] * dsa;
                }
                gp[a] = acc / g->vs;      /* voxel units -> world units */
            }
            /* Eq. 14: dp/do = 1, dp/dd = t_i */
            for (int a = 0; a < 3; ++a) { go[a] += gp[a]; gd[a] += tr->t[i] * gp[a]; }
            if (flags & FLAG_POSE_VIEWDIR) {
                double val[NREC];
                interp(&cc, val);
                for (int a = 0; a < 3; ++a) {
                    double acc = 0.0;
                    for (int ch = 0; ch < 3; ++ch)
                        for (int k = 0; k < g->nsh; ++k)
                            acc += dL_ds[ch] * GY[k][a] * val[1 + ch * g->nsh + k];
                    gview[a] += acc;
                }
            }
        }
    }
    if (out6) {
        double gphi[3];
        gphi[0] = o[1] * go[2] - o[2] * go[1] + d[1] * gd[2] - d[2] * gd[1];
        gphi[1] = o[2] * go[0] - o[0] * go[2] + d[2] * gd[0] - d[0] * gd[2];
        gphi[2] = o[0] * go[1] - o[1] * go[0] + d[0] * gd[1] - d[1] * gd[0];
        if (flags & FLAG_POSE_VIEWDIR) {
            gphi[0] += d[1] * gview[2] - d[2] * gview[1];
            gphi[1] += d[2] * gview[0] - d[0] * gview[2];
            gphi[2] += d[0] * gview[1] - d[1] * gview[0];
        }
        for (int a = 0; a < 3; ++a) { out6[a] = go[a]; out6[3 + a] = gphi[a]; }
    }
}

/*
 * Backward pass.  With the upstream gradients dL/dC-hat (g_rgb, [n][3]) and
 * dL/d(z-depth) (g_depth, [n]):
 *   grad_data ([n_alloc][28], accumulated, may be NULL): Eq. 6-10 scattered
 *     through the trilinear weights onto the allocated corner vertices;
 *   grad_pose ([F][6], accumulated, may be NULL): Eq. 12-14 with the
 *     Appendix A spatial gradients, reduced to (rho, phi) per frame.
 */
void orc_backward(const int32_t *R, const float *lo, double vs, const int32_t *link,
                  const float *data, int32_t deg, int32_t F, const double *c2w, const double *intr,
                  const int32_t *off, const int32_t *pix, int64_t n_rays,
                  double step_vox, int32_t max_samples, double t_near, double t_stop, int32_t act,
                  int32_t flags, const double *g_rgb, const double *g_depth,
                  double *grad_data, double *grad_pose)
{
    ogrid g;
    load_grid(&g, R, lo, vs, link, data, deg);
    oopts op = {step_vox, max_samples, t_near, t_stop, act};
#pragma omp parallel
    {
        otrace tr;
        trace_alloc(&tr, 256);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n_rays; ++r) {
            const double *gC = g_rgb + 3 * r;
            if (gC[0] == 0.0 && gC[1] == 0.0 && gC[2] == 0.0 && g_depth[r] == 0.0) continue;
            const int f = frame_of(off, F, r);
            double six[6];
            ray_backward(&g, &op, flags, c2w + 12 * f, intr + 4 * f, pix[2 * r], pix[2 * r + 1],
                         gC, g_depth[r], &tr, grad_data, grad_pose ? six : NULL);
            if (grad_pose) {
                double *dst = grad_pose + 6 * f;
                for (int a = 0; a < 6; ++a) {
#pragma omp atomic
                    dst[a] += six[a];
                }
            }
        }
        trace_free(&tr);
    }
}

/*
 * Per-ray pose Jacobian of the rendered outputs (colour R, G, B and z-depth)
 * with respect to the left se(3) perturbation (rho, phi): row k of J[r] is
 * the pose gradient of output k alone (upstream 1 on output k, 0 elsewhere),
 * so J is built from the same Eq. 12-14 chain as the pose gradient.
 *   J: [n][4][6], fully written (rows of rays that miss the grid are 0).
 */
void orc_pose_jacobian(const int32_t *R, const float *lo, double vs, const int32_t *link,
                       const float *data, int32_t deg, int32_t F, const double *c2w, const double *intr,
                       const int32_t *off, const int32_t *pix, int64_t n_rays,
                       double step_vox, int32_t max_samples, double t_near, double t_stop,
                       int32_t act, int32_t flags, double *J)
{
    ogrid g;
    load_grid(&g, R, lo, vs, link, data, deg);
    oopts op = {step_vox, max_samples, t_near, t_stop, act};
#pragma omp parallel
    {
        otrace tr;
        trace_alloc(&tr, 256);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n_rays; ++r) {
            const int f = frame_of(off, F, r);
            for (int k = 0; k < 4; ++k) {
                double gC[3] = {0.0, 0.0, 0.0};
                double gz = 0.0;
                if (k < 3) gC[k] = 1.0;
                else gz = 1.0;
                ray_backward(&g, &op, flags, c2w + 12 * f, intr + 4 * f, pix[2 * r],
                             pix[2 * r + 1], gC, gz, &tr, NULL, J + 24 * r + 6 * k);
            }
        }
        trace_free(&tr);
    }
}

/*
 * Total variation over the allocated vertices (a Plenoxel-style regulariser;
 * the paper itself does not define one):
 *   TV = sum_m lambda_m sum_{v} sqrt(dx^2 + dy^2 + dz^2 + eps)
 * with forward differences to the +x, +y, +z neighbours (empty reads as 0),
 * vertices on an upper face excluded, lambda_0 = lambda_sigma for density
 * and lambda_sh for each of the 27 SH fields.  The gradient is obtained by
 * differentiating each term and adding into the allocated vertices it reads.
 */
double orc_tv(const int32_t *R, const int32_t *link, const float *data, int32_t deg,
              double lambda_sigma, double lambda_sh, double eps, double *grad)
{
    const int nrec = 1 + 3 * (deg + 1) * (deg + 1);
    const int64_t S = orc_record_floats(deg);
    double total = 0.0;
    const int64_t n = (int64_t)R[0] * R[1] * R[2];
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (int64_t lin = 0; lin < n; ++lin) {
        int32_t id = link[lin];
        if (id < 0) continue;
        int x = (int)(lin / ((int64_t)R[1] * R[2]));
        int y = (int)((lin / R[2]) % R[1]);
        int z = (int)(lin % R[2]);
        if (x >= R[0] - 1 || y >= R[1] - 1 || z >= R[2] - 1) continue;
        int32_t nx = link[lin + (int64_t)R[1] * R[2]];
        int32_t ny = link[lin + R[2]];
        int32_t nz = link[lin + 1];
        for (int m = 0; m < nrec; ++m) {
            double lam = m == 0 ? lambda_sigma : lambda_sh;
            double v0 = data[(int64_t)id * S + m];
            double vx = nx >= 0 ? data[(int64_t)nx * S + m] : 0.0;
            double vy = ny >= 0 ? data[(int64_t)ny * S + m] : 0.0;
            double vz = nz >= 0 ? data[(int64_t)nz * S + m] : 0.0;
            double dx = vx - v0, dy = vy - v0, dz = vz - v0;
            double root = sqrt(dx * dx + dy * dy + dz * dz + eps);
            total += lam * root;
            if (grad) {
                double g0 = -lam * (dx + dy + dz) / root;
#pragma omp atomic
                grad[(int64_t)id * S + m] += g0;
                if (nx >= 0) {
                    double gx = lam * dx / root;
#pragma omp atomic
                    grad[(int64_t)nx * S + m] += gx;
                }
                if (ny >= 0) {
                    double gy = lam * dy / root;
#pragma omp atomic
                    grad[(int64_t)ny * S + m] += gy;
                }
                if (nz >= 0) {
                    double gz = lam * dz / root;
#pragma omp atomic
                    grad[(int64_t)nz * S + m] += gz;
                }
            }
        }
    }
    return total;
}
