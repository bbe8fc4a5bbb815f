"""FP64 CPU oracle for the sparse-voxel volume renderer and its gradients.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path never does.
It shares no code with the HIP kernels.  Its C core (``oracle.c``) follows the
paper's equations one ray at a time in double precision; this module only
marshals numpy arrays, plus small textbook pieces in numpy (the SE(3)
exponential map, an Adam step for tracking, a sparse RMSProp step for
mapping, and the dynamic-grid edits: coarse-to-fine growth and pruning).

Parity unpinned by the paper: the colour activation, the SH sign/order
convention, the se(3) pose parametrisation, the default (position-only)
pose chain, early termination, the TV regulariser and the growth/pruning
rules of the dynamic grid (Sec. 6.1 names a dynamic grid with a 512^3 peak
and gives no policy) are readings; they are
pinned by finite differences, closed forms and invariants, not by numbers
the paper prints (it prints none for this path).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# A test that plants a mistake in a copy of oracle.c (to show that the pins
# catch it) points this variable at the library built from that copy.
_LIB_OVERRIDE = os.environ.get("PXM_ORACLE_LIB")
_lib = None

NREC = 28   # floats per record at SH degree 2 (the paper's nine coefficients per channel)


def record_floats(deg: int) -> int:
    """Floats per record of SH degree deg: 4, 16 (13 used) or 28."""
    return {0: 4, 1: 16, 2: 28}[int(deg)]


def used_fields(deg: int) -> int:
    """Density plus (deg+1)^2 SH coefficients for each of three channels."""
    return 1 + 3 * (int(deg) + 1) ** 2


GCC_FLAGS = ["-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off"]


def build(verbose=False, src=None, out=None, extra=()) -> str:
    """Compile the oracle with gcc (plain IEEE double, no FMA contraction).
    `src`, `out` and `extra` flags serve the tests that build instrumented or
    deliberately broken copies; the default builds oracle.c in place."""
    out = out or _LIB_PATH
    cmd = ["gcc", *GCC_FLAGS, *extra, "-o", out, src or os.path.join(_HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    src = os.path.join(_HERE, "oracle.c")
    if _LIB_OVERRIDE:
        lib = C.CDLL(_LIB_OVERRIDE)
    else:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
            build()
        lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
    lib.orc_render.argtypes = [P, P, f64, P, P, i32, i32, P, P, P, P, i64, f64, i32, f64, f64,
                               i32, P, P, P, P]
    lib.orc_render.restype = None
    lib.orc_backward.argtypes = [P, P, f64, P, P, i32, i32, P, P, P, P, i64, f64, i32, f64, f64,
                                 i32, i32, P, P, P, P]
    lib.orc_backward.restype = None
    lib.orc_pose_jacobian.argtypes = [P, P, f64, P, P, i32, i32, P, P, P, P, i64, f64, i32, f64,
                                      f64, i32, i32, P]
    lib.orc_pose_jacobian.restype = None
    lib.orc_loss.argtypes = [i32, P, P, P, P, P, P, i32, f64, P, P, P]
    lib.orc_loss.restype = None
    lib.orc_tv.argtypes = [P, P, P, i32, f64, f64, f64, P]
    lib.orc_tv.restype = f64
    lib.orc_trace.argtypes = [P, P, f64, P, P, i32, P, P, f64, i32, f64, f64, i32, i32, P, P, P, P,
                              P, P]
    lib.orc_trace.restype = C.c_int
    lib.orc_interp.argtypes = [P, P, f64, P, P, i32, P, P, P]
    lib.orc_interp.restype = None
    lib.orc_sh_basis.argtypes = [P, P]
    lib.orc_sh_basis_grad.argtypes = [P, P]
    lib.orc_ray.argtypes = [P, P, C.c_int, C.c_int, P, P, P]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_set_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _grid_args(grid):
    R = _c(grid.reso, np.int32)
    lo = _c(grid.aabb_min, np.float32)
    link = _c(grid.link, np.int32)
    deg = int(getattr(grid, "sh_degree", 2))
    data = _c(grid.data, np.float32).reshape(-1, record_floats(deg))
    return (R, lo, float(grid.voxel_size), link, data, deg)


def _ray_args(rays):
    return (_c(rays.c2w, np.float64), _c(rays.intr, np.float64),
            _c(rays.frame_offsets, np.int32), _c(rays.pix, np.int32))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int):
    _load().orc_set_threads(int(n))


def render(grid, rays, opts):
    """Forward render: rgb f64[n,3], z-depth f64[n], nsamp i32[n], stats i64[n,3]."""
    lib = _load()
    R, lo, vs, link, data, deg = _grid_args(grid)
    c2w, intr, off, pix = _ray_args(rays)
    n = rays.n_rays
    rgb = np.zeros((n, 3))
    depth = np.zeros(n)
    nsamp = np.zeros(n, np.int32)
    stats = np.zeros((n, 3), np.int64)
    lib.orc_render(_p(R), _p(lo), vs, _p(link), _p(data), deg, rays.n_frames, _p(c2w), _p(intr),
                   _p(off), _p(pix), n, opts.step_vox, opts.max_samples, opts.t_near,
                   opts.t_stop, opts.color_act, _p(rgb), _p(depth), _p(nsamp), _p(stats))
    return rgb, depth, nsamp, stats


def loss(rays, rgb, depth, targets, opts):
    """Per-frame loss (Eq. 4, 5, 11) and dL/d rgb, dL/d z-depth."""
    lib = _load()
    n = rays.n_rays
    rgb = _c(rgb, np.float64)
    depth = _c(depth, np.float64)
    trgb = _c(targets.rgb, np.float32)
    tdep = _c(targets.depth, np.float32)
    fw = _c(targets.frame_weight, np.float32)
    off = _c(rays.frame_offsets, np.int32)
    L = np.zeros(rays.n_frames)
    g_rgb = np.zeros((n, 3))
    g_depth = np.zeros(n)
    lib.orc_loss(rays.n_frames, _p(off), _p(rgb), _p(depth), _p(trgb), _p(tdep), _p(fw),
                 opts.depth_loss, float(opts.lambda_depth), _p(L), _p(g_rgb), _p(g_depth))
    return L, g_rgb, g_depth


def backward(grid, rays, opts, g_rgb, g_depth, want_grid=True, want_pose=True, flags=None):
    """Gradients: grid f64[n_alloc, record floats] (Eq. 6-10) and pose
    f64[F,6] (Eq. 12-14)."""
    lib = _load()
    R, lo, vs, link, data, deg = _grid_args(grid)
    c2w, intr, off, pix = _ray_args(rays)
    g_rgb = _c(g_rgb, np.float64)
    g_depth = _c(g_depth, np.float64)
    gd = np.zeros((data.shape[0], record_floats(deg))) if want_grid else None
    gp = np.zeros((rays.n_frames, 6)) if want_pose else None
    fl = opts.flags if flags is None else flags
    lib.orc_backward(_p(R), _p(lo), vs, _p(link), _p(data), deg, rays.n_frames, _p(c2w), _p(intr),
                     _p(off), _p(pix), rays.n_rays, opts.step_vox, opts.max_samples, opts.t_near,
                     opts.t_stop, opts.color_act, int(fl), _p(g_rgb), _p(g_depth), _p(gd), _p(gp))
    return gd, gp


def fused(grid, rays, targets, opts, want_grid=True, want_pose=True):
    """Forward, loss and backward of one batch, the way a training step runs it."""
    rgb, depth, nsamp, stats = render(grid, rays, opts)
    L, g_rgb, g_depth = loss(rays, rgb, depth, targets, opts)
    gd, gp = backward(grid, rays, opts, g_rgb, g_depth, want_grid, want_pose)
    return dict(rgb=rgb, depth=depth, nsamp=nsamp, stats=stats, loss=L, g_rgb=g_rgb,
                g_depth=g_depth, grad_data=gd, grad_pose=gp)


def pose_jacobian(grid, rays, opts, flags=None):
    """Per-ray Jacobian f64[n,4,6] of (R, G, B, z-depth) with respect to the
    left se(3) perturbation (rho, phi) of the ray's camera (Eq. 12-14)."""
    lib = _load()
    R, lo, vs, link, data, deg = _grid_args(grid)
    c2w, intr, off, pix = _ray_args(rays)
    J = np.zeros((rays.n_rays, 4, 6))
    fl = opts.flags if flags is None else flags
    lib.orc_pose_jacobian(_p(R), _p(lo), vs, _p(link), _p(data), deg, rays.n_frames, _p(c2w), _p(intr),
                          _p(off), _p(pix), rays.n_rays, opts.step_vox, opts.max_samples,
                          opts.t_near, opts.t_stop, opts.color_act, int(fl), _p(J))
    return J


def gn_system(grid, rays, targets, opts, flags=None):
    """Gauss-Newton normal equations of each frame's squared photometric +
    depth error (Eq. 4, 5 and 11 with the squared depth norm), linearised in
    the frame's se(3) perturbation:
        E_f = w_f sum_r (|C-hat_r - C_r|^2 + lambda (z_r - D_r)^2),
        H_f = w_f sum_r J_r^T W J_r,  g_f = w_f sum_r J_r^T W e_r,
    W = diag(1, 1, 1, lambda), e_r the 4-residual, over the rays with a valid
    depth target.  Returns H f64[F,6,6], g f64[F,6], E f64[F]."""
    rgb, depth, _, _ = render(grid, rays, opts)
    J = pose_jacobian(grid, rays, opts, flags)
    tr = np.asarray(targets.rgb, np.float64)
    td = np.asarray(targets.depth, np.float64)
    with np.errstate(invalid="ignore"):
        valid = np.isfinite(td) & (td > 0)
    lam = float(np.float32(opts.lambda_depth))
    W = np.array([1.0, 1.0, 1.0, lam])
    F = rays.n_frames
    off = np.asarray(rays.frame_offsets)
    H = np.zeros((F, 6, 6))
    g = np.zeros((F, 6))
    E = np.zeros(F)
    for f in range(F):
        sl = slice(int(off[f]), int(off[f + 1]))
        v = valid[sl]
        wf = float(np.float32(targets.frame_weight[f]))
        e = np.concatenate([rgb[sl][v] - tr[sl][v], (depth[sl][v] - td[sl][v])[:, None]], axis=1)
        Jf = J[sl][v]
        H[f] = wf * np.einsum("rki,k,rkj->ij", Jf, W, Jf)
        g[f] = wf * np.einsum("rki,k,rk->i", Jf, W, e)
        E[f] = wf * float(np.sum(W[None, :] * e * e))
    return H, g, E


def gn_pose_step(c2w, H, g, damping):
    """One damped Gauss-Newton step per frame: xi = -(H + damping I)^-1 g,
    then the left retraction c2w <- exp(xi^) c2w."""
    c2w = np.asarray(c2w, np.float64)
    out = np.empty_like(c2w)
    for f in range(c2w.shape[0]):
        xi = -np.linalg.solve(H[f] + damping * np.eye(6), g[f])
        out[f] = apply_left(xi, c2w[f])
    return out


def tv(grid, lambda_sigma, lambda_sh, eps, want_grad=True):
    """Total-variation value and its gradient f64[n_alloc, record floats]."""
    lib = _load()
    R, lo, vs, link, data, deg = _grid_args(grid)
    g = np.zeros((data.shape[0], record_floats(deg))) if want_grad else None
    val = lib.orc_tv(_p(R), _p(link), _p(data), deg, float(lambda_sigma), float(lambda_sh),
                     float(eps), _p(g))
    return float(val), g


def trace(grid, o, d, opts, cap=4096):
    """Per-sample record of one ray: t, sigma_raw, colour, T_i (n+1), w, (C-hat, D-hat)."""
    lib = _load()
    R, lo, vs, link, data, deg = _grid_args(grid)
    o = _c(o, np.float64)
    d = _c(d, np.float64)
    t = np.zeros(cap)
    sr = np.zeros(cap)
    cs = np.zeros((cap, 3))
    T = np.zeros(cap + 1)
    w = np.zeros(cap)
    out = np.zeros(4)
    n = lib.orc_trace(_p(R), _p(lo), vs, _p(link), _p(data), deg, _p(o), _p(d), opts.step_vox,
                      opts.max_samples, opts.t_near, opts.t_stop, opts.color_act, cap,
                      _p(t), _p(sr), _p(cs), _p(T), _p(w), _p(out))
    n = min(n, cap)
    return dict(n=n, t=t[:n], sigma_raw=sr[:n], c=cs[:n], T=T[:n + 1], w=w[:n],
                rgb=out[:3].copy(), D=float(out[3]))


def interp(grid, q, want_grad=True):
    """Interpolated record fields (density, then SH) at voxel point q and
    their Appendix A gradients; the used fields only (28 at degree 2)."""
    lib = _load()
    R, lo, vs, link, data, deg = _grid_args(grid)
    q = _c(q, np.float64)
    val = np.zeros(NREC)
    g = np.zeros((NREC, 3))
    lib.orc_interp(_p(R), _p(lo), vs, _p(link), _p(data), deg, _p(q), _p(val), _p(g))
    m = used_fields(deg)
    return val[:m].copy(), (g[:m].copy() if want_grad else None)


def sh_basis(d):
    lib = _load()
    d = _c(d, np.float64)
    Y = np.zeros(9)
    lib.orc_sh_basis(_p(d), _p(Y))
    return Y


def sh_basis_grad(d):
    lib = _load()
    d = _c(d, np.float64)
    G = np.zeros((9, 3))
    lib.orc_sh_basis_grad(_p(d), _p(G))
    return G


def ray(c2w, intr, u, v):
    """Camera centre o, unit world direction d and |d_cam| for pixel (u, v)."""
    lib = _load()
    c2w = _c(c2w, np.float64)
    intr = _c(intr, np.float64)
    o, d, s = np.zeros(3), np.zeros(3), np.zeros(1)
    lib.orc_ray(_p(c2w), _p(intr), int(u), int(v), _p(o), _p(d), _p(s))
    return o, d, float(s[0])


# ---------------------------------------------------------------------------
# Tracking update: SE(3) exponential and Adam (textbook forms, numpy FP64)
# ---------------------------------------------------------------------------

def hat(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]], np.float64)


def se3_exp(xi):
    """4x4 exp of the twist xi = (rho, phi) (rotation by Rodrigues' formula)."""
    rho, phi = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    th = np.linalg.norm(phi)
    K = hat(phi)
    if th < 1e-12:
        Rm = np.eye(3) + K
        V = np.eye(3) + 0.5 * K
    else:
        Rm = np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * (K @ K)
        V = np.eye(3) + (1 - np.cos(th)) / th ** 2 * K + (th - np.sin(th)) / th ** 3 * (K @ K)
    T = np.eye(4)
    T[:3, :3] = Rm
    T[:3, 3] = V @ rho
    return T


def apply_left(xi, c2w):
    """exp(xi^) * [c2w; 0 0 0 1] as a 3x4 matrix (left, world-frame update)."""
    T = np.eye(4)
    T[:3, :] = np.asarray(c2w, np.float64)
    return (se3_exp(xi) @ T)[:3, :]


def adam_pose_step(c2w, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on each frame's se(3) tangent, then the
    left retraction c2w <- exp(-lr * m_hat / (sqrt(v_hat) + eps)) c2w."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    upd = -lr * mh / (np.sqrt(vh) + eps)
    out = np.stack([apply_left(upd[f], c2w[f]) for f in range(len(c2w))])
    return out, m, v


def rmsprop_grid(data, grad, state, lr_density, lr_sh, alpha, eps):
    """One sparse RMSProp step on the vertex records (mapping optimiser,
    Sec. 5.4).  A record is touched when any of its 28 gradient entries is
    non-zero; touched records update every entry,
        v <- alpha v + (1 - alpha) g^2,   x <- x - lr g / (sqrt(v) + eps),
    with lr_density for entry 0 and lr_sh for the 27 SH entries; untouched
    records keep both their values and their running average.  Returns the
    new (data, state) in FP64; the gradient is consumed (the caller zeroes it)."""
    data = np.array(data, np.float64)
    state = np.array(state, np.float64)
    g = np.asarray(grad, np.float64)
    touched = np.any(g != 0.0, axis=1)
    lr = np.full(g.shape[1], float(lr_sh))
    lr[0] = float(lr_density)
    gt = g[touched]
    v = alpha * state[touched] + (1.0 - alpha) * gt * gt
    state[touched] = v
    data[touched] = data[touched] - lr[None, :] * gt / (np.sqrt(v) + eps)
    return data, state


def grid_upsample(grid):
    """Coarse-to-fine growth of the dynamic grid (Sec. 6.1; the rule is a
    reading, the paper gives none): the lattice of R vertices per axis
    becomes 2R - 1, fine vertex 2v sitting on coarse vertex v (voxel size
    halved, same origin).  A fine vertex is allocated when it lies in (the
    closure of) a coarse cell with an allocated corner, in lattice order;
    its record is the coarse trilinear interpolant at its position (empty
    corners read 0), with the density halved: density is per voxel, so the
    optical depth of a world-length step is unchanged.  Returns a new grid
    (float32 records rounded from FP64)."""
    import dataclasses
    R = np.asarray(grid.reso, np.int64)
    link = np.asarray(grid.link, np.int64).reshape(tuple(R))
    data = np.asarray(grid.data, np.float64)
    alloc = link >= 0
    occ = np.zeros(tuple(R - 1), bool)                      # cell has an allocated corner
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                occ |= alloc[dx:R[0] - 1 + dx, dy:R[1] - 1 + dy, dz:R[2] - 1 + dz]
    Rf = 2 * R - 1

    def cells(axis_n, Rc):
        # coarse cells containing each fine coordinate: even -> v-1, v; odd -> (v-1)/2
        lo = np.where(axis_n % 2 == 0, axis_n // 2 - 1, (axis_n - 1) // 2)
        hi = np.where(axis_n % 2 == 0, axis_n // 2, (axis_n - 1) // 2)
        return np.clip(lo, 0, Rc - 2), np.clip(hi, 0, Rc - 2)

    X, Y, Z = (np.arange(n) for n in Rf)
    xl, xh = cells(X, R[0])
    yl, yh = cells(Y, R[1])
    zl, zh = cells(Z, R[2])
    mask = np.zeros(tuple(Rf), bool)
    for xs in (xl, xh):
        for ys in (yl, yh):
            for zs in (zl, zh):
                mask |= occ[xs[:, None, None], ys[None, :, None], zs[None, None, :]]
    flat = mask.ravel()
    new_link = np.full(flat.size, -1, np.int32)
    idx = np.flatnonzero(flat)
    new_link[idx] = np.arange(idx.size, dtype=np.int32)
    # fine vertex positions in coarse voxel units, and their interpolated records
    fx, fy, fz = np.unravel_index(idx, tuple(Rf))
    q = np.stack([fx, fy, fz], 1) / 2.0
    c = np.minimum(np.floor(q).astype(np.int64), R - 2)
    f = q - c
    vals = np.zeros((idx.size, data.shape[1]))
    for b in range(8):
        o = np.array([(b >> 2) & 1, (b >> 1) & 1, b & 1])
        w = np.prod(np.where(o[None, :] == 1, f, 1.0 - f), axis=1)
        v = c + o[None, :]
        lid = link[v[:, 0], v[:, 1], v[:, 2]]
        ok = lid >= 0
        vals[ok] += w[ok, None] * data[lid[ok]]
    vals[:, 0] *= 0.5
    return dataclasses.replace(grid, reso=tuple(int(r) for r in Rf),
                               voxel_size=np.float32(grid.voxel_size / 2), link=new_link,
                               data=vals.astype(np.float32))


def grid_prune(grid, tau):
    """Prune the dynamic grid (Sec. 6.1; the rule is a reading): records
    whose density is <= tau are dropped, the others keep their order and
    are renumbered, and the link table is rewritten (a dropped vertex
    becomes empty).  Returns a new grid."""
    import dataclasses
    data = np.asarray(grid.data)
    keep = data[:, 0] > np.float32(tau)
    new_id = np.full(data.shape[0], -1, np.int64)
    new_id[keep] = np.arange(int(keep.sum()))
    link = np.asarray(grid.link, np.int64)
    new_link = np.full(link.shape, -1, np.int32)
    live = link >= 0
    new_link[live] = new_id[link[live]]
    return dataclasses.replace(grid, link=new_link, data=data[keep].copy())
