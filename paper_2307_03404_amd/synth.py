"""Seeded synthetic workloads for the five benchmark configurations.

This module only *builds inputs*: voxel grids, camera poses, pixel lists and
RGB-D targets.  It holds none of the rendering arithmetic (no sampling, no
interpolation, no compositing, no gradients).  The FP64 oracle and the HIP
path both consume its outputs; neither shares any other code.

The paper evaluates on Replica and ScanNet (Sec. 6.1), neither of which is
available here.  These generators stand in for them with the shapes the paper
works at: 1200x680 RGB-D frames, grids up to 512^3 vertices (Sec. 6.1,
implementation details), indoor room-like geometry, and missing depth
(pixels with invalid depth are dropped, Sec. 6.1).

Sensor targets come from a small analytic ray caster over the generating
primitives (planes, boxes, spheres): it is a simulated RGB-D camera looking at
the true surfaces, not the volume renderer being tested.

Seeds: ``numpy.random.default_rng(1000 * cfg + component)`` with component
0 = scene, 1 = cameras, 2 = ray subsets, 3 = targets, 4 = perturbations.
"""
from __future__ import annotations

import dataclasses
import os
from dataclasses import dataclass, field

import numpy as np

# Vertex record: 28 floats = 1 density + 3 colour channels x 9 SH coefficients
# (Sec. 5.2, model representation).
REC = 28

COLOR_RELU_SHIFT = 0
COLOR_SIGMOID = 1
COLOR_IDENTITY = 2

DEPTH_L1 = 0
DEPTH_L2 = 1

FLAG_POSE_VIEWDIR = 1


@dataclass
class Grid:
    reso: tuple            # (Rx, Ry, Rz) vertices per axis
    aabb_min: np.ndarray   # f32[3], world position of vertex (0,0,0)
    voxel_size: float      # world length of one voxel edge
    link: np.ndarray       # i32[Rx*Ry*Rz], index (x*Ry+y)*Rz+z, -1 = empty
    data: np.ndarray       # f32[n_alloc][record_floats(sh_degree)]: density, then sh[ch][k]
    sh_degree: int = 2     # 2: the paper's nine coefficients per channel; 0 or 1: the first 1 or 4

    @property
    def n_alloc(self) -> int:
        return int(self.data.shape[0])


def record_floats(sh_degree: int) -> int:
    """Floats per vertex record: density + 3 (d+1)^2 SH coefficients, padded
    to a multiple of four (16-byte records): 4, 16 (13 used) or 28."""
    return {0: 4, 1: 16, 2: 28}[int(sh_degree)]


def with_sh_degree(grid: Grid, sh_degree: int) -> Grid:
    """The same map with records of a lower SH degree: the density and the
    first (d+1)^2 coefficients of each channel, the padding zeroed."""
    d = int(sh_degree)
    if d == grid.sh_degree:
        return grid
    assert d < grid.sh_degree, "only lowers the degree"
    k_old, k_new = (grid.sh_degree + 1) ** 2, (d + 1) ** 2
    src = np.asarray(grid.data, np.float32)
    out = np.zeros((src.shape[0], record_floats(d)), np.float32)
    out[:, 0] = src[:, 0]
    for c in range(3):
        out[:, 1 + c * k_new:1 + (c + 1) * k_new] = src[:, 1 + c * k_old:1 + c * k_old + k_new]
    return dataclasses.replace(grid, data=out, sh_degree=d)


@dataclass
class Rays:
    c2w: np.ndarray            # f32[F][3][4] camera-to-world [R|t], OpenCV axes
    intr: np.ndarray           # f32[F][4] fx, fy, cx, cy
    frame_offsets: np.ndarray  # i32[F+1] CSR: rays of frame f are [off[f], off[f+1])
    pix: np.ndarray            # i32[n_rays][2] (u, v) pixel, centre at +0.5

    @property
    def n_frames(self) -> int:
        return int(self.c2w.shape[0])

    @property
    def n_rays(self) -> int:
        return int(self.pix.shape[0])


@dataclass
class Targets:
    rgb: np.ndarray           # f32[n_rays][3]
    depth: np.ndarray         # f32[n_rays] z-depth; <=0 or non-finite = invalid
    frame_weight: np.ndarray  # f32[F] loss weight of each frame's rays (1/M)


def f32(x) -> float:
    """Round to the nearest float32 so both consumers see identical scalars."""
    return float(np.float32(x))


@dataclass
class Opts:
    step_vox: float = 0.5
    max_samples: int = 2**31 - 1
    t_near: float = 0.0
    t_stop: float = f32(1e-6)
    color_act: int = COLOR_RELU_SHIFT
    depth_loss: int = DEPTH_L1
    lambda_depth: float = 1.0
    flags: int = 0


@dataclass
class Workload:
    name: str
    grid: Grid
    rays: Rays
    targets: Targets
    opts: Opts
    true_c2w: np.ndarray = None     # tracking configs: the unperturbed poses
    meta: dict = field(default_factory=dict)

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


def _rng(cfg: int, comp: int) -> np.random.Generator:
    return np.random.default_rng(1000 * cfg + comp)


# ----------------------------------------------------------------------------
# camera helpers (scene set-up, not rendering)
# ----------------------------------------------------------------------------

def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """3x4 camera-to-world matrix, OpenCV axes (x right, y down, z forward)."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    up = np.asarray(up, np.float64)
    if abs(np.dot(z, up)) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    x = np.cross(z, up)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    m = np.zeros((3, 4))
    m[:, 0], m[:, 1], m[:, 2], m[:, 3] = x, y, z, eye
    return m


def _rotation_about(axis, angle) -> np.ndarray:
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    k = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(angle) * k + (1 - np.cos(angle)) * (k @ k)


def perturb_grid(grid, rng, sigma_scale=(0.5, 1.5), sh_noise=0.05):
    """A starting map for mapping: density scaled by U(sigma_scale), SH plus
    N(0, sh_noise); same link table."""
    data = grid.data.copy()
    data[:, 0] *= rng.uniform(*sigma_scale, size=data.shape[0]).astype(np.float32)
    data[:, 1:] += rng.normal(0.0, sh_noise, size=data[:, 1:].shape).astype(np.float32)
    return dataclasses.replace(grid, data=data)


def perturb_pose(c2w, rng, trans_sigma, rot_sigma_rad) -> np.ndarray:
    """Left-multiplied random rigid perturbation of a 3x4 pose."""
    axis = rng.normal(size=3)
    ang = rng.normal() * rot_sigma_rad
    r = _rotation_about(axis, ang)
    out = np.array(c2w, np.float64)
    out[:, :3] = r @ out[:, :3]
    out[:, 3] = r @ out[:, 3] + rng.normal(size=3) * trans_sigma
    return out


def tile_order(width: int, height: int, tile: int = 8) -> np.ndarray:
    """All pixels of a frame as (u, v), grouped in tile x tile blocks.

    Rays of one block traverse nearly the same voxels, which is what the
    kernels' gather and atomic locality relies on.
    """
    v, u = np.mgrid[0:height, 0:width]
    key = ((v // tile) * ((width + tile - 1) // tile) + (u // tile)) * tile * tile \
        + (v % tile) * tile + (u % tile)
    order = np.argsort(key.ravel(), kind="stable")
    pix = np.stack([u.ravel(), v.ravel()], 1)[order]
    return pix.astype(np.int32)


def subsample_pixels(width, height, n, rng) -> np.ndarray:
    """n distinct pixels, uniform without replacement, in the batch order of
    a sparse subset (Z-order of (u, v); see rayorder.py)."""
    from .rayorder import morton_sort
    flat = np.sort(rng.choice(width * height, size=n, replace=False))
    pix = np.stack([flat % width, flat // width], 1).astype(np.int32)
    return pix[morton_sort(pix)]


# ----------------------------------------------------------------------------
# analytic primitives: unsigned distances (allocation) and a sensor ray caster
# ----------------------------------------------------------------------------

@dataclass
class Scene:
    """Analytic surfaces in world units."""
    room: tuple = None                               # (lo[3], hi[3]) seen from inside
    boxes: list = field(default_factory=list)        # [(lo[3], hi[3])]
    planes: list = field(default_factory=list)       # [(n[3], c)] n.x = c, clipped to room
    spheres: list = field(default_factory=list)      # [(centre[3], radius)]
    background: tuple = None                         # plane (n, c) hit by every ray


def _box_dist(p, lo, hi):
    """Unsigned distance from points p[...,3] to the surface of box [lo,hi]."""
    c = (lo + hi) * 0.5
    h = (hi - lo) * 0.5
    q = np.abs(p - c) - h
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
    inside = np.minimum(np.max(q, axis=-1), 0.0)
    return np.abs(outside + inside)


def scene_distance(scene: Scene, p: np.ndarray) -> np.ndarray:
    d = np.full(p.shape[:-1], np.inf, np.float64)
    if scene.room is not None:
        d = np.minimum(d, _box_dist(p, *scene.room))
    for lo, hi in scene.boxes:
        d = np.minimum(d, _box_dist(p, lo, hi))
    if scene.planes:
        lo, hi = scene.room
        inroom = np.all((p >= lo) & (p <= hi), axis=-1)
        for n, c in scene.planes:
            dp = np.abs(p @ n - c)
            d = np.minimum(d, np.where(inroom, dp, np.inf))
    for cen, rad in scene.spheres:
        d = np.minimum(d, np.abs(np.linalg.norm(p - cen, axis=-1) - rad))
    return d


def _sensor_cast(scene: Scene, o, dz):
    """First-hit parameter along dz (camera z component = 1, so the parameter
    is the sensor's z-depth) and a per-hit primitive id."""
    n = dz.shape[0]
    best = np.full(n, np.inf)
    pid = np.full(n, -1, np.int64)
    inv = 1.0 / np.where(np.abs(dz) < 1e-12, 1e-12, dz)

    def take(t, k):
        nonlocal best, pid
        ok = np.isfinite(t) & (t > 1e-6) & (t < best)
        best = np.where(ok, t, best)
        pid = np.where(ok, k, pid)

    k = 0
    if scene.room is not None:
        lo, hi = scene.room
        t1 = (lo - o) * inv
        t2 = (hi - o) * inv
        take(np.min(np.maximum(t1, t2), axis=1), k)
    k += 1
    for lo, hi in scene.boxes:
        t1 = (lo - o) * inv
        t2 = (hi - o) * inv
        tn = np.max(np.minimum(t1, t2), axis=1)
        tf = np.min(np.maximum(t1, t2), axis=1)
        take(np.where(tf >= tn, tn, np.inf), k)
        k += 1
    for nrm, c in scene.planes:
        den = dz @ nrm
        t = (c - o @ nrm) / np.where(np.abs(den) < 1e-12, 1e-12, den)
        x = o + t[:, None] * dz
        lo, hi = scene.room
        inroom = np.all((x >= lo) & (x <= hi), axis=1)
        take(np.where(inroom, t, np.inf), k)
        k += 1
    for cen, rad in scene.spheres:
        oc = o - cen
        a = np.einsum("ij,ij->i", dz, dz)
        b = np.einsum("ij,ij->i", oc, dz)
        cc = np.einsum("ij,ij->i", oc, oc) - rad * rad
        disc = b * b - a * cc
        sq = np.sqrt(np.maximum(disc, 0.0))
        t = np.where(disc >= 0, (-b - sq) / a, np.inf)
        t = np.where(t > 1e-6, t, np.where(disc >= 0, (-b + sq) / a, np.inf))
        take(t, k)
        k += 1
    if scene.background is not None:
        nrm, c = scene.background
        den = dz @ nrm
        t = (c - o @ nrm) / np.where(np.abs(den) < 1e-12, 1e-12, den)
        take(t, k)
    return best, pid


def sensor_targets(scene: Scene, rays: Rays, rng, depth_noise=0.0, missing=0.0,
                   n_nonfinite=0) -> tuple:
    """Simulated RGB-D measurements of the analytic scene for every ray."""
    rgb = np.zeros((rays.n_rays, 3), np.float32)
    depth = np.zeros(rays.n_rays, np.float32)
    off = rays.frame_offsets
    for f in range(rays.n_frames):
        a, b = int(off[f]), int(off[f + 1])
        if a == b:
            continue
        fx, fy, cx, cy = [float(x) for x in rays.intr[f]]
        px = rays.pix[a:b].astype(np.float64)
        dcam = np.stack([(px[:, 0] + 0.5 - cx) / fx, (px[:, 1] + 0.5 - cy) / fy,
                         np.ones(b - a)], 1)
        m = rays.c2w[f].astype(np.float64)
        dz = dcam @ m[:, :3].T
        o = np.broadcast_to(m[:, 3], dz.shape)
        t, pid = _sensor_cast(scene, o, dz)
        hit = o + np.where(np.isfinite(t), t, 0.0)[:, None] * dz
        phase = (pid[:, None] * np.array([1.3, 2.1, 0.7]))
        col = 0.5 + 0.4 * np.sin(3.0 * hit[:, [0, 1, 2]] + hit[:, [1, 2, 0]] * 1.7 + phase)
        rgb[a:b] = col.astype(np.float32)
        dd = np.where(np.isfinite(t), t, 0.0)
        if depth_noise > 0:
            dd = dd + rng.normal(size=dd.shape) * depth_noise
        if missing > 0:
            dd = np.where(rng.random(dd.shape) < missing, 0.0, dd)
        depth[a:b] = dd.astype(np.float32)
    if n_nonfinite:
        idx = rng.choice(rays.n_rays, size=n_nonfinite, replace=False)
        depth[idx[: n_nonfinite // 2]] = np.nan
        depth[idx[n_nonfinite // 2:]] = np.inf
    return rgb, depth


def frame_weights(depth, frame_offsets, per_frame: bool) -> np.ndarray:
    """1/M: per frame (tracking) or over the whole batch (mapping); Eq. 4-5."""
    valid = np.isfinite(depth) & (depth > 0)
    F = len(frame_offsets) - 1
    w = np.zeros(F, np.float32)
    if per_frame:
        for f in range(F):
            m = int(valid[frame_offsets[f]:frame_offsets[f + 1]].sum())
            w[f] = 1.0 / m if m else 0.0
    else:
        m = int(valid.sum())
        w[:] = 1.0 / m if m else 0.0
    return w


# ----------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------

def _fill_payload(n, rng, dense_sigma):
    data = np.empty((n, REC), np.float32)
    data[:, 0] = dense_sigma
    data[:, 1:] = rng.normal(0.0, 0.3, size=(n, REC - 1)).astype(np.float32)
    return data


def grid_from_mask(reso, aabb_min, vs, mask_flat, sigma_vals, rng) -> Grid:
    link = np.full(mask_flat.size, -1, np.int32)
    idx = np.flatnonzero(mask_flat)
    link[idx] = np.arange(idx.size, dtype=np.int32)
    data = _fill_payload(idx.size, rng, sigma_vals)
    return Grid(tuple(int(r) for r in reso), np.asarray(aabb_min, np.float32), f32(vs), link, data)


def sphere_grid(cfg: int = 1, R: int = 32) -> tuple:
    """Dense R^3 grid on [-1,1]^3; sigma = relu(N(0,1)) inside 3 spheres."""
    rng = _rng(cfg, 0)
    vs = f32(2.0 / (R - 1))
    cen = rng.uniform(-0.6, 0.6, size=(3, 3))
    rad = rng.uniform(0.15, 0.4, size=3)
    i = np.arange(R)
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    p = -1.0 + vs * np.stack([X, Y, Z], -1).reshape(-1, 3)
    inside = np.zeros(p.shape[0], bool)
    for c, r in zip(cen, rad):
        inside |= np.linalg.norm(p - c, axis=1) <= r
    sig = np.where(inside, np.maximum(rng.normal(size=p.shape[0]), 0.0), 0.0)
    grid = grid_from_mask((R, R, R), (-1.0, -1.0, -1.0), vs, np.ones(p.shape[0], bool),
                          sig.astype(np.float32), rng)
    scene = Scene(spheres=[(c, r) for c, r in zip(cen, rad)])
    return grid, scene


def room_grid(cfg: int, R: int, extent: float, occupancy: float) -> tuple:
    """Sparse R^3 room: walls inset 8 voxels, 4 boxes, 2 oblique panels.

    Vertices within distance b of a surface are allocated, with b chosen so
    that the allocated fraction equals ``occupancy``.
    """
    rng = _rng(cfg, 0)
    vs = f32(extent / R)
    aabb_min = np.zeros(3)
    inset = 8 * vs
    top = (R - 1) * vs
    room = (np.full(3, inset), np.full(3, top - inset))
    s = R / 256.0
    boxes = []
    for _ in range(4):
        half = rng.uniform(8, 32, size=3) * s * vs
        cen = rng.uniform(room[0] + half + 16 * vs, room[1] - half - 16 * vs)
        boxes.append((cen - half, cen + half))
    planes = []
    for _ in range(2):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        pt = rng.uniform(room[0] + 0.25 * (room[1] - room[0]), room[1] - 0.25 * (room[1] - room[0]))
        planes.append((n, float(n @ pt)))
    scene = Scene(room=room, boxes=boxes, planes=planes)

    # unsigned distance at every vertex, in voxels, one x-slab at a time
    # (slabs are independent; numpy releases the GIL, so threads share them)
    dist = np.empty(R * R * R, np.float32)
    j = np.arange(R)
    Y, Z = np.meshgrid(j, j, indexing="ij")
    yz = np.stack([Y.ravel(), Z.ravel()], 1).astype(np.float64) * vs

    def slab(x):
        p = np.concatenate([np.full((yz.shape[0], 1), x * vs), yz], 1)
        dist[x * R * R:(x + 1) * R * R] = (scene_distance(scene, p) / vs).astype(np.float32)

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        list(ex.map(slab, range(R)))
    # axis-aligned surfaces put many vertices at exactly the same distance;
    # a tiny seeded jitter breaks those ties so the quantile hits the target
    dist += rng.uniform(0.0, 1e-3, size=dist.size).astype(np.float32)
    sample = dist[rng.integers(0, dist.size, size=min(dist.size, 8_000_000))]
    b = float(np.quantile(sample, occupancy))
    mask = dist <= b
    n = int(mask.sum())
    near = dist[mask] <= 1.0
    sig = np.where(near, np.maximum(rng.normal(3.0, 1.0, size=n), 0.0),
                   np.maximum(rng.normal(0.0, 1.0, size=n), 0.0)).astype(np.float32)
    grid = grid_from_mask((R, R, R), aabb_min, vs, mask, sig, rng)
    return grid, scene


def _room_camera(rng, R, vs, scene=None, clearance_vox=32, pitch_deg=15.0):
    lo = (8 + clearance_vox) * vs
    hi = (R - 1 - 8 - clearance_vox) * vs
    for _ in range(1000):
        eye = rng.uniform(lo, hi, size=3)
        if scene is None or scene_distance(scene, eye[None])[0] >= clearance_vox * vs:
            break
    yaw = rng.uniform(0, 2 * np.pi)
    pitch = np.deg2rad(rng.uniform(-pitch_deg, pitch_deg))
    fwd = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), np.sin(pitch)])
    return look_at(eye, eye + fwd)


W_FULL, H_FULL = 1200, 680
INTR_FULL = (600.0, 600.0, 600.0, 340.0)


def _pack(c2ws, intrs, pix_list) -> Rays:
    off = np.zeros(len(pix_list) + 1, np.int64)
    off[1:] = np.cumsum([p.shape[0] for p in pix_list])
    pix = np.concatenate(pix_list, 0) if pix_list else np.zeros((0, 2), np.int32)
    return Rays(np.asarray(c2ws, np.float32), np.asarray(intrs, np.float32),
                off.astype(np.int32), pix.astype(np.int32))


# ----------------------------------------------------------------------------
# the five configurations
# ----------------------------------------------------------------------------

def config1() -> Workload:
    """Dense 32^3, one 64x64 camera, <=128 samples, L2 colour + L1 depth."""
    grid, scene = sphere_grid(1, 32)
    rng = _rng(1, 1)
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    c2w = look_at(3.0 * v, np.zeros(3))
    scene.background = (-v, 0.0)          # a plane through the origin facing the camera
    v_, u_ = np.mgrid[0:64, 0:64]
    pix = np.stack([u_.ravel(), v_.ravel()], 1).astype(np.int32)
    rays = _pack([c2w], [(64.0, 64.0, 32.0, 32.0)], [pix])
    rgb, depth = sensor_targets(scene, rays, _rng(1, 3), depth_noise=0.01, missing=0.05,
                                n_nonfinite=8)
    tg = Targets(rgb, depth, frame_weights(depth, rays.frame_offsets, False))
    opts = Opts(step_vox=0.5, max_samples=128, t_near=0.0, t_stop=f32(1e-6),
                color_act=COLOR_RELU_SHIFT, depth_loss=DEPTH_L1, lambda_depth=1.0)
    return Workload("c1_dense32_64x64", grid, rays, tg, opts, meta={"scene": scene})


def config2() -> Workload:
    """Sparse 256^3 room (~10 % allocated), one 1200x680 frame, mapping + TV."""
    grid, scene = room_grid(2, 256, 5.12, 0.10)
    rng = _rng(2, 1)
    c2w = _room_camera(rng, 256, grid.voxel_size, scene)
    rays = _pack([c2w], [INTR_FULL], [tile_order(W_FULL, H_FULL)])
    rgb, depth = sensor_targets(scene, rays, _rng(2, 3), depth_noise=0.01, missing=0.0)
    tg = Targets(rgb, depth, frame_weights(depth, rays.frame_offsets, False))
    opts = Opts(step_vox=0.5, depth_loss=DEPTH_L1)
    return Workload("c2_room256_1200x680_mapping", grid, rays, tg, opts,
                    meta={"scene": scene, "tv": (1e-5, 1e-6, 1e-9)})


def config3(grid_scene=None) -> Workload:
    """Tracking on the 32^3 grid: 16 frames x 2k-50k rays, perturbed poses."""
    grid, scene = grid_scene if grid_scene is not None else sphere_grid(1, 32)
    rng = _rng(3, 1)
    cen, rad = scene.spheres[0] if scene.spheres else (np.zeros(3), 0.3)
    true, start, pix = [], [], []
    counts = rng.integers(2000, 50001, size=16)
    rsub = _rng(3, 2)
    rper = _rng(3, 4)
    for f in range(16):
        sidx = f % len(scene.spheres)
        cen, rad = scene.spheres[sidx]
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        surf = cen + rad * n
        eye = surf + n * rng.uniform(0.3, 0.8)
        tgt = surf + rng.normal(size=3) * np.tan(np.deg2rad(10.0)) * np.linalg.norm(eye - surf) / np.sqrt(3)
        m = look_at(eye, tgt)
        true.append(m)
        start.append(perturb_pose(m, rper, 0.5 * grid.voxel_size, np.deg2rad(0.5)))
        pix.append(subsample_pixels(W_FULL, H_FULL, int(counts[f]), rsub))
    rays_true = _pack(true, [INTR_FULL] * 16, pix)
    scene_bg = dataclasses.replace(scene, background=None)
    rgb, depth = sensor_targets(scene_bg, rays_true, _rng(3, 3))
    rays = dataclasses.replace(rays_true, c2w=np.asarray(start, np.float32))
    tg = Targets(rgb, depth, frame_weights(depth, rays.frame_offsets, True))
    opts = Opts(step_vox=0.5, max_samples=128, depth_loss=DEPTH_L1)
    return Workload("c3_track32_16frames", grid, rays, tg, opts,
                    true_c2w=np.asarray(true, np.float32), meta={"scene": scene, "mode": "tracking", "iters": 20})


_C4_CACHE = {}


def room512():
    if "g" not in _C4_CACHE:
        _C4_CACHE["g"] = room_grid(4, 512, 10.24, 0.03)
    return _C4_CACHE["g"]


def config4() -> Workload:
    """Sparse 512^3 room (~3 %), 8 keyframes x 1200x680, fused mapping."""
    grid, scene = room512()
    rng = _rng(4, 1)
    c2ws = [_room_camera(rng, 512, grid.voxel_size, scene) for _ in range(8)]
    full = tile_order(W_FULL, H_FULL)
    rays = _pack(c2ws, [INTR_FULL] * 8, [full] * 8)
    rgb, depth = sensor_targets(scene, rays, _rng(4, 3), depth_noise=0.01, missing=0.05)
    tg = Targets(rgb, depth, frame_weights(depth, rays.frame_offsets, False))
    opts = Opts(step_vox=0.5, depth_loss=DEPTH_L1)
    return Workload("c4_room512_8x1200x680_mapping", grid, rays, tg, opts, meta={"scene": scene})


def config5() -> Workload:
    """512^3 room, 64 frames with 1k-200k rays each: mapping + tracking."""
    grid, scene = room512()
    rng = _rng(5, 1)
    rsub = _rng(5, 2)
    c2ws, pix = [], []
    counts = rng.integers(1000, 200001, size=64)
    for f in range(64):
        c2ws.append(_room_camera(rng, 512, grid.voxel_size, scene))
        pix.append(subsample_pixels(W_FULL, H_FULL, int(counts[f]), rsub))
    rays = _pack(c2ws, [INTR_FULL] * 64, pix)
    rgb, depth = sensor_targets(scene, rays, _rng(5, 3), depth_noise=0.01, missing=0.05)
    tg = Targets(rgb, depth, frame_weights(depth, rays.frame_offsets, True))
    opts = Opts(step_vox=0.5, depth_loss=DEPTH_L1)
    return Workload("c5_room512_64frames_mixed", grid, rays, tg, opts, meta={"scene": scene})


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def subset_rays(wl: Workload, n: int, seed: int = 7) -> Workload:
    """Seeded ray subset shared by both sides of a parity test (CSR kept)."""
    R = wl.rays.n_rays
    if n >= R:
        return wl
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(R, size=n, replace=False))
    off = wl.rays.frame_offsets
    fid = np.searchsorted(off, sel, side="right") - 1
    new_off = np.zeros_like(off)
    new_off[1:] = np.cumsum(np.bincount(fid, minlength=wl.rays.n_frames))
    rays = dataclasses.replace(wl.rays, pix=wl.rays.pix[sel].copy(), frame_offsets=new_off.astype(np.int32))
    tg = dataclasses.replace(wl.targets, rgb=wl.targets.rgb[sel].copy(), depth=wl.targets.depth[sel].copy())
    return wl.replace(rays=rays, targets=tg)


def random_tiny_grid(rng, R=6, margin=2, sh_degree0=False, sigma_lo=0.1, sigma_hi=2.0,
                     occupancy=1.0) -> Grid:
    """Small grid for pins: random payload, empty `margin`-vertex shell."""
    n = R ** 3
    i = np.arange(R)
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    core = ((X >= margin) & (X < R - margin) & (Y >= margin) & (Y < R - margin)
            & (Z >= margin) & (Z < R - margin)).ravel()
    mask = core & (rng.random(n) < occupancy)
    sig = rng.uniform(sigma_lo, sigma_hi, size=int(mask.sum())).astype(np.float32)
    g = grid_from_mask((R, R, R), (-1.0, -1.0, -1.0), 2.0 / (R - 1), mask, sig, rng)
    if sh_degree0:
        keep = np.zeros(REC, bool)
        keep[[0, 1, 10, 19]] = True
        g.data[:, ~keep] = 0.0
    return g
