"""Batching around the fused kernel: ray packer, autotuner, captured tracking loop.

* pack_frames: many frames with uneven ray counts -> one CSR ray batch whose
  rays are ordered inside each frame for coherent waves (8x8 pixel tiles for
  a full frame, Z-order for a sparse subset; rayorder.py), plus the
  permutation back to the caller's order.
* Autotuner: times pxm_render_fused over launch shapes (rays per workgroup x
  plain/persistent tile queue) on the real inputs and caches the winner per
  problem signature in a JSON file.  Run it before any graph capture.
* TrackingGraph: `iters` tracking iterations (fused forward + loss + pose
  backward for every frame, then the Adam pose update) captured once into a
  HIP graph and replayed without host round trips (Sec. 5.3-5.4).
* MappingLoop: mapping iterations over keyframes (random rays, fused grid
  gradient, TV, sparse RMSProp), and image_metrics (PSNR, L1 depth).
"""
from __future__ import annotations

import dataclasses

import json
import os
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import pxm
from .rayorder import frame_order, morton_sort, tile_sort  # noqa: F401 (re-exported)


@dataclass
class PackedRays:
    c2w: np.ndarray            # f32 [F, 3, 4]
    intr: np.ndarray           # f32 [F, 4]
    frame_offsets: np.ndarray  # i32 [F + 1]
    pix: np.ndarray            # i32 [n, 2]
    order: np.ndarray          # i64 [n]: packed ray j is input ray order[j]

    @property
    def n_frames(self):
        return int(self.c2w.shape[0])

    @property
    def n_rays(self):
        return int(self.pix.shape[0])


def pack_frames(frames, width: int, tile: int = 8, height: int | None = None) -> PackedRays:
    """frames: iterable of (c2w [3,4], intr [4], pix [n_f, 2]) of images
    `width` x `height` pixels (height defaults to the largest v + 1 seen).
    Rays keep their frame grouping (CSR); inside a frame they are reordered
    for coherent waves (rayorder.frame_order)."""
    frames = [(m, k, np.asarray(p, np.int32).reshape(-1, 2)) for m, k, p in frames]
    if height is None:
        height = max([int(p[:, 1].max()) + 1 for _, _, p in frames if p.shape[0]] or [1])
    c2w, intr, pix, order, counts = [], [], [], [], []
    base = 0
    for m, k, p in frames:
        perm = frame_order(p, width, height, tile)
        c2w.append(np.asarray(m, np.float32).reshape(3, 4))
        intr.append(np.asarray(k, np.float32).reshape(4))
        pix.append(p[perm])
        order.append(base + perm)
        counts.append(p.shape[0])
        base += p.shape[0]
    off = np.zeros(len(counts) + 1, np.int64)
    off[1:] = np.cumsum(counts)
    if off[-1] > np.iinfo(np.int32).max:
        raise ValueError("too many rays for int32 CSR offsets")
    return PackedRays(np.stack(c2w), np.stack(intr), off.astype(np.int32),
                      np.concatenate(pix) if pix else np.zeros((0, 2), np.int32),
                      np.concatenate(order) if order else np.zeros(0, np.int64))


# ----------------------------------------------------------------------------
# autotuner
# ----------------------------------------------------------------------------

CANDIDATES = [(b, v) for b in (64, 128, 256) for v in (0, 1, 2)]


def _signature(grid, rays, opts, want) -> str:
    return "r%s_n%d_rays%d_f%d_w%d_fl%d_act%d" % (
        "x".join(str(int(x)) for x in grid.reso), grid.n_alloc, rays.n_rays, rays.n_frames,
        int(want), int(opts.flags), int(opts.color_act))


class Autotuner:
    """Chooses pxm_set_tuning(block, variant) for pxm_render_fused by timing."""

    def __init__(self, cache_path: str | None = None, reps: int = 5, warmup: int = 2):
        self.cache_path = cache_path or os.path.join(
            os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "pxm", "tune.json")
        self.reps, self.warmup = reps, warmup
        self.cache = {}
        if os.path.exists(self.cache_path):
            try:
                with open(self.cache_path) as fh:
                    self.cache = json.load(fh)
            except (OSError, ValueError):
                self.cache = {}

    def _save(self):
        try:
            os.makedirs(os.path.dirname(self.cache_path), exist_ok=True)
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(self.cache, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)
        except OSError:
            pass

    def tune(self, grid, rays, opts, tgt_rgb, tgt_depth, frame_weight, want, grad_data=None,
             grad_pose=None, force=False):
        """Returns ((block, variant), {candidate: ms}) and applies the winner."""
        sig = _signature(grid, rays, opts, want)
        if not force and sig in self.cache:
            b, v = self.cache[sig]["best"]
            pxm.set_tuning(b, v)
            return (b, v), self.cache[sig]["ms"]
        dev = grid.data.device
        if grad_data is None and want & pxm.WANT_GRID:
            grad_data = torch.zeros_like(grid.data)
        if grad_pose is None and want & pxm.WANT_POSE:
            grad_pose = torch.zeros(rays.n_frames, 6, dtype=torch.float64, device=dev)
        ws = pxm.new_workspace(grid, rays, opts, want)
        results = {}
        old = pxm.get_tuning()
        try:
            for b, v in CANDIDATES:
                pxm.set_tuning(b, v)
                call = lambda: pxm.render_fused(grid, rays, opts, tgt_rgb, tgt_depth, frame_weight,
                                                want, grad_data=grad_data, grad_pose=grad_pose,
                                                ws=ws)
                for _ in range(self.warmup):
                    call()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(self.reps):
                    call()
                e1.record()
                torch.cuda.synchronize()
                results["%d/%d" % (b, v)] = e0.elapsed_time(e1) / self.reps
        finally:
            pxm.set_tuning(*old)
        best = min(results, key=results.get)
        b, v = (int(x) for x in best.split("/"))
        pxm.set_tuning(b, v)
        self.cache[sig] = {"best": [b, v], "ms": results, "time": time.time()}
        self._save()
        return (b, v), results


# ----------------------------------------------------------------------------
# captured tracking loop
# ----------------------------------------------------------------------------

class TrackingGraph:
    """`iters` tracking iterations for all frames of `rays`, captured once.

    method "adam": each iteration is the fused forward + loss + pose backward
    (PXM_WANT_POSE) into grad_pose, then pxm_pose_adam, which updates rays.c2w
    in place and zeroes grad_pose.  method "gauss-newton": pxm_render_gn
    accumulates every frame's normal equations, then pxm_pose_gn solves and
    retracts (and zeroes them).  losses[it, f] holds the energy of frame f
    before update it.
    """

    def __init__(self, grid, rays, opts, tgt_rgb, tgt_depth, frame_weight, iters=20, lr=1e-3,
                 betas=(0.9, 0.999), eps=1e-8, method="adam", damping=1e-6):
        dev = grid.data.device
        F = rays.n_frames
        if method not in ("adam", "gauss-newton"):
            raise ValueError("method must be 'adam' or 'gauss-newton'")
        self.grid, self.rays, self.opts = grid, rays, opts
        self.tgt = (tgt_rgb, tgt_depth, frame_weight)
        self.iters, self.lr, self.betas, self.eps = iters, lr, betas, eps
        self.method, self.damping = method, float(damping)
        self.grad_pose = torch.zeros(F, 6, dtype=torch.float64, device=dev)
        self.gn = torch.zeros(F, pxm.GN_VALUES, dtype=torch.float64, device=dev)
        self.state = torch.zeros(F, 16, dtype=torch.float64, device=dev)
        self.losses = torch.zeros(iters, F, dtype=torch.float64, device=dev)
        self.ws = pxm.new_workspace(grid, rays, opts, pxm.WANT_POSE)
        self.graph = None

    def _body(self):
        self.grad_pose.zero_()
        self.gn.zero_()
        self.losses.zero_()
        for it in range(self.iters):
            if self.method == "adam":
                pxm.render_fused(self.grid, self.rays, self.opts, *self.tgt, pxm.WANT_POSE,
                                 loss=self.losses[it], grad_pose=self.grad_pose, ws=self.ws)
                pxm.pose_adam(self.rays.c2w, self.grad_pose, self.state, self.lr, self.betas[0],
                              self.betas[1], self.eps)
            else:
                # losses hold the squared (Gauss-Newton) energy of each frame
                pxm.render_gn(self.grid, self.rays, self.opts, *self.tgt, gn=self.gn)
                self.losses[it].copy_(self.gn[:, pxm.GN_VALUES - 1])
                pxm.pose_gn(self.rays.c2w, self.gn, self.damping)

    def run_eager(self):
        self._body()

    def capture(self):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):          # warm-up outside the capture
            pass
        torch.cuda.current_stream().wait_stream(s)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._body()
        return self

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def reset(self, c2w: torch.Tensor):
        """Restore the starting poses and clear the optimiser state."""
        self.rays.c2w.copy_(c2w)
        self.state.zero_()
        self.gn.zero_()


class MappingLoop:
    """Mapping iterations over a set of keyframes (Sec. 5.4, Sec. 6.1).

    Each iteration draws `n_rays` rays uniformly (with replacement) from all
    keyframe pixels, runs one fused launch for the loss and its grid gradient
    (rays without a valid depth are dropped by the kernel; the loss weight is
    1/M over the valid rays of the batch), adds the TV gradient and applies one
    sparse RMSProp step to the vertex records, which also clears the gradient.
    The random draw is the only host-side decision and stays on the device
    (a seeded torch generator); `last_indices` keeps the rays of the latest
    iteration so that a test can replay it.
    """

    def __init__(self, grid, keyframes, tgt_rgb, tgt_depth, opts, n_rays, lr_density, lr_sh,
                 alpha=0.95, eps=1e-8, tv=(1e-5, 1e-6, 1e-9), seed=0):
        dev = grid.data.device
        self.grid, self.kf, self.opts = grid, keyframes, opts
        self.tgt_rgb, self.tgt_depth = tgt_rgb, tgt_depth
        self.n_rays = int(n_rays)
        self.lr = (float(lr_density), float(lr_sh))
        self.alpha, self.eps, self.tv = float(alpha), float(eps), tuple(tv)
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(int(seed))
        self.grad = torch.zeros_like(grid.data)
        self.state = torch.zeros_like(grid.data)
        F = keyframes.c2w.shape[0]
        self.loss = torch.zeros(F, dtype=torch.float64, device=dev)
        self.ws = None
        self.last_indices = None
        self._frame_ids = torch.repeat_interleave(
            torch.arange(F, device=dev),
            (keyframes.frame_offsets[1:] - keyframes.frame_offsets[:-1]).long())

    def sample(self, indices=None):
        """The ray batch of one iteration: sorted keyframe ray indices -> CSR
        rays (frames in order), their targets and the 1/M weight."""
        kf, dev = self.kf, self.grid.data.device
        n_all = int(kf.pix.shape[0])
        if indices is None:
            indices = torch.randint(0, n_all, (self.n_rays,), device=dev, generator=self.gen)
        idx = torch.sort(indices).values
        fid = self._frame_ids[idx]
        F = kf.c2w.shape[0]
        counts = torch.bincount(fid, minlength=F)
        off = torch.zeros(F + 1, dtype=torch.int32, device=dev)
        off[1:] = torch.cumsum(counts, 0).to(torch.int32)
        rays = pxm.DeviceRays(kf.c2w, kf.intr, off, kf.pix[idx].contiguous())
        rgb = self.tgt_rgb[idx].contiguous()
        depth = self.tgt_depth[idx].contiguous()
        valid = torch.isfinite(depth) & (depth > 0)
        w = (1.0 / valid.sum().clamp(min=1).to(torch.float32)).expand(F).contiguous()
        return idx, rays, rgb, depth, w

    def grow(self):
        """Coarse-to-fine growth of the map (Sec. 6.1's dynamic grid; see
        pxm.grid_upsample): the voxel size halves while step_vox stays, so
        samples along a ray become twice as dense, and max_samples doubles
        to keep covering the same distance.  The records are new, so the
        RMSProp running averages restart at zero."""
        self.grid = pxm.grid_upsample(self.grid)
        self.opts = dataclasses.replace(self.opts, max_samples=min(2 * int(self.opts.max_samples),
                                                                   2 ** 31 - 1))
        self._new_records()
        return self.grid

    def prune(self, tau):
        """Drop the records with density <= tau (pxm.grid_prune); the
        running averages restart at zero."""
        self.grid = pxm.grid_prune(self.grid, tau)
        self._new_records()
        return self.grid

    def _new_records(self):
        self.grad = torch.zeros_like(self.grid.data)
        self.state = torch.zeros_like(self.grid.data)

    def step(self, indices=None):
        idx, rays, rgb, depth, w = self.sample(indices)
        self.last_indices = idx
        if self.ws is None:
            self.ws = pxm.new_workspace(self.grid, rays, self.opts, pxm.WANT_GRID)
        self.loss.zero_()
        # the gradient is zero here (grid_rmsprop clears it): the TV term is
        # written first and the rendering backward adds onto it
        if self.tv[0] or self.tv[1]:
            pxm.tv_grad_set(self.grid, self.tv[0], self.tv[1], self.tv[2], self.grad)
        pxm.render_fused(self.grid, rays, self.opts, rgb, depth, w, pxm.WANT_GRID, loss=self.loss,
                         grad_data=self.grad, ws=self.ws)
        pxm.grid_rmsprop(self.grid.data, self.grad, self.state, self.lr[0], self.lr[1],
                         self.alpha, self.eps, sh_degree=self.grid.sh_degree)
        return self.loss.sum()


def image_metrics(grid, rays, opts, tgt_rgb, tgt_depth):
    """PSNR of the rendered colour and mean absolute z-depth error over the
    pixels with a valid depth (the map-quality metrics of Sec. 6.1)."""
    rgb, depth, _ = pxm.render_forward(grid, rays, opts)
    valid = torch.isfinite(tgt_depth) & (tgt_depth > 0)
    mse = ((rgb - tgt_rgb) ** 2)[valid].mean()
    psnr = -10.0 * torch.log10(mse)
    l1 = (depth - tgt_depth)[valid].abs().mean()
    return float(psnr), float(l1)
