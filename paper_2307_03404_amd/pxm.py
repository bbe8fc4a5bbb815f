"""Python binding of libpxm (ctypes over the C ABI in include/pxm.h).

Argument marshalling only: every step of rendering and differentiation runs in
the HIP kernels of libpxm.so.  torch supplies device memory and the current
stream.  If the library is missing it is built once with hipcc; if that is not
possible every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from dataclasses import dataclass

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# PXM_LIBRARY selects another build of the same library (e.g. one whose host
# code is built with sanitizers, for the CPU-side argument-check tests)
LIB_PATH = os.environ.get("PXM_LIBRARY") or os.path.join(_PKG, "libpxm.so")
REC = 28                      # floats per record at SH degree 2


def record_floats(sh_degree: int) -> int:
    """Floats per vertex record of SH degree 0, 1 or 2 (PXM_RECORD_FLOATS)."""
    return {0: 4, 1: 16, 2: 28}[int(sh_degree)]

COLOR_RELU_SHIFT, COLOR_SIGMOID, COLOR_IDENTITY = 0, 1, 2
DEPTH_L1, DEPTH_L2 = 0, 1
FLAG_POSE_VIEWDIR = 1
WANT_GRID, WANT_POSE, WANT_STATS, WANT_DETERMINISTIC = 1, 2, 4, 8

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "device error",
          4: "workspace too small"}


class PxmError(RuntimeError):
    def __init__(self, fn, status, detail):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {detail}")
        self.status = status


class _Grid(C.Structure):
    _fields_ = [("reso", C.c_int32 * 3), ("aabb_min", C.c_float * 3), ("voxel_size", C.c_float),
                ("link", C.c_void_p), ("n_alloc", C.c_int64), ("data", C.c_void_p),
                ("occ", C.c_void_p), ("sh_degree", C.c_int32)]


class _Rays(C.Structure):
    _fields_ = [("n_frames", C.c_int32), ("c2w", C.c_void_p), ("intr", C.c_void_p),
                ("n_rays", C.c_int64), ("frame_offsets", C.c_void_p), ("pix", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("step_vox", C.c_float), ("max_samples", C.c_int32), ("t_near", C.c_float),
                ("t_stop", C.c_float), ("color_act", C.c_int32), ("depth_loss", C.c_int32),
                ("lambda_depth", C.c_float), ("flags", C.c_int32)]


_lib = None
_lock = threading.Lock()
EXPORTS = ("pxm_render_forward", "pxm_render_backward_grid", "pxm_render_backward_pose",
           "pxm_tv_grad", "pxm_tv_grad_set", "pxm_render_fused", "pxm_render_fused_noalloc",
           "pxm_pose_adam", "pxm_grid_rmsprop", "pxm_render_gn", "pxm_pose_gn",
           "pxm_grid_edit_workspace_bytes", "pxm_grid_upsample_link", "pxm_grid_upsample_data",
           "pxm_probe_read_bandwidth",
           "pxm_grid_prune",
           "pxm_workspace_bytes",
           "pxm_occupancy_words", "pxm_build_occupancy",
           "pxm_set_tuning", "pxm_get_tuning", "pxm_status_string", "pxm_last_error",
           "pxm_abi_version")


def lib():
    """Load libpxm.so (building it once with hipcc if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        L = C.CDLL(LIB_PATH)
        P, i32, i64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
        G, R, O = C.POINTER(_Grid), C.POINTER(_Rays), C.POINTER(_Opts)
        L.pxm_render_forward.argtypes = [G, R, O, P, P, P, P]
        L.pxm_render_backward_grid.argtypes = [G, R, O, P, P, P, P, P, P, P]
        L.pxm_render_backward_pose.argtypes = [G, R, O, P, P, P, P, P, P, P]
        L.pxm_tv_grad.argtypes = [G, f32, f32, f32, P, P]
        L.pxm_tv_grad_set.argtypes = [G, f32, f32, f32, P, P]
        L.pxm_render_fused.argtypes = [G, R, O, P, P, P, i32, P, P, P, P, P, P, P, sz, P]
        L.pxm_render_fused_noalloc.argtypes = [G, R, O, P, P, P, i32, P, P, P, P, P, P, P]
        L.pxm_pose_adam.argtypes = [i32, P, P, P, f32, f32, f32, f32, P]
        L.pxm_grid_rmsprop.argtypes = [i64, i32, P, P, P, f32, f32, f32, f32, P]
        L.pxm_render_gn.argtypes = [G, R, O, P, P, P, P, P]
        L.pxm_pose_gn.argtypes = [i32, P, P, f32, P]
        L.pxm_probe_read_bandwidth.argtypes = [P, sz, i32, P, sz, P]
        L.pxm_probe_read_bandwidth.restype = C.c_int
        L.pxm_grid_edit_workspace_bytes.argtypes = [G]
        L.pxm_grid_edit_workspace_bytes.restype = sz
        L.pxm_grid_upsample_link.argtypes = [G, P, P, P, sz, P]
        L.pxm_grid_upsample_data.argtypes = [G, P, i64, P, P]
        L.pxm_grid_prune.argtypes = [G, f32, P, P, P, P, sz, P]
        L.pxm_occupancy_words.argtypes = [G]
        L.pxm_occupancy_words.restype = sz
        L.pxm_build_occupancy.argtypes = [G, P, sz, P]
        L.pxm_build_occupancy.restype = C.c_int
        L.pxm_workspace_bytes.argtypes = [G, R, O, i32]
        L.pxm_workspace_bytes.restype = sz
        L.pxm_set_tuning.argtypes = [i32, i32]
        L.pxm_get_tuning.argtypes = [C.POINTER(i32), C.POINTER(i32)]
        L.pxm_get_tuning.restype = None
        L.pxm_status_string.argtypes = [C.c_int]
        L.pxm_status_string.restype = C.c_char_p
        L.pxm_last_error.restype = C.c_char_p
        for name in ("pxm_render_forward", "pxm_render_backward_grid", "pxm_render_backward_pose",
                     "pxm_tv_grad", "pxm_tv_grad_set", "pxm_render_fused", "pxm_render_fused_noalloc",
                     "pxm_pose_adam", "pxm_set_tuning",
                     "pxm_grid_upsample_link", "pxm_grid_upsample_data", "pxm_grid_prune"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(fn, status):
    if status != 0:
        raise PxmError(fn, status, lib().pxm_last_error().decode(errors="replace"))


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, name, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on a GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    return t


# ----------------------------------------------------------------------------
# device-resident inputs
# ----------------------------------------------------------------------------

@dataclass
class DeviceGrid:
    reso: tuple
    aabb_min: tuple
    voxel_size: float
    link: torch.Tensor      # int32 [Rx*Ry*Rz]
    data: torch.Tensor      # float32 [n_alloc, record_floats(sh_degree)]
    occ: torch.Tensor = None  # int32 words of the occupancy bitfield (optional)
    sh_degree: int = 2      # 2: nine SH coefficients per channel (the paper's); 1 or 0

    @property
    def n_alloc(self):
        return int(self.data.shape[0])

    def struct(self, data=None) -> _Grid:
        d = self.data if data is None else data
        _need(self.link, "grid.link", torch.int32, (int(np.prod(self.reso)),))
        _need(d, "grid.data", torch.float32, (self.n_alloc, record_floats(self.sh_degree)))
        g = _Grid()
        g.reso[:] = [int(x) for x in self.reso]
        g.aabb_min[:] = [float(x) for x in self.aabb_min]
        g.voxel_size = float(self.voxel_size)
        g.link = self.link.data_ptr()
        g.n_alloc = self.n_alloc
        g.data = d.data_ptr()
        g.occ = self.occ.data_ptr() if self.occ is not None else None
        g.sh_degree = int(self.sh_degree)
        return g

    def with_data(self, data) -> "DeviceGrid":
        """Same structure (links, occupancy) with another payload tensor."""
        return DeviceGrid(self.reso, self.aabb_min, self.voxel_size, self.link, data, self.occ,
                          self.sh_degree)

    def build_occupancy(self, stream=None) -> "DeviceGrid":
        """(Re)build the occupancy bitfield from the link table."""
        g = self.struct()
        g.occ = None
        n = int(lib().pxm_occupancy_words(C.byref(g)))
        occ = torch.empty(n, dtype=torch.int32, device=self.link.device)
        _check("build_occupancy", lib().pxm_build_occupancy(C.byref(g), _ptr(occ), n,
                                                           _stream(stream)))
        self.occ = occ
        return self


@dataclass
class DeviceRays:
    c2w: torch.Tensor            # float32 [F, 3, 4]
    intr: torch.Tensor           # float32 [F, 4]
    frame_offsets: torch.Tensor  # int32 [F+1]
    pix: torch.Tensor            # int32 [n_rays, 2]

    @property
    def n_frames(self):
        return int(self.c2w.shape[0])

    @property
    def n_rays(self):
        return int(self.pix.shape[0])

    def struct(self) -> _Rays:
        F = self.n_frames
        _need(self.c2w, "rays.c2w", torch.float32, (F, 3, 4))
        _need(self.intr, "rays.intr", torch.float32, (F, 4))
        _need(self.frame_offsets, "rays.frame_offsets", torch.int32, (F + 1,))
        _need(self.pix, "rays.pix", torch.int32, (self.n_rays, 2))
        r = _Rays()
        r.n_frames = F
        r.c2w = self.c2w.data_ptr()
        r.intr = self.intr.data_ptr()
        r.n_rays = self.n_rays
        r.frame_offsets = self.frame_offsets.data_ptr()
        r.pix = self.pix.data_ptr()
        return r


def opts_struct(o) -> _Opts:
    s = _Opts()
    s.step_vox = float(o.step_vox)
    s.max_samples = int(o.max_samples)
    s.t_near = float(o.t_near)
    s.t_stop = float(o.t_stop)
    s.color_act = int(o.color_act)
    s.depth_loss = int(o.depth_loss)
    s.lambda_depth = float(o.lambda_depth)
    s.flags = int(o.flags)
    return s


def grid_to_device(grid, device="cuda", occupancy=True) -> DeviceGrid:
    g = DeviceGrid(tuple(int(r) for r in grid.reso), tuple(float(x) for x in grid.aabb_min),
                   float(grid.voxel_size),
                   torch.from_numpy(np.ascontiguousarray(grid.link, np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(grid.data, np.float32)).to(device),
                   sh_degree=int(getattr(grid, "sh_degree", 2)))
    if occupancy:
        g.build_occupancy()
    return g


def rays_to_device(rays, device="cuda") -> DeviceRays:
    off = np.ascontiguousarray(rays.frame_offsets, np.int32)
    return DeviceRays(torch.from_numpy(np.ascontiguousarray(rays.c2w, np.float32)).to(device),
                      torch.from_numpy(np.ascontiguousarray(rays.intr, np.float32)).to(device),
                      torch.from_numpy(off).to(device),
                      torch.from_numpy(np.ascontiguousarray(rays.pix, np.int32)).to(device))


# ----------------------------------------------------------------------------
# entry points (same names as the C ABI without the pxm_ prefix)
# ----------------------------------------------------------------------------

def render_forward(grid: DeviceGrid, rays: DeviceRays, opts, rgb=None, depth=None, nsamp=None,
                   stream=None):
    n = rays.n_rays
    dev = grid.data.device
    rgb = torch.empty(n, 3, device=dev) if rgb is None else _need(rgb, "rgb", torch.float32, (n, 3))
    depth = torch.empty(n, device=dev) if depth is None else _need(depth, "depth", torch.float32, (n,))
    nsamp = (torch.empty(n, dtype=torch.int32, device=dev) if nsamp is None
             else _need(nsamp, "nsamp", torch.int32, (n,)))
    g, r, o = grid.struct(), rays.struct(), opts_struct(opts)
    _check("render_forward", lib().pxm_render_forward(C.byref(g), C.byref(r), C.byref(o), _ptr(rgb),
                                                      _ptr(depth), _ptr(nsamp), _stream(stream)))
    return rgb, depth, nsamp


def _bwd_inputs(rays, rgb, depth, nsamp, g_rgb, g_depth):
    n = rays.n_rays
    _need(rgb, "rgb", torch.float32, (n, 3))
    _need(depth, "depth", torch.float32, (n,))
    _need(nsamp, "nsamp", torch.int32, (n,))
    _need(g_rgb, "g_rgb", torch.float32, (n, 3))
    _need(g_depth, "g_depth", torch.float32, (n,))


def render_backward_grid(grid, rays, opts, rgb, depth, nsamp, g_rgb, g_depth, grad_data=None,
                         stream=None):
    _bwd_inputs(rays, rgb, depth, nsamp, g_rgb, g_depth)
    if grad_data is None:
        grad_data = torch.zeros_like(grid.data)
    _need(grad_data, "grad_data", torch.float32, tuple(grid.data.shape))
    g, r, o = grid.struct(), rays.struct(), opts_struct(opts)
    _check("render_backward_grid", lib().pxm_render_backward_grid(
        C.byref(g), C.byref(r), C.byref(o), _ptr(rgb), _ptr(depth), _ptr(nsamp), _ptr(g_rgb),
        _ptr(g_depth), _ptr(grad_data), _stream(stream)))
    return grad_data


def render_backward_pose(grid, rays, opts, rgb, depth, nsamp, g_rgb, g_depth, grad_pose=None,
                         stream=None):
    _bwd_inputs(rays, rgb, depth, nsamp, g_rgb, g_depth)
    if grad_pose is None:
        grad_pose = torch.zeros(rays.n_frames, 6, dtype=torch.float64, device=grid.data.device)
    _need(grad_pose, "grad_pose", torch.float64, (rays.n_frames, 6))
    g, r, o = grid.struct(), rays.struct(), opts_struct(opts)
    _check("render_backward_pose", lib().pxm_render_backward_pose(
        C.byref(g), C.byref(r), C.byref(o), _ptr(rgb), _ptr(depth), _ptr(nsamp), _ptr(g_rgb),
        _ptr(g_depth), _ptr(grad_pose), _stream(stream)))
    return grad_pose


def tv_grad(grid, lambda_density, lambda_sh, eps, grad_data=None, stream=None):
    """grad_data += dTV/d record (pxm_tv_grad)."""
    if grad_data is None:
        grad_data = torch.zeros_like(grid.data)
    _need(grad_data, "grad_data", torch.float32, tuple(grid.data.shape))
    g = grid.struct()
    _check("tv_grad", lib().pxm_tv_grad(C.byref(g), float(lambda_density), float(lambda_sh),
                                        float(eps), _ptr(grad_data), _stream(stream)))
    return grad_data


def tv_grad_set(grid, lambda_density, lambda_sh, eps, grad_data=None, stream=None):
    """grad_data = dTV/d record on the used fields of every linked record
    (pxm_tv_grad_set); other entries keep their contents."""
    if grad_data is None:
        grad_data = torch.zeros_like(grid.data)
    _need(grad_data, "grad_data", torch.float32, tuple(grid.data.shape))
    g = grid.struct()
    _check("tv_grad_set", lib().pxm_tv_grad_set(C.byref(g), float(lambda_density), float(lambda_sh),
                                                float(eps), _ptr(grad_data), _stream(stream)))
    return grad_data


def workspace_bytes(grid, rays, opts, want) -> int:
    g, r, o = grid.struct(), rays.struct(), opts_struct(opts)
    return int(lib().pxm_workspace_bytes(C.byref(g), C.byref(r), C.byref(o), int(want)))


def new_workspace(grid, rays, opts, want):
    """Zeroed workspace for render_fused (the kernel leaves it zeroed again)."""
    nb = workspace_bytes(grid, rays, opts, want)
    return torch.zeros((nb + 7) // 8, dtype=torch.int64, device=grid.data.device)


def render_fused(grid, rays, opts, tgt_rgb, tgt_depth, frame_weight, want, rgb=None, depth=None,
                 loss=None, grad_data=None, grad_pose=None, stats=None, ws=None, stream=None):
    n, F = rays.n_rays, rays.n_frames
    _need(tgt_rgb, "tgt_rgb", torch.float32, (n, 3))
    _need(tgt_depth, "tgt_depth", torch.float32, (n,))
    _need(frame_weight, "frame_weight", torch.float32, (F,))
    if rgb is not None:
        _need(rgb, "rgb", torch.float32, (n, 3))
    if depth is not None:
        _need(depth, "depth", torch.float32, (n,))
    if loss is not None:
        _need(loss, "loss", torch.float64, (F,))
    if grad_data is not None:
        _need(grad_data, "grad_data", torch.float32, tuple(grid.data.shape))
    if grad_pose is not None:
        _need(grad_pose, "grad_pose", torch.float64, (F, 6))
    if stats is not None:
        _need(stats, "stats", torch.int64, (4,))
    if ws is None:
        ws = new_workspace(grid, rays, opts, want)
    g, r, o = grid.struct(), rays.struct(), opts_struct(opts)
    _check("render_fused", lib().pxm_render_fused(
        C.byref(g), C.byref(r), C.byref(o), _ptr(tgt_rgb), _ptr(tgt_depth), _ptr(frame_weight),
        int(want), _ptr(rgb), _ptr(depth), _ptr(loss), _ptr(grad_data), _ptr(grad_pose),
        _ptr(stats), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return dict(rgb=rgb, depth=depth, loss=loss, grad_data=grad_data, grad_pose=grad_pose,
                stats=stats)


NOALLOC_SCRATCH_BYTES = 32 << 20
NOALLOC_MAX_SPLIT_RAYS = 182336


def render_fused_noalloc(grid, rays, opts, tgt_rgb, tgt_depth, frame_weight, want, rgb=None,
                         depth=None, loss=None, grad_data=None, grad_pose=None, stats=None,
                         stream=None):
    """render_fused without a workspace: the library's static per-GPU scratch
    serves instead (calls that overlap on one GPU race).  Raises PxmError
    (unsupported) above NOALLOC_MAX_SPLIT_RAYS rays under launch variant 2."""
    n, F = rays.n_rays, rays.n_frames
    _need(tgt_rgb, "tgt_rgb", torch.float32, (n, 3))
    _need(tgt_depth, "tgt_depth", torch.float32, (n,))
    _need(frame_weight, "frame_weight", torch.float32, (F,))
    for t, name, dt, shp in ((rgb, "rgb", torch.float32, (n, 3)), (depth, "depth", torch.float32, (n,)),
                             (loss, "loss", torch.float64, (F,)),
                             (grad_data, "grad_data", torch.float32, tuple(grid.data.shape)),
                             (grad_pose, "grad_pose", torch.float64, (F, 6)),
                             (stats, "stats", torch.int64, (4,))):
        if t is not None:
            _need(t, name, dt, shp)
    g, r, o = grid.struct(), rays.struct(), opts_struct(opts)
    _check("render_fused_noalloc", lib().pxm_render_fused_noalloc(
        C.byref(g), C.byref(r), C.byref(o), _ptr(tgt_rgb), _ptr(tgt_depth), _ptr(frame_weight),
        int(want), _ptr(rgb), _ptr(depth), _ptr(loss), _ptr(grad_data), _ptr(grad_pose),
        _ptr(stats), _stream(stream)))
    return dict(rgb=rgb, depth=depth, loss=loss, grad_data=grad_data, grad_pose=grad_pose,
                stats=stats)


def pose_adam(c2w, grad_pose, state, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    F = int(c2w.shape[0])
    _need(c2w, "c2w", torch.float32, (F, 3, 4))
    _need(grad_pose, "grad_pose", torch.float64, (F, 6))
    _need(state, "state", torch.float64, (F, 16))
    _check("pose_adam", lib().pxm_pose_adam(F, _ptr(c2w), _ptr(grad_pose), _ptr(state), float(lr),
                                            float(beta1), float(beta2), float(eps),
                                            _stream(stream)))


GN_VALUES = 28


def render_gn(grid, rays, opts, tgt_rgb, tgt_depth, frame_weight, gn=None, stream=None):
    """Gauss-Newton normal equations per frame, accumulated into gn f64[F, 28]
    (H upper triangle 21, g 6, E 1)."""
    n, F = rays.n_rays, rays.n_frames
    dev = grid.data.device
    _need(tgt_rgb, "tgt_rgb", torch.float32, (n, 3))
    _need(tgt_depth, "tgt_depth", torch.float32, (n,))
    _need(frame_weight, "frame_weight", torch.float32, (F,))
    if gn is None:
        gn = torch.zeros(F, GN_VALUES, dtype=torch.float64, device=dev)
    _need(gn, "gn", torch.float64, (F, GN_VALUES))
    g, r, o = grid.struct(), rays.struct(), opts_struct(opts)
    _check("render_gn", lib().pxm_render_gn(C.byref(g), C.byref(r), C.byref(o), _ptr(tgt_rgb),
                                            _ptr(tgt_depth), _ptr(frame_weight), _ptr(gn),
                                            _stream(stream)))
    return gn


def pose_gn(c2w, gn, damping=1e-6, stream=None):
    """Damped Gauss-Newton pose step per frame (in place); zeroes gn."""
    F = int(c2w.shape[0])
    _need(c2w, "c2w", torch.float32, (F, 3, 4))
    _need(gn, "gn", torch.float64, (F, GN_VALUES))
    _check("pose_gn", lib().pxm_pose_gn(F, _ptr(c2w), _ptr(gn), float(damping), _stream(stream)))


def gn_unpack(gn):
    """(H [F,6,6], g [F,6], E [F]) from the packed rows of render_gn."""
    gn = torch.as_tensor(gn)
    F = gn.shape[0]
    H = torch.zeros(F, 6, 6, dtype=gn.dtype, device=gn.device)
    iu = torch.triu_indices(6, 6)
    H[:, iu[0], iu[1]] = gn[:, :21]
    H[:, iu[1], iu[0]] = gn[:, :21]
    return H, gn[:, 21:27], gn[:, 27]


def grid_rmsprop(data, grad_data, state, lr_density, lr_sh, alpha=0.95, eps=1e-8, stream=None,
                 sh_degree=2):
    """Sparse RMSProp step on the vertex records (in place); zeroes grad_data."""
    n = int(data.shape[0])
    S = record_floats(sh_degree)
    _need(data, "data", torch.float32, (n, S))
    _need(grad_data, "grad_data", torch.float32, (n, S))
    _need(state, "state", torch.float32, (n, S))
    _check("grid_rmsprop", lib().pxm_grid_rmsprop(n, int(sh_degree), _ptr(data), _ptr(grad_data), _ptr(state),
                                                  float(lr_density), float(lr_sh), float(alpha),
                                                  float(eps), _stream(stream)))


# ----------------------------------------------------------------------------
# dynamic grid: coarse-to-fine growth and pruning
# ----------------------------------------------------------------------------

def grid_edit_workspace(grid: DeviceGrid) -> torch.Tensor:
    """Scratch for grid_upsample / grid_prune on this grid (contents free)."""
    n = int(lib().pxm_grid_edit_workspace_bytes(C.byref(grid.struct())))
    return torch.empty(max(n, 256), dtype=torch.uint8, device=grid.link.device)


def _sync(stream):
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()


def grid_upsample_link(grid: DeviceGrid, ws=None, stream=None):
    """Link table of the doubled lattice and its record count (device int64)."""
    g = grid.struct()
    reso = tuple(2 * int(r) - 1 for r in grid.reso)
    link = torch.empty(int(np.prod(reso)), dtype=torch.int32, device=grid.link.device)
    n = torch.zeros(1, dtype=torch.int64, device=grid.link.device)
    ws = grid_edit_workspace(grid) if ws is None else ws
    _check("grid_upsample_link", lib().pxm_grid_upsample_link(
        C.byref(g), _ptr(link), _ptr(n), _ptr(ws), ws.numel(), _stream(stream)))
    return reso, link, n


def grid_upsample(grid: DeviceGrid, ws=None, occupancy=True, stream=None) -> DeviceGrid:
    """Coarse-to-fine growth: 2R - 1 vertices per axis, voxel size halved.
    Synchronises `stream` once to read the fine record count."""
    reso, link, n = grid_upsample_link(grid, ws, stream)
    _sync(stream)
    n_fine = int(n.item())
    data = torch.empty((n_fine, record_floats(grid.sh_degree)), dtype=torch.float32,
                       device=grid.link.device)
    _check("grid_upsample_data", lib().pxm_grid_upsample_data(
        C.byref(grid.struct()), _ptr(link), n_fine, _ptr(data), _stream(stream)))
    out = DeviceGrid(reso, grid.aabb_min, float(np.float32(grid.voxel_size) / np.float32(2)), link, data,
                     sh_degree=grid.sh_degree)
    if occupancy:
        out.build_occupancy(stream)
    return out


def grid_prune(grid: DeviceGrid, tau: float, ws=None, in_place=False, occupancy=True,
               stream=None) -> DeviceGrid:
    """Drop records with density <= tau; survivors keep their order.  With
    in_place the link table of `grid` itself is rewritten, so `grid` (old
    payload, new links) must not be used afterwards: use the returned grid.
    Synchronises `stream` once to read the surviving count."""
    g = grid.struct()
    link = grid.link if in_place else torch.empty_like(grid.link)
    data = torch.empty_like(grid.data)
    n = torch.zeros(1, dtype=torch.int64, device=grid.link.device)
    ws = grid_edit_workspace(grid) if ws is None else ws
    _check("grid_prune", lib().pxm_grid_prune(C.byref(g), float(tau), _ptr(link), _ptr(data), _ptr(n),
                                              _ptr(ws), ws.numel(), _stream(stream)))
    _sync(stream)
    out = DeviceGrid(grid.reso, grid.aabb_min, grid.voxel_size, link, data[:int(n.item())],
                     sh_degree=grid.sh_degree)
    if occupancy:
        out.build_occupancy(stream)
    return out


def probe_read_bandwidth(buf: torch.Tensor, passes: int, sink: torch.Tensor = None, stream=None):
    """Streaming reads of `buf` (each XCD its own eighth), `passes` times:
    a cache-level read ceiling to compare the fused kernel's traffic with."""
    if sink is None:
        sink = torch.empty(2048 * 256, dtype=torch.float32, device=buf.device)
    nbytes = buf.numel() * buf.element_size()
    _check("probe_read_bandwidth", lib().pxm_probe_read_bandwidth(
        _ptr(buf), nbytes, int(passes), _ptr(sink), sink.numel(), _stream(stream)))
    return sink


def set_tuning(block: int, variant: int):
    _check("set_tuning", lib().pxm_set_tuning(int(block), int(variant)))


def get_tuning():
    b, v = C.c_int32(), C.c_int32()
    lib().pxm_get_tuning(C.byref(b), C.byref(v))
    return int(b.value), int(v.value)


def abi_version() -> int:
    return int(lib().pxm_abi_version())
