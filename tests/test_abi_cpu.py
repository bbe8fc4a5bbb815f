"""The C ABI library loads, exports every declared symbol, and rejects bad
arguments on the host (before anything touches a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2307_03404_amd import pxm, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pxm.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pxm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = pxm.lib()
    names = declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(pxm.EXPORTS) == set(names)
    assert pxm.abi_version() == 7


def test_status_strings():
    L = pxm.lib()
    assert L.pxm_status_string(0) == b"ok"
    assert L.pxm_status_string(4) == b"workspace too small"
    assert L.pxm_status_string(99) == b"unknown status"


FAKE = 0x10000   # never dereferenced: every call below fails validation first


def good_grid():
    g = pxm._Grid()
    g.reso[:] = [8, 8, 8]
    g.aabb_min[:] = [0.0, 0.0, 0.0]
    g.voxel_size = 0.1
    g.link = FAKE
    g.n_alloc = 10
    g.data = FAKE
    g.sh_degree = 2
    return g


def good_rays(n=5):
    r = pxm._Rays()
    r.n_frames = 1
    r.c2w = FAKE
    r.intr = FAKE
    r.n_rays = n
    r.frame_offsets = FAKE
    r.pix = FAKE
    return r


def good_opts():
    o = pxm._Opts()
    o.step_vox = 0.5
    o.max_samples = 128
    o.t_near = 0.0
    o.t_stop = 1e-6
    o.color_act = 0
    o.depth_loss = 0
    o.lambda_depth = 1.0
    o.flags = 0
    return o


def fwd(g, r, o, outs=(FAKE, FAKE, FAKE)):
    return pxm.lib().pxm_render_forward(C.byref(g) if g is not None else None,
                                        C.byref(r) if r is not None else None,
                                        C.byref(o) if o is not None else None, *outs, None)


@pytest.mark.parametrize("mutate,code", [
    (lambda g, r, o: g.reso.__setitem__(1, 1), 2),
    (lambda g, r, o: setattr(g, "voxel_size", 0.0), 1),
    (lambda g, r, o: setattr(g, "voxel_size", float("nan")), 1),
    (lambda g, r, o: g.aabb_min.__setitem__(0, float("inf")), 1),
    (lambda g, r, o: setattr(g, "link", None), 1),
    (lambda g, r, o: setattr(g, "data", FAKE + 4), 1),
    (lambda g, r, o: setattr(g, "n_alloc", -1), 1),
    (lambda g, r, o: setattr(r, "n_frames", 0), 1),
    (lambda g, r, o: setattr(r, "n_rays", -3), 1),
    (lambda g, r, o: setattr(r, "pix", None), 1),
    (lambda g, r, o: setattr(o, "step_vox", 0.0), 1),
    (lambda g, r, o: setattr(o, "step_vox", float("inf")), 1),
    (lambda g, r, o: setattr(o, "max_samples", 0), 1),
    (lambda g, r, o: setattr(o, "t_stop", 1.0), 1),
    (lambda g, r, o: setattr(o, "t_stop", -0.1), 1),
    (lambda g, r, o: setattr(o, "t_near", -1.0), 1),
    (lambda g, r, o: setattr(o, "color_act", 3), 1),
    (lambda g, r, o: setattr(o, "depth_loss", 2), 1),
    (lambda g, r, o: setattr(o, "flags", 8), 1),
    (lambda g, r, o: setattr(g, "sh_degree", 3), 1),
    (lambda g, r, o: setattr(g, "sh_degree", -1), 1),
])
def test_forward_rejects_bad_arguments(mutate, code):
    g, r, o = good_grid(), good_rays(), good_opts()
    mutate(g, r, o)
    assert fwd(g, r, o) == code
    assert pxm.lib().pxm_last_error()


def test_null_descriptors_and_outputs():
    assert fwd(None, good_rays(), good_opts()) == 1
    assert fwd(good_grid(), None, good_opts()) == 1
    assert fwd(good_grid(), good_rays(), None) == 1
    assert fwd(good_grid(), good_rays(), good_opts(), (FAKE, None, FAKE)) == 1


def test_zero_rays_is_a_noop():
    assert fwd(good_grid(), good_rays(0), good_opts()) == 0


def test_backward_and_fused_argument_checks():
    L = pxm.lib()
    g, r, o = good_grid(), good_rays(), good_opts()
    args = [C.byref(g), C.byref(r), C.byref(o)]
    assert L.pxm_render_backward_grid(*args, FAKE, FAKE, FAKE, FAKE, FAKE, None, None) == 1
    assert L.pxm_render_backward_pose(*args, FAKE, FAKE, FAKE, None, FAKE, FAKE, None) == 1
    # fused: unknown want bit, missing grad buffers, small workspace
    assert L.pxm_render_fused(*args, FAKE, FAKE, FAKE, 16, None, None, None, None, None, None,
                              FAKE, 4096, None) == 1
    assert L.pxm_render_fused(*args, FAKE, FAKE, FAKE, 1, None, None, None, None, None, None,
                              FAKE, 4096, None) == 1
    assert L.pxm_render_fused(*args, FAKE, FAKE, FAKE, 2, None, None, None, None, None, None,
                              FAKE, 4096, None) == 1
    assert L.pxm_render_fused(*args, FAKE, FAKE, FAKE, 0, None, None, None, None, None, None,
                              FAKE, 8, None) == 4
    assert L.pxm_render_fused(*args, FAKE, FAKE, FAKE, 0, None, None, None, None, None, None,
                              None, 4096, None) == 1
    assert L.pxm_render_fused(*args, FAKE, FAKE, FAKE, 0, None, None, None, None, None, None,
                              FAKE + 8, 1 << 20, None) == 1
    # queue counters, then 184 bytes of per-ray state for n_rays rounded up to 64
    assert L.pxm_workspace_bytes(*args, 3) == 256 + 64 * 184


def test_tv_adam_and_tuning_checks():
    L = pxm.lib()
    g = good_grid()
    assert L.pxm_tv_grad(C.byref(g), 1.0, 1.0, 0.0, FAKE, None) == 1
    assert L.pxm_tv_grad(C.byref(g), float("nan"), 1.0, 1e-9, FAKE, None) == 1
    assert L.pxm_tv_grad(C.byref(g), 1.0, 1.0, 1e-9, None, None) == 1
    assert L.pxm_tv_grad_set(C.byref(g), 1.0, 1.0, 0.0, FAKE, None) == 1
    assert L.pxm_tv_grad_set(C.byref(g), 1.0, float("inf"), 1e-9, FAKE, None) == 1
    assert L.pxm_tv_grad_set(C.byref(g), 1.0, 1.0, 1e-9, None, None) == 1
    assert L.pxm_tv_grad_set(C.byref(g), 1.0, 1.0, 1e-9, FAKE + 4, None) == 1   # 16-byte alignment
    assert L.pxm_pose_adam(0, FAKE, FAKE, FAKE, 1e-3, 0.9, 0.999, 1e-8, None) == 1
    assert L.pxm_pose_adam(2, FAKE, FAKE, FAKE, 1e-3, 1.0, 0.999, 1e-8, None) == 1
    assert L.pxm_pose_adam(2, FAKE, FAKE, None, 1e-3, 0.9, 0.999, 1e-8, None) == 1
    assert L.pxm_grid_rmsprop(0, 2, None, None, None, 0.1, 0.01, 0.9, 1e-8, None) == 0
    assert L.pxm_grid_rmsprop(-1, 2, FAKE, FAKE, FAKE, 0.1, 0.01, 0.9, 1e-8, None) == 1
    assert L.pxm_grid_rmsprop(4, 2, FAKE, FAKE, FAKE, 0.1, 0.01, 1.0, 1e-8, None) == 1
    assert L.pxm_grid_rmsprop(4, 2, FAKE, FAKE, FAKE, -0.1, 0.01, 0.9, 1e-8, None) == 1
    assert L.pxm_grid_rmsprop(4, 2, FAKE, FAKE, FAKE, 0.1, 0.01, 0.9, 0.0, None) == 1
    assert L.pxm_grid_rmsprop(4, 2, FAKE, None, FAKE, 0.1, 0.01, 0.9, 1e-8, None) == 1
    assert L.pxm_grid_rmsprop(4, 3, FAKE, FAKE, FAKE, 0.1, 0.01, 0.9, 1e-8, None) == 1
    assert L.pxm_grid_rmsprop(4, -1, FAKE, FAKE, FAKE, 0.1, 0.01, 0.9, 1e-8, None) == 1
    assert L.pxm_grid_rmsprop(4, 2, FAKE + 4, FAKE, FAKE, 0.1, 0.01, 0.9, 1e-8,
                              None) == 1
    assert L.pxm_set_tuning(100, 0) == 1
    assert L.pxm_set_tuning(256, 3) == 1
    before = pxm.get_tuning()
    pxm.set_tuning(64, 2)
    assert pxm.get_tuning() == (64, 2)
    pxm.set_tuning(128, 1)
    assert pxm.get_tuning() == (128, 1)
    pxm.set_tuning(*before)


def test_grid_edit_checks():
    """Workspace sizing and host-side rejection of the dynamic-grid calls."""
    L = pxm.lib()
    g = good_grid()
    need = L.pxm_grid_edit_workspace_bytes(C.byref(g))
    # coarse row bits (64 rows x 1 word), 15 x 15 fine rows x 1 word of flags and of prefixes, one chunk total
    assert need == 256 + 2 * 1024 + 256
    big = good_grid()
    big.n_alloc = 100_000
    assert L.pxm_grid_edit_workspace_bytes(C.byref(big)) == 2 * 12544 + 256 + 400_000
    bad = good_grid()
    bad.reso[0] = 1
    assert L.pxm_grid_edit_workspace_bytes(C.byref(bad)) == 0
    WS = 0x100000            # 256-byte aligned, never dereferenced
    up = L.pxm_grid_upsample_link
    assert up(C.byref(g), FAKE, FAKE, WS, need - 1, None) == 4
    assert up(C.byref(g), FAKE, FAKE, WS + 16, need, None) == 1
    assert up(C.byref(g), None, FAKE, WS, need, None) == 1
    assert up(C.byref(g), FAKE, None, WS, need, None) == 1
    huge = good_grid()
    huge.reso[:] = [1025, 1025, 1025]     # 2049^3 fine vertices > 2^31 - 1
    assert up(C.byref(huge), FAKE, FAKE, WS, 1 << 40, None) == 2
    ud = L.pxm_grid_upsample_data
    assert ud(C.byref(g), FAKE, 0, None, None) == 0          # nothing to write
    assert ud(C.byref(g), FAKE, -1, FAKE, None) == 1
    assert ud(C.byref(g), FAKE, 15 ** 3 + 1, FAKE, None) == 1
    assert ud(C.byref(g), FAKE, 10, FAKE + 4, None) == 1
    assert ud(C.byref(g), None, 10, FAKE, None) == 1
    pr = L.pxm_grid_prune
    out = 0x200000
    assert pr(C.byref(g), float("nan"), out, out, FAKE, WS, need, None) == 1
    assert pr(C.byref(g), 0.0, None, out, FAKE, WS, need, None) == 1
    assert pr(C.byref(g), 0.0, out, out, None, WS, need, None) == 1
    assert pr(C.byref(g), 0.0, out, FAKE, FAKE, WS, need, None) == 1      # data_out is grid.data
    assert pr(C.byref(g), 0.0, out, FAKE + 512, FAKE, WS, need, None) == 1  # overlaps it
    assert pr(C.byref(g), 0.0, FAKE + 4, out, FAKE, WS, need, None) == 1   # link_out overlaps link
    assert pr(C.byref(g), 0.0, out, out + 4, FAKE, WS, need, None) == 1    # misaligned data_out
    assert pr(C.byref(g), 0.0, out, out, FAKE, WS, need - 1, None) == 4


def test_binding_rejects_host_tensors():
    import torch
    grid = pxm.DeviceGrid((2, 2, 2), (0, 0, 0), 1.0, torch.zeros(8, dtype=torch.int32),
                          torch.zeros(1, 28))
    with pytest.raises(ValueError):
        grid.struct()


def test_upload_helpers_build_descriptors():
    """grid_to_device / rays_to_device assemble their dataclasses (on host
    tensors here); handing them to the library is refused off the GPU."""
    wl = synth.subset_rays(synth.config1(), 10)
    g = pxm.grid_to_device(wl.grid, device="cpu", occupancy=False)
    r = pxm.rays_to_device(wl.rays, device="cpu")
    assert tuple(g.data.shape) == (wl.grid.n_alloc, 28) and g.link.numel() == 32 ** 3
    assert r.n_rays == 10 and r.n_frames == 1 and r.frame_offsets.tolist() == [0, 10]
    with pytest.raises(ValueError):
        r.struct()


def test_noalloc_fused_argument_checks_and_size_limit():
    """The allocation-free fused step checks its arguments like
    pxm_render_fused, and refuses, on the host, a two-launch call whose
    per-ray state would not fit its static scratch."""
    L = pxm.lib()
    g, r, o = good_grid(), good_rays(), good_opts()
    args = [C.byref(g), C.byref(r), C.byref(o)]
    assert L.pxm_render_fused_noalloc(*args, FAKE, FAKE, FAKE, 16, None, None, None, None, None,
                                      None, None) == 1
    assert L.pxm_render_fused_noalloc(*args, FAKE, FAKE, FAKE, 1, None, None, None, None, None,
                                      None, None) == 1
    assert L.pxm_render_fused_noalloc(*args, FAKE, FAKE, FAKE, 2, None, None, None, None, None,
                                      None, None) == 1
    assert L.pxm_render_fused_noalloc(*args, None, FAKE, FAKE, 0, None, None, None, None, None,
                                      None, None) == 1
    old = (C.c_int32(), C.c_int32())
    L.pxm_get_tuning(C.byref(old[0]), C.byref(old[1]))
    try:
        assert L.pxm_set_tuning(64, 2) == 0
        big = good_rays(pxm.NOALLOC_MAX_SPLIT_RAYS + 1)
        st = L.pxm_render_fused_noalloc(C.byref(g), C.byref(big), C.byref(o), FAKE, FAKE, FAKE, 3,
                                        None, None, None, FAKE, FAKE, None, None)
        assert st == 2 and b"static scratch" in L.pxm_last_error()
        zero = good_rays(0)
        assert L.pxm_render_fused_noalloc(C.byref(g), C.byref(zero), C.byref(o), FAKE, FAKE, FAKE,
                                          3, None, None, None, FAKE, FAKE, None, None) == 0
    finally:
        L.pxm_set_tuning(old[0].value, old[1].value)
    # the limit in the binding is the header's
    text = open(HEADER).read()
    assert f"#define PXM_NOALLOC_MAX_SPLIT_RAYS {pxm.NOALLOC_MAX_SPLIT_RAYS}" in text
    assert pxm.NOALLOC_SCRATCH_BYTES == 32 << 20 and "(32u << 20)" in text


def test_deterministic_scatter_workspace_and_noalloc_refusal():
    """The deterministic grid scatter adds an n_alloc x S int64 buffer to the
    fused workspace, and the allocation-free entry point refuses it."""
    L = pxm.lib()
    g, r, o = good_grid(), good_rays(), good_opts()
    args = [C.byref(g), C.byref(r), C.byref(o)]
    base = 256 + 64 * 184
    assert L.pxm_workspace_bytes(*args, 3) == base
    assert L.pxm_workspace_bytes(*args, 3 | 8) == base + 256 * ((10 * 28 * 8 + 255) // 256)
    assert L.pxm_workspace_bytes(*args, 2 | 8) == base          # no grid gradient, no buffer
    g.sh_degree = 1
    assert L.pxm_workspace_bytes(*args, 1 | 8) == base + 256 * ((10 * 16 * 8 + 255) // 256)
    g.sh_degree = 2
    assert L.pxm_render_fused(*args, FAKE, FAKE, FAKE, 1 | 8, None, None, None, FAKE, None, None,
                              FAKE, base, None) == 4                # workspace too small
    assert L.pxm_render_fused(*args, FAKE, FAKE, FAKE, 16, None, None, None, FAKE, None, None,
                              FAKE, 1 << 20, None) == 1             # unknown bit
    st = L.pxm_render_fused_noalloc(*args, FAKE, FAKE, FAKE, 1 | 8, None, None, None, FAKE, None,
                                    None, None)
    assert st == 2 and b"workspace" in L.pxm_last_error()


def test_read_probe_argument_checks():
    L = pxm.lib()
    assert L.pxm_probe_read_bandwidth(None, 1 << 20, 1, FAKE, 2048 * 256, None) == 1
    assert L.pxm_probe_read_bandwidth(FAKE, 1 << 20, 1, None, 2048 * 256, None) == 1
    assert L.pxm_probe_read_bandwidth(FAKE + 4, 1 << 20, 1, FAKE, 2048 * 256, None) == 1
    assert L.pxm_probe_read_bandwidth(FAKE, 100, 1, FAKE, 2048 * 256, None) == 1
    assert L.pxm_probe_read_bandwidth(FAKE, 1 << 20, 0, FAKE, 2048 * 256, None) == 1
    assert L.pxm_probe_read_bandwidth(FAKE, 1 << 20, 1, FAKE, 1000, None) == 4
