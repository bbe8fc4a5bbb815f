"""Parity on the 512^3 room (4,027,586 records, 3 % occupancy): the eight
1200x680 keyframes (6,528,000 rays) and the mixed batch of 64 frames with
1k-200k rays each (6.8 M rays).

* Seeded 32k-ray subsets of both batches (rays of many frames, incoherent
  within a wave: the broadcast form of the grid scatter) and a contiguous
  block of 8x8 pixel tiles of one keyframe (coherent: the matrix-core
  form), in one launch and in two: every output element against the oracle.
* The whole batches, in the launch configuration the benchmark times
  (64 rays per workgroup, persistent tile queue, one or two launches).
  Rays are independent, so sampled rays' colour and depth are checked one by
  one.  The grid gradient is a sum over every ray; to compare it element by
  element, the same full-size launch is repeated with the loss weight of all
  but a few frames set to zero, which leaves exactly the oracle's gradient
  of those frames' rays (their loss and pose gradients are checked too, and
  every other frame's must be exactly zero).
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2307_03404_amd import synth
from tests._parity import TAU_FWD, TAU_GRAD, assert_pose, assert_r28, reference

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_03404_amd import pxm
    return pxm


def np_(t):
    return t.detach().cpu().numpy()


def _frame(wl, f):
    off = wl.rays.frame_offsets
    a, b = int(off[f]), int(off[f + 1])
    rays = synth.Rays(wl.rays.c2w[f:f + 1], wl.rays.intr[f:f + 1],
                      np.array([0, b - a], np.int32), wl.rays.pix[a:b])
    tg = synth.Targets(wl.targets.rgb[a:b], wl.targets.depth[a:b],
                       wl.targets.frame_weight[f:f + 1])
    return wl.replace(name=f"{wl.name} frame {f}", rays=rays, targets=tg), a, b


@pytest.fixture(scope="module")
def c4():
    return synth.config4()


@pytest.fixture(scope="module")
def c5():
    return synth.config5()


def run_fused(wl, block, variant, fw=None, tgt_depth=None, want=3):
    pxm = _dev()
    n, F = wl.rays.n_rays, wl.rays.n_frames
    print(f"[gpu] {wl.name}: {n} rays, {F} frames, block {block}, variant {variant}", flush=True)
    g = pxm.grid_to_device(wl.grid)
    r = pxm.rays_to_device(wl.rays)
    trgb = torch.from_numpy(wl.targets.rgb).cuda()
    tdep = torch.from_numpy(wl.targets.depth if tgt_depth is None else tgt_depth).cuda()
    fwt = torch.from_numpy(wl.targets.frame_weight if fw is None else fw).cuda()
    rgb = torch.empty(n, 3, device="cuda")
    depth = torch.empty(n, device="cuda")
    loss = torch.zeros(F, dtype=torch.float64, device="cuda")
    gd = torch.zeros_like(g.data)
    gp = torch.zeros(F, 6, dtype=torch.float64, device="cuda")
    old = pxm.get_tuning()
    pxm.set_tuning(block, variant)
    try:
        ws = pxm.new_workspace(g, r, wl.opts, want)
        pxm.render_fused(g, r, wl.opts, trgb, tdep, fwt, want, rgb=rgb, depth=depth, loss=loss,
                         grad_data=gd, grad_pose=gp, ws=ws)
        torch.cuda.synchronize()
    finally:
        pxm.set_tuning(*old)
    return dict(rgb=np_(rgb), depth=np_(depth), loss=np_(loss), grad_data=np_(gd),
                grad_pose=np_(gp))


def check_all(out, ref, what, want=3):
    assert_r28(out["rgb"], ref["rgb"], TAU_FWD, what + " rgb")
    assert_r28(out["depth"], ref["depth"], TAU_FWD, what + " depth")
    assert_r28(out["loss"], ref["loss"], TAU_FWD, what + " loss")
    if want & 1:
        assert np.abs(ref["grad_data"]).max() > 0
        assert_r28(out["grad_data"][:, 0], ref["grad_data"][:, 0], TAU_GRAD, what + " grad density")
        assert_r28(out["grad_data"][:, 1:], ref["grad_data"][:, 1:], TAU_GRAD, what + " grad sh")
    if want & 2:
        assert_pose(out["grad_pose"], ref["grad_pose"], TAU_GRAD, what + " pose")


# ------------------------------------------------------------ ray subsets

@pytest.fixture(scope="module")
def c4_subset(c4):
    return reference(synth.subset_rays(c4, 32768, seed=401))


@pytest.fixture(scope="module")
def c5_subset(c5):
    return reference(synth.subset_rays(c5, 32768, seed=501))


@pytest.mark.parametrize("variant", [1, 2])
def test_c4_keyframes_ray_subset(c4_subset, variant):
    """32,768 rays drawn from all eight keyframes."""
    wl, ref = c4_subset
    check_all(run_fused(wl, 64, variant), ref, f"c4 subset v{variant}")


@pytest.mark.parametrize("variant", [1, 2])
def test_c5_mixed_batch_ray_subset(c5_subset, variant):
    """32,768 rays drawn from the 64 frames; per-frame pose gradients."""
    wl, ref = c5_subset
    assert (np.diff(wl.rays.frame_offsets) > 0).sum() == 64
    check_all(run_fused(wl, 64, variant), ref, f"c5 subset v{variant}")


@pytest.fixture(scope="module")
def c4_tiles(c4):
    off = c4.rays.frame_offsets
    a = int(off[3]) + 400_000
    b = a + 40_000 + 29
    rays = dataclasses.replace(c4.rays, c2w=c4.rays.c2w[3:4], intr=c4.rays.intr[3:4],
                               pix=c4.rays.pix[a:b], frame_offsets=np.array([0, b - a], np.int32))
    tg = synth.Targets(c4.targets.rgb[a:b], c4.targets.depth[a:b], c4.targets.frame_weight[3:4])
    return reference(c4.replace(rays=rays, targets=tg))


@pytest.mark.parametrize("variant", [1, 2])
def test_c4_keyframe_tile_block(c4_tiles, variant):
    """40,029 consecutive rays (8x8 pixel tiles and a ragged tail) of one
    keyframe: coherent waves, the matrix-core form of the grid scatter."""
    wl, ref = c4_tiles
    check_all(run_fused(wl, 64, variant), ref, f"c4 tiles v{variant}")


# ------------------------------------------------------------ full batches

def _frames_reference(wl, frames):
    """Oracle loss, pose and grid gradients of the given frames alone (their
    targets moved off the L1 kink: the moved depths are returned too)."""
    gd = np.zeros((wl.grid.n_alloc, 28))
    gp = np.zeros((wl.rays.n_frames, 6))
    loss = np.zeros(wl.rays.n_frames)
    depth = np.array(wl.targets.depth, np.float32)
    for f in frames:
        wf, a, b = _frame(wl, int(f))
        wf, rf = reference(wf)
        depth[a:b] = wf.targets.depth
        gd += rf["grad_data"]
        gp[f] = rf["grad_pose"][0]
        loss[f] = rf["loss"][0]
    return dict(grad_data=gd, grad_pose=gp, loss=loss), depth


def _full_batch_check(wl, frames, fref, tdep, variant, what):
    n, F = wl.rays.n_rays, wl.rays.n_frames
    # all frames weighted: sampled rays, one by one
    out = run_fused(wl, 64, variant, tgt_depth=tdep)
    sel = np.sort(np.random.default_rng(95).choice(n, size=3000, replace=False))
    sub = synth.subset_rays(wl, 3000, seed=95)
    assert np.array_equal(wl.rays.pix[sel], sub.rays.pix)              # the same rays
    ref_rgb, ref_depth, _, _ = oracle.render(sub.grid, sub.rays, sub.opts)
    assert_r28(out["rgb"][sel], ref_rgb, TAU_FWD, what + " sampled rgb")
    assert_r28(out["depth"][sel], ref_depth, TAU_FWD, what + " sampled depth")
    assert np.all(np.isfinite(out["grad_data"])) and np.abs(out["grad_data"]).max() > 0
    for f in frames:
        assert_r28(out["loss"][f:f + 1], fref["loss"][f:f + 1], TAU_FWD, f"{what} frame {f} loss")
        assert_pose(out["grad_pose"][f:f + 1], fref["grad_pose"][f:f + 1], TAU_GRAD,
                    f"{what} frame {f} pose")
    # only `frames` weighted: the full-size launch's grid gradient is theirs
    fw = np.zeros(F, np.float32)
    fw[frames] = wl.targets.frame_weight[frames]
    out = run_fused(wl, 64, variant, fw=fw, tgt_depth=tdep)
    others = np.setdiff1d(np.arange(F), frames)
    assert np.all(out["grad_pose"][others] == 0) and np.all(out["loss"][others] == 0)
    touched = np.abs(fref["grad_data"]).sum(1) > 0
    print(f"{what}: frames {list(map(int, frames))}, {int(touched.sum())} records with a gradient",
          flush=True)
    assert touched.sum() > 1000
    assert np.all(out["grad_data"][~touched] == 0)
    assert_r28(out["grad_data"][:, 0], fref["grad_data"][:, 0], TAU_GRAD, what + " grad density")
    assert_r28(out["grad_data"][:, 1:], fref["grad_data"][:, 1:], TAU_GRAD, what + " grad sh")
    assert_pose(out["grad_pose"][frames], fref["grad_pose"][frames], TAU_GRAD, what + " pose")


@pytest.fixture(scope="module")
def c4_full_ref(c4):
    frames = np.array([5])
    fref, tdep = _frames_reference(c4, frames)
    return frames, fref, tdep


@pytest.mark.parametrize("variant", [1, 2])
def test_c4_eight_keyframes_full_size(c4, c4_full_ref, variant):
    frames, fref, tdep = c4_full_ref
    _full_batch_check(c4, frames, fref, tdep, variant, f"c4 full v{variant}")


@pytest.fixture(scope="module")
def c5_full_ref(c5):
    counts = np.diff(c5.rays.frame_offsets)
    order = np.argsort(counts)
    frames = np.sort(np.concatenate([order[:3], order[len(order) // 2:len(order) // 2 + 1]]))
    fref, tdep = _frames_reference(c5, frames)
    return frames, fref, tdep


@pytest.mark.parametrize("variant", [1, 2])
def test_c5_mixed_64_frame_batch_full_size(c5, c5_full_ref, variant):
    frames, fref, tdep = c5_full_ref
    _full_batch_check(c5, frames, fref, tdep, variant, f"c5 full v{variant}")
