"""Parity at full size, in the launch configuration the benchmark times.

The mixed 64-frame batch on the 512^3 room (6.8M rays, 1k-200k per frame,
64 rays per workgroup, persistent tile queue): rays are independent, so
sampled rays' colour and depth are checked one by one against the oracle,
and the smaller frames' loss and pose gradient (sums over that frame's rays
only) against the oracle run on those frames alone."""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_03404_amd import synth
from tests._parity import TAU_FWD, TAU_GRAD, align_depth_decisions, assert_pose, assert_r28

pytestmark = pytest.mark.gpu


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
    return wl.replace(rays=rays, targets=tg), a, b


@pytest.fixture(scope="module")
def c5():
    return synth.config5()


@pytest.mark.parametrize("variant", [1, 2])
def test_fused_mixed_64_frame_batch_full_size(c5, variant):
    """In one launch (variant 1) and in two (variant 2, the form the autotuner
    picks for this batch)."""
    pxm = _dev()
    wl = c5
    n, F = wl.rays.n_rays, wl.rays.n_frames
    print(f"{wl.name}: {n} rays, {F} frames, variant {variant}", flush=True)
    g = pxm.grid_to_device(wl.grid)
    r = pxm.rays_to_device(wl.rays)
    trgb = torch.from_numpy(wl.targets.rgb).cuda()
    tdep = torch.from_numpy(wl.targets.depth).cuda()
    fw = torch.from_numpy(wl.targets.frame_weight).cuda()
    rgb = torch.empty(n, 3, device="cuda")
    depth = torch.empty(n, device="cuda")
    loss = torch.zeros(F, dtype=torch.float64, device="cuda")
    gd = torch.zeros_like(g.data)
    gp = torch.zeros(F, 6, dtype=torch.float64, device="cuda")
    old = pxm.get_tuning()
    pxm.set_tuning(64, variant)
    try:
        ws = pxm.new_workspace(g, r, wl.opts, 3)
        pxm.render_fused(g, r, wl.opts, trgb, tdep, fw, 3, rgb=rgb, depth=depth, loss=loss,
                         grad_data=gd, grad_pose=gp, ws=ws)
        torch.cuda.synchronize()
    finally:
        pxm.set_tuning(*old)
    rgb, depth, loss, gp = np_(rgb), np_(depth), np_(loss), np_(gp)
    # sampled rays, one by one
    sub = synth.subset_rays(wl, 3000, seed=95)
    sel = np.sort(np.random.default_rng(95).choice(n, size=3000, replace=False))
    assert np.array_equal(wl.rays.pix[sel], sub.rays.pix)     # the same rays
    ref_rgb, ref_depth, _, _ = oracle.render(sub.grid, sub.rays, sub.opts)
    assert_r28(rgb[sel], ref_rgb, TAU_FWD, "sampled rgb")
    assert_r28(depth[sel], ref_depth, TAU_FWD, "sampled depth")
    # the three smallest frames: loss and pose gradient against the oracle on those rays
    counts = np.diff(wl.rays.frame_offsets)
    for f in np.argsort(counts)[:3]:
        wf, a, b = _frame(wl, int(f))
        ref = oracle.fused(wf.grid, wf.rays, wf.targets, wf.opts, want_grid=False, want_pose=True)
        assert_r28(loss[f:f + 1], ref["loss"], TAU_FWD, f"frame {f} loss")
        ref, nflip = align_depth_decisions(wf, ref, depth[a:b])
        assert_pose(gp[f:f + 1], ref["grad_pose"], TAU_GRAD, f"frame {f} ({b - a} rays) pose")
    # the grid gradient is a sum over every ray: check that it is finite and
    # touches only allocated records that rays reached
    gdn = np_(gd)
    assert np.all(np.isfinite(gdn)) and np.abs(gdn).sum() > 0
