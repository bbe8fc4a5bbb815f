"""Ray packer (CPU), autotuner and captured tracking loop (GPU)."""
import dataclasses

import numpy as np
import pytest

from paper_2307_03404_amd import synth
from paper_2307_03404_amd.batch import pack_frames, tile_sort


def test_tile_sort_groups_8x8_blocks():
    rng = np.random.default_rng(0)
    pix = synth.subsample_pixels(1200, 680, 5000, rng)
    perm = tile_sort(pix, 1200)
    assert sorted(perm.tolist()) == list(range(5000))
    p = pix[perm]
    tile = (p[:, 1] // 8) * 150 + p[:, 0] // 8
    assert np.all(np.diff(tile) >= 0)
    full = synth.tile_order(1200, 680)
    np.testing.assert_array_equal(full[tile_sort(full, 1200)], full)


def test_morton_sort_is_a_z_curve():
    from paper_2307_03404_amd.rayorder import morton_sort
    v, u = np.mgrid[0:64, 0:64]
    pix = np.stack([u.ravel(), v.ravel()], 1)
    p = pix[morton_sort(pix)]
    # every aligned 2^k x 2^k block is one contiguous run, blocks in Z order
    for k in (1, 3, 5):
        blk = (p[:, 1] >> k) * (64 >> k) + (p[:, 0] >> k)
        runs = blk[np.r_[True, np.diff(blk) != 0]]
        assert len(runs) == (64 >> k) ** 2 and len(set(runs.tolist())) == len(runs)
    np.testing.assert_array_equal(p[:4], [[0, 0], [1, 0], [0, 1], [1, 1]])
    # on a sparse subset, 64 consecutive rays stay in a compact patch
    rng = np.random.default_rng(3)
    sub = synth.subsample_pixels(1200, 680, 100000, rng)
    spans = [np.ptp(sub[i:i + 64], axis=0).max() for i in range(0, 100000 - 64, 64)]
    assert np.median(spans) < 64
    flat = sub[:, 1] * 1200 + sub[:, 0]
    assert len(np.unique(flat)) == 100000


def test_frame_order_tiles_full_frames_and_z_orders_subsets():
    from paper_2307_03404_amd.rayorder import frame_order, morton_sort, tile_sort
    full = synth.tile_order(1200, 680)
    np.testing.assert_array_equal(frame_order(full, 1200, 680), tile_sort(full, 1200))
    rng = np.random.default_rng(4)
    sub = synth.subsample_pixels(1200, 680, 3000, rng)
    np.testing.assert_array_equal(frame_order(sub, 1200, 680), morton_sort(sub))


def test_pack_frames_csr_and_inverse_order():
    rng = np.random.default_rng(1)
    frames = []
    for n in (100, 0, 37, 2000):
        frames.append((np.eye(4)[:3], np.array([600, 600, 600, 340]),
                       synth.subsample_pixels(1200, 680, n, rng) if n else np.zeros((0, 2))))
    pk = pack_frames(frames, 1200)
    np.testing.assert_array_equal(pk.frame_offsets, [0, 100, 100, 137, 2137])
    allpix = np.concatenate([f[2] for f in frames if len(f[2])]).astype(np.int32)
    np.testing.assert_array_equal(pk.pix, allpix[pk.order])
    for f in range(4):
        a, b = pk.frame_offsets[f], pk.frame_offsets[f + 1]
        assert np.all((pk.order[a:b] >= a) & (pk.order[a:b] < b))


# ----------------------------------------------------------------------------- GPU

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_03404_amd import pxm
    return pxm


@pytest.mark.gpu
def test_autotuner_picks_a_candidate_and_caches(tmp_path):
    pxm = _gpu()
    from paper_2307_03404_amd.batch import CANDIDATES, Autotuner
    wl = synth.subset_rays(synth.config1(), 3000, seed=4)
    g, r = pxm.grid_to_device(wl.grid), pxm.rays_to_device(wl.rays)
    t = [torch.from_numpy(x).cuda() for x in (wl.targets.rgb, wl.targets.depth, wl.targets.frame_weight)]
    old = pxm.get_tuning()
    try:
        tuner = Autotuner(str(tmp_path / "tune.json"), reps=2, warmup=1)
        best, ms = tuner.tune(g, r, wl.opts, *t, 3)
        assert best in CANDIDATES and len(ms) == len(CANDIDATES)
        assert pxm.get_tuning() == best
        again = Autotuner(str(tmp_path / "tune.json"))
        assert again.tune(g, r, wl.opts, *t, 3)[0] == best
    finally:
        pxm.set_tuning(*old)


@pytest.mark.gpu
@pytest.mark.parametrize("tuning", [(256, 0), (64, 2)])
def test_tracking_graph_replays_match_eager_and_reduce_loss(tuning):
    """20 captured Adam iterations over 16 frames: every replay (with eager
    work between replays) matches the eager run; the loss goes down.  Also
    with the two-launch variant, whose graph holds two launches per
    iteration and hands per-ray state through the workspace."""
    pxm = _gpu()
    old = pxm.get_tuning()
    pxm.set_tuning(*tuning)
    try:
        _tracking_graph_check(pxm)
    finally:
        pxm.set_tuning(*old)


def _tracking_graph_check(pxm):
    from paper_2307_03404_amd.batch import TrackingGraph
    wl = synth.config3()
    wl = synth.subset_rays(wl, 60000, seed=2)
    g = pxm.grid_to_device(wl.grid)
    # targets: the render at the true poses (a GPU-only property test: no oracle here)
    true_rays = pxm.rays_to_device(dataclasses.replace(wl.rays, c2w=wl.true_c2w))
    rgb, depth, _ = pxm.render_forward(g, true_rays, wl.opts)
    fw = torch.from_numpy(wl.targets.frame_weight).cuda()
    opts = dataclasses.replace(wl.opts, depth_loss=synth.DEPTH_L2)
    r = pxm.rays_to_device(wl.rays)
    c2w0 = r.c2w.clone()
    tg = TrackingGraph(g, r, opts, rgb, depth, fw, iters=20, lr=2e-3)
    tg.run_eager()
    torch.cuda.synchronize()
    eager_c2w = r.c2w.clone()
    eager_loss = tg.losses.clone()
    assert float(eager_loss[-1].sum()) < 0.8 * float(eager_loss[0].sum())
    tg.reset(c2w0)
    tg.capture()
    for rep in range(3):
        tg.reset(c2w0)
        scratch = torch.randn(1000, device="cuda").sum()      # eager work between replays
        tg.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(scratch)
        np.testing.assert_allclose(r.c2w.cpu().numpy(), eager_c2w.cpu().numpy(), atol=1e-5)
        np.testing.assert_allclose(tg.losses.cpu().numpy(), eager_loss.cpu().numpy(), rtol=1e-4,
                                   atol=1e-9)
