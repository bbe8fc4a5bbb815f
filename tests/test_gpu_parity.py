"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, element by element, with the forward within 1e-5 and the
gradients within 1e-4 (relative with an RMS floor, see _parity.py)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2307_03404_amd import synth
from tests._parity import TAU_FWD, TAU_GRAD, assert_pose, assert_r28, r28_ratio, reference

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_03404_amd import pxm
    return pxm


def to_dev(wl):
    pxm = _dev()
    g = pxm.grid_to_device(wl.grid)
    r = pxm.rays_to_device(wl.rays)
    t = dict(rgb=torch.from_numpy(wl.targets.rgb).cuda(),
             depth=torch.from_numpy(wl.targets.depth).cuda(),
             fw=torch.from_numpy(wl.targets.frame_weight).cuda())
    return g, r, t


def np_(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def c1():
    return reference(synth.config1())


# ------------------------------------------------------------------ forward

def test_forward_c1(c1):
    pxm = _dev()
    wl, ref = c1
    g, r, _ = to_dev(wl)
    rgb, depth, nsamp = pxm.render_forward(g, r, wl.opts)
    torch.cuda.synchronize()
    assert_r28(np_(rgb), ref["rgb"], TAU_FWD, "rgb")
    assert_r28(np_(depth), ref["depth"], TAU_FWD, "depth")
    check_nsamp(wl, np_(nsamp), ref["nsamp"])


def check_nsamp(wl, got, want, max_fraction=1e-3):
    """Kept sample counts agree, except on rays whose early-termination test
    T_{i+1} < t_stop (Sec. 4 reading: stop once T falls below t_stop) is
    decided by rounding: there the oracle's transmittance at the earlier of
    the two stopping points must lie within 1e-4 (relative) of t_stop."""
    bad = np.flatnonzero(got != want)
    assert bad.size <= max(2, max_fraction * got.size), f"{bad.size} rays disagree on nsamp"
    off = wl.rays.frame_offsets
    for r in bad:
        f = int(np.searchsorted(off, r, side="right") - 1)
        o, d, _ = oracle.ray(wl.rays.c2w[f], wl.rays.intr[f], *wl.rays.pix[r])
        tr = oracle.trace(wl.grid, o, d, wl.opts)
        m = int(min(got[r], want[r]))
        T = tr["T"][m]
        assert abs(T / wl.opts.t_stop - 1.0) < 1e-4, \
            f"ray {r}: nsamp {got[r]} vs {want[r]} with T = {T:.6e}, t_stop {wl.opts.t_stop:.6e}"
    return bad.size


def test_forward_cap_and_tail_and_misses(c1):
    pxm = _dev()
    wl, _ = c1
    # 1000 rays (ragged tail of a 256-ray block), cap of 5 positions
    sub = synth.subset_rays(wl, 1000, seed=3)
    opts = dataclasses.replace(wl.opts, max_samples=5)
    ref_rgb, ref_d, ref_n, _ = oracle.render(sub.grid, sub.rays, opts)
    g, r, _ = to_dev(sub)
    rgb, depth, nsamp = pxm.render_forward(g, r, opts)
    torch.cuda.synchronize()
    assert ref_n.max() == 5
    np.testing.assert_array_equal(np_(nsamp), ref_n)
    assert_r28(np_(rgb), ref_rgb, TAU_FWD, "rgb cap")
    assert_r28(np_(depth), ref_d, TAU_FWD, "depth cap")
    # a camera looking away from the box: every ray misses
    c2w = synth.look_at((0.0, 0.0, 3.0), (0.0, 0.0, 6.0))
    away = dataclasses.replace(sub.rays, c2w=c2w[None].astype(np.float32))
    ra = pxm.rays_to_device(away)
    rgb, depth, nsamp = pxm.render_forward(g, ra, opts)
    torch.cuda.synchronize()
    assert np.all(np_(rgb) == 0) and np.all(np_(depth) == 0) and np.all(np_(nsamp) == 0)


def test_forward_one_ray_and_empty(c1):
    pxm = _dev()
    wl, ref = c1
    one = synth.subset_rays(wl, 1, seed=5)
    ref_rgb, ref_d, ref_n, _ = oracle.render(one.grid, one.rays, one.opts)
    g, r, _ = to_dev(one)
    rgb, depth, nsamp = pxm.render_forward(g, r, one.opts)
    torch.cuda.synchronize()
    assert_r28(np_(rgb), ref_rgb, TAU_FWD, "rgb one")
    empty = dataclasses.replace(one.rays, pix=np.zeros((0, 2), np.int32),
                                frame_offsets=np.array([0, 0], np.int32))
    re = pxm.rays_to_device(empty)
    rgb, depth, nsamp = pxm.render_forward(g, re, one.opts)
    assert rgb.shape == (0, 3)


# ------------------------------------------------------------------ backward

def _upstream(ref):
    return (torch.from_numpy(ref["g_rgb"].astype(np.float32)).cuda(),
            torch.from_numpy(ref["g_depth"].astype(np.float32)).cuda())


def test_backward_grid_c1(c1):
    pxm = _dev()
    wl, _ = c1
    rgb_o, dep_o, _, _ = oracle.render(wl.grid, wl.rays, wl.opts)
    L, g_rgb, g_dep = oracle.loss(wl.rays, rgb_o, dep_o, wl.targets, wl.opts)
    # the oracle's backward sees the same float32 upstream gradients as the GPU
    g_rgb32, g_dep32 = g_rgb.astype(np.float32), g_dep.astype(np.float32)
    ref, _ = oracle.backward(wl.grid, wl.rays, wl.opts, g_rgb32, g_dep32, True, False)
    g, r, _ = to_dev(wl)
    rgb, depth, nsamp = pxm.render_forward(g, r, wl.opts)
    grad = pxm.render_backward_grid(g, r, wl.opts, rgb, depth, nsamp,
                                    torch.from_numpy(g_rgb32).cuda(), torch.from_numpy(g_dep32).cuda())
    torch.cuda.synchronize()
    assert np.abs(ref).max() > 0
    assert_r28(np_(grad)[:, 0], ref[:, 0], TAU_GRAD, "grad density")
    assert_r28(np_(grad)[:, 1:], ref[:, 1:], TAU_GRAD, "grad sh")


@pytest.mark.parametrize("viewdir", [False, True])
def test_backward_pose_c1(c1, viewdir):
    pxm = _dev()
    wl, _ = c1
    opts = dataclasses.replace(wl.opts, flags=synth.FLAG_POSE_VIEWDIR if viewdir else 0)
    rgb_o, dep_o, _, _ = oracle.render(wl.grid, wl.rays, opts)
    L, g_rgb, g_dep = oracle.loss(wl.rays, rgb_o, dep_o, wl.targets, opts)
    g_rgb32, g_dep32 = g_rgb.astype(np.float32), g_dep.astype(np.float32)
    _, ref = oracle.backward(wl.grid, wl.rays, opts, g_rgb32, g_dep32, False, True)
    g, r, _ = to_dev(wl)
    rgb, depth, nsamp = pxm.render_forward(g, r, opts)
    gp = pxm.render_backward_pose(g, r, opts, rgb, depth, nsamp,
                                  torch.from_numpy(g_rgb32).cuda(), torch.from_numpy(g_dep32).cuda())
    torch.cuda.synchronize()
    assert_pose(np_(gp), ref, TAU_GRAD, "pose")


# ------------------------------------------------------------------ fused

def _fused_check(wl, want, what, ref=None, block=None, variant=None):
    """`ref` comes from reference(wl), with `wl` the workload it returned."""
    pxm = _dev()
    if ref is None:
        wl, ref = reference(wl)
    g, r, t = to_dev(wl)
    n, F = wl.rays.n_rays, wl.rays.n_frames
    rgb = torch.empty(n, 3, device="cuda")
    depth = torch.empty(n, device="cuda")
    loss = torch.zeros(F, dtype=torch.float64, device="cuda")
    gd = torch.zeros_like(g.data)
    gp = torch.zeros(F, 6, dtype=torch.float64, device="cuda")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    old = pxm.get_tuning()
    if block is not None:
        pxm.set_tuning(block, variant)
    try:
        ws = pxm.new_workspace(g, r, wl.opts, want)
        for _ in range(2):      # twice: the persistent queue must re-arm itself
            for x in (loss, gd, gp, stats):
                x.zero_()
            pxm.render_fused(g, r, wl.opts, t["rgb"], t["depth"], t["fw"], want | pxm.WANT_STATS,
                             rgb=rgb, depth=depth, loss=loss, grad_data=gd, grad_pose=gp,
                             stats=stats, ws=ws)
            torch.cuda.synchronize()
            assert_r28(np_(rgb), ref["rgb"], TAU_FWD, what + " rgb")
            assert_r28(np_(depth), ref["depth"], TAU_FWD, what + " depth")
            assert_r28(np_(loss), ref["loss"], TAU_FWD, what + " loss")
            gref = ref
            if want & pxm.WANT_GRID:
                assert_r28(np_(gd)[:, 0], gref["grad_data"][:, 0], TAU_GRAD, what + " grad density")
                assert_r28(np_(gd)[:, 1:], gref["grad_data"][:, 1:], TAU_GRAD, what + " grad sh")
            else:
                assert np.all(np_(gd) == 0)
            if want & pxm.WANT_POSE:
                assert_pose(np_(gp), gref["grad_pose"], TAU_GRAD, what + " pose")
            st = np_(stats)
            valid = np.isfinite(wl.targets.depth) & (wl.targets.depth > 0)
            assert st[3] == int(valid.sum())
            occ = ref["stats"].sum(0)
            assert abs(int(st[0]) - int(occ[0])) <= max(2, 1e-4 * occ[0])
            assert abs(int(st[1]) - int(occ[1])) <= max(16, 1e-4 * occ[1])
    finally:
        pxm.set_tuning(*old)
    return ref


def test_fused_c1_grid_and_pose(c1):
    wl, ref = c1
    _fused_check(wl, 3, "c1 fused", ref)


@pytest.mark.parametrize("block,variant", [(64, 0), (128, 1), (64, 1), (256, 1), (64, 2), (256, 2)])
def test_fused_c1_launch_shapes(c1, block, variant):
    wl, ref = c1
    _fused_check(wl, 3, f"c1 b{block} v{variant}", ref, block, variant)


@pytest.mark.parametrize("block,variant", [(256, 0), (64, 2)])
def test_fused_c1_grid_only_and_pose_only(c1, block, variant):
    """Grid gradient only, pose gradient only, and neither (forward and loss)."""
    wl, ref = c1
    _fused_check(wl, 1, f"c1 grid {block}/{variant}", ref, block, variant)
    _fused_check(wl, 2, f"c1 pose {block}/{variant}", ref, block, variant)
    _fused_check(wl, 0, f"c1 loss only {block}/{variant}", ref, block, variant)


def test_fused_all_targets_invalid(c1):
    pxm = _dev()
    wl, _ = c1
    bad = dataclasses.replace(wl.targets, depth=np.zeros_like(wl.targets.depth))
    wl2 = wl.replace(targets=bad)
    g, r, t = to_dev(wl2)
    gd = torch.zeros_like(g.data)
    gp = torch.zeros(1, 6, dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    pxm.render_fused(g, r, wl.opts, t["rgb"], t["depth"], t["fw"], 3, loss=loss, grad_data=gd,
                     grad_pose=gp)
    torch.cuda.synchronize()
    assert np.all(np_(gd) == 0) and np.all(np_(gp) == 0) and np_(loss)[0] == 0


@pytest.fixture(scope="module")
def c3():
    return synth.config3()


def test_fused_c3_tracking_all_frames(c3):
    """16 frames, 2k-50k rays each, one launch, per-frame pose reduction."""
    _fused_check(c3, 2, "c3 pose")


def test_fused_view_direction_pose_term(c1):
    """The exact view-direction pose term (PXM_FLAG_POSE_VIEWDIR) in the fused
    kernel, grid + pose and pose only, against the oracle with the same flag."""
    wl, _ = c1
    wlv, ref = reference(wl.replace(opts=dataclasses.replace(wl.opts, flags=synth.FLAG_POSE_VIEWDIR)))
    plain = oracle.fused(wl.grid, wl.rays, wl.targets, wl.opts)
    # the term moves the rotation gradient well beyond the tolerance: a kernel
    # that ignored the flag would fail
    assert r28_ratio(plain["grad_pose"][:, 3:], ref["grad_pose"][:, 3:]) > 10 * TAU_GRAD
    _fused_check(wlv, 3, "c1 grid+pose viewdir", ref)
    _fused_check(wlv, 2, "c1 pose viewdir", ref)
    _fused_check(wlv, 3, "c1 grid+pose viewdir two launches", ref, 64, 2)
    _fused_check(wlv, 2, "c1 pose viewdir two launches", ref, 64, 2)


def test_fused_c3_tracking_view_direction(c3):
    sub = synth.subset_rays(c3, 40000, seed=12)
    subv, ref = reference(sub.replace(opts=dataclasses.replace(sub.opts, flags=synth.FLAG_POSE_VIEWDIR)),
                          want_grid=False)
    plain = oracle.fused(sub.grid, sub.rays, sub.targets, sub.opts, want_grid=False)
    assert r28_ratio(plain["grad_pose"][:, 3:], ref["grad_pose"][:, 3:]) > 10 * TAU_GRAD
    _fused_check(subv, 2, "c3 pose viewdir", ref)


def test_fused_frames_with_no_rays(c3):
    wl = c3
    off = wl.rays.frame_offsets.copy()
    # make frames 3 and 7 empty by moving their rays to the previous frame's end
    keep = np.ones(wl.rays.n_rays, bool)
    keep[off[3]:off[4]] = False
    keep[off[7]:off[8]] = False
    counts = np.diff(off)
    counts[3] = counts[7] = 0
    new_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    rays = dataclasses.replace(wl.rays, pix=wl.rays.pix[keep], frame_offsets=new_off)
    tg = dataclasses.replace(wl.targets, rgb=wl.targets.rgb[keep], depth=wl.targets.depth[keep])
    sub = synth.subset_rays(wl.replace(rays=rays, targets=tg), 40000, seed=9)
    ref = _fused_check(sub, 3, "c3 empty frames")
    assert np.all(ref["grad_pose"][[3, 7]] == 0)


@pytest.fixture(scope="module")
def c2():
    return synth.config2()


def test_fused_c2_tile_block(c2):
    """A contiguous block of 8x8 pixel tiles of the 1200x680 frame (the bench
    launch configuration, grid and pose gradients) plus a ragged tail."""
    wl = c2
    a, b = 300_000, 300_000 + 40_000 + 37
    rays = dataclasses.replace(wl.rays, pix=wl.rays.pix[a:b],
                               frame_offsets=np.array([0, b - a], np.int32))
    tg = dataclasses.replace(wl.targets, rgb=wl.targets.rgb[a:b], depth=wl.targets.depth[a:b])
    _fused_check(wl.replace(rays=rays, targets=tg), 3, "c2 tiles")


def _occupancy_numpy(grid):
    """Cell and brick occupancy bits recomputed on the host from the link table."""
    R = np.array(grid.reso)
    L = (grid.link.reshape(*grid.reso) >= 0)
    cell = np.zeros(tuple(R - 1), bool)
    for i in (0, 1):
        for j in (0, 1):
            for k in (0, 1):
                cell |= L[i:R[0] - 1 + i, j:R[1] - 1 + j, k:R[2] - 1 + k]
    # level 0: a 64-bit word per 4^3 block, bit (x&3)*16 + (y&3)*4 + (z&3)
    Q = (R - 1 + 3) // 4
    qpad = np.zeros(tuple(Q * 4), bool)
    qpad[:R[0] - 1, :R[1] - 1, :R[2] - 1] = cell
    blocks = qpad.reshape(Q[0], 4, Q[1], 4, Q[2], 4).transpose(0, 2, 4, 1, 3, 5).reshape(-1, 64)
    words = (blocks.astype(np.uint64) << np.arange(64, dtype=np.uint64)).sum(axis=1, dtype=np.uint64)
    w0 = words.view(np.uint32)                  # little-endian: low half first
    B = (R - 1 + 7) // 8
    bpad = np.zeros(tuple(B * 8), bool)
    bpad[:R[0] - 1, :R[1] - 1, :R[2] - 1] = cell
    brick = bpad.reshape(B[0], 8, B[1], 8, B[2], 8).any(axis=(1, 3, 5)).ravel()
    nb = ((brick.size + 31) // 32) * 32
    bp = np.zeros(nb, bool)
    bp[:brick.size] = brick
    w1 = np.packbits(bp.reshape(-1, 32)[:, ::-1], axis=1).view(">u4").ravel().astype(np.uint32)
    return np.concatenate([w0, w1])


def test_occupancy_bitfield_matches_link_table(c2):
    pxm = _dev()
    for grid in (c2.grid, synth.random_tiny_grid(np.random.default_rng(3), R=37, margin=3,
                                                  occupancy=0.3)):
        g = pxm.grid_to_device(grid)
        torch.cuda.synchronize()
        got = np_(g.occ).view(np.uint32)
        np.testing.assert_array_equal(got, _occupancy_numpy(grid))


def test_fused_c2_tiles_without_occupancy(c2):
    """Skipping is exact: the same tile block without the bitfield."""
    pxm = _dev()
    wl = c2
    a, b = 500_000, 500_000 + 20_000
    rays = dataclasses.replace(wl.rays, pix=wl.rays.pix[a:b],
                               frame_offsets=np.array([0, b - a], np.int32))
    tg = dataclasses.replace(wl.targets, rgb=wl.targets.rgb[a:b], depth=wl.targets.depth[a:b])
    sub, ref = reference(wl.replace(rays=rays, targets=tg))
    tg = sub.targets
    outs = []
    for occ in (True, False):
        g = pxm.grid_to_device(sub.grid, occupancy=occ)
        r = pxm.rays_to_device(sub.rays)
        t = [torch.from_numpy(x).cuda() for x in (tg.rgb, tg.depth, tg.frame_weight)]
        rgb = torch.empty(b - a, 3, device="cuda")
        depth = torch.empty(b - a, device="cuda")
        gd = torch.zeros_like(g.data)
        gp = torch.zeros(1, 6, dtype=torch.float64, device="cuda")
        st = torch.zeros(4, dtype=torch.int64, device="cuda")
        pxm.render_fused(g, r, sub.opts, *t, 3 | pxm.WANT_STATS, rgb=rgb, depth=depth,
                         grad_data=gd, grad_pose=gp, stats=st)
        torch.cuda.synchronize()
        assert_r28(np_(rgb), ref["rgb"], TAU_FWD, f"rgb occ={occ}")
        assert_r28(np_(gd), ref["grad_data"], TAU_GRAD, f"grad occ={occ}")
        assert_pose(np_(gp), ref["grad_pose"], TAU_GRAD, f"pose occ={occ}")
        outs.append((np_(rgb), np_(st)))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])      # forward bitwise identical
    np.testing.assert_array_equal(outs[0][1], outs[1][1])      # same samples counted


@pytest.fixture(scope="module")
def c2_ref(c2):
    return reference(c2)


@pytest.mark.parametrize("variant", [1, 2])
def test_fused_c2_full_frame(c2_ref, variant):
    """The whole 816,000-ray frame at the bench launch configuration (one
    launch, persistent) and in the two-launch form."""
    wl, ref = c2_ref
    _fused_check(wl, 3, f"c2 full v{variant}", ref, block=64, variant=variant)


def test_tv_c2(c2):
    pxm = _dev()
    lam_d, lam_sh, eps = 1e-3, 1e-4, 1e-9
    _, ref = oracle.tv(c2.grid, lam_d, lam_sh, eps)
    g = pxm.grid_to_device(c2.grid)
    grad = pxm.tv_grad(g, lam_d, lam_sh, eps)
    put = pxm.tv_grad_set(g, lam_d, lam_sh, eps, grad_data=torch.ones_like(g.data))
    torch.cuda.synchronize()
    assert_r28(np_(grad)[:, 0], ref[:, 0], TAU_GRAD, "tv density")
    assert_r28(np_(grad)[:, 1:], ref[:, 1:], TAU_GRAD, "tv sh")
    assert np.array_equal(np_(put), np_(grad))


@pytest.mark.parametrize("occupancy", [True, False])
def test_tv_dense_c1(c1, occupancy):
    pxm = _dev()
    wl, _ = c1
    _, ref = oracle.tv(wl.grid, 0.3, 0.05, 1e-4)
    g = pxm.grid_to_device(wl.grid, occupancy=occupancy)
    base = torch.full_like(g.data, 0.25)
    grad = pxm.tv_grad(g, 0.3, 0.05, 1e-4, grad_data=base)     # accumulates
    torch.cuda.synchronize()
    assert_r28(np_(grad) - 0.25, ref, TAU_GRAD, "tv dense")


@pytest.mark.parametrize("occupancy", [True, False])
def test_tv_set_writes_the_gradient(c1, occupancy):
    """pxm_tv_grad_set overwrites the used fields of every linked record with
    dTV (the oracle's, to the gradient tolerance, whatever the buffer held)
    and equals pxm_tv_grad on a zeroed buffer value for value."""
    pxm = _dev()
    wl, _ = c1
    _, ref = oracle.tv(wl.grid, 0.3, 0.05, 1e-4)
    g = pxm.grid_to_device(wl.grid, occupancy=occupancy)
    junk = torch.full_like(g.data, 7.5)
    got = np_(pxm.tv_grad_set(g, 0.3, 0.05, 1e-4, grad_data=junk))
    acc = np_(pxm.tv_grad(g, 0.3, 0.05, 1e-4, grad_data=torch.zeros_like(g.data)))
    torch.cuda.synchronize()
    assert_r28(got, ref, TAU_GRAD, "tv set")
    assert np.array_equal(got, acc)


@pytest.mark.parametrize("reso", [(17, 9, 24), (9, 16, 25)])
def test_tv_ragged_bricks(reso):
    """Lattices that are not whole 8^3 bricks, sparse blobs (whole bricks
    empty), with and without the occupancy bitfield: matches the oracle, and
    the two launches agree bitwise (one writer per vertex and field)."""
    pxm = _dev()
    rng = np.random.default_rng(61)
    X, Y, Z = np.meshgrid(*[np.arange(r) for r in reso], indexing="ij")
    mask = np.zeros(reso, bool)
    for _ in range(3):
        c = rng.uniform(0, 1, 3) * np.array(reso)
        mask |= ((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) < rng.uniform(4, 16)
    mask &= rng.random(reso) < 0.7
    sig = rng.uniform(0.1, 2.0, size=int(mask.sum())).astype(np.float32)
    grid = synth.grid_from_mask(reso, (-1.0, -1.0, -1.0), 0.125, mask.ravel(), sig, rng)
    _, ref = oracle.tv(grid, 0.3, 0.05, 1e-4)
    outs = []
    for occ in (True, False):
        g = pxm.grid_to_device(grid, occupancy=occ)
        outs.append(np_(pxm.tv_grad(g, 0.3, 0.05, 1e-4)))
        outs.append(np_(pxm.tv_grad_set(g, 0.3, 0.05, 1e-4, grad_data=torch.full_like(g.data, -3.0))))
    torch.cuda.synchronize()
    assert_r28(outs[0], ref, TAU_GRAD, f"tv {reso}")
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_empty_grid_every_entry_point():
    """A map with no allocated vertex (n_alloc = 0, data and gradients may be
    NULL): transparent everywhere, zero gradients, a loss made of the targets
    alone, TV and RMSProp no-ops, an all-empty occupancy bitfield."""
    pxm = _dev()
    wl = synth.subset_rays(synth.config1(), 500, seed=63)
    R = wl.grid.reso
    empty = synth.Grid(R, wl.grid.aabb_min, wl.grid.voxel_size,
                       np.full(int(np.prod(R)), -1, np.int32), np.zeros((0, 28), np.float32))
    wl, ref = reference(wl.replace(grid=empty))
    g, r, t = to_dev(wl)
    assert g.data.numel() == 0 and int(g.occ.sum()) == 0
    n, F = wl.rays.n_rays, wl.rays.n_frames
    rgb, depth, ns = pxm.render_forward(g, r, wl.opts)
    loss = torch.zeros(F, dtype=torch.float64, device="cuda")
    gd = torch.zeros_like(g.data)
    gp = torch.zeros(F, 6, dtype=torch.float64, device="cuda")
    pxm.render_fused(g, r, wl.opts, t["rgb"], t["depth"], t["fw"], 3, loss=loss, grad_data=gd,
                     grad_pose=gp)
    pxm.tv_grad(g, 0.1, 0.1, 1e-6, gd)
    pxm.tv_grad_set(g, 0.1, 0.1, 1e-6, gd)
    pxm.grid_rmsprop(g.data, gd, torch.zeros_like(g.data), 0.1, 0.1)
    torch.cuda.synchronize()
    assert np.all(np_(rgb) == 0) and np.all(np_(depth) == 0)
    assert np.array_equal(np_(ns), ref["nsamp"])
    assert_r28(np_(loss), ref["loss"], TAU_FWD, "empty-map loss")
    assert np.all(np_(gp) == 0) and np.all(ref["grad_pose"] == 0)


def test_axis_aligned_rays():
    """Rays exactly parallel to lattice axes and lattice planes (direction
    components exactly 0: the zero-step branches of the box entry and of the
    brick jump), through a sparse grid with and without the occupancy
    bitfield, against the oracle: forward, grid and pose gradients."""
    pxm = _dev()
    rng = np.random.default_rng(64)
    grid = synth.random_tiny_grid(rng, R=40, margin=3, occupancy=0.15)
    mats = []
    for perm in ([0, 1, 2], [1, 2, 0], [2, 0, 1]):
        Rm = np.eye(3)[:, perm]
        if np.linalg.det(Rm) < 0:
            Rm[:, 0] *= -1
        c2w = np.zeros((3, 4))
        c2w[:, :3] = Rm
        c2w[:, 3] = -2.5 * Rm[:, 2] + 0.013 * rng.normal(size=3)
        mats.append(c2w)
    intr = np.array([[20.0, 20.0, 8.5, 8.5]] * 3)        # pixel (8, 8) looks along the optical axis
    u, v = np.meshgrid(np.arange(17), np.arange(17))
    pix = np.stack([u.ravel(), v.ravel()], 1).astype(np.int32)
    keep = (pix[:, 0] == 8) | (pix[:, 1] == 8) | (rng.random(len(pix)) < 0.3)
    pix = pix[keep]
    rays = synth.Rays(np.asarray(mats, np.float32), intr.astype(np.float32),
                      np.array([0, len(pix), 2 * len(pix), 3 * len(pix)], np.int32),
                      np.concatenate([pix] * 3))
    rgb0, depth0, _, _ = oracle.render(grid, rays, synth.Opts(step_vox=0.5, depth_loss=synth.DEPTH_L1))
    tg = synth.Targets((rgb0 + 0.05).astype(np.float32), (depth0 * 1.02 + 0.01).astype(np.float32),
                       synth.frame_weights(depth0 * 1.02 + 0.01, rays.frame_offsets, True))
    wl, ref = reference(synth.Workload("axis", grid, rays, tg,
                                       synth.Opts(step_vox=0.5, depth_loss=synth.DEPTH_L2)))
    for occ in (True, False):
        g = pxm.grid_to_device(grid, occupancy=occ)
        r = pxm.rays_to_device(rays)
        t = {k: torch.from_numpy(x).cuda() for k, x in
             (("rgb", tg.rgb), ("depth", tg.depth), ("fw", tg.frame_weight))}
        n, F = rays.n_rays, rays.n_frames
        out_rgb = torch.empty(n, 3, device="cuda")
        out_d = torch.empty(n, device="cuda")
        gd = torch.zeros_like(g.data)
        gp = torch.zeros(F, 6, dtype=torch.float64, device="cuda")
        pxm.render_fused(g, r, wl.opts, t["rgb"], t["depth"], t["fw"], 3, rgb=out_rgb,
                         depth=out_d, grad_data=gd, grad_pose=gp)
        torch.cuda.synchronize()
        what = f"axis-aligned (occupancy {occ})"
        assert_r28(np_(out_rgb), ref["rgb"], TAU_FWD, what + " rgb")
        assert_r28(np_(out_d), ref["depth"], TAU_FWD, what + " depth")
        assert_r28(np_(gd), ref["grad_data"], TAU_GRAD, what + " grid")
        assert_pose(np_(gp), ref["grad_pose"], TAU_GRAD, what + " pose")


def test_fused_long_rays_fall_back_to_scanning():
    """Rays with more than 1024 work positions (a 600-voxel, nearly
    transparent column) overflow the per-lane work mask the forward records,
    and their wave's backward scans the grid instead; the other frame's
    short rays, in another wave of the same launch, use the mask.  Both
    against the oracle, with and without the occupancy bitfield."""
    pxm = _dev()
    rng = np.random.default_rng(66)
    R = (6, 6, 600)
    n = int(np.prod(R))
    link = np.arange(n, dtype=np.int32)
    data = np.zeros((n, 28), np.float32)
    data[:, 0] = rng.uniform(0.001, 0.003, n)
    data[:, 1:] = rng.normal(0, 0.3, (n, 27))
    grid = synth.Grid(R, np.zeros(3, np.float32), synth.f32(0.01), link, data)
    along = np.zeros((3, 4))
    along[:, :3] = np.eye(3)
    along[:, 3] = [0.025, 0.025, -0.3]                     # looking along +z down the column
    across = np.zeros((3, 4))
    across[:, :3] = np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], float).T
    across[:, 3] = [0.3, 0.025, 3.0]                      # looking along -x across it
    intr = np.array([[2000.0, 2000.0, 8.0, 8.0], [40.0, 40.0, 8.0, 8.0]], np.float32)
    u, v = np.meshgrid(np.arange(4, 12), np.arange(4, 12))
    pix = np.stack([u.ravel(), v.ravel()], 1).astype(np.int32)          # 64 rays per frame
    rays = synth.Rays(np.stack([along, across]).astype(np.float32), intr,
                      np.array([0, 64, 128], np.int32), np.concatenate([pix, pix]))
    opts = synth.Opts(step_vox=0.5, depth_loss=synth.DEPTH_L2)
    rgb0, depth0, nsamp, _ = oracle.render(grid, rays, opts)
    assert nsamp[:64].max() > 1100 and nsamp[64:].max() < 1024
    tg = synth.Targets((rgb0 + 0.05).astype(np.float32), (depth0 * 1.01).astype(np.float32),
                       synth.frame_weights(depth0 * 1.01, rays.frame_offsets, True))
    wl, ref = reference(synth.Workload("long", grid, rays, tg, opts))
    tg = wl.targets
    for occ in (True, False):
        g = pxm.grid_to_device(grid, occupancy=occ)
        r = pxm.rays_to_device(rays)
        t = [torch.from_numpy(x).cuda() for x in (tg.rgb, tg.depth, tg.frame_weight)]
        out_rgb = torch.empty(128, 3, device="cuda")
        out_d = torch.empty(128, device="cuda")
        gd = torch.zeros_like(g.data)
        gp = torch.zeros(2, 6, dtype=torch.float64, device="cuda")
        old = pxm.get_tuning()
        pxm.set_tuning(64, 1)
        try:
            pxm.render_fused(g, r, opts, *t, 3, rgb=out_rgb, depth=out_d, grad_data=gd, grad_pose=gp)
            torch.cuda.synchronize()
        finally:
            pxm.set_tuning(*old)
        what = f"long rays (occupancy {occ})"
        assert_r28(np_(out_rgb), ref["rgb"], TAU_FWD, what + " rgb")
        assert_r28(np_(out_d), ref["depth"], TAU_FWD, what + " depth")
        assert_r28(np_(gd), ref["grad_data"], TAU_GRAD, what + " grid")
        assert_pose(np_(gp), ref["grad_pose"], TAU_GRAD, what + " pose")
        # the per-lane marches (pose only, Gauss-Newton) fall back lane by lane
        gp.zero_()
        pxm.render_fused(g, r, opts, *t, 2, grad_pose=gp)
        H, gv, E = oracle.gn_system(grid, rays, tg, opts)
        gn = pxm.render_gn(g, r, opts, *t)
        torch.cuda.synchronize()
        assert_pose(np_(gp), ref["grad_pose"], TAU_GRAD, what + " pose-only launch")
        Hg, gg, Eg = (np_(x) for x in pxm.gn_unpack(gn))
        assert_r28(Hg, H, TAU_GRAD, what + " Gauss-Newton H")
        assert_r28(gg, gv, TAU_GRAD, what + " Gauss-Newton g")


# ------------------------------------------------------------------ tracking update

def test_pose_adam_matches_oracle(c3):
    pxm = _dev()
    rng = np.random.default_rng(60)
    F = c3.rays.n_frames
    c2w = c3.rays.c2w.astype(np.float64)
    m = np.zeros((F, 6))
    v = np.zeros((F, 6))
    dc2w = torch.from_numpy(c3.rays.c2w.copy()).cuda()
    state = torch.zeros(F, 16, dtype=torch.float64, device="cuda")
    for it in range(1, 4):
        grad = rng.normal(size=(F, 6))
        c2w, m, v = oracle.adam_pose_step(c2w, grad, m, v, it, 1e-3)
        dg = torch.from_numpy(grad).cuda()
        pxm.pose_adam(dc2w, dg, state, 1e-3)
        torch.cuda.synchronize()
        assert np.all(np_(dg) == 0)
        np.testing.assert_allclose(np_(dc2w), c2w, atol=2e-6)
        c2w = np_(dc2w).astype(np.float64)


# ------------------------------------------------------------------ autograd

def _autograd_check(wl, ref, what):
    """Eq. 4, 5, 11 written in torch over the differentiable render (saved
    state: rgb, depth, nsamp per ray; the backward recomputes the samples),
    against the oracle's grid and pose gradients of the same loss."""
    pxm = _dev()
    from paper_2307_03404_amd import autograd as AG
    g, r, t = to_dev(wl)
    data = g.data.clone().requires_grad_(True)
    xi = torch.zeros(1, 6, dtype=torch.float64, device="cuda", requires_grad=True)
    rgb, depth, _ = AG.render(g, r, wl.opts, data=data, xi=xi)
    valid = torch.isfinite(t["depth"]) & (t["depth"] > 0)
    m = valid.sum()
    dd = torch.where(valid, depth - torch.where(valid, t["depth"], 0.0), 0.0)
    ec = torch.where(valid[:, None], rgb - t["rgb"], 0.0)
    loss = (ec ** 2).sum() / m + dd.abs().sum() / m
    loss.backward()
    torch.cuda.synchronize()
    assert_r28(np_(rgb), ref["rgb"], TAU_FWD, what + " rgb")
    assert_r28(np_(data.grad), ref["grad_data"], TAU_GRAD, what + " grid")
    assert_pose(np_(xi.grad), ref["grad_pose"], TAU_GRAD, what + " pose")


def test_autograd_matches_direct_calls(c1):
    wl, ref = c1
    _autograd_check(wl, ref, "autograd c1")


def test_autograd_full_frame_c2(c2_ref):
    """A whole 1200x680 frame (816,000 rays) through the autograd.Function:
    20 bytes of saved state per ray, recomputation in the backward."""
    wl, ref = c2_ref
    _autograd_check(wl, ref, "autograd c2 full frame")


def _small_lattice_workload(reso, seed):
    """A lattice at or near the minimum size: one cell (2x2x2), or two
    vertices thick, seen by a 24x24 camera from outside the box."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(reso))
    mask = np.ones(n, bool) if n == 8 else rng.random(n) < 0.6
    sig = rng.uniform(0.2, 2.0, int(mask.sum())).astype(np.float32)
    vs = 0.1
    g = synth.grid_from_mask(reso, (0.0, 0.0, 0.0), vs, mask, sig, rng)
    centre = vs * (np.array(reso, np.float64) - 1) / 2
    eye = centre + np.array([0.35, -0.3, 0.25]) * (0.5 + max(reso) * vs)
    c2w = synth.look_at(eye, centre)
    W = 24
    intr = np.array([W, W, W / 2, W / 2], np.float64)
    v_, u_ = np.mgrid[0:W, 0:W]
    pix = np.stack([u_.ravel(), v_.ravel()], 1).astype(np.int32)
    rays = synth.Rays(c2w[None], intr[None], np.array([0, W * W], np.int32), pix)
    opts = synth.Opts(step_vox=0.5, max_samples=100_000, t_near=0.0, t_stop=synth.f32(1e-6),
                      color_act=synth.COLOR_SIGMOID, depth_loss=synth.DEPTH_L1, lambda_depth=1.0)
    rgb, depth, _, _ = oracle.render(g, rays, opts)
    tgt_rgb = (rgb + 0.05 * rng.normal(size=rgb.shape)).astype(np.float32)
    tgt_depth = np.where(depth > 0, 1.02 * depth, 0.0).astype(np.float32)   # misses: invalid
    tg = synth.Targets(tgt_rgb, tgt_depth, np.array([1.0 / (W * W)], np.float32))
    return synth.Workload(f"lattice{reso}", g, rays, tg, opts)


@pytest.mark.parametrize("reso", [(2, 2, 2), (2, 3, 70), (70, 2, 3)])
def test_minimum_and_thin_lattices(reso):
    """Degenerate lattice sizes through every grid entry point: the fused
    step in one and two launches, TV, growth and pruning."""
    pxm = _dev()
    wl, ref = reference(_small_lattice_workload(reso, 81 + sum(reso)))
    hit = ref["depth"] > 0
    assert hit.sum() > 20, "the camera must see the box"
    _fused_check(wl, 3, f"lattice {reso}", ref, block=64, variant=1)
    _fused_check(wl, 3, f"lattice {reso} two launches", ref, block=64, variant=2)
    g = pxm.grid_to_device(wl.grid)
    _, tv_ref = oracle.tv(wl.grid, 1e-2, 1e-3, 1e-6)
    tv = pxm.tv_grad(g, 1e-2, 1e-3, 1e-6)
    torch.cuda.synchronize()
    assert_r28(np_(tv), tv_ref, TAU_GRAD, f"lattice {reso} tv")
    up_ref = oracle.grid_upsample(wl.grid)
    up = pxm.grid_upsample(g)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(up.link), up_ref.link)
    assert np.array_equal(np_(up.data), up_ref.data)
    tau = float(np.median(wl.grid.data[:, 0]))
    pr_ref = oracle.grid_prune(wl.grid, np.float32(tau))
    pr = pxm.grid_prune(g, tau)
    np.testing.assert_array_equal(np_(pr.link), pr_ref.link)
    assert np.array_equal(np_(pr.data), pr_ref.data)


@pytest.mark.parametrize("variant", [1, 2])
def test_fused_sample_cap_near_plane_and_early_stop(c1, variant):
    """A cap that cuts most rays (20 kept positions), a near plane inside the
    grid and early termination: the backward replays exactly the samples the
    forward kept, in one launch and in two."""
    wl, _ = c1
    opts = dataclasses.replace(wl.opts, max_samples=20, t_near=synth.f32(2.4),
                               t_stop=synth.f32(0.05))
    wlc, ref = reference(wl.replace(opts=opts))
    assert (ref["nsamp"] == 20).sum() > 100, "the cap must bind on many rays"
    _fused_check(wlc, 3, f"c1 capped v{variant}", ref, block=64, variant=variant)


@pytest.mark.parametrize("act,depth_loss", [(synth.COLOR_SIGMOID, synth.DEPTH_L2),
                                            (synth.COLOR_IDENTITY, synth.DEPTH_L1)])
def test_fused_colour_activations_and_depth_norms(c1, act, depth_loss):
    """The fused step for the other colour activations (c1 itself uses the
    shifted ReLU) and both depth norms of the loss."""
    wl, _ = c1
    wla, ref = reference(wl.replace(opts=dataclasses.replace(wl.opts, color_act=act,
                                                             depth_loss=depth_loss)))
    _fused_check(wla, 3, f"c1 act {act} depth {depth_loss}", ref)
