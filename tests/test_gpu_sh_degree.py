"""GPU parity on records of SH degree 0 and 1 (4 and 16 floats: density and
the first 1 or 4 SH functions per channel; Sec. 5.2 uses nine) against the
FP64 oracle: forward, the two backward entry points, the fused step in its
three launch forms (coherent tiles on the matrix-core scatter, a random ray
subset on the broadcast scatter), Gauss-Newton normal equations, TV, the
RMSProp step and the grid edits (bit-exact)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2307_03404_amd import synth
from tests._parity import TAU_FWD, TAU_GRAD, assert_pose, assert_r28, reference
from tests.test_gpu_parity import _fused_check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEGREES = [0, 1]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_03404_amd import pxm
    return pxm


def np_(t):
    return t.detach().cpu().numpy()


def _c1(deg):
    wl = synth.config1()
    return wl.replace(name=f"{wl.name} degree {deg}", grid=synth.with_sh_degree(wl.grid, deg))


@pytest.fixture(scope="module", params=DEGREES)
def c1d(request):
    return reference(_c1(request.param))


def _to_dev(wl):
    pxm = _dev()
    return pxm.grid_to_device(wl.grid), pxm.rays_to_device(wl.rays)


def test_forward(c1d):
    pxm = _dev()
    wl, ref = c1d
    g, r = _to_dev(wl)
    assert g.data.shape[1] == synth.record_floats(wl.grid.sh_degree)
    rgb, depth, ns = pxm.render_forward(g, r, wl.opts)
    torch.cuda.synchronize()
    assert_r28(np_(rgb), ref["rgb"], TAU_FWD, "rgb")
    assert_r28(np_(depth), ref["depth"], TAU_FWD, "depth")
    assert np.mean(np_(ns) != ref["nsamp"]) <= 1e-3


def test_backward_entry_points(c1d):
    pxm = _dev()
    wl, ref = c1d
    # the oracle's backward sees the same float32 upstream gradients as the GPU
    g_rgb32, g_dep32 = ref["g_rgb"].astype(np.float32), ref["g_depth"].astype(np.float32)
    gref, pref = oracle.backward(wl.grid, wl.rays, wl.opts, g_rgb32, g_dep32, True, True)
    g, r = _to_dev(wl)
    rgb, depth, ns = pxm.render_forward(g, r, wl.opts)
    g_rgb = torch.from_numpy(g_rgb32).cuda()
    g_dep = torch.from_numpy(g_dep32).cuda()
    gd = torch.zeros_like(g.data)
    pxm.render_backward_grid(g, r, wl.opts, rgb, depth, ns, g_rgb, g_dep, gd)
    gp = torch.zeros(1, 6, dtype=torch.float64, device="cuda")
    pxm.render_backward_pose(g, r, wl.opts, rgb, depth, ns, g_rgb, g_dep, gp)
    torch.cuda.synchronize()
    used = oracle.used_fields(wl.grid.sh_degree)
    assert np.all(np_(gd)[:, used:] == 0.0)
    assert_r28(np_(gd)[:, 0], gref[:, 0], TAU_GRAD, "grad density")
    assert_r28(np_(gd)[:, 1:used], gref[:, 1:used], TAU_GRAD, "grad sh")
    assert_pose(np_(gp), pref, TAU_GRAD, "pose")


@pytest.mark.parametrize("block,variant", [(64, 0), (64, 1), (256, 2)])
def test_fused_launch_forms(c1d, block, variant):
    wl, ref = c1d
    _fused_check(wl, 3, f"deg {wl.grid.sh_degree} b{block} v{variant}", ref, block, variant)


@pytest.mark.parametrize("deg", DEGREES)
def test_fused_view_direction_pose_term(deg):
    wl = _c1(deg)
    wl = wl.replace(opts=dataclasses.replace(wl.opts, flags=synth.FLAG_POSE_VIEWDIR))
    _fused_check(wl, 2, f"deg {deg} viewdir")


@pytest.fixture(scope="module")
def c2():
    return synth.config2()


@pytest.mark.parametrize("deg", DEGREES)
def test_fused_room_tile_block_and_random_subset(c2, deg):
    """A block of whole 8x8 tiles of the 256^3 room frame (coherent: the
    matrix-core scatter) and a seeded random ray subset of it (incoherent:
    the broadcast scatter)."""
    wl = c2.replace(grid=synth.with_sh_degree(c2.grid, deg))
    off = 64 * 3000
    n = 64 * 250
    tiles = wl.replace(rays=dataclasses.replace(wl.rays, pix=wl.rays.pix[off:off + n].copy(),
                                                frame_offsets=np.array([0, n], np.int32)),
                       targets=dataclasses.replace(wl.targets, rgb=wl.targets.rgb[off:off + n].copy(),
                                                   depth=wl.targets.depth[off:off + n].copy()))
    _fused_check(tiles, 3, f"room tiles deg {deg}", None, 64, 1)
    sub = synth.subset_rays(wl, 12000, seed=17)
    _fused_check(sub, 3, f"room subset deg {deg}", None, 64, 2)


@pytest.mark.parametrize("deg", DEGREES)
def test_gauss_newton_normal_equations(deg):
    pxm = _dev()
    wl = synth.subset_rays(synth.config3(), 12000, seed=92)
    wl = wl.replace(grid=synth.with_sh_degree(wl.grid, deg),
                    opts=dataclasses.replace(wl.opts, flags=synth.FLAG_POSE_VIEWDIR))
    H, gv, E = oracle.gn_system(wl.grid, wl.rays, wl.targets, wl.opts)
    g, r = _to_dev(wl)
    t = [torch.from_numpy(x).cuda() for x in (wl.targets.rgb, wl.targets.depth, wl.targets.frame_weight)]
    gn = pxm.render_gn(g, r, wl.opts, *t)
    torch.cuda.synchronize()
    Hg, gg, Eg = (np_(x) for x in pxm.gn_unpack(gn))
    assert_r28(Hg, H, TAU_GRAD, "H")
    assert_r28(gg[:, :3], gv[:, :3], TAU_GRAD, "g rho")
    assert_r28(gg[:, 3:], gv[:, 3:], TAU_GRAD, "g phi")
    assert_r28(Eg, E, TAU_GRAD, "E")


@pytest.mark.parametrize("deg", DEGREES)
def test_tv(deg):
    pxm = _dev()
    for wl in (synth.config1(), synth.config2()):
        grid = synth.with_sh_degree(wl.grid, deg)
        _, ref = oracle.tv(grid, 0.3, 0.05, 1e-4)
        g = pxm.grid_to_device(grid)
        base = torch.full_like(g.data, 0.25)
        grad = pxm.tv_grad(g, 0.3, 0.05, 1e-4, grad_data=base)
        put = pxm.tv_grad_set(g, 0.3, 0.05, 1e-4, grad_data=torch.full_like(g.data, 0.25))
        torch.cuda.synchronize()
        used = oracle.used_fields(deg)
        assert np.all(np_(grad)[:, used:] == 0.25) and np.all(np_(put)[:, used:] == 0.25)
        assert_r28(np_(grad)[:, :used] - 0.25, ref[:, :used], TAU_GRAD, f"tv {wl.name} deg {deg}")
        assert_r28(np_(put)[:, :used], ref[:, :used], TAU_GRAD, f"tv set {wl.name} deg {deg}")


@pytest.mark.parametrize("deg", DEGREES)
def test_rmsprop(deg):
    pxm = _dev()
    S = synth.record_floats(deg)
    used = oracle.used_fields(deg)
    rng = np.random.default_rng(73 + deg)
    n = 1001
    data = rng.normal(size=(n, S)).astype(np.float32)
    data[:, used:] = 0.0
    state = rng.uniform(0.0, 1.0, size=(n, S)).astype(np.float32)
    dd, ds = torch.from_numpy(data).cuda(), torch.from_numpy(state).cuda()
    for step in range(2):
        gr = rng.normal(size=(n, S)).astype(np.float32)
        gr[:, used:] = 0.0
        gr[rng.random(n) < 0.3] = 0.0
        ref_d, ref_s = oracle.rmsprop_grid(np_(dd), gr, np_(ds), 0.3, 0.02, 0.9, 1e-8)
        dg = torch.from_numpy(gr).cuda()
        pxm.grid_rmsprop(dd, dg, ds, 0.3, 0.02, alpha=0.9, eps=1e-8, sh_degree=deg)
        torch.cuda.synchronize()
        assert np.all(np_(dg) == 0.0)
        assert_r28(np_(dd), ref_d, TAU_FWD, f"rmsprop data step {step}")
        assert_r28(np_(ds), ref_s, TAU_FWD, f"rmsprop state step {step}")


@pytest.mark.parametrize("deg", DEGREES)
def test_grid_edits_bit_exact(deg):
    pxm = _dev()
    g = synth.with_sh_degree(synth.config1().grid, deg)
    want = oracle.grid_upsample(g)
    got = pxm.grid_upsample(pxm.grid_to_device(g))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(got.link), want.link)
    assert got.sh_degree == deg and np.array_equal(np_(got.data), want.data)
    tau = float(np.median(g.data[:, 0]))
    want = oracle.grid_prune(g, np.float32(tau))
    got = pxm.grid_prune(pxm.grid_to_device(g), tau)
    np.testing.assert_array_equal(np_(got.link), want.link)
    assert got.sh_degree == deg and np.array_equal(np_(got.data), want.data)
