"""The allocation-free fused step (pxm_render_fused_noalloc) against the
fused step with a caller workspace (pxm_render_fused), through the C ABI:
two calls in a row on one GPU, the second on a smaller batch, in each launch
form.  Forward outputs must agree bit for bit (each ray's march is the same
code on the same inputs); loss, grid and pose gradients to the gradient
tolerance (atomic additions in any order).  The first call also goes against
the FP64 oracle."""
import numpy as np
import pytest

from paper_2307_03404_amd import synth
from tests._parity import TAU_FWD, TAU_GRAD, assert_pose, assert_r28, reference

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_03404_amd import pxm
    return pxm


def np_(t):
    return t.detach().cpu().numpy()


def _run(pxm, wl, want, noalloc):
    g = pxm.grid_to_device(wl.grid)
    r = pxm.rays_to_device(wl.rays)
    trgb = torch.from_numpy(wl.targets.rgb).cuda()
    tdep = torch.from_numpy(wl.targets.depth).cuda()
    fw = torch.from_numpy(wl.targets.frame_weight).cuda()
    n, F = wl.rays.n_rays, wl.rays.n_frames
    out = dict(rgb=torch.full((n, 3), -1.0, device="cuda"), depth=torch.full((n,), -1.0, device="cuda"),
               loss=torch.zeros(F, dtype=torch.float64, device="cuda"),
               grad_data=torch.zeros_like(g.data),
               grad_pose=torch.zeros(F, 6, dtype=torch.float64, device="cuda"))
    if noalloc:
        pxm.render_fused_noalloc(g, r, wl.opts, trgb, tdep, fw, want, **out)
    else:
        pxm.render_fused(g, r, wl.opts, trgb, tdep, fw, want, **out)
    torch.cuda.synchronize()
    return {k: np_(v) for k, v in out.items()}


def _compare(a, b, what):
    assert np.array_equal(a["rgb"], b["rgb"]), what + " rgb"
    assert np.array_equal(a["depth"], b["depth"]), what + " depth"
    assert_r28(a["loss"], b["loss"], TAU_FWD, what + " loss")
    assert_r28(a["grad_data"][:, 0], b["grad_data"][:, 0], TAU_GRAD, what + " grad density")
    assert_r28(a["grad_data"][:, 1:], b["grad_data"][:, 1:], TAU_GRAD, what + " grad sh")
    assert_pose(a["grad_pose"], b["grad_pose"], TAU_GRAD, what + " pose")


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_noalloc_matches_workspace_entry_point(variant):
    pxm = _dev()
    wl, ref = reference(synth.config1())
    small, _ = reference(synth.subset_rays(wl, 1500, seed=5))
    want = pxm.WANT_GRID | pxm.WANT_POSE
    old = pxm.get_tuning()
    pxm.set_tuning(64, variant)
    try:
        for i, w in enumerate((wl, small)):
            print(f"[gpu] noalloc variant {variant} call {i + 1}: {w.rays.n_rays} rays", flush=True)
            a = _run(pxm, w, want, noalloc=True)
            b = _run(pxm, w, want, noalloc=False)
            _compare(a, b, f"v{variant} call {i + 1}")
            if i == 0:
                assert_r28(a["rgb"], ref["rgb"], TAU_FWD, "rgb vs oracle")
                assert_r28(a["grad_data"], ref["grad_data"], TAU_GRAD, "grad vs oracle")
                assert_pose(a["grad_pose"], ref["grad_pose"], TAU_GRAD, "pose vs oracle")
    finally:
        pxm.set_tuning(*old)


def test_noalloc_many_frames_pose_only_then_smaller():
    """Tracking batch of 16 frames (453k rays, persistent form, pose only),
    then a 20k-ray subset of it."""
    pxm = _dev()
    wl = synth.config3()
    small = synth.subset_rays(wl, 20000, seed=9)
    old = pxm.get_tuning()
    pxm.set_tuning(256, 1)
    try:
        for i, w in enumerate((wl, small)):
            print(f"[gpu] noalloc pose-only call {i + 1}: {w.rays.n_rays} rays", flush=True)
            a = _run(pxm, w, pxm.WANT_POSE, noalloc=True)
            b = _run(pxm, w, pxm.WANT_POSE, noalloc=False)
            assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["depth"], b["depth"])
            assert_r28(a["loss"], b["loss"], TAU_FWD, "loss")
            assert_pose(a["grad_pose"], b["grad_pose"], TAU_GRAD, "pose")
            assert np.all(a["grad_data"] == 0)
    finally:
        pxm.set_tuning(*old)
