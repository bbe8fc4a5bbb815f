"""Shared helpers of the GPU parity tests (no GPU needed to import)."""
import numpy as np

# Tolerances: forward outputs within 1e-5 and gradients within 1e-4, relative
# elementwise with an RMS floor, |x - x*| <= tau * max(|x*|, rms(x*)).  The
# floor lets entries that are tiny compared with the tensor's typical
# magnitude (e.g. a vertex touched only by nearly transparent samples, whose
# FP32 rounding is set by the large terms it is summed with) be judged
# against that typical magnitude.  Atomic additions happen in any order, so
# gradients cannot be bitwise reproducible.
TAU_FWD = 1e-5
TAU_GRAD = 1e-4


def r28_ratio(x, ref):
    """max |x - ref| / max(|ref|, rms(ref)); <= tau passes."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    rms = float(np.sqrt(np.mean(ref * ref)))
    scale = np.maximum(np.abs(ref), rms)
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(x - ref) / scale))


def assert_r28(x, ref, tau, what):
    ratio = r28_ratio(x, ref)
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    nrm = float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))
    assert ratio <= tau, f"{what}: max scaled error {ratio:.3e} > {tau:.1e} (normwise {nrm:.3e})"
    return ratio


def assert_pose(gp, ref, tau, what):
    """Pose gradients checked per group: translation (rho) and rotation (phi)."""
    a = assert_r28(np.asarray(gp)[:, :3], np.asarray(ref)[:, :3], tau, what + " rho")
    b = assert_r28(np.asarray(gp)[:, 3:], np.asarray(ref)[:, 3:], tau, what + " phi")
    return max(a, b)
