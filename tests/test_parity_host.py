"""Host logic of the parity harness (no GPU): targets moved off the L1 kink
using oracle values only."""
import numpy as np
import pytest

from paper_2307_03404_amd import synth
from tests._parity import KINK_MAX_FRACTION, kink_band, kink_free_targets, r28_ratio


def _wl(depth_tgt, depth_loss=synth.DEPTH_L1):
    n = len(depth_tgt)
    rays = synth.Rays(np.zeros((1, 3, 4), np.float32), np.ones((1, 4), np.float32),
                      np.array([0, n], np.int32), np.zeros((n, 2), np.int32))
    tg = synth.Targets(np.zeros((n, 3), np.float32), np.asarray(depth_tgt, np.float32),
                       np.ones(1, np.float32))
    grid = synth.Grid((2, 2, 2), np.zeros(3, np.float32), 1.0, np.full(8, -1, np.int32),
                      np.zeros((0, 28), np.float32))
    return synth.Workload("host", grid, rays, tg, synth.Opts(depth_loss=depth_loss))


def test_targets_near_the_kink_move_to_the_side_of_their_residual():
    rng = np.random.default_rng(1)
    z = rng.uniform(1.0, 4.0, 1000)                      # the oracle's z-depth
    z[11] = float(np.float32(z[11]))                     # so that D[11] = z[11] exactly
    D = (z + rng.normal(0, 0.01, 1000)).astype(np.float32)
    D[[3, 7, 11]] = (z[[3, 7, 11]] + np.array([1e-6, -2e-6, 0.0])).astype(np.float32)
    D[20] = np.nan
    D[21] = 0.0
    wl, n = kink_free_targets(_wl(D), z)
    band = kink_band(z)
    Dn = wl.targets.depth
    assert n >= 3
    moved = np.flatnonzero((Dn != D) & np.isfinite(D))
    assert {3, 7, 11} <= set(moved.tolist())
    assert np.isnan(Dn[20]) and Dn[21] == 0.0            # invalid targets untouched
    assert np.all(np.abs(z[moved] - Dn[moved]) > band[moved])
    assert np.sign(z[3] - Dn[3]) == np.sign(z[3] - float(D[3])) or z[3] == float(D[3])
    assert z[11] - Dn[11] > 0                           # a zero residual goes positive
    far = np.setdiff1d(np.arange(1000), np.concatenate([moved, [20, 21]]))
    assert np.array_equal(Dn[far], D[far])


def test_other_norms_and_too_many_kinks():
    z = np.linspace(1.0, 2.0, 100)
    wl, n = kink_free_targets(_wl(z, synth.DEPTH_L2), z)
    assert n == 0                                        # the squared norm has no kink
    with pytest.raises(AssertionError, match="L1 kink"):
        kink_free_targets(_wl(z), z)                      # every target on the kink
    assert KINK_MAX_FRACTION <= 0.01


def test_r28_ratio_uses_the_rms_floor():
    ref = np.array([1.0, 1e-9, -1.0])
    assert r28_ratio(ref + np.array([0.0, 1e-6, 0.0]), ref) == pytest.approx(1e-6 / np.sqrt(2 / 3))
