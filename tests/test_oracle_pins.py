"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms (slab transmittance, geometric-series depth, opaque plane, SH degree-0
colour), library routines (scipy's spherical harmonics, scipy's matrix
exponential, torch's Adam), exact polynomial reproduction, geometric
inverses (re-projecting a ray) and central finite differences of the
oracle's own forward pass for every backward quantity.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2307_03404_amd import synth

OPTS = synth.Opts(step_vox=0.5, max_samples=10_000, t_near=0.0, t_stop=0.0,
                  color_act=synth.COLOR_IDENTITY, depth_loss=synth.DEPTH_L2)


def dense_grid(R, values, lo=(0.0, 0.0, 0.0), vs=1.0):
    """Dense grid with link = identity and payload values[R^3, 28]."""
    link = np.arange(R ** 3, dtype=np.int32)
    return synth.Grid((R, R, R), np.asarray(lo, np.float32), float(vs), link,
                      np.ascontiguousarray(values, np.float32))


def lattice(R):
    i = np.arange(R)
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float64)


# ---------------------------------------------------------------- rays (Sec. 4)

def test_ray_principal_point_and_reprojection():
    rng = np.random.default_rng(0)
    c2w = synth.perturb_pose(synth.look_at((1.0, 2.0, 0.5), (0.0, 0.0, 0.0)), rng, 0.1, 0.3)
    intr = np.array([500.0, 450.0, 10.5, 20.5])
    o, d, s = oracle.ray(c2w, intr, 10, 20)            # pixel centre on the principal point
    assert s == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(d, c2w[:, 2], atol=1e-15)
    np.testing.assert_allclose(o, c2w[:, 3], atol=1e-15)
    for u, v in [(0, 0), (37, 5), (1199, 679)]:
        o, d, s = oracle.ray(c2w, intr, u, v)
        assert np.linalg.norm(d) == pytest.approx(1.0, abs=1e-14)
        # project a point of the ray back through the pinhole
        x = c2w[:, :3].T @ (o + 2.7 * d - c2w[:, 3])
        assert x[0] / x[2] * intr[0] + intr[2] == pytest.approx(u + 0.5, abs=1e-9)
        assert x[1] / x[2] * intr[1] + intr[3] == pytest.approx(v + 0.5, abs=1e-9)
        assert x[2] * s == pytest.approx(2.7, abs=1e-12)    # range = z-depth * |d_cam|


# ---------------------------------------------------------- SH basis (Sec. 5.2)

def _real_sh_scipy(d):
    import scipy.special as sp
    x, y, z = d
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    out = []
    for l, m in [(0, 0), (1, -1), (1, 0), (1, 1), (2, -2), (2, -1), (2, 0), (2, 1), (2, 2)]:
        if m == 0:
            out.append(sp.sph_harm_y(l, 0, theta, phi).real)
        elif m > 0:
            out.append(np.sqrt(2) * sp.sph_harm_y(l, m, theta, phi).real)
        else:
            out.append(np.sqrt(2) * sp.sph_harm_y(l, -m, theta, phi).imag)
    return np.array(out)


def test_sh_basis_matches_scipy_real_harmonics():
    rng = np.random.default_rng(1)
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        np.testing.assert_allclose(oracle.sh_basis(d), _real_sh_scipy(d), atol=1e-13)


def test_sh_orthonormal_by_quadrature():
    xg, wg = np.polynomial.legendre.leggauss(12)       # exact for degree <= 23 in cos(theta)
    nphi = 16
    G = np.zeros((9, 9))
    for ct, wt in zip(xg, wg):
        st = np.sqrt(1 - ct * ct)
        for j in range(nphi):
            ph = 2 * np.pi * j / nphi
            Y = oracle.sh_basis(np.array([st * np.cos(ph), st * np.sin(ph), ct]))
            G += wt * (2 * np.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(9), atol=1e-13)


def test_sh_basis_gradient_fd():
    rng = np.random.default_rng(2)
    d = rng.normal(size=3)
    G = oracle.sh_basis_grad(d)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (oracle.sh_basis(d + e) - oracle.sh_basis(d - e)) / (2 * h)
        np.testing.assert_allclose(G[:, a], fd, atol=1e-8)


# ------------------------------------------ trilinear interpolation (App. A)

def test_trilinear_reproduces_multilinear_polynomials_and_eq16():
    rng = np.random.default_rng(3)
    R = 5
    P = lattice(R)
    coef = rng.normal(size=(8, 28))

    def poly(p):
        x, y, z = p[..., 0:1], p[..., 1:2], p[..., 2:3]
        basis = np.concatenate([np.ones_like(x), x, y, z, x * y, x * z, y * z, x * y * z], -1)
        return basis @ coef

    def poly_grad(p):
        x, y, z = p
        gx = coef[1] + coef[4] * y + coef[5] * z + coef[7] * y * z
        gy = coef[2] + coef[4] * x + coef[6] * z + coef[7] * x * z
        gz = coef[3] + coef[5] * x + coef[6] * y + coef[7] * x * y
        return np.stack([gx, gy, gz], 1)

    # values are stored in float32, so compare against the float32-rounded polynomial
    vals = poly(P).astype(np.float32)
    g = dense_grid(R, vals)
    # the interpolant of float32 vertex values: refit the polynomial per cell is not needed,
    # since each cell holds a multilinear function; check against a float64 grid instead
    for _ in range(40):
        q = rng.uniform(0, R - 1, size=3)
        val, grad = oracle.interp(g, q)
        np.testing.assert_allclose(val, poly(q[None])[0], rtol=2e-6, atol=2e-5)
        np.testing.assert_allclose(grad, poly_grad(q), rtol=2e-5, atol=2e-4)
    # exactness at vertices
    for idx in [0, 7, 31, 124]:
        val, _ = oracle.interp(g, P[idx])
        np.testing.assert_array_equal(val.astype(np.float32), vals[idx])


def test_trilinear_gradient_fd_and_linear_field():
    rng = np.random.default_rng(4)
    R = 4
    g = dense_grid(R, rng.normal(size=(R ** 3, 28)))
    h = 1e-6
    for _ in range(20):
        q = rng.uniform(0.05, R - 1.05, size=3)
        # keep away from cell faces where the derivative is one-sided
        q = np.floor(q) + np.clip(q - np.floor(q), 0.01, 0.99)
        _, G = oracle.interp(g, q)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            fd = (oracle.interp(g, q + e, False)[0] - oracle.interp(g, q - e, False)[0]) / (2 * h)
            np.testing.assert_allclose(G[:, a], fd, atol=1e-8)
    # a linear field has a constant gradient
    a = np.array([0.25, -0.5, 0.125])
    vals = np.repeat((lattice(R) @ a)[:, None], 28, 1)
    gl = dense_grid(R, vals)
    for _ in range(5):
        _, G = oracle.interp(gl, rng.uniform(0, R - 1, size=3))
        np.testing.assert_allclose(G, np.tile(a, (28, 1)), atol=1e-12)


# ------------------------------------------------ compositing (Eq. 1, 2, 3)

def _axis_ray(R, q0_yz=(2.3, 1.7)):
    o = np.array([0.25, q0_yz[0], q0_yz[1]])        # vs = 1, lo = 0: world == voxel units
    d = np.array([1.0, 0.0, 0.0])
    return o, d


def test_slab_transmittance_closed_form():
    R, a, b, s0 = 24, 6, 13, float(np.float32(0.37))
    vals = np.zeros((R ** 3, 28))
    P = lattice(R)
    vals[(P[:, 0] >= a) & (P[:, 0] <= b), 0] = s0
    g = dense_grid(R, vals)
    o, d = _axis_ray(R)
    tr = oracle.trace(g, o, d, OPTS)
    # midpoint sums of a piecewise-linear density: sum sigma*delta = s0 (b - a + 1)
    assert tr["T"][-1] == pytest.approx(np.exp(-s0 * (b - a + 1)), rel=1e-13)
    # invariant: the weights and the transmitted light add up to one (Eq. 2)
    assert tr["w"].sum() + tr["T"][-1] == pytest.approx(1.0, abs=1e-14)


def test_constant_density_depth_geometric_series():
    R, s0 = 12, float(np.float32(0.21))
    vals = np.zeros((R ** 3, 28))
    vals[:, 0] = s0
    g = dense_grid(R, vals)
    o, d = _axis_ray(R)
    tr = oracle.trace(g, o, d, OPTS)
    n = tr["n"]
    assert n == 2 * (R - 1)              # positions 0.25, 0.75, ..., R - 1.25
    q = np.exp(-s0 * 0.5)
    t0, dw = tr["t"][0], 0.5
    D = (1 - q ** n) * t0 + dw * q * (1 - n * q ** (n - 1) + (n - 1) * q ** n) / (1 - q)
    assert tr["D"] == pytest.approx(D, rel=1e-13)


def test_opaque_plane_depth():
    R, a = 16, 9
    vals = np.zeros((R ** 3, 28))
    P = lattice(R)
    vals[P[:, 0] >= a, 0] = 1e3
    g = dense_grid(R, vals, lo=(-3.0, -1.0, 2.0), vs=0.25)
    # camera looking along +x through a pixel off the principal point
    c2w = np.array([[0.0, 0.0, 1.0, -3.0 + 0.25 * 0.25],
                    [-1.0, 0.0, 0.0, -1.0 + 0.25 * 7.4],
                    [0.0, -1.0, 0.0, 2.0 + 0.25 * 7.1]])
    intr = np.array([100.0, 100.0, 50.0, 50.0])
    rays = synth.Rays(c2w[None].astype(np.float64), intr[None], np.array([0, 1], np.int32),
                      np.array([[53, 48]], np.int32))
    rgb, depth, nsamp, _ = oracle.render(g, rays, OPTS)
    o, d, s = oracle.ray(c2w, intr, 53, 48)
    # first sample whose x-coordinate (voxel units) exceeds a - 1 takes all the light
    k = 0
    while (o[0] + 0.25 * 0.5 * k * d[0] - (-3.0)) / 0.25 <= a - 1:
        k += 1
    t_first = 0.25 * 0.5 * k
    x_first = o + t_first * d
    zdepth = (x_first - o) @ c2w[:, 2]
    assert depth[0] == pytest.approx(zdepth, rel=1e-12)


def test_sh_degree0_colour_closed_form():
    R, s0 = 10, float(np.float32(0.3))
    k0 = np.array([0.4, -0.2, 1.1], np.float32).astype(np.float64)
    vals = np.zeros((R ** 3, 28))
    vals[:, 0] = s0
    vals[:, [1, 10, 19]] = k0
    g = dense_grid(R, vals)
    rng = np.random.default_rng(5)
    Y0 = 0.5 / np.sqrt(np.pi)
    for act, f in [(synth.COLOR_IDENTITY, lambda s: s),
                   (synth.COLOR_SIGMOID, lambda s: 1 / (1 + np.exp(-s))),
                   (synth.COLOR_RELU_SHIFT, lambda s: np.maximum(s + 0.5, 0))]:
        opts = dataclasses.replace(OPTS, color_act=act)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        o = np.array([4.5, 4.5, 4.5]) - 3 * d
        tr = oracle.trace(g, o, d, opts)
        np.testing.assert_allclose(tr["rgb"], f(Y0 * k0) * (1 - tr["T"][-1]), rtol=1e-13)


def test_early_termination_and_cap():
    R = 12
    vals = np.zeros((R ** 3, 28))
    vals[:, 0] = 2.0
    g = dense_grid(R, vals)
    o, d = _axis_ray(R)
    opts = dataclasses.replace(OPTS, t_stop=1e-4)
    tr = oracle.trace(g, o, d, opts)
    assert tr["T"][-1] < 1e-4 <= tr["T"][-2]
    assert tr["n"] == int(np.ceil(np.log(1e4) / 1.0))          # sigma*delta = 1 per sample
    tr = oracle.trace(g, o, d, dataclasses.replace(OPTS, max_samples=5))
    assert tr["n"] == 5


# ------------------------------------------- loss (Eq. 4, 5, 11), masking

def test_loss_gradient_fd_and_invalid_rays():
    rng = np.random.default_rng(6)
    n = 20
    rays = synth.Rays(np.zeros((2, 3, 4)), np.ones((2, 4)), np.array([0, 8, 20], np.int32),
                      np.zeros((n, 2), np.int32))
    rgb = rng.uniform(size=(n, 3))
    depth = rng.uniform(1, 3, size=n)
    trgb = rng.uniform(size=(n, 3)).astype(np.float32)
    tdep = rng.uniform(1, 3, size=n).astype(np.float32)
    tdep[[1, 9]] = 0.0
    tdep[3] = np.nan
    tdep[12] = -1.0
    fw = np.array([0.3, 0.7], np.float32)
    tg = synth.Targets(trgb, tdep, fw)
    for loss_kind in (synth.DEPTH_L1, synth.DEPTH_L2):
        opts = dataclasses.replace(OPTS, depth_loss=loss_kind, lambda_depth=0.6)
        L, gr, gd = oracle.loss(rays, rgb, depth, tg, opts)
        h = 1e-7
        for r in range(n):
            f = 0 if r < 8 else 1
            for ch in range(3):
                rp, rm = rgb.copy(), rgb.copy()
                rp[r, ch] += h
                rm[r, ch] -= h
                fd = (oracle.loss(rays, rp, depth, tg, opts)[0][f]
                      - oracle.loss(rays, rm, depth, tg, opts)[0][f]) / (2 * h)
                assert gr[r, ch] == pytest.approx(fd, abs=1e-7)
            dp, dm = depth.copy(), depth.copy()
            dp[r] += h
            dm[r] -= h
            fd = (oracle.loss(rays, rgb, dp, tg, opts)[0][f]
                  - oracle.loss(rays, rgb, dm, tg, opts)[0][f]) / (2 * h)
            assert gd[r] == pytest.approx(fd, abs=1e-7)
        for r in (1, 3, 9, 12):
            assert gd[r] == 0.0 and np.all(gr[r] == 0.0)


# ------------------------------------------------ grid backward (Eq. 6-10)

def _tiny_workload(seed, sh_degree0=False, act=synth.COLOR_SIGMOID, n_pix=24, R=7,
                   occupancy=1.0, depth_loss=synth.DEPTH_L2):
    rng = np.random.default_rng(seed)
    g = synth.random_tiny_grid(rng, R=R, margin=2, sh_degree0=sh_degree0, occupancy=occupancy)
    eye = rng.normal(size=3)
    eye = 2.2 * eye / np.linalg.norm(eye)
    c2w = synth.look_at(eye, rng.normal(size=3) * 0.05)
    intr = np.array([12.0, 12.0, 8.0, 8.0])
    pix = np.stack([rng.integers(3, 13, n_pix), rng.integers(3, 13, n_pix)], 1).astype(np.int32)
    rays = synth.Rays(c2w[None], intr[None], np.array([0, n_pix], np.int32), pix)
    opts = synth.Opts(step_vox=0.5, max_samples=100_000, t_near=0.0, t_stop=0.0,
                      color_act=act, depth_loss=depth_loss)
    g_rgb = rng.normal(size=(n_pix, 3))
    g_depth = rng.normal(size=n_pix)
    return g, rays, opts, g_rgb, g_depth


def _objective(g, rays, opts, g_rgb, g_depth):
    rgb, depth, _, _ = oracle.render(g, rays, opts)
    return float((g_rgb * rgb).sum() + (g_depth * depth).sum())


@pytest.mark.parametrize("act", [synth.COLOR_SIGMOID, synth.COLOR_IDENTITY])
def test_grid_backward_matches_finite_differences(act):
    g, rays, opts, g_rgb, g_depth = _tiny_workload(10 + act, act=act)
    gd, _ = oracle.backward(g, rays, opts, g_rgb, g_depth, True, False)
    rng = np.random.default_rng(11)
    hit = np.flatnonzero(np.abs(gd).sum(1) > 0)
    assert hit.size > 5
    checked = 0
    for v in rng.choice(hit, size=min(6, hit.size), replace=False):
        for m in [0, 1, 5, 13, 27]:
            base = g.data[v, m]
            h = np.float32(2.0 ** -10)
            gp = dataclasses.replace(g, data=g.data.copy())
            gm = dataclasses.replace(g, data=g.data.copy())
            gp.data[v, m] = base + h
            gm.data[v, m] = base - h
            hh = (np.float64(gp.data[v, m]) - np.float64(gm.data[v, m])) / 2
            fd = (_objective(gp, rays, opts, g_rgb, g_depth)
                  - _objective(gm, rays, opts, g_rgb, g_depth)) / (2 * hh)
            assert gd[v, m] == pytest.approx(fd, rel=2e-5, abs=1e-9), (v, m)
            checked += 1
    assert checked >= 25


def test_grid_backward_negative_density_gets_no_density_gradient():
    g, rays, opts, g_rgb, g_depth = _tiny_workload(20)
    g.data[:, 0] = -np.abs(g.data[:, 0])
    gd, _ = oracle.backward(g, rays, opts, g_rgb, g_depth, True, False)
    assert np.all(gd[:, 0] == 0.0)
    rgb, _, _, _ = oracle.render(g, rays, opts)
    assert np.all(rgb == 0.0)


def test_eq9_prefix_form_matches_bruteforce_per_sample():
    """Eq. 9/10 against the O(N^2) derivative of Eq. 1/3 for one ray."""
    g, rays, opts, _, _ = _tiny_workload(21, act=synth.COLOR_IDENTITY)
    o, d, s = oracle.ray(rays.c2w[0], rays.intr[0], 8, 8)
    tr = oracle.trace(g, o, d, opts)
    n, delta = tr["n"], opts.step_vox
    sig = np.maximum(tr["sigma_raw"], 0)
    assert n > 4
    # brute force: differentiate C = sum_i T_i a_i c_i term by term
    for k in range(n):
        dC = tr["T"][k] * np.exp(-sig[k] * delta) * delta * tr["c"][k]
        dD = tr["T"][k] * np.exp(-sig[k] * delta) * delta * tr["t"][k]
        for i in range(k + 1, n):
            dC = dC - delta * tr["w"][i] * tr["c"][i]
            dD = dD - delta * tr["w"][i] * tr["t"][i]
        # the paper's prefix form
        pre_c = (tr["w"][:k + 1, None] * tr["c"][:k + 1]).sum(0)
        pre_d = (tr["w"][:k + 1] * tr["t"][:k + 1]).sum()
        eq9 = delta * (tr["c"][k] * tr["T"][k + 1] - tr["rgb"] + pre_c)
        eq10 = delta * (tr["t"][k] * tr["T"][k + 1] - tr["D"] + pre_d)
        np.testing.assert_allclose(eq9, dC, atol=1e-13)
        assert eq10 == pytest.approx(dD, abs=1e-12)


# ------------------------------------------------ pose backward (Eq. 12-14)

def _pose_objective(g, rays, opts, g_rgb, g_depth, xi):
    c2w = np.stack([oracle.apply_left(xi, rays.c2w[f]) for f in range(rays.n_frames)])
    r2 = dataclasses.replace(rays, c2w=c2w)
    return _objective(g, r2, opts, g_rgb, g_depth)


@pytest.mark.parametrize("viewdir", [False, True])
def test_pose_backward_matches_finite_differences(viewdir):
    # position-only chain (the paper's Eq. 12) is exact when colour does not depend
    # on the view direction, i.e. on SH-degree-0 grids; the flagged mode on any grid
    g, rays, opts, g_rgb, g_depth = _tiny_workload(30 + viewdir, sh_degree0=not viewdir)
    flags = synth.FLAG_POSE_VIEWDIR if viewdir else 0
    _, gp = oracle.backward(g, rays, opts, g_rgb, g_depth, False, True, flags=flags)
    h = 1e-6
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        fd = (_pose_objective(g, rays, opts, g_rgb, g_depth, e)
              - _pose_objective(g, rays, opts, g_rgb, g_depth, -e)) / (2 * h)
        assert gp[0, j] == pytest.approx(fd, rel=1e-5, abs=1e-7), j


def test_pose_default_differs_from_exact_on_view_dependent_grid():
    g, rays, opts, g_rgb, g_depth = _tiny_workload(33, sh_degree0=False)
    _, gp0 = oracle.backward(g, rays, opts, g_rgb, g_depth, False, True, flags=0)
    _, gp1 = oracle.backward(g, rays, opts, g_rgb, g_depth, False, True,
                             flags=synth.FLAG_POSE_VIEWDIR)
    np.testing.assert_array_equal(gp0[0, :3], gp1[0, :3])      # translation unaffected
    assert np.abs(gp0[0, 3:] - gp1[0, 3:]).max() > 1e-6


def test_pose_multi_frame_segments_and_empty_frame():
    g, rays, opts, g_rgb, g_depth = _tiny_workload(34, sh_degree0=True, n_pix=30)
    c2w2 = np.stack([rays.c2w[0], rays.c2w[0], oracle.apply_left(
        np.array([0.01, 0, 0.02, 0.0, 0.03, 0.0]), rays.c2w[0])])
    rays3 = synth.Rays(c2w2, np.repeat(rays.intr, 3, 0), np.array([0, 10, 10, 30], np.int32),
                       rays.pix)
    _, gp = oracle.backward(g, rays3, opts, g_rgb, g_depth, False, True)
    assert np.all(gp[1] == 0.0)
    # frame 0 equals the single-frame gradient of its own rays
    one = synth.Rays(rays.c2w, rays.intr, np.array([0, 10], np.int32), rays.pix[:10])
    _, g0 = oracle.backward(g, one, opts, g_rgb[:10], g_depth[:10], False, True)
    np.testing.assert_allclose(gp[0], g0[0], rtol=1e-12, atol=1e-15)


def test_pose_zero_gradient_at_true_pose():
    """Targets rendered at the true pose: an L2 loss is stationary there."""
    g, rays, opts, _, _ = _tiny_workload(35, sh_degree0=True, n_pix=40)
    rgb, depth, _, _ = oracle.render(g, rays, opts)
    tg = synth.Targets(rgb.astype(np.float32), depth.astype(np.float32),
                       np.array([1.0 / 40], np.float32))
    # float32 targets leave a tiny residual; the gradient scales with it
    L, g_rgb, g_depth = oracle.loss(rays, rgb, depth, tg, opts)
    _, gp = oracle.backward(g, rays, opts, g_rgb, g_depth, False, True)
    assert np.abs(gp).max() < 1e-6


# ---------------------------------------------------------- TV regulariser

def test_tv_ramp_closed_form():
    R, a, eps = 6, 0.3, 1e-9
    P = lattice(R)
    vals = np.repeat((a * P[:, 0])[:, None], 28, 1)
    g = dense_grid(R, vals)
    val, grad = oracle.tv(g, 0.7, 0.2, eps)
    per = np.sqrt(np.float32(a) ** 2 + eps)
    assert val == pytest.approx((R - 1) ** 3 * (0.7 + 27 * 0.2) * per, rel=1e-6)
    inner = (P[:, 0] >= 1) & (P[:, 0] < R - 1) & (P[:, 1] < R - 1) & (P[:, 2] < R - 1)
    assert np.abs(grad[inner]).max() < 1e-6


def test_tv_gradient_fd_sparse():
    rng = np.random.default_rng(40)
    R = 5
    mask = rng.random(R ** 3) < 0.7
    g = synth.grid_from_mask((R, R, R), (0, 0, 0), 1.0, mask,
                             rng.normal(size=int(mask.sum())).astype(np.float32), rng)
    val, grad = oracle.tv(g, 0.9, 0.4, 1e-3)
    for v in rng.choice(g.n_alloc, 10, replace=False):
        for m in (0, 4, 27):
            h = np.float32(2.0 ** -12)
            gp = dataclasses.replace(g, data=g.data.copy())
            gm = dataclasses.replace(g, data=g.data.copy())
            gp.data[v, m] += h
            gm.data[v, m] -= h
            hh = (np.float64(gp.data[v, m]) - np.float64(gm.data[v, m])) / 2
            fd = (oracle.tv(gp, 0.9, 0.4, 1e-3, False)[0] - oracle.tv(gm, 0.9, 0.4, 1e-3, False)[0]) / (2 * hh)
            assert grad[v, m] == pytest.approx(fd, rel=1e-4, abs=1e-6)


# ------------------------------------------------- tracking update (Adam)

def test_se3_exp_matches_matrix_exponential():
    import scipy.linalg
    rng = np.random.default_rng(50)
    for _ in range(5):
        xi = rng.normal(size=6) * 0.4
        M = np.zeros((4, 4))
        M[:3, :3] = oracle.hat(xi[3:])
        M[:3, 3] = xi[:3]
        np.testing.assert_allclose(oracle.se3_exp(xi), scipy.linalg.expm(M), atol=1e-12)


def test_adam_step_matches_torch():
    import torch
    rng = np.random.default_rng(51)
    F = 3
    grads = [rng.normal(size=(F, 6)) for _ in range(4)]
    p = torch.zeros(F, 6, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    c2w = np.stack([np.eye(4)[:3]] * F)
    m = np.zeros((F, 6))
    v = np.zeros((F, 6))
    for it, gr in enumerate(grads, 1):
        before = p.detach().clone().numpy()
        opt.zero_grad()
        p.grad = torch.from_numpy(gr.copy())
        opt.step()
        step_torch = p.detach().numpy() - before
        new, m, v = oracle.adam_pose_step(c2w, gr, m, v, it, 1e-3)
        expect = np.stack([oracle.apply_left(step_torch[f], c2w[f]) for f in range(F)])
        np.testing.assert_allclose(new, expect, atol=1e-14)
        c2w = new


def test_rmsprop_dense_matches_torch():
    """Every record touched: the sparse step is plain RMSProp (torch's
    non-centred form, two parameter groups for the density and SH learning
    rates), over several steps."""
    import torch
    rng = np.random.default_rng(52)
    n = 5
    x0 = rng.normal(size=(n, oracle.NREC))
    dens = torch.tensor(x0[:, :1].copy(), requires_grad=True)
    sh = torch.tensor(x0[:, 1:].copy(), requires_grad=True)
    opt = torch.optim.RMSprop([{"params": [dens], "lr": 0.3}, {"params": [sh], "lr": 0.02}],
                              alpha=0.95, eps=1e-8)
    data, state = x0.copy(), np.zeros_like(x0)
    for _ in range(4):
        g = rng.normal(size=(n, oracle.NREC))
        opt.zero_grad()
        dens.grad = torch.from_numpy(g[:, :1].copy())
        sh.grad = torch.from_numpy(g[:, 1:].copy())
        opt.step()
        data, state = oracle.rmsprop_grid(data, g, state, 0.3, 0.02, 0.95, 1e-8)
        ref = np.concatenate([dens.detach().numpy(), sh.detach().numpy()], axis=1)
        np.testing.assert_allclose(data, ref, rtol=0, atol=1e-13)


def test_rmsprop_sparse_rule():
    """Untouched records keep value and running average (dense RMSProp would
    decay the average); a record with one non-zero entry is touched as a
    whole: its other entries keep their values but their averages decay."""
    rng = np.random.default_rng(53)
    n = 4
    data = rng.normal(size=(n, oracle.NREC))
    state = rng.uniform(0.1, 1.0, size=(n, oracle.NREC))
    g = np.zeros((n, oracle.NREC))
    g[1] = rng.normal(size=oracle.NREC)
    g[3, 7] = 0.5
    new, st = oracle.rmsprop_grid(data, g, state, 0.1, 0.01, 0.9, 1e-8)
    for r in (0, 2):
        assert np.array_equal(new[r], data[r]) and np.array_equal(st[r], state[r])
    others = np.arange(oracle.NREC) != 7
    assert np.array_equal(new[3, others], data[3, others])
    np.testing.assert_allclose(st[3, others], 0.9 * state[3, others], rtol=1e-15)
    v = 0.9 * state[3, 7] + 0.1 * 0.25
    np.testing.assert_allclose(new[3, 7], data[3, 7] - 0.01 * 0.5 / (np.sqrt(v) + 1e-8), rtol=1e-14)
    np.testing.assert_allclose(st[1], 0.9 * state[1] + 0.1 * g[1] ** 2, rtol=1e-15)


# ---------------------------------------------------------- Gauss-Newton tracking

@pytest.mark.parametrize("viewdir", [False, True])
def test_pose_jacobian_matches_finite_differences(viewdir):
    """Every row of every ray's Jacobian against central differences of that
    output under left se(3) perturbations of the camera (position-only chain
    on an SH-degree-0 grid, the exact chain on a view-dependent one)."""
    g, rays, opts, _, _ = _tiny_workload(80 + viewdir, sh_degree0=not viewdir)
    flags = synth.FLAG_POSE_VIEWDIR if viewdir else 0
    J = oracle.pose_jacobian(g, rays, opts, flags=flags)
    h = 1e-6
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        outs = []
        for sgn in (1.0, -1.0):
            c2w = np.stack([oracle.apply_left(sgn * e, rays.c2w[0])])
            rgb, depth, _, _ = oracle.render(g, dataclasses.replace(rays, c2w=c2w), opts)
            outs.append(np.concatenate([rgb, depth[:, None]], 1))
        fd = (outs[0] - outs[1]) / (2 * h)
        np.testing.assert_allclose(J[:, :, j], fd, rtol=1e-5, atol=1e-6)


def test_gn_gradient_is_half_the_squared_loss_pose_gradient():
    """J^T W e summed per frame is half the pose gradient of the squared loss
    (Eq. 4, 5, 11 with the squared depth norm), computed by the backward."""
    g, rays, opts, _, _ = _tiny_workload(82, sh_degree0=True, n_pix=40)
    rng = np.random.default_rng(83)
    rgb, depth, _, _ = oracle.render(g, rays, opts)
    td = (depth + rng.normal(0, 0.05, depth.shape)).astype(np.float32)
    td[:3] = np.nan
    tg = synth.Targets((rgb + rng.normal(0, 0.05, rgb.shape)).astype(np.float32), td,
                       np.array([1.0 / 37], np.float32))
    opts2 = dataclasses.replace(opts, lambda_depth=0.5)
    H, gvec, E = oracle.gn_system(g, rays, tg, opts2)
    ref = oracle.fused(g, rays, tg, opts2, want_grid=False, want_pose=True)
    np.testing.assert_allclose(gvec[0], 0.5 * ref["grad_pose"][0], rtol=1e-9, atol=1e-12)
    assert E[0] == pytest.approx(ref["loss"][0], rel=1e-12)
    assert np.allclose(H[0], H[0].T) and np.linalg.eigvalsh(H[0]).min() > -1e-12


def test_gn_steps_recover_the_pose():
    """Targets rendered at a true pose, start perturbed (2 voxels, 2 degrees):
    damped Gauss-Newton steps bring the pose back and the error down to the
    float32 rounding of the targets (superlinear once close: a zero-residual
    problem)."""
    g, rays, opts, _, _ = _tiny_workload(84, sh_degree0=True, n_pix=60)
    rgb, depth, _, _ = oracle.render(g, rays, opts)
    tg = synth.Targets(rgb.astype(np.float32), depth.astype(np.float32),
                       np.array([1.0 / 60], np.float32))
    true = rays.c2w.astype(np.float64)
    start = np.stack([synth.perturb_pose(true[0], np.random.default_rng(85),
                                         2 * float(g.voxel_size), np.deg2rad(2.0))])
    c2w, errs = start, []
    for _ in range(8):
        r = dataclasses.replace(rays, c2w=c2w)
        H, gvec, E = oracle.gn_system(g, r, tg, opts)
        errs.append(E[0])
        c2w = oracle.gn_pose_step(c2w, H, gvec, 1e-9)
    assert all(b < a for a, b in zip(errs[:5], errs[1:6]))
    assert errs[-1] < 1e-12 * errs[0]
    np.testing.assert_allclose(c2w, true, atol=1e-6)


# ------------------------------------------- dynamic grid (Sec. 5, peak 512^3)

def _fine_bruteforce(g):
    """Allocation mask and records of the doubled lattice by brute force:
    a fine vertex is allocated when some coarse cell whose closed box holds
    it has an allocated corner; its record is the separable midpoint average
    of the coarse records along each odd axis (empty corners read 0)."""
    R = g.reso[0]
    link = g.link.reshape(R, R, R)
    Rf = 2 * R - 1
    mask = np.zeros((Rf, Rf, Rf), bool)
    vals = np.zeros((Rf, Rf, Rf, oracle.NREC))

    def rec(x, y, z):
        i = link[x, y, z]
        return np.zeros(oracle.NREC) if i < 0 else g.data[i].astype(np.float64)

    for fx in range(Rf):
        for fy in range(Rf):
            for fz in range(Rf):
                p = np.array([fx, fy, fz]) / 2.0
                for cx in range(R - 1):
                    for cy in range(R - 1):
                        for cz in range(R - 1):
                            c = np.array([cx, cy, cz])
                            if np.all(p >= c) and np.all(p <= c + 1) and \
                                    (link[cx:cx + 2, cy:cy + 2, cz:cz + 2] >= 0).any():
                                mask[fx, fy, fz] = True
                # midpoint averages: axis coordinate 2a -> a, 2a+1 -> {a, a+1}
                sets = [[f // 2] if f % 2 == 0 else [f // 2, f // 2 + 1] for f in (fx, fy, fz)]
                acc = np.zeros(oracle.NREC)
                for x in sets[0]:
                    for y in sets[1]:
                        for z in sets[2]:
                            acc += rec(x, y, z)
                vals[fx, fy, fz] = acc / (len(sets[0]) * len(sets[1]) * len(sets[2]))
    vals[..., 0] *= 0.5
    return mask.ravel(), vals.reshape(-1, oracle.NREC)


def test_upsample_matches_bruteforce_allocation_and_midpoint_records():
    rng = np.random.default_rng(61)
    g = synth.random_tiny_grid(rng, R=5, margin=1, occupancy=0.4)
    g.link[0] = g.data.shape[0] - 1          # a corner vertex too (clipped cells)
    fine = oracle.grid_upsample(g)
    assert fine.reso == (9, 9, 9) and fine.voxel_size == np.float32(g.voxel_size / 2)
    np.testing.assert_array_equal(fine.aabb_min, g.aabb_min)
    mask, vals = _fine_bruteforce(g)
    np.testing.assert_array_equal(fine.link >= 0, mask)
    idx = np.flatnonzero(mask)
    np.testing.assert_array_equal(fine.link[idx], np.arange(idx.size))   # lattice order
    np.testing.assert_allclose(fine.data, vals[idx], rtol=1e-7, atol=1e-7)


def test_upsample_keeps_the_interpolated_field():
    """Trilinear fields restrict exactly to the eight sub-cells of a cell, so
    the fine map interpolates to the coarse field (density halved: it is per
    voxel) at every point, not only at vertices."""
    rng = np.random.default_rng(62)
    g = synth.random_tiny_grid(rng, R=7, margin=1, occupancy=0.5)
    fine = oracle.grid_upsample(g)
    scale = np.abs(g.data).max()
    for q in rng.uniform(0.0, 6.0, size=(60, 3)):
        vc, _ = oracle.interp(g, q, want_grad=False)
        vf, _ = oracle.interp(fine, 2.0 * q, want_grad=False)
        vf[0] *= 2.0
        np.testing.assert_allclose(vf, vc, rtol=0, atol=2e-7 * scale)


@pytest.mark.parametrize("act", [synth.COLOR_SIGMOID, synth.COLOR_IDENTITY])
def test_upsample_render_at_half_step_is_unchanged(act):
    """Rendering the doubled map with twice the step in voxel units samples the
    same world points with the same optical depth per sample (Eq. 1-3)."""
    g, rays, opts, _, _ = _tiny_workload(63 + act, act=act, occupancy=0.6)
    fine = oracle.grid_upsample(g)
    rgb_c, dep_c, n_c, _ = oracle.render(g, rays, opts)
    rgb_f, dep_f, _, _ = oracle.render(fine, rays, dataclasses.replace(opts, step_vox=2 * opts.step_vox))
    assert (n_c > 0).sum() > 10
    np.testing.assert_allclose(rgb_f, rgb_c, rtol=0, atol=2e-6)
    np.testing.assert_allclose(dep_f, dep_c, rtol=0, atol=2e-6)


def test_prune_drops_low_density_records_in_order():
    rng = np.random.default_rng(64)
    g = synth.random_tiny_grid(rng, R=7, margin=1, occupancy=0.7)
    tau = np.float32(np.median(g.data[:, 0]))
    p = oracle.grid_prune(g, tau)
    keep = g.data[:, 0] > tau
    assert p.n_alloc == int(keep.sum()) and 0 < p.n_alloc < g.n_alloc
    for v in range(g.link.size):
        old = g.link[v]
        if old < 0 or not keep[old]:
            assert p.link[v] == -1
        else:
            assert np.array_equal(p.data[p.link[v]], g.data[old])
    live = p.link[p.link >= 0]
    assert np.array_equal(np.sort(live), np.arange(p.n_alloc))
    assert np.all(np.diff(live) > 0)                        # order kept
    same = oracle.grid_prune(g, np.float32(g.data[:, 0].min()) - 1)
    assert np.array_equal(same.link, g.link) and np.array_equal(same.data, g.data)


def test_prune_of_zero_records_leaves_renders_unchanged():
    """An all-zero record reads the same as an empty vertex."""
    g, rays, opts, _, _ = _tiny_workload(65, occupancy=0.9)
    rng = np.random.default_rng(66)
    zero = rng.random(g.n_alloc) < 0.3
    g.data[zero] = 0.0
    g.data[~zero, 0] = np.abs(g.data[~zero, 0]) + 0.01
    p = oracle.grid_prune(g, 0.0)
    assert p.n_alloc == int((~zero).sum())
    rgb0, dep0, _, _ = oracle.render(g, rays, opts)
    rgb1, dep1, _, _ = oracle.render(p, rays, opts)
    np.testing.assert_allclose(rgb1, rgb0, rtol=0, atol=1e-13)
    np.testing.assert_allclose(dep1, dep0, rtol=0, atol=1e-13)


def test_dynamic_grid_edits_of_an_empty_map():
    rng = np.random.default_rng(67)
    g = synth.grid_from_mask((4, 5, 6), (0.0, 0.0, 0.0), 0.5, np.zeros(120, bool),
                             np.zeros(0, np.float32), rng)
    p = oracle.grid_prune(g, 0.0)
    assert p.n_alloc == 0 and np.all(p.link == -1)
    f = oracle.grid_upsample(g)
    assert f.reso == (7, 9, 11) and f.n_alloc == 0 and np.all(f.link == -1)
