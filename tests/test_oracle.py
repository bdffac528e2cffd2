"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

None of these compare the oracle with itself: each checks a closed form, an
invariant, an independent library routine (SciPy's spherical harmonics), an
independent NumPy implementation of the per-pixel definition, or finite
differences.  Equation numbers refer to GSFusion (arXiv 2408.12677).
"""
import math

import numpy as np
import pytest

import oracle
import scenes
from oracle import brute

I3 = np.eye(3, dtype=np.float32)
Z3 = np.zeros(3, np.float32)


def cam(W, H, f, cx=None, cy=None, R=I3, t=Z3):
    return scenes.Camera(W, H, float(f), float(f), float(W / 2 if cx is None else cx),
                         float(H / 2 if cy is None else cy), np.asarray(R, np.float32), np.asarray(t, np.float32))


def gaussians(means, scales, quats=None, opac=None, rgb=None, sh=None, deg=0):
    n = len(means)
    means = np.asarray(means, np.float32).reshape(n, 3)
    scales = np.asarray(scales, np.float32).reshape(n, 3)
    quats = np.tile([1, 0, 0, 0], (n, 1)).astype(np.float32) if quats is None else np.asarray(quats, np.float32)
    opac = np.full(n, 0.5, np.float32) if opac is None else np.asarray(opac, np.float32)
    if sh is None:
        rgb = np.full((n, 3), 0.5) if rgb is None else np.asarray(rgb, np.float64)
        sh = scenes.dc_from_rgb(rgb).reshape(n, 1, 3).astype(np.float32)
    return [means, scales, quats, opac, np.asarray(sh, np.float32)]


def rot_z(theta):
    return [math.cos(theta / 2), 0.0, 0.0, math.sin(theta / 2)]


# ---------------------------------------------------------------------------------------
# spherical harmonics (colour model, Sec. III-A-2)
# ---------------------------------------------------------------------------------------

def test_sh_matches_scipy_definition():
    rng = np.random.default_rng(1)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    np.testing.assert_allclose(oracle.sh_eval(3, d), brute.real_sh(3, d), atol=1e-13)


def test_sh_orthonormal_by_quadrature():
    # product Gauss-Legendre (in cos theta) x uniform phi is exact for degree <= 6 products
    xg, wg = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    Y = oracle.sh_eval(3, dirs)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_addition_theorem_and_constant():
    rng = np.random.default_rng(2)
    d = rng.standard_normal((100, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = oracle.sh_eval(3, d)
    np.testing.assert_allclose(Y[:, 0], 1 / (2 * math.sqrt(math.pi)), rtol=1e-15)
    for l in range(4):
        s = (Y[:, l * l:(l + 1) ** 2] ** 2).sum(1)
        np.testing.assert_allclose(s, (2 * l + 1) / (4 * math.pi), rtol=1e-12)
    # Condon-Shortley phase: Y_1^1 = -sqrt(3/4pi) x, Y_1^-1 = -sqrt(3/4pi) y, Y_1^0 = +sqrt(3/4pi) z
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(Y[:, 1:4], np.stack([-c1 * d[:, 1], c1 * d[:, 2], -c1 * d[:, 0]], 1), atol=1e-14)


def test_sh_gradient_is_surface_gradient():
    rng = np.random.default_rng(3)
    d = rng.standard_normal((20, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    _, dY = oracle.sh_eval(3, d, grad=True)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        dp, dm = d + e, d - e
        fd = (oracle.sh_eval(3, dp / np.linalg.norm(dp, axis=1, keepdims=True)) -
              oracle.sh_eval(3, dm / np.linalg.norm(dm, axis=1, keepdims=True))) / (2 * h)
        # chain rule of normalisation: (I - v v^T) grad
        proj = dY[:, :, j] - d[:, None, j] * np.einsum("nki,ni->nk", dY, d)
        np.testing.assert_allclose(fd, proj, atol=1e-7)


# ---------------------------------------------------------------------------------------
# projection (Eq. 2, 4, 5)
# ---------------------------------------------------------------------------------------

def test_projection_on_axis_closed_form():
    f, z = 100.0, 2.0
    sx, sy, sz = 0.05, 0.07, 0.01
    c = cam(64, 48, f)
    p = gaussians([[0, 0, z]], [[sx, sy, sz]])
    o = oracle.Oracle(p, 0, [c], oracle.Settings(mu_fp32=False))
    r = o.records()
    assert r["visible"][0]
    np.testing.assert_array_equal(r["mu"][0], [32.0, 24.0])
    f32 = lambda v: float(np.float32(v))     # binary32 inputs promoted exactly
    cov = np.array([[(f * f32(sx) / z) ** 2 + f32(0.3), 0],
                    [0, (f * f32(sy) / z) ** 2 + f32(0.3)]])
    np.testing.assert_allclose(r["conic"][0], [1 / cov[0, 0], 0.0, 1 / cov[1, 1]], rtol=1e-12, atol=1e-15)


def test_projection_isotropic_ignores_rotation():
    c = cam(48, 40, 80.0)
    base = gaussians([[0.1, -0.05, 2.0]], [[0.04, 0.04, 0.04]], quats=[[1, 0, 0, 0]], opac=[0.8], rgb=[[0.2, 0.6, 0.9]])
    rot = [a.copy() for a in base]
    rot[2] = np.array([[0.3, -0.5, 0.7, 0.2]], np.float32)
    s = oracle.Settings(mu_fp32=False)
    a = oracle.Oracle(base, 0, [c], s).forward()[0]
    b = oracle.Oracle(rot, 0, [c], s).forward()[0]
    np.testing.assert_allclose(a["color"], b["color"], atol=1e-13)
    g = oracle.Oracle(rot, 0, [c], s).backward([np.ones((3, 40, 48))], [np.ones((40, 48))], None)
    assert np.abs(g["quats"]).max() < 1e-9 * max(1.0, np.abs(g["means"]).max())
    assert np.abs(g["means"]).max() > 1e-3


def test_view_frustum_cull_with_guard_band():
    # only Gaussians lying in the view frustum are rendered (Sec. III-B-3): the centre must
    # project inside the image widened by guard x (W, H) per side, in front of znear
    W, H, f, z = 64, 48, 50.0, 2.0
    xs = [(W * 1.10 - W / 2) / f * z, (W * 1.20 - W / 2) / f * z, 0.0, 0.0]
    p = gaussians([[xs[0], 0, z], [xs[1], 0, z], [0, 0, 0.005], [0, 0, -1.0]], [[0.3, 0.3, 0.3]] * 4)
    r = oracle.Oracle(p, 0, [cam(W, H, f)], oracle.Settings(guard=0.15)).records()
    assert r["visible"].tolist() == [True, False, False, False]
    r = oracle.Oracle(p, 0, [cam(W, H, f)], oracle.Settings(guard=0.25)).records()
    assert r["visible"].tolist() == [True, True, False, False]


# ---------------------------------------------------------------------------------------
# compositing closed forms (Eq. 3, 11)
# ---------------------------------------------------------------------------------------

def _splat(W, H, f, z, s, theta, o):
    """Closed-form alpha of an on-axis Gaussian rotated by theta about the optical axis."""
    q32 = np.asarray(rot_z(theta), np.float32).astype(np.float64)
    theta = 2.0 * math.atan2(q32[3], q32[0])          # angle of the binary32 quaternion
    Rz = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    s32 = np.float32(s)
    cov = (f / z) ** 2 * Rz @ np.diag([float(s32[0]) ** 2, float(s32[1]) ** 2]) @ Rz.T + float(np.float32(0.3)) * np.eye(2)
    Q = np.linalg.inv(cov)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    dx, dy = xs - W / 2, ys - H / 2
    q = Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
    a = float(np.float32(o)) * np.exp(-0.5 * q)
    alpha = np.where(a < float(np.float32(1 / 255)), 0.0, np.minimum(a, float(np.float32(0.99))))
    return alpha, cov, np.exp(-0.5 * q)


def test_single_gaussian_closed_form():
    W, H, f, z = 64, 48, 100.0, 2.0
    s, th, o, rgb, bg = [0.05, 0.08, 0.01], 0.6, 0.7, [0.9, 0.3, 0.1], (0.2, 0.4, 0.6)
    p = gaussians([[0, 0, z]], [s], quats=[rot_z(th)], opac=[o], rgb=[rgb])
    out = oracle.Oracle(p, 0, [cam(W, H, f)], oracle.Settings(mu_fp32=False, bg=bg)).forward()[0]
    alpha, _, _ = _splat(W, H, f, z, s, th, o)
    c = np.float32(scenes.dc_from_rgb(rgb)).astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5
    np.testing.assert_allclose(out["alpha"], alpha, atol=1e-12)
    np.testing.assert_allclose(out["depth"], float(np.float32(z)) * alpha, atol=1e-12)
    exp_c = c[:, None, None] * alpha + np.asarray(bg, np.float64)[:, None, None] * (1 - alpha)
    np.testing.assert_allclose(out["color"], exp_c, atol=1e-12)


def test_opacity_clamp_and_skip_rule():
    W, H, f, z = 32, 32, 100.0, 2.0
    # o = 0.999 -> centre clamps to 0.99; faint tail below 1/255 is dropped entirely
    p = gaussians([[0, 0, z]], [[0.03, 0.03, 0.03]], opac=[0.999])
    out = oracle.Oracle(p, 0, [cam(W, H, f)], oracle.Settings(mu_fp32=False)).forward()[0]
    assert out["alpha"].max() == pytest.approx(float(np.float32(0.99)), abs=1e-15)
    nz = out["alpha"][out["alpha"] > 0]
    assert nz.min() >= float(np.float32(1 / 255))


def test_two_gaussians_closed_form():
    W, H, f = 48, 40, 90.0
    z1, z2 = 1.5, 3.0
    s1, s2 = [0.04, 0.06, 0.01], [0.09, 0.05, 0.02]
    o1, o2 = 0.6, 0.8
    c1, c2 = [0.1, 0.7, 0.3], [0.8, 0.2, 0.5]
    # list them back to front to check the depth sort
    p = gaussians([[0, 0, z2], [0, 0, z1]], [s2, s1], quats=[rot_z(1.0), rot_z(0.3)], opac=[o2, o1], rgb=[c2, c1])
    out = oracle.Oracle(p, 0, [cam(W, H, f)], oracle.Settings(mu_fp32=False, T_min=0.0)).forward()[0]
    a1, _, _ = _splat(W, H, f, float(np.float32(z1)), s1, 0.3, o1)
    a2, _, _ = _splat(W, H, f, float(np.float32(z2)), s2, 1.0, o2)
    col = lambda c: (np.float32(scenes.dc_from_rgb(c)).astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5)[:, None, None]
    C = col(c1) * a1 + col(c2) * a2 * (1 - a1)
    D = float(np.float32(z1)) * a1 + float(np.float32(z2)) * a2 * (1 - a1)
    np.testing.assert_allclose(out["color"], C, atol=1e-6)   # splats use the binary32 quaternion
    np.testing.assert_allclose(out["depth"], D, atol=1e-6)
    np.testing.assert_allclose(out["T_final"], (1 - a1) * (1 - a2), atol=1e-6)


def test_riemann_mass_pins_conic_scale_and_skip_rule():
    # sum_u alpha(u) -> 2 pi sqrt(det Sigma_hat) (o - 1/255) for a wide unclamped splat
    W, H, f, z, o = 96, 96, 100.0, 2.0, 0.6
    s, th = [0.05, 0.08, 0.01], 0.4
    p = gaussians([[0, 0, z]], [s], quats=[rot_z(th)], opac=[o])
    out = oracle.Oracle(p, 0, [cam(W, H, f)], oracle.Settings(mu_fp32=False)).forward()[0]
    _, cov, _ = _splat(W, H, f, z, s, th, o)
    mass = 2 * math.pi * math.sqrt(np.linalg.det(cov)) * (float(np.float32(o)) - float(np.float32(1 / 255)))
    assert out["alpha"].sum() == pytest.approx(mass, rel=1e-3)


def test_single_gaussian_opacity_gradient_closed_form():
    # d alpha / d o = G(u) where the splat is neither skipped nor clamped
    W, H, f, z = 40, 40, 100.0, 2.0
    s, th, o = [0.04, 0.06, 0.02], 0.2, 0.5
    p = gaussians([[0, 0, z]], [s], quats=[rot_z(th)], opac=[o])
    orc = oracle.Oracle(p, 0, [cam(W, H, f)], oracle.Settings(mu_fp32=False))
    alpha, _, G = _splat(W, H, f, z, s, th, o)
    gA = np.zeros((H, W))
    gA[20, 20] = 1.0
    gA[23, 18] = 1.0
    g = orc.backward(None, None, [gA])
    assert g["opacities"][0] == pytest.approx(G[20, 20] + G[23, 18], rel=1e-10)


# ---------------------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------------------

def test_transmittance_non_increasing_along_list():
    w = scenes.make_cfg1(n=300)
    g = w.gaussians
    c = cam(64, 48, 55.0)
    s = oracle.Settings(mu_fp32=False)
    z = np.asarray(g.means[:, 2])
    order = np.argsort(z, kind="stable")
    prev = np.ones((48, 64))
    for k in (10, 40, 80, 160, 300):
        sub = g.subset(np.sort(order[:k]))
        out = oracle.Oracle(sub.arrays(), 0, [c], s).forward()[0]
        assert np.all(out["T_final"] <= prev + 1e-15)
        prev = out["T_final"]
    out = oracle.Oracle(g.arrays(), 0, [c], s).forward()[0]
    assert np.all(out["alpha"] >= 0) and np.all(out["alpha"] < 1)
    cmax = (0.5 + g.sh[:, 0, :].astype(np.float64) / (2 * math.sqrt(math.pi))).max(0)   # per-channel max splat colour
    assert np.all(out["color"] <= cmax[:, None, None] * out["alpha"] + 1e-12)


def test_permutation_invariance():
    w = scenes.make_cfg1(n=200)
    g = w.gaussians
    c = cam(64, 48, 55.0)
    s = oracle.Settings()
    perm = np.random.default_rng(5).permutation(g.n)
    a = oracle.Oracle(g.arrays(), 0, [c], s)
    b = oracle.Oracle(g.subset(perm).arrays(), 0, [c], s)
    fa, fb = a.forward()[0], b.forward()[0]
    np.testing.assert_array_equal(fa["color"], fb["color"])
    gC = [np.random.default_rng(6).standard_normal((3, 48, 64))]
    ga, gb = a.backward(gC), b.backward(gC)
    np.testing.assert_array_equal(ga["means"][perm], gb["means"])
    np.testing.assert_array_equal(ga["sh"][perm], gb["sh"])


def test_shift_principal_point_by_one_tile():
    w = scenes.make_cfg1(n=300)
    g = w.gaussians
    s = oracle.Settings(mu_fp32=False)
    a = oracle.Oracle(g.arrays(), 0, [cam(96, 64, 60.0, cx=40.0, cy=32.0)], s).forward()[0]
    b = oracle.Oracle(g.arrays(), 0, [cam(96, 64, 60.0, cx=56.0, cy=32.0)], s).forward()[0]
    np.testing.assert_allclose(b["color"][:, :, 16:], a["color"][:, :, :80], atol=1e-12)


# ---------------------------------------------------------------------------------------
# brute force (no tiles) and literal Eq. 11
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("deg", [0, 3])
def test_tiles_equal_brute_force(deg):
    rng = np.random.default_rng(10 + deg)
    n = 150
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-0.8, 0.8, n), rng.uniform(1, 4, n)], 1)
    g = scenes.random_gaussians(rng, means * 0.5, deg)
    g.scales *= 3
    c = cam(40, 32, 30.0, cx=19.5, cy=16.25)
    out = oracle.Oracle(g.arrays(), deg, [c], oracle.Settings(mu_fp32=False, tile=8)).forward()[0]
    b = brute.render(g.arrays(), deg, c)
    for k in ("color", "depth", "alpha", "T_final"):
        np.testing.assert_allclose(out[k], b[k], atol=1e-12, err_msg=k)
    assert out["n_used"].sum() > 200


def test_literal_eq11_without_rules():
    rng = np.random.default_rng(12)
    n = 30
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.4, 0.4, n), rng.uniform(1, 3, n)], 1)
    g = scenes.random_gaussians(rng, means, 0)
    g.scales *= 4
    c = cam(24, 20, 25.0)
    s = oracle.Settings(mu_fp32=False, extent_k=1e4, alpha_min=0.0, alpha_max=1.0, T_min=0.0, tile=8)
    out = oracle.Oracle(g.arrays(), 0, [c], s).forward()[0]
    # Eq. 11 word for word, Gaussians sorted by depth
    pr = brute.project(g.arrays(), 0, c)
    order = np.argsort(pr["z"], kind="stable")
    ys, xs = np.mgrid[0:20, 0:24].astype(np.float64)
    I = np.zeros((3, 20, 24))
    for i, gi in enumerate(order):
        def Ghat(j):
            Q = pr["conic"][j]
            dx, dy = xs - pr["mu"][j, 0], ys - pr["mu"][j, 1]
            return np.exp(-0.5 * (Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy))
        prod = np.ones((20, 24))
        for gj in order[:i]:
            prod *= 1 - pr["opacity"][gj] * Ghat(gj)
        I += pr["color"][gi][:, None, None] * pr["opacity"][gi] * Ghat(gi) * prod
    np.testing.assert_allclose(out["color"], I, atol=1e-12)


# ---------------------------------------------------------------------------------------
# discrete stage: an independent float32 transcription of the documented op sequence
# ---------------------------------------------------------------------------------------

def discrete_stage_f32(p, s, q, c, k=3.33, lowpass=0.3, full=False, guard=0.15):
    f = np.float32
    p, s, q = (np.asarray(a, np.float32) for a in (p, s, q))
    W = np.asarray(c.R, np.float32).reshape(9)
    t = np.asarray(c.t, np.float32)
    tx = ((W[0] * p[:, 0] + W[1] * p[:, 1]) + W[2] * p[:, 2]) + t[0]
    ty = ((W[3] * p[:, 0] + W[4] * p[:, 1]) + W[5] * p[:, 2]) + t[1]
    tz = ((W[6] * p[:, 0] + W[7] * p[:, 1]) + W[8] * p[:, 2]) + t[2]
    nq = np.sqrt(((q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2]) + q[:, 3] * q[:, 3])
    w, x, y, z = (q[:, i] / nq for i in range(4))
    one, two = f(1), f(2)
    r = [one - two * (y * y + z * z), two * (x * y - w * z), two * (x * z + w * y),
         two * (x * y + w * z), one - two * (x * x + z * z), two * (y * z - w * x),
         two * (x * z - w * y), two * (y * z + w * x), one - two * (x * x + y * y)]
    m = [r[i * 3 + j] * s[:, j] for i in range(3) for j in range(3)]
    fx, fy = f(c.fx), f(c.fy)
    tz2 = tz * tz
    j00, j11 = fx / tz, fy / tz
    j02, j12 = -(fx * tx) / tz2, -(fy * ty) / tz2
    T = [j00 * W[cc] + j02 * W[6 + cc] for cc in range(3)] + [j11 * W[3 + cc] + j12 * W[6 + cc] for cc in range(3)]
    U = [((T[i * 3] * m[cc] + T[i * 3 + 1] * m[3 + cc]) + T[i * 3 + 2] * m[6 + cc]) for i in range(2) for cc in range(3)]
    lp = f(lowpass)
    a = ((U[0] * U[0] + U[1] * U[1]) + U[2] * U[2]) + lp
    b = (U[0] * U[3] + U[1] * U[4]) + U[2] * U[5]
    cc_ = ((U[3] * U[3] + U[4] * U[4]) + U[5] * U[5]) + lp
    det = a * cc_ - b * b
    mux = fx * (tx / tz) + f(c.cx)
    muy = fy * (ty / tz) + f(c.cy)
    gx, gy = f(guard) * f(c.width), f(guard) * f(c.height)
    infrustum = (mux >= -gx) & (mux <= f(c.width) + gx) & (muy >= -gy) & (muy <= f(c.height) + gy)
    kk = f(k)
    rx, ry = kk * np.sqrt(a), kk * np.sqrt(cc_)
    x0, x1 = np.ceil(mux - rx), np.floor(mux + rx)
    y0, y1 = np.ceil(muy - ry), np.floor(muy + ry)
    x0 = np.where(x0 < 0, f(0), x0)
    y0 = np.where(y0 < 0, f(0), y0)
    x1 = np.where(x1 > f(c.width - 1), f(c.width - 1), x1)
    y1 = np.where(y1 > f(c.height - 1), f(c.height - 1), y1)
    vis = (tz > f(c.znear)) & (nq > 0) & (det > 0) & infrustum & (x0 <= x1) & (y0 <= y1)
    if full:
        return vis, tz, np.stack([mux, muy], 1), np.stack([x0, x1, y0, y1], 1), a
    return vis, tz, np.stack([mux, muy], 1), np.stack([x0, x1, y0, y1], 1)


@pytest.mark.parametrize("posed", [False, True])
def test_discrete_stage_matches_float32_transcription(posed):
    w = scenes.make_cfg1(n=20000)
    g = w.gaussians
    c = w.cameras[0]
    if posed:   # a general rotation and translation so every product and sum matters
        R, t = scenes.look_at([0.3, -0.2, -0.5], [0.1, 0.05, 3.0], up=(0.1, -1, 0))
        c = scenes.Camera(c.width, c.height, c.fx, c.fy, 63.7, 47.9, R, t)
    with np.errstate(all="ignore"):
        vis, tz, mu, rect = discrete_stage_f32(g.means, g.scales, g.quats, c)
    r = oracle.Oracle(g.arrays(), 0, [c]).records()
    assert vis.sum() > 1000
    np.testing.assert_array_equal(r["visible"], vis)
    np.testing.assert_array_equal(r["z"][vis].view(np.uint32), tz[vis].view(np.uint32))
    np.testing.assert_array_equal(r["mu"][vis].view(np.uint32), mu[vis].view(np.uint32))
    np.testing.assert_array_equal(r["cov"][vis][:, 0].view(np.uint32), _cov_a(g, c)[vis].view(np.uint32))
    np.testing.assert_array_equal(r["rect"][vis], rect[vis].astype(np.int32))


def _cov_a(g, c):
    """First entry of the binary32 projected covariance, recomputed via the transcription."""
    with np.errstate(all="ignore"):
        return discrete_stage_f32(g.means, g.scales, g.quats, c, full=True)[4]


def test_keys_sorted_unique_and_ranges_partition():
    w = scenes.make_cfg1()
    g = w.gaussians
    c = w.cameras[0]
    o = oracle.Oracle(g.arrays(), 0, [c, c.crop(10, 8, 100, 70)], oracle.Settings(tile=16))
    keys, vals, ranges = o.keys()
    assert np.all(keys[1:] >= keys[:-1])
    r = o.records()
    tiles = keys >> np.uint64(32)
    pairs = set(zip(tiles.tolist(), vals.tolist()))
    assert len(pairs) == len(keys)                       # each (tile, Gaussian) once
    rect = r["rect"][r["visible"]]
    area = ((rect[:, 1] // 16 - rect[:, 0] // 16 + 1) * (rect[:, 3] // 16 - rect[:, 2] // 16 + 1)).sum()
    assert area == len(keys)                             # M = sum of tile-rect areas
    nz = ranges[ranges[:, 1] > ranges[:, 0]]
    assert nz[0, 0] == 0 and nz[-1, 1] == len(keys)
    assert np.all(nz[1:, 0] == nz[:-1, 1])               # ranges partition [0, M)
    for t in np.unique(tiles)[:20]:
        s, e = ranges[t]
        assert np.all(tiles[s:e] == t)
        z = (keys[s:e] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        v = vals[s:e]
        assert np.all((z[1:] > z[:-1]) | ((z[1:] == z[:-1]) & (v[1:] > v[:-1])))   # ties by index


# ---------------------------------------------------------------------------------------
# gradients: central finite differences in FP64
# ---------------------------------------------------------------------------------------

def _fd_scene(deg, seed):
    rng = np.random.default_rng(seed)
    n = 24
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.4, 0.4, n), rng.uniform(1.5, 3.0, n)], 1)
    g = scenes.random_gaussians(rng, means, deg)
    g.scales *= 3
    g.opacities[:] = np.float32(0.3 + 0.6 * rng.random(n))
    c = scenes.Camera(40, 32, 35.0, 35.0, 20.0, 16.0, *scenes.look_at([0.05, -0.02, -0.1], [0.0, 0.0, 2.0], up=(0, -1, 0)))
    return g, c


def _fd_check(g, c, deg, s, seed, trials=100):
    """Central differences (h = 1e-6, FP64) of <w, outputs> at random parameters against the
    analytic gradient; stencils that change a discrete decision (keys, order, contributors
    or the stop position) are left out.  Returns the checked (group, index) pairs."""
    rng = np.random.default_rng(seed + 100)
    H, W = c.height, c.width
    wC, wD, wA = rng.standard_normal((3, H, W)), rng.standard_normal((H, W)), rng.standard_normal((H, W))
    base = [np.asarray(a, np.float64).copy() for a in g.arrays()]
    orc = oracle.Oracle(base, deg, [c], s)
    ref_keys = orc.keys()
    ref_out = orc.forward()[0]
    an = orc.backward([wC], [wD], [wA])

    def f(params):
        o = oracle.Oracle(params, deg, [c], s)
        out = o.forward()[0]
        val = (wC * out["color"]).sum() + (wD * out["depth"]).sum() + (wA * out["alpha"]).sum()
        k = o.keys()
        same = (np.array_equal(k[0] >> np.uint64(32), ref_keys[0] >> np.uint64(32)) and np.array_equal(k[1], ref_keys[1])
                and np.array_equal(out["n_contrib"], ref_out["n_contrib"]) and np.array_equal(out["n_used"], ref_out["n_used"]))
        return val, same

    names = ["means", "scales", "quats", "opacities", "sh"]
    h = 1e-6
    checked = []
    for trial in range(trials):
        gi = trial % 5
        arr = base[gi]
        idx = tuple(rng.integers(0, d) for d in arr.shape)
        plus = [a.copy() for a in base]
        minus = [a.copy() for a in base]
        plus[gi][idx] += h
        minus[gi][idx] -= h
        fp, sp = f(plus)
        fm, sm = f(minus)
        if not (sp and sm):
            continue
        fd = (fp - fm) / (2 * h)
        a = an[names[gi]][idx]
        scale = max(abs(a), 1e-2 * np.abs(an[names[gi]]).max(), 1e-6)
        assert abs(fd - a) <= 1e-4 * scale, (names[gi], idx, fd, a)
        checked.append((gi, idx, a))
    return checked, ref_out


@pytest.mark.parametrize("norm", [False, True])
@pytest.mark.parametrize("deg,seed", [(0, 20), (3, 21)])
def test_backward_matches_central_differences(deg, seed, norm):
    g, c = _fd_scene(deg, seed)
    s = oracle.Settings(mu_fp32=False, tile=8, bg=(0.1, 0.2, 0.3), normalized_depth=norm)
    checked, _ = _fd_check(g, c, deg, s, seed)
    assert len(checked) >= 80


def test_loss_l1_gradient():
    rng = np.random.default_rng(30)
    C, D = rng.random((3, 8, 9)), rng.random((8, 9)) * 3
    tc, td = rng.random((3, 8, 9)), rng.random((8, 9)) * 3
    td[0, :4] = 0.0
    L, gC, gD = oracle.l1_loss(C, D, tc, td, 0.1)
    h = 1e-7
    for idx in [(0, 1, 2), (2, 7, 8)]:
        Cp = C.copy()
        Cp[idx] += h
        assert (oracle.l1_loss(Cp, D, tc, td)[0] - L) / h == pytest.approx(gC[idx], rel=1e-5)
    assert np.all(gD[0, :4] == 0)
    assert L == pytest.approx(np.abs(C - tc).mean() + 0.1 * np.abs(D - td)[td > 0].sum() / D.size)


# ---------------------------------------------------------------------------------------
# exact ellipse-tile culling (a variant of the tile lists: same images, fewer pairs)
# ---------------------------------------------------------------------------------------

def _thin_scene(seed, n=120, deg=0):
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-0.8, 0.8, n), rng.uniform(1, 4, n)], 1)
    g = scenes.random_gaussians(rng, means * 0.5, deg)
    g.scales *= 3
    g.scales[:, 0] *= 4                           # elongated splats, most of their rectangle empty
    return g


@pytest.mark.parametrize("tile", [8, 16])
def test_exact_tiles_equal_brute_force_and_the_rectangle_path(tile):
    g = _thin_scene(30 + tile)
    c = cam(56, 40, 30.0, cx=27.5, cy=19.75)
    box = oracle.Oracle(g.arrays(), 0, [c], oracle.Settings(mu_fp32=False, tile=tile))
    ex = oracle.Oracle(g.arrays(), 0, [c], oracle.Settings(mu_fp32=False, tile=tile, exact_tiles=True))
    ob, oe = box.forward()[0], ex.forward()[0]
    b = brute.render(g.arrays(), 0, c)
    for k in ("color", "depth", "alpha", "T_final"):
        np.testing.assert_allclose(oe[k], b[k], atol=1e-12, err_msg=k)
        np.testing.assert_array_equal(oe[k], ob[k], err_msg=k)      # same contributors, same order
    np.testing.assert_array_equal(oe["n_used"], ob["n_used"])
    kb, vb, _ = box.keys()
    ke, ve, _ = ex.keys()
    pb = set(zip((kb >> np.uint64(32)).tolist(), vb.tolist()))
    pe = set(zip((ke >> np.uint64(32)).tolist(), ve.tolist()))
    assert pe <= pb and len(pe) < 0.9 * len(pb)


def test_dropped_tiles_hold_no_pixel_of_the_ellipse():
    # every (tile, Gaussian) pair the exact lists drop has no pixel centre with
    # d^T Q d <= k^2 (FP64, conic from the binary32 covariance), so dropping it cannot
    # change any pixel; pairs kept beyond that are allowed (the band test is conservative)
    g = _thin_scene(41, n=80)
    c = cam(64, 48, 36.0, cx=31.5, cy=23.5)
    ts, k = 8, np.float64(np.float32(3.33))
    box = oracle.Oracle(g.arrays(), 0, [c], oracle.Settings(tile=ts))
    ex = oracle.Oracle(g.arrays(), 0, [c], oracle.Settings(tile=ts, exact_tiles=True))
    kb, vb, _ = box.keys()
    ke, ve, _ = ex.keys()
    dropped = set(zip((kb >> np.uint64(32)).tolist(), vb.tolist())) - set(zip((ke >> np.uint64(32)).tolist(), ve.tolist()))
    assert len(dropped) > 50
    r = box.records()
    tx_n = -(-64 // ts)
    for tile, gi in dropped:
        a, b_, cc = (float(x) for x in r["cov"][gi])
        det = a * cc - b_ * b_
        Q = np.array([[cc, -b_], [-b_, a]]) / det
        mx, my = (float(x) for x in r["mu"][gi])
        ty, tx = divmod(tile, tx_n)
        ys, xs = np.mgrid[ty * ts:min(ty * ts + ts, 48), tx * ts:min(tx * ts + ts, 64)]
        dx, dy = xs - mx, ys - my
        qv = Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
        assert qv.min() > k * k * (1 - 1e-5), (tile, gi, qv.min())


def test_normalized_depth_closed_forms():
    # one Gaussian alone on a pixel: D = z a, A = a, so D / A = z whatever its opacity;
    # two on the same line of sight: the alpha-weighted mean of their depths
    c = cam(16, 16, 20.0, cx=8.0, cy=8.0)    # pixel (8, 8) sits on both centres: G = 1
    g1 = gaussians([[0.0, 0.0, 2.0]], [[0.3, 0.3, 0.3]], opac=[0.37])
    o = oracle.Oracle(g1, 0, [c], oracle.Settings(normalized_depth=True)).forward()[0]
    hit = o["alpha"] > 0
    assert hit.sum() > 20
    np.testing.assert_allclose(o["depth"][hit], np.float64(np.float32(2.0)), rtol=1e-12)
    assert (o["depth"][~hit] == 0).all()
    g2 = gaussians([[0.0, 0.0, 2.0], [0.0, 0.0, 3.0]], [[0.3, 0.3, 0.3], [0.5, 0.5, 0.5]], opac=[0.4, 0.6])
    raw = oracle.Oracle(g2, 0, [c], oracle.Settings()).forward()[0]
    nrm = oracle.Oracle(g2, 0, [c], oracle.Settings(normalized_depth=True)).forward()[0]
    hit = raw["alpha"] > 0
    np.testing.assert_allclose(nrm["depth"][hit], raw["depth"][hit] / raw["alpha"][hit], rtol=1e-12)
    assert ((nrm["depth"][hit] > 2.0 - 1e-6) & (nrm["depth"][hit] < 3.0 + 1e-6)).all()
    centre = nrm["depth"][8, 8]
    a1 = 0.4
    a2 = 0.6
    assert centre == pytest.approx((2.0 * a1 + 3.0 * a2 * (1 - a1)) / (a1 + a2 * (1 - a1)), rel=1e-6)


# ---------------------------------------------------------------------------------------
# dense scenes where most pixels stop (T < T_min, the crossing Gaussian included)
# ---------------------------------------------------------------------------------------

T_MIN32 = float(np.float32(1e-4))


def _dense_scene(seed, n, deg):
    """n large, nearly opaque Gaussians (opacity 0.9-0.99) piled on a 32x24 image."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.4, 0.4, n), rng.uniform(1.5, 3.0, n)], 1)
    g = scenes.random_gaussians(rng, means, deg)
    g.scales = np.exp(rng.uniform(np.log(0.15), np.log(0.4), (n, 3))).astype(np.float32)
    g.opacities = rng.uniform(0.9, 0.99, n).astype(np.float32)
    return g, cam(32, 24, 30.0, cx=15.7, cy=11.4)


@pytest.mark.parametrize("deg,seed", [(0, 30), (3, 31)])
def test_dense_stopping_scene_equals_brute_force(deg, seed):
    g, c = _dense_scene(seed, 300, deg)
    orc = oracle.Oracle(g.arrays(), deg, [c], oracle.Settings(mu_fp32=False, tile=8))
    out = orc.forward()[0]
    b = brute.render(g.arrays(), deg, c)
    assert b["stopped"].mean() >= 0.5, b["stopped"].mean()
    np.testing.assert_array_equal(out["T_final"] < T_MIN32, b["stopped"])
    for k in ("color", "depth", "alpha", "T_final"):
        np.testing.assert_allclose(out[k], b[k], atol=1e-12, rtol=0, err_msg=k)
    # the same contributors, and the same Gaussian last (where a pixel stopped: the one
    # that took T below T_min)
    np.testing.assert_array_equal(out["n_used"], b["count"])
    _, vals, ranges = orc.keys()
    H, W = c.height, c.width
    tiles_x = (W + 7) // 8
    last = np.full((H, W), -1, np.int64)
    for y in range(H):
        for x in range(W):
            k = out["n_contrib"][y, x]
            if k > 0:
                last[y, x] = vals[ranges[(y // 8) * tiles_x + x // 8, 0] + k - 1] % g.n
    np.testing.assert_array_equal(last, b["last"])


@pytest.mark.parametrize("deg,seed", [(0, 40), (3, 41)])
def test_backward_matches_central_differences_where_pixels_stop(deg, seed):
    g, c = _dense_scene(seed, 120, deg)
    s = oracle.Settings(mu_fp32=False, tile=8, bg=(0.1, 0.2, 0.3))
    checked, out = _fd_check(g, c, deg, s, seed, trials=140)
    stopped = out["T_final"] < T_MIN32
    assert stopped.mean() >= 0.3, stopped.mean()
    assert len(checked) >= 80
    # the check reaches Gaussians whose reverse pass starts at a stopped pixel
    _, vals, ranges = oracle.Oracle(g.arrays(), deg, [c], s).keys()
    tiles_x = (c.width + 7) // 8
    crossing = set()
    for y, x in zip(*np.nonzero(stopped)):
        k = out["n_contrib"][y, x]
        crossing.add(int(vals[ranges[(y // 8) * tiles_x + x // 8, 0] + k - 1] % g.n))
    hit = [a for gi, idx, a in checked if idx[0] in crossing and a != 0.0]
    assert len(hit) >= 20, len(hit)


# ---------------------------------------------------------------------------------------
# several correct results: every outcome of a decision inside its margin is enumerated
# ---------------------------------------------------------------------------------------

A_MIN32 = float(np.float32(1 / 255))
A_MAX32 = float(np.float32(0.99))


def _stack(opac, rgb=None):
    """Four wide Gaussians on the optical axis at depths 1.5, 2, 2.5, 3 (front to back);
    at the principal point (12, 10) each splat value equals its opacity exactly."""
    n = len(opac)
    means = [[0.0, 0.0, 1.5 + 0.5 * i] for i in range(n)]
    scales = [[0.6 + 0.1 * i, 0.5, 0.4] for i in range(n)]
    rgb = rgb or [[0.9, 0.1, 0.2], [0.2, 0.8, 0.3], [0.1, 0.3, 0.9], [0.7, 0.6, 0.1]][:n]
    p = gaussians(means, scales, rgb=rgb)
    p[3] = np.asarray(opac, np.float64)   # opacities in binary64: the oracle takes them as given
    return [np.asarray(a, np.float64) for a in p]


def _run(p, gC=None):
    c = cam(24, 20, 40.0, cx=12.0, cy=10.0)
    s = oracle.Settings(mu_fp32=True, tile=8)
    orc = oracle.Oracle(p, 0, [c], s)
    out = orc.forward()[0]
    rng = np.random.default_rng(5)
    gC = rng.standard_normal((3, 20, 24)) if gC is None else gC
    gD = rng.standard_normal((20, 24))
    return orc, out, gC, gD


def _covers(out_ref, out_alt, bck_ref, bck_alt, slack_img=0.0, slack_grad=0.0):
    """The alternative outcome lies inside the reference's bounds (image and gradients)."""
    gpu_like = np.concatenate([out_alt["color"], out_alt["depth"][None], out_alt["alpha"][None]], 0)
    assert (gpu_like >= out_ref["lo"] - slack_img).all() and (gpu_like <= out_ref["hi"] + slack_img).all()
    biggest = 0.0
    for k in ("means", "scales", "quats", "opacities", "sh"):
        d = np.abs(bck_alt[k] - bck_ref[k])
        env = bck_ref["envelope"][k]
        assert (d <= env * (1 + 1e-9) + slack_grad + 1e-15).all(), (k, (d - env).max())
        biggest = max(biggest, d.max())
    # the change is real, and well above the slack the alternative's own input change needs
    assert biggest > 10.0 * slack_grad and biggest > 0.0
    assert not bck_ref["flagged"].any()


def test_envelope_covers_the_other_skip_decision():
    # splat 1 sits at alpha_min (1 + 3e-6) at the principal point: included there, but a
    # binary32 renderer may skip it; with alpha_min (1 - 1e-9) it is skipped
    o = [0.5, A_MIN32 * (1 + 3e-6), 0.6, 0.7]
    orc, out, gC, gD = _run(_stack(o))
    assert out["events"][10, 12] == 1 and out["ambiguous"].sum() == 1
    assert (out["hi"] - out["lo"]).max() > 1e-4          # the two outcomes differ visibly
    bref = orc.backward([gC], [gD])
    o_alt = list(o)
    o_alt[1] = A_MIN32 * (1 - 1e-9)
    orc2, out2, _, _ = _run(_stack(o_alt), gC)
    # the skipped splat contributes nowhere, so this is exactly the other outcome
    _covers(out, out2, bref, orc2.backward([gC], [gD]))


def test_envelope_covers_the_other_stop_decision():
    # T after splat 2 is T_min (1 + 5e-5): the pass goes on to splat 3, but it may stop there
    a0, a1 = 0.95, 0.9
    T_prev = (1 - a0) * (1 - a1)
    a2 = 1 - T_MIN32 * (1 + 5e-5) / T_prev
    orc, out, gC, gD = _run(_stack([a0, a1, a2, 0.6]))
    assert out["events"][10, 12] == 1
    assert out["n_used"][10, 12] == 4
    bref = orc.backward([gC], [gD])
    a2_alt = 1 - T_MIN32 * (1 - 1e-9) / T_prev
    orc2, out2, _, _ = _run(_stack([a0, a1, a2_alt, 0.6]), gC)
    assert out2["n_used"][10, 12] == 3
    assert (out["hi"] - out["lo"])[:, 10, 12].max() > 1e-5   # splat 3 behind the stop is visible
    # the alternative moved splat 2's opacity by ~1e-6 relative as well (every pixel)
    scale = max(np.abs(bref[k]).max() for k in ("means", "scales", "opacities", "sh"))
    _covers(out, out2, bref, orc2.backward([gC], [gD]), slack_img=1e-6, slack_grad=1e-5 * scale)


def test_envelope_covers_the_other_clamp_decision():
    # splat 0 sits at alpha_max (1 + 2e-6) at the principal point: clamped, so its value
    # gradient there is 0; unclamped (alpha_max (1 - 1e-9)) it is not
    orc, out, gC, gD = _run(_stack([A_MAX32 * (1 + 2e-6), 0.5]))
    assert out["events"][10, 12] == 0          # a clamp changes no value, only a gradient
    bref = orc.backward([gC], [gD])
    orc2, out2, _, _ = _run(_stack([A_MAX32 * (1 - 1e-9), 0.5]), gC)
    # the alternative moved splat 0's opacity by 2e-6 relative (every pixel)
    scale = max(np.abs(bref[k]).max() for k in ("means", "scales", "opacities", "sh"))
    _covers(out, out2, bref, orc2.backward([gC], [gD]), slack_img=1e-5, slack_grad=1e-5 * scale)


def test_envelope_covers_a_flipped_loss_sign():
    # output 0 (red) of one pixel has a non-unique gradient: its sign may flip
    orc, out, gC, gD = _run(_stack([0.5, 0.6, 0.3]))
    tie = np.zeros((20, 24), np.uint8)
    tie[9, 13] = 1
    bref = orc.backward([gC], [gD], ambiguous_pixels=[tie])
    gC2 = gC.copy()
    gC2[0, 9, 13] = -gC[0, 9, 13]
    _covers(out, out, bref, orc.backward([gC2], [gD]))
    # a pixel without a mark keeps its gradient unique
    assert sum(np.abs(orc.backward([gC], [gD])["envelope"][k]).max() for k in ("means", "sh")) == 0.0


def test_window_renders_and_differentiates_only_its_pixels():
    # a window of a view equals the same pixels of the full render, and its gradient is the
    # full gradient of output gradients that vanish outside the window
    w = scenes.make_cfg1(n=400)
    g, c = w.gaussians, w.cameras[0]
    s = oracle.Settings(mu_fp32=True, tile=16)
    full = oracle.Oracle(g.arrays(), 0, [c], s)
    win = (37, 21, 101, 70)
    sw = oracle.Settings(mu_fp32=True, tile=16, window=win)
    part = oracle.Oracle(g.arrays(), 0, [c], sw)
    a, b = full.forward()[0], part.forward()[0]
    x0, y0, x1, y1 = win
    for k in ("color", "depth", "alpha", "T_final", "lo", "hi"):
        np.testing.assert_array_equal(a[k][..., y0:y1, x0:x1], b[k][..., y0:y1, x0:x1])
        outside = np.ones(b[k].shape[-2:], bool)
        outside[y0:y1, x0:x1] = False
        assert (b[k][..., outside] == 0).all()
    rng = np.random.default_rng(3)
    gC = rng.standard_normal((3, c.height, c.width))
    gD = rng.standard_normal((c.height, c.width))
    mask = np.zeros((c.height, c.width))
    mask[y0:y1, x0:x1] = 1
    ga = full.backward([gC * mask], [gD * mask])
    gb = part.backward([gC], [gD])
    for k in ("means", "scales", "quats", "opacities", "sh"):
        np.testing.assert_allclose(gb[k], ga[k], rtol=1e-12, atol=1e-14 * np.abs(ga[k]).max())


# ---------------------------------------------------------------------------------------
# guard-band clamp of the projection's Jacobian (x/z, y/z clamped to 1.3 half-FOVs)
# ---------------------------------------------------------------------------------------

def _offcentre_scene(seed, n=150, deg=0):
    """Gaussians in front of a camera whose principal point sits near the left edge, so
    that many lie beyond 1.3 half fields of view to the right of the optical axis."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(1.5, 3.0, n)
    means = np.stack([rng.uniform(-0.3, 1.6, n) * z, rng.uniform(-0.5, 0.5, n) * z, z], 1)
    g = scenes.random_gaussians(rng, means, deg)
    g.scales = (g.scales * 4).astype(np.float32)
    c = cam(40, 32, 30.0, cx=6.0, cy=16.0)
    return g, c


def test_jacobian_clamp_closed_form():
    # an axis-aligned Gaussian at x/z = 1.6 > 1.3 W / (2 fx) = 1.04: J's x/z entry is held at the limit
    W, H, f, z = 64, 48, 40.0, 2.0
    lim = float(np.float32(1.3) * (np.float32(0.5 * W) / np.float32(f)))
    p = gaussians([[1.6 * z, 0.0, z]], [[0.05, 0.04, 0.3]])
    c = cam(W, H, f, cx=0.0, cy=24.0)
    rec = oracle.Oracle(p, 0, [c], oracle.Settings(mu_fp32=False, jclamp=1.3, guard=10.0)).records()
    s32 = np.float32([0.05, 0.04, 0.3]).astype(np.float64)
    zz = float(np.float32(z))
    sxx = (f / zz) ** 2 * s32[0] ** 2 + (f * lim / zz) ** 2 * s32[2] ** 2 + float(np.float32(0.3))
    syy = (f / zz) ** 2 * s32[1] ** 2 + float(np.float32(0.3))
    np.testing.assert_allclose(rec["conic"][0], [1 / sxx, 0.0, 1 / syy], rtol=1e-12, atol=1e-15)
    # unclamped the x/z entry would be 1.6 (a wider splat)
    rec0 = oracle.Oracle(p, 0, [c], oracle.Settings(mu_fp32=False, guard=10.0)).records()
    assert rec0["conic"][0][0] < rec["conic"][0][0]


@pytest.mark.parametrize("deg", [0, 3])
def test_jacobian_clamp_equals_brute_force(deg):
    g, c = _offcentre_scene(50 + deg, deg=deg)
    out = oracle.Oracle(g.arrays(), deg, [c], oracle.Settings(mu_fp32=False, tile=8, jclamp=1.3)).forward()[0]
    b = brute.render(g.arrays(), deg, c, jclamp=1.3)
    for k in ("color", "depth", "alpha", "T_final"):
        np.testing.assert_allclose(out[k], b[k], atol=1e-12, rtol=0, err_msg=k)
    # the clamp acts on rendered Gaussians here and changes the image
    pr = brute.project(g.arrays(), deg, c)
    lim = float(np.float32(1.3) * (np.float32(0.5 * c.width) / np.float32(c.fx)))
    t = np.asarray(g.means, np.float64) @ np.eye(3).T
    assert (pr["front"] & (t[:, 0] / t[:, 2] > lim)).sum() >= 10
    b0 = brute.render(g.arrays(), deg, c)
    assert np.abs(b0["color"] - b["color"]).max() > 1e-3
    # a limit nobody reaches changes nothing
    far = oracle.Oracle(g.arrays(), deg, [c], oracle.Settings(mu_fp32=False, tile=8, jclamp=100.0)).forward()[0]
    off = oracle.Oracle(g.arrays(), deg, [c], oracle.Settings(mu_fp32=False, tile=8)).forward()[0]
    np.testing.assert_array_equal(far["color"], off["color"])


@pytest.mark.parametrize("deg,seed", [(0, 60), (3, 61)])
def test_jacobian_clamp_backward_matches_central_differences(deg, seed):
    g, c = _offcentre_scene(seed, n=40, deg=deg)
    s = oracle.Settings(mu_fp32=False, tile=8, jclamp=1.3)
    checked, _ = _fd_check(g, c, deg, s, seed, trials=120)
    assert len(checked) >= 80
    lim = float(np.float32(1.3) * (np.float32(0.5 * c.width) / np.float32(c.fx)))
    t = np.asarray(g.means, np.float64)
    clamped = set(np.nonzero(t[:, 0] / t[:, 2] > lim)[0].tolist())
    hit = [a for gi, idx, a in checked if gi in (0, 1, 2) and idx[0] in clamped and a != 0.0]
    assert len(hit) >= 10, len(hit)
