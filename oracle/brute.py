"""Brute-force per-pixel compositing in NumPy/SciPy (FP64), for tiny scenes only.

TEST INFRASTRUCTURE ONLY.  Written independently of ``oracle.cpp``: no tiles,
no sort of duplicated keys, SH values from ``scipy.special`` rather than from
Legendre polynomials, covariance products through ``numpy.linalg``.  Every
Gaussian in front of the near plane is composited at every pixel in ascending
(binary32 depth bits, index) order, following Eq. 2-5 and Eq. 11 of GSFusion.

With extent_k >= sqrt(2 ln 255) the tile path visits exactly the Gaussians that
can pass the skip rule, so a tile renderer must agree with this.  With
alpha_min = 0, alpha_max = 1, T_min = 0 the loop is Eq. 11 word for word.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def real_sh(degree, dirs):
    """Orthonormal real SH that keep the Condon-Shortley phase, from scipy's complex ones.

    scipy's complex Y_l^m = N P_l^m(cos t) e^{i m phi} already carries the phase in
    P_l^m, so Y_l^m(real) = sqrt2 Re(Y_l^|m|) for m > 0, sqrt2 Im(Y_l^|m|) for m < 0
    and Y_l^0 for m = 0 (e.g. Y_1^1 = -sqrt(3/(4 pi)) x); index k = l^2 + l + m.
    """
    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))       # polar
    phi = np.arctan2(d[:, 1], d[:, 0])                   # azimuth
    K = (degree + 1) ** 2
    out = np.zeros((d.shape[0], K))
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            if hasattr(special, "sph_harm_y"):
                Yc = special.sph_harm_y(l, am, theta, phi)
            else:  # older SciPy: sph_harm(m, l, azimuth, polar)
                Yc = special.sph_harm(am, l, phi, theta)
            if m == 0:
                val = Yc.real
            elif m > 0:
                val = np.sqrt(2.0) * Yc.real
            else:
                val = np.sqrt(2.0) * Yc.imag
            out[:, l * l + l + m] = val
    return out


def quat_to_rot(q):
    q = np.asarray(q, np.float64)
    w, x, y, z = (q / np.linalg.norm(q, axis=-1, keepdims=True)).T
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def project(params, sh_degree, cam, lowpass=0.3, guard=0.15, jclamp=0.0):
    """FP64 splat parameters of every Gaussian: dict(mu, conic, z, color, opacity, front).

    ``front`` marks the Gaussians in the view frustum: binary32 depth above znear and
    binary32 projected centre inside the image widened by guard x (W, H) per side.
    """
    means, scales, quats, opac, sh = (np.asarray(a, np.float64) for a in params)
    W = np.asarray(cam.R, np.float32).astype(np.float64)
    tc = np.asarray(cam.t, np.float32).astype(np.float64)
    t = means @ W.T + tc
    tx, ty, tz = t.T
    R = quat_to_rot(quats)
    S = np.einsum("nij,nj->nij", R, scales)             # R diag(s)
    Sigma = S @ np.transpose(S, (0, 2, 1))               # Eq. 2
    fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    J = np.zeros((means.shape[0], 2, 3))
    txj, tyj = tx, ty
    if jclamp > 0:   # guard band inside J: x/z, y/z clamped to +-jclamp times the half field of view
        f = np.float32
        limx = float(f(jclamp) * (f(0.5) * f(cam.width) / f(cam.fx)))
        limy = float(f(jclamp) * (f(0.5) * f(cam.height) / f(cam.fy)))
        txj = np.clip(tx / tz, -limx, limx) * tz
        tyj = np.clip(ty / tz, -limy, limy) * tz
        txj = np.where(np.abs(tx / tz) > limx, txj, tx)
        tyj = np.where(np.abs(ty / tz) > limy, tyj, ty)
    J[:, 0, 0] = fx / tz
    J[:, 0, 2] = -fx * txj / tz ** 2
    J[:, 1, 1] = fy / tz
    J[:, 1, 2] = -fy * tyj / tz ** 2
    JW = J @ W
    cov = JW @ Sigma @ np.transpose(JW, (0, 2, 1)) + float(np.float32(lowpass)) * np.eye(2)   # Eq. 5
    conic = np.linalg.inv(cov)
    mu = np.stack([fx * tx / tz + float(np.float32(cam.cx)), fy * ty / tz + float(np.float32(cam.cy))], 1)
    centre = -(W.T @ tc)
    dirs = means - centre
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    Y = real_sh(sh_degree, dirs)
    color = np.maximum(0.0, 0.5 + np.einsum("nk,nkc->nc", Y, sh))
    # binary32 camera coordinates and centre, same operation order as the discrete stage,
    # for the ordering and the frustum decision
    p32 = np.asarray(params[0], np.float32)
    W32 = np.asarray(cam.R, np.float32)
    t32 = np.asarray(cam.t, np.float32)
    c32 = []
    for r in range(3):
        v = (W32[r, 0] * p32[:, 0] + W32[r, 1] * p32[:, 1]).astype(np.float32)
        v = (v + W32[r, 2] * p32[:, 2]).astype(np.float32)
        c32.append((v + t32[r]).astype(np.float32))
    x32, y32, z32 = c32
    f = np.float32
    with np.errstate(all="ignore"):
        mux = f(cam.fx) * (x32 / z32) + f(cam.cx)
        muy = f(cam.fy) * (y32 / z32) + f(cam.cy)
    gx, gy = f(guard) * f(cam.width), f(guard) * f(cam.height)
    inside = (mux >= -gx) & (mux <= f(cam.width) + gx) & (muy >= -gy) & (muy <= f(cam.height) + gy)
    front = (z32 > np.float32(cam.znear)) & inside
    return dict(mu=mu, conic=conic, z=tz, z32=z32, color=color, opacity=opac, front=front)


def render(params, sh_degree, cam, alpha_min=1 / 255, alpha_max=0.99, T_min=1e-4, bg=(0, 0, 0), lowpass=0.3,
           guard=0.15, jclamp=0.0):
    """Per-pixel front-to-back compositing over all Gaussians in the frustum (no tiles)."""
    pr = project(params, sh_degree, cam, lowpass, guard, jclamp)
    idx = np.nonzero(pr["front"])[0]
    zb = pr["z32"][idx].view(np.uint32)
    order = idx[np.lexsort((idx, zb))]
    H, W = cam.height, cam.width
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    T = np.ones((H, W))
    C = np.zeros((3, H, W))
    D = np.zeros((H, W))
    done = np.zeros((H, W), bool)
    last = np.full((H, W), -1, np.int64)   # Gaussian index of the last contributor
    count = np.zeros((H, W), np.int64)     # contributors
    amin = float(np.float32(alpha_min))
    amax = float(np.float32(alpha_max))
    tmin = float(np.float32(T_min))
    for g in order:
        A, B = pr["conic"][g, 0, 0], pr["conic"][g, 0, 1]
        Cc = pr["conic"][g, 1, 1]
        dx = xs - pr["mu"][g, 0]
        dy = ys - pr["mu"][g, 1]
        power = -0.5 * (A * dx * dx + 2.0 * B * dx * dy + Cc * dy * dy)
        a = pr["opacity"][g] * np.exp(power)
        use = (~done) & ~(a < amin)
        alpha = np.minimum(a, amax)
        w = np.where(use, alpha * T, 0.0)
        C += pr["color"][g][:, None, None] * w
        D += pr["z"][g] * w
        T = np.where(use, T * (1.0 - alpha), T)
        last = np.where(use, g, last)
        count += use
        done |= use & (T < tmin)
    C += np.asarray(bg, np.float64)[:, None, None] * T
    return dict(color=C, depth=D, alpha=1.0 - T, T_final=T, last=last, count=count, stopped=done)
