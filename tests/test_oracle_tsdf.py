"""Pins of the TSDF oracle (oracle/tsdf.py) against closed forms: a plane facing the camera
at a known depth (any camera pose) has sdf = Z - z_v at every voxel, so Eq. 7 fixes every
fused value; repeated and alternating frames fix Eq. 8 and both readings of Eq. 9; the
allocation must contain every surface point's block; the seeding check turns off after a
second observation."""
import numpy as np
import pytest

import scenes
from oracle import tsdf as T


def _pose(seed):
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]], np.float32)
    return R, rng.uniform(-0.5, 0.5, 3).astype(np.float32)


def _cam(W, H, f, R=None, t=None):
    return scenes.Camera(W, H, f, f, W / 2 - 0.5, H / 2 - 0.5, np.eye(3, dtype=np.float32) if R is None else R,
                         np.zeros(3, np.float32) if t is None else t)


def _voxels(m):
    """(global index [n,3], tsdf, weight) of every voxel of the map, x fastest."""
    g, ts, ws = [], [], []
    for b, (t, w) in m.blocks.items():
        k, j, i = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
        g.append(np.stack([i.ravel(), j.ravel(), k.ravel()], 1) + np.asarray(b) * 8)
        ts.append(t.ravel())
        ws.append(w.ravel())
    return np.concatenate(g), np.concatenate(ts), np.concatenate(ws)


def _camera_z(g, cam, voxel):
    p = (g + 0.5) * voxel
    return (p @ np.asarray(cam.R, np.float64).T + np.asarray(cam.t, np.float64))[:, 2]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plane_facing_the_camera(seed):
    R, t = _pose(seed)
    cam = _cam(48, 36, 40.0, R, t)
    Z = 1.3
    m = T.TsdfMap(voxel=0.01)
    met = m.integrate(np.full((36, 48), Z, np.float32), cam)
    assert met and set(met) == set(m.blocks)
    g, ts, ws = _voxels(m)
    zv = _camera_z(g, cam, 0.01)
    upd = ws > 0
    assert set(np.unique(ws)) <= {0.0, 1.0}
    np.testing.assert_allclose(ts[upd], np.clip((Z - zv[upd]) / m.eps, -1, 1), atol=1e-5)
    # with depth everywhere, a voxel of a met block is updated exactly when it projects
    # into the image (nearest pixel); voxels within 1e-3 px of the image edge are skipped
    p = (g + 0.5) * 0.01 @ np.asarray(cam.R, np.float64).T + np.asarray(cam.t, np.float64)
    uh = 40 * p[:, 0] / p[:, 2] + 23.5 + 0.5
    vh = 40 * p[:, 1] / p[:, 2] + 17.5 + 0.5
    inside = (p[:, 2] > 0) & (uh >= 0) & (uh < 48) & (vh >= 0) & (vh < 36)
    clear_edge = (np.minimum(np.abs(uh), np.abs(uh - 48)) > 1e-3) & (np.minimum(np.abs(vh), np.abs(vh - 36)) > 1e-3)
    assert inside.sum() > 1000
    np.testing.assert_array_equal(upd[clear_edge], inside[clear_edge])
    # every block holding a surface point is allocated
    ys, xs = np.mgrid[0:36, 0:48]
    pc = np.stack([(xs - 23.5) / 40 * Z, (ys - 17.5) / 40 * Z, np.full(xs.shape, Z)], -1).reshape(-1, 3)
    pw = (pc - t.astype(np.float64)) @ R.astype(np.float64)
    blk = np.floor(pw / 0.08).astype(np.int64)
    frac = pw / 0.08 - np.floor(pw / 0.08)
    clear = ((frac > 1e-4) & (frac < 1 - 1e-4)).all(1)
    assert clear.mean() > 0.9
    assert {tuple(b) for b in blk[clear]} <= set(m.blocks)


def test_repeated_and_alternating_frames_follow_eq8_and_eq9():
    cam = _cam(24, 18, 20.0)
    Z1, Z2 = 1.0, 1.03
    d1, d2 = np.full((18, 24), Z1, np.float32), np.full((18, 24), Z2, np.float32)
    for weighting in ("eq9", "unit"):
        m = T.TsdfMap(voxel=0.01, w_max=5, weighting=weighting)
        m.integrate(d1, cam)
        m.integrate(d2, cam)
        g, ts, ws = _voxels(m)
        zv = _camera_z(g, cam, 0.01)
        both = ws == 2
        assert both.sum() > 100
        t1 = np.clip((Z1 - zv) / m.eps, -1, 1)
        t2 = np.clip((Z2 - zv) / m.eps, -1, 1)
        expect = (t1 + 2 * t2) / 3 if weighting == "eq9" else (t1 + t2) / 2
        np.testing.assert_allclose(ts[both], expect[both], atol=1e-6)
        # the same frame again and again: the weight saturates at w_max (Eq. 8) ...
        for _ in range(6):
            m.integrate(d2, cam)
        g, ts2, ws2 = _voxels(m)
        assert ws2.max() == 5 and (ws2[both] == 5).all()
        # ... and the value converges to the repeated frame's: at the cap, Eq. 9 halves the
        # distance each time (w_k = w_(k-1) = w_max), the running average by 1/(w_max + 1)
        if weighting == "eq9":
            # 2 -> 3 -> 4 -> 5 (three steps below the cap), then three at the cap
            k = 2
            r = 1.0
            for _ in range(3):
                r *= k / (2 * k + 1)
                k += 1
            r *= 0.5 ** 3
        else:
            r = (2 / 3) * (3 / 4) * (4 / 5) * (5 / 6) ** 3
        # ts2 - t2 = r (ts - t2) per voxel: the fixed point recovered from the two states
        # must be the repeated frame's value (to the binary32 voxel depth, ~1e-6)
        rec = (ts2[both] - r * ts[both]) / (1 - r)
        np.testing.assert_allclose(rec, t2[both], atol=5e-6)
        assert np.abs(ts[both] - t2[both]).max() > 0.05     # far enough to tell the factors apart


def test_empty_and_invalid_depth():
    cam = _cam(16, 12, 15.0)
    m = T.TsdfMap()
    assert m.integrate(np.zeros((12, 16), np.float32), cam) == set() and not m.blocks
    d = np.full((12, 16), -1.0, np.float32)
    d[5, 7] = 0.5
    met = m.integrate(d, cam)
    assert 1 <= len(met) <= 8      # one ray segment of 16 cm crosses at most a few blocks


def test_band_sample_count():
    assert T.band_samples(0.08, 0.01) == 17
    assert T.band_samples(0.05, 0.02) == 6
    assert T.band_samples(0.01, 0.05) == 1


def test_seeding_check_weights():
    cam = _cam(32, 24, 30.0)
    Z = 2.0
    m = T.TsdfMap(voxel=0.01)
    depth = np.full((24, 32), Z, np.float32)
    pts = np.stack([np.linspace(-0.5, 0.5, 7) * Z / 3, np.zeros(7), np.full(7, Z + 0.001)], 1)
    assert (m.voxel_weight(pts) == 0).all()            # nothing allocated yet
    m.integrate(depth, cam)
    assert (m.voxel_weight(pts) == 1).all()            # first observation: new Gaussians
    m.integrate(depth, cam)
    assert (m.voxel_weight(pts) == 2).all()            # seen before: none
    assert (m.voxel_weight(np.array([[0.0, 0.0, 40.0]])) == 0).all()


@pytest.mark.parametrize("seed", [3, 4])
def test_single_ray_allocates_the_blocks_of_its_band(seed):
    # the blocks met by one pixel's samples are blocks that the continuous band segment
    # [d - eps, d + eps] passes through, and they include every block the segment spends
    # more than one step in
    R, t = _pose(seed)
    cam = _cam(20, 16, 18.0, R, t)
    d = np.full((16, 20), -1.0, np.float32)
    d[9, 4] = 1.7
    m = T.TsdfMap(voxel=0.01)
    met = m.integrate(d, cam)
    z = np.linspace(1.7 - m.eps, 1.7 + m.eps, 20001)
    pc = np.stack([(4 - cam.cx) / 18.0 * z, (9 - cam.cy) / 18.0 * z, z], 1)
    pw = (pc - t.astype(np.float64)) @ R.astype(np.float64)
    blk = [tuple(b) for b in np.floor(pw / 0.08).astype(np.int64)]
    seg = set(blk)
    assert met <= seg
    runs = {b: blk.count(b) for b in seg}
    long_runs = {b for b, c in runs.items() if c * (2 * m.eps / 20000) > m.step * 1.01}
    assert long_runs <= met
