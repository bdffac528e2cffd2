"""Pins of the seeding oracle (oracle/seed.py) against facts that do not come from it:
hand-derived cases, invariants of the quadtree, an independent integral-image seeder,
and the closed forms of the back-projection (Eq. 10) and of the initial Gaussian."""
import math

import numpy as np
import pytest

import scenes
from oracle import seed as S


def _img(W, H, value=0.5):
    return np.full((3, H, W), value, np.float32)


def _cam(W, H, f=100.0, R=None, t=None):
    return scenes.Camera(W, H, f, f, W / 2, H / 2,
                         np.eye(3, dtype=np.float32) if R is None else R,
                         np.zeros(3, np.float32) if t is None else t)


def test_uniform_image_one_leaf_per_root():
    W, H = 200, 130  # roots clipped at both borders
    rgb, depth = _img(W, H), np.full((H, W), 2.0, np.float32)
    for measure in ("contrast", "depth_variance"):
        leaves, _ = S.quadtree(rgb, depth, measure)
        assert len(leaves) == math.ceil(W / 64) * math.ceil(H / 64)
        assert {tuple(l) for l in leaves} == {(x, y, min(64, W - x), min(64, H - y))
                                            for y in range(0, H, 64) for x in range(0, W, 64)}


def test_step_edge_by_hand():
    # 8x8 image, root 8, min side 4: a colour step between x = 1 and x = 2 splits the root
    # once; the four 4x4 quadrants are leaves (side 4 is the minimum)
    rgb = _img(8, 8, 0.0)
    rgb[:, :, 2:] = 1.0
    depth = np.ones((8, 8), np.float32)
    leaves, cells = S.quadtree(rgb, depth, "contrast", 0.1, root=8, min_side=4)
    assert [tuple(l) for l in leaves] == [(0, 0, 4, 4), (4, 0, 4, 4), (0, 4, 4, 4), (4, 4, 4, 4)]
    # min side 2: the quadrants holding the step split again; the right ones are uniform
    leaves, _ = S.quadtree(rgb, depth, "contrast", 0.1, root=8, min_side=2)
    assert [tuple(l) for l in leaves] == [
        (0, 0, 2, 2), (2, 0, 2, 2), (0, 2, 2, 2), (2, 2, 2, 2), (4, 0, 4, 4),
        (0, 4, 2, 2), (2, 4, 2, 2), (0, 6, 2, 2), (2, 6, 2, 2), (4, 4, 4, 4)]
    # a contrast exactly at the threshold splits (a leaf's contrast is below it)
    rgb2 = _img(8, 8, 0.0)
    rgb2[:, :, 4:] = 0.25
    assert len(S.quadtree(rgb2, depth, "contrast", 0.25, root=8, min_side=4)[0]) == 4
    assert len(S.quadtree(rgb2, depth, "contrast", 0.2500001, root=8, min_side=4)[0]) == 1


@pytest.mark.parametrize("measure,thr", [("contrast", 0.1), ("contrast", 0.4), ("depth_variance", 0.01)])
@pytest.mark.parametrize("seed", [0, 1])
def test_quadtree_invariants(measure, thr, seed):
    rng = np.random.default_rng(seed)
    W, H = 150, 97
    rgb = rng.random((3, H, W)).astype(np.float32) ** 4        # mostly dark, some bright pixels
    depth = (1 + 2 * rng.random((H, W)) ** 8).astype(np.float32)
    depth[rng.random((H, W)) < 0.05] = 0.0
    depth[:30, :30] = 0.0                                        # a region without depth
    leaves, cells = S.quadtree(rgb, depth, measure, thr, root=64, min_side=2)
    cover = np.zeros((H, W), np.int32)
    for x0, y0, w, h in leaves:
        cover[y0:y0 + h, x0:x0 + w] += 1
    assert cover.max() == 1                                      # disjoint
    if measure == "contrast":
        assert cover.min() == 1                                  # the whole image
    else:                                                        # every valid depth is covered
        assert (cover[depth > 0] == 1).all()
    for x0, y0, side, n, m, s in cells:
        if s:
            assert side > 2 and (m >= thr if measure == "contrast" else m > thr)
        elif n > 0:
            assert side == 2 or (m < thr if measure == "contrast" else m <= thr)


def test_depth_variance_matches_integral_image_seeder():
    # the workload seeder computes the same quadtree from integral images
    room = scenes.Room(np.random.default_rng(7), (6.0, 5.0, 3.0), 20)
    cam = room.random_camera(np.random.default_rng(8), 320, 240)
    depth, rgb = room.raycast(cam)   # depth [H,W], colour [3,H,W]
    leaves, cells = S.quadtree(rgb, depth, "depth_variance", 0.01, root=64, min_side=4)
    ref = scenes.quadtree_leaves(depth, root=64, min_side=4, var_thresh=0.01)
    near = [c for c in cells if abs(c[4] - 0.01) < 1e-9]
    assert not near
    assert sorted(map(tuple, leaves)) == sorted(map(tuple, ref))
    assert len(leaves) > 100


def test_initial_gaussians_closed_forms():
    rng = np.random.default_rng(3)
    W, H = 96, 80
    rgb = rng.random((3, H, W)).astype(np.float32)
    depth = (0.5 + 3 * rng.random((H, W))).astype(np.float32)
    depth[::7, ::5] = 0.0
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]], np.float32)
    cam = _cam(W, H, 90.0, R, np.array([0.3, -0.2, 1.1], np.float32))
    leaves, _ = S.quadtree(rgb, depth, "contrast", 0.3, root=32, min_side=4)
    g = S.initial_gaussians(leaves, rgb, depth, cam, opacity=0.5, sh_degree=2)
    n = len(g["means"])
    assert 0 < n <= len(leaves)
    Rd, td = R.astype(np.float64), cam.t.astype(np.float64)
    for i in range(n):
        x0, y0, lw, lh = g["leaves"][i]
        xc, yc = x0 + lw // 2, y0 + lh // 2
        # back into the camera; R^T inverts the binary32 rotation to ~1e-7
        pcam = Rd @ g["means"][i] + td
        d = float(depth[yc, xc])
        assert pcam[2] == pytest.approx(d, rel=1e-6)
        assert pcam[0] / pcam[2] * cam.fx + cam.cx == pytest.approx(xc, abs=1e-4)
        assert pcam[1] / pcam[2] * cam.fy + cam.cy == pytest.approx(yc, abs=1e-4)
        expect = d * math.hypot((xc - x0) / cam.fx, (yc - y0) / cam.fy)
        assert g["scales"][i] == pytest.approx([expect] * 3, rel=1e-12)
        assert np.allclose(0.5 + g["sh"][i, 0] * S.Y00, rgb[:, yc, xc], atol=1e-12)
        assert not g["sh"][i, 1:].any()
    assert (g["quats"] == [1, 0, 0, 0]).all() and (g["opacities"] == 0.5).all()
    # leaves whose centre depth is missing give no Gaussian
    missing = [tuple(l) for l in leaves if not depth[l[1] + l[3] // 2, l[0] + l[2] // 2] > 0]
    assert n == len(leaves) - len(missing)


def test_back_projection_matches_workload_seeder():
    room = scenes.Room(np.random.default_rng(11), (6.0, 5.0, 3.0), 20)
    cam = room.random_camera(np.random.default_rng(12), 160, 120)
    depth, _ = room.raycast(cam, with_color=False)
    rgb = np.zeros((3, 120, 160), np.float32)
    leaves, _ = S.quadtree(rgb, depth, "depth_variance", 0.01, root=64, min_side=4)
    g = S.initial_gaussians(leaves, rgb, depth, cam)
    pw, scale = scenes.seed_from_view(cam, depth)
    order = np.lexsort(g["means"].T)
    ref = np.lexsort(pw.T)
    assert np.allclose(g["means"][order], pw[ref], atol=1e-9)
    assert np.allclose(g["scales"][order, 0], scale[ref], atol=1e-9)


def test_y00_is_the_normalised_constant():
    # integral of Y00^2 over the unit sphere is 1
    assert 4 * math.pi * S.Y00 ** 2 == pytest.approx(1.0, rel=1e-15)


def test_voxel_weight_check_against_a_fused_map():
    # a wall facing the camera: after the frame is fused every leaf's mean sits in a voxel
    # first seen by that frame (weight 1), so every leaf gives a Gaussian; fusing the
    # same frame again raises the weights to 2 and the check then keeps none
    from oracle import tsdf as T
    W, H = 64, 48
    cam = _cam(W, H, 50.0)
    rng = np.random.default_rng(4)
    rgb = rng.random((3, H, W)).astype(np.float32)
    depth = np.full((H, W), 1.5, np.float32)
    leaves, _ = S.quadtree(rgb, depth, "contrast", 0.3, root=16, min_side=4)
    m = T.TsdfMap(voxel=0.01)
    m.integrate(depth, cam)
    first = S.initial_gaussians(leaves, rgb, depth, cam, tsdf_map=m)
    assert len(first["means"]) == len(leaves) > 10
    m.integrate(depth, cam)
    assert len(S.initial_gaussians(leaves, rgb, depth, cam, tsdf_map=m)["means"]) == 0
    # a fresh map that never saw the frame: weight 0 everywhere, no Gaussians either
    assert len(S.initial_gaussians(leaves, rgb, depth, cam, tsdf_map=T.TsdfMap(voxel=0.01))["means"]) == 0
