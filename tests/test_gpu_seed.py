"""GPU quadtree seeding (gsr_seed) against the seeding oracle: the leaves must match
exactly and in order (integer decisions taken from binary64 statistics on both sides),
the initial Gaussians within binary32 rounding of the binary64 oracle."""
import numpy as np
import pytest
import torch

import scenes
from oracle import seed as S

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
REL = 2e-6  # binary32 results of binary64 arithmetic


def _room_frame(seed, W, H):
    room = scenes.Room(np.random.default_rng(seed), (6.0, 5.0, 3.0), 20)
    cam = room.random_camera(np.random.default_rng(seed + 100), W, H)
    depth, rgb = room.raycast(cam, perturbed=True)   # depth [H,W], colour [3,H,W]
    return cam, np.ascontiguousarray(rgb, np.float32), depth.astype(np.float32)


def _random_frame(seed, W, H):
    rng = np.random.default_rng(seed)
    rgb = (rng.random((3, H, W)) ** 3).astype(np.float32)
    rgb[:, : H // 2, : W // 3] = 0.4                   # a flat region
    depth = (0.5 + 4 * rng.random((H, W)) ** 6).astype(np.float32)
    depth[rng.random((H, W)) < 0.1] = 0.0
    cam = scenes.Camera(W, H, 0.8 * W, 0.8 * W, W / 2 - 0.3, H / 2 + 0.2, np.eye(3, dtype=np.float32),
                        np.array([0.1, 0.2, -0.3], np.float32))
    return cam, rgb, depth


def _check(cam, rgb, depth, measure, thr, min_side, sh_degree=0, opacity=0.5):
    from paper_2408_12677_amd import rasterize as R
    thr32 = float(np.float32(thr))
    leaves, cells = S.quadtree(rgb, depth, measure, thr32, root=64, min_side=min_side)
    near = [c for c in cells if c[3] > 0 and abs(c[4] - thr32) <= 1e-9 * max(thr32, 1e-30)]
    assert not near, "a cell's measure lies within rounding of the threshold: pick another case"
    ref = S.initial_gaussians(leaves, rgb, depth, cam, opacity=opacity, sh_degree=sh_degree)
    out = R.seed(torch.from_numpy(rgb).to(DEV), torch.from_numpy(depth).to(DEV), cam, measure, thr32, min_side,
                 opacity, sh_degree)
    got = {k: v.cpu().numpy() for k, v in out.items()}
    np.testing.assert_array_equal(got["leaves"], ref["leaves"])
    for k in ("means", "scales", "sh"):
        np.testing.assert_allclose(got[k], ref[k], rtol=REL, atol=REL * max(1.0, np.abs(ref[k]).max(initial=0)))
    assert (got["quats"] == np.array([1, 0, 0, 0], np.float32)).all()
    assert (got["opacities"] == np.float32(opacity)).all()
    return len(got["leaves"])


@pytest.mark.parametrize("measure,thr", [("contrast", 0.1), ("depth_variance", 0.01)])
@pytest.mark.parametrize("min_side", [1, 4, 16])
def test_room_frames(measure, thr, min_side):
    cam, rgb, depth = _room_frame(3, 320, 240)
    n = _check(cam, rgb, depth, measure, thr, min_side, sh_degree=1)
    assert n > 50


@pytest.mark.parametrize("shape", [(1, 1), (7, 5), (64, 64), (65, 130), (200, 97)])
@pytest.mark.parametrize("min_side", [1, 2, 4, 64])
def test_random_frames_and_ragged_sizes(shape, min_side):
    W, H = shape
    cam, rgb, depth = _random_frame(W * 1000 + H, W, H)
    for measure, thr in (("contrast", 0.3), ("depth_variance", 0.05)):
        _check(cam, rgb, depth, measure, thr, min_side, sh_degree=3, opacity=0.9)


def test_headline_resolution_room():
    cam, rgb, depth = _room_frame(5, 640, 480)
    assert _check(cam, rgb, depth, "contrast", 0.1, 4) > 500


def test_no_valid_depth_gives_nothing():
    from paper_2408_12677_amd import rasterize as R
    cam, rgb, depth = _random_frame(1, 100, 60)
    out = R.seed(torch.from_numpy(rgb).to(DEV), torch.zeros((60, 100), device=DEV), cam)
    assert out["means"].shape[0] == 0


def test_capacity_too_small_is_reported():
    import ctypes
    from paper_2408_12677_amd import _native as N
    from paper_2408_12677_amd import rasterize as R
    cam, rgb, depth = _room_frame(3, 128, 96)
    need = len(S.initial_gaussians(S.quadtree(rgb, depth, "contrast", float(np.float32(0.1)))[0], rgb, depth,
                                   cam)["means"])
    ctx = R.context(DEV)
    cap = need - 1
    bufs = [torch.full((max(cap, 1), c), 7.0, device=DEV) for c in (3, 3, 4, 1, 3)]
    so = N.SeedOut(*(b.data_ptr() for b in bufs), None)
    s = N.SeedSettings()
    assert ctx.lib.gsr_seed_settings_default(ctypes.byref(s)) == N.OK
    n = ctypes.c_int64()
    rgb_d, depth_d = torch.from_numpy(rgb).to(DEV), torch.from_numpy(depth).to(DEV)
    cams = R._cams([cam])
    st = ctx.lib.gsr_seed(ctx.h, ctypes.byref(cams[0]), ctypes.c_void_p(rgb_d.data_ptr()),
                          ctypes.c_void_p(depth_d.data_ptr()), ctypes.byref(s), None, ctypes.byref(so), cap,
                          ctypes.byref(n))
    torch.cuda.synchronize()
    assert st == N.ECAPACITY and n.value == need
    assert all((b == 7.0).all() for b in bufs)   # nothing written
