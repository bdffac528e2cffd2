"""GPU TSDF fusion (gsr_tsdf_*) and the seeding voxel-weight check against the oracle
(oracle/tsdf.py, oracle/seed.py) on seeded frames.

Bars: the allocated blocks (a set of block coordinates) and every voxel weight are
bit-exact (integer decisions taken by the same binary32 operation sequences on both
sides); the fused distances are binary32 against the FP64 oracle, within 1e-5 per fused
frame (a handful of roundings of values in [-1, 1] per update); the seeding check keeps
exactly the oracle's leaves, except that a mean within 1e-5 voxel of a voxel boundary may
round to the other voxel on one side (its binary32 mean comes from a binary64 value that
the two sides sum in different orders)."""
import sys

import numpy as np
import pytest

import scenes
from oracle import seed as S
from oracle import tsdf as T

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_12677_amd import rasterize
    return rasterize


def _frames(seed, W, H, n):
    room = scenes.Room(np.random.default_rng(seed), (6.0, 5.0, 3.0), 20)
    out = []
    for k in range(n):
        cam = room.random_camera(np.random.default_rng(seed * 100 + k), W, H)
        depth, rgb = room.raycast(cam, perturbed=True)
        out.append((cam, depth.astype(np.float32), np.ascontiguousarray(rgb, np.float32)))
    return out


def _compare(gpu_map, ref, frames_fused, label=""):
    coords, ts, ws = gpu_map.export()
    got = {tuple(int(v) for v in c): n for n, c in enumerate(coords)}
    # (counts, not the sets themselves: pytest's explanation of two large unequal sets is slow)
    missing, extra = len(set(ref.blocks) - set(got)), len(set(got) - set(ref.blocks))
    assert missing == 0 and extra == 0, f"{label}: {len(got)} blocks vs {len(ref.blocks)} " \
                                        f"({missing} missing, {extra} extra)"
    tol = 1e-5 * frames_fused + 1e-6
    worst = 0.0
    for b, (rt, rw) in ref.blocks.items():
        n = got[b]
        np.testing.assert_array_equal(ws[n], rw, err_msg=f"{label} weights of block {b}")
        d = np.abs(ts[n].astype(np.float64) - rt).max()
        worst = max(worst, d)
        assert d <= tol, f"{label} block {b}: tsdf differs by {d:.3g}"
    return worst


@pytest.mark.parametrize("weighting", ["eq9", "unit"])
def test_fusion_of_room_frames_matches_oracle(R, weighting):
    frames = _frames(3, 160, 120, 3)
    m = R.TsdfMap(DEV, weighting=weighting, max_blocks=1 << 15)
    ref = T.TsdfMap(voxel=0.01, weighting=weighting)
    for k, (cam, depth, _) in enumerate(frames):
        m.integrate(torch.from_numpy(depth).to(DEV), cam)
        met = ref.integrate(depth, cam)
        inf = m.info()
        assert inf["flags"] == 0 and inf["met_last"] == len(met)
        worst = _compare(m, ref, k + 1, f"frame {k}")
        say(weighting, "frame", k, "blocks", inf["blocks"], "met", inf["met_last"], "worst", worst)
    m.free()


@pytest.mark.parametrize("shape", [(1, 1), (37, 23), (64, 48)])
def test_ragged_frames_and_other_settings(R, shape):
    W, H = shape
    frames = _frames(7, W, H, 2)
    kw = dict(voxel=0.02, trunc=0.05, w_max=3.0, step=0.015)
    m = R.TsdfMap(DEV, max_blocks=1 << 12, **kw)
    ref = T.TsdfMap(voxel=0.02, eps=0.05, w_max=3.0, step=0.015)
    for k in range(4):                       # past the weight cap
        cam, depth, _ = frames[k % 2]
        depth = depth.copy()
        depth[::3, ::2] = 0.0                # holes
        m.integrate(torch.from_numpy(depth).to(DEV), cam)
        ref.integrate(depth, cam)
        _compare(m, ref, k + 1, f"{shape} frame {k}")
    m.free()


def test_empty_frame_and_capacity_flags(R):
    cam, depth, _ = _frames(5, 96, 72, 1)[0]
    m = R.TsdfMap(DEV, max_blocks=64)
    m.integrate(torch.zeros((72, 96), device=DEV), cam)
    assert m.info() == dict(blocks=0, met_last=0, flags=0)
    m.integrate(torch.from_numpy(depth).to(DEV), cam)   # needs far more than 64 blocks
    inf = m.info()
    assert inf["blocks"] == 64 and inf["flags"] & 2      # pool full, reported
    m.free()


def test_voxel_weight_queries(R):
    frames = _frames(9, 120, 90, 2)
    m = R.TsdfMap(DEV, max_blocks=1 << 15)
    ref = T.TsdfMap(voxel=0.01)
    for cam, depth, _ in frames:
        m.integrate(torch.from_numpy(depth).to(DEV), cam)
        ref.integrate(depth, cam)
    say("query test: fused", m.info())
    rng = np.random.default_rng(2)
    c, _, w = m.export()
    # points inside allocated blocks (every weight occurs) and anywhere in the room
    b = c[rng.integers(0, len(c), 3000)]
    pts = np.concatenate([(b * 8 + rng.uniform(0, 8, (3000, 3))) * 0.01,
                          rng.uniform([-1, -1, -1], [7, 6, 4], (2000, 3))]).astype(np.float32)
    _compare(m, ref, 2, "query map")
    say("query test: maps equal")
    got = m.weights(torch.from_numpy(pts).to(DEV)).cpu().numpy()
    say("query test: queried")
    want = ref.voxel_weight(pts)
    bad = np.nonzero(got != want)[0]
    for i in bad[:5]:
        g = np.floor(pts[i] / np.float32(0.01))
        say("query mismatch", i, pts[i].tolist(), (pts[i] / np.float32(0.01)).tolist(), g.tolist(), got[i], want[i])
    assert len(bad) == 0, f"{len(bad)} query weights differ"
    assert (got == 1).any() and (got == 2).any() and (got == 0).any()
    m.free()


def test_seeding_check_with_fused_map(R):
    (cam, depth, rgb), (cam2, depth2, rgb2) = _frames(11, 320, 240, 2)
    m = R.TsdfMap(DEV, max_blocks=1 << 16)
    ref = T.TsdfMap(voxel=0.01)
    thr = float(np.float32(0.1))
    kept = []
    for c, d, im in ((cam, depth, rgb), (cam2, depth2, rgb2), (cam, depth, rgb)):
        m.integrate(torch.from_numpy(d).to(DEV), c)
        ref.integrate(d, c)
        leaves, _ = S.quadtree(im, d, "contrast", thr, root=64, min_side=4)
        want = S.initial_gaussians(leaves, im, d, c, tsdf_map=ref)
        allg = S.initial_gaussians(leaves, im, d, c)
        out = R.seed(torch.from_numpy(im).to(DEV), torch.from_numpy(d).to(DEV), c, "contrast", thr, 4, tsdf=m)
        got = {tuple(l) for l in out["leaves"].cpu().numpy()}
        exp = {tuple(l) for l in want["leaves"]}
        # leaves whose binary32 mean lies within 1e-5 voxel of a voxel boundary may differ
        g = allg["means"].astype(np.float32) / np.float32(0.01)
        near = np.abs(g - np.round(g)) < 1e-5
        edge = {tuple(l) for l, nb in zip(allg["leaves"], near.any(1)) if nb}
        diff = got ^ exp
        assert len(diff - edge) == 0, (len(diff), len(edge))
        kept.append(len(got))
        say("seeding check: kept", len(got), "of", len(allg["leaves"]), "oracle", len(exp))
    assert kept[0] > 100 and kept[2] == 0      # the first frame seeds, seeing it again seeds nothing
    m.free()
