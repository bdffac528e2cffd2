"""Time steps of the keyframe-list optimisation run as captured iterations (rasterize.KeyframeSteps).

* the views the iterations render are the schedule oracle's (oracle/keyframes.py), frame
  by frame;
* the parameters after the time steps equal those of the same iterations run eagerly
  (forward, L1 loss, backward fused with Adam, per view in the same order), within the
  replay tolerance of the captured Adam step (the single captured step is checked against
  the Adam oracle in test_gpu_adam.py);
* every view's graph is captured once and replayed for its later iterations.
"""
import sys

import numpy as np
import pytest

import scenes
from oracle import keyframes as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from parity_util import to_dev  # noqa: E402

GROUPS = ("means", "scales", "quats", "opacities", "sh")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_12677_amd import rasterize
    return rasterize


def frames():
    """cfg1's Gaussians seen from six poses around the scene, with seeded targets."""
    w = scenes.make_cfg1()
    rng = np.random.default_rng(12)
    cams = []
    for i in range(6):
        pos = [0.3 * np.cos(i), 0.2 * np.sin(i), -0.2 - 0.05 * i]
        R1, t1 = scenes.look_at(pos, [0.0, 0.0, 3.0], up=(0, -1, 0))
        W, H = (96, 72) if i % 2 else (80, 64)
        cams.append(scenes.Camera(W, H, 80.0, 80.0, W / 2 + 0.3, H / 2 - 0.2, R1, t1))
    targets = [(rng.random((3, c.height, c.width)).astype(np.float32),
                (1 + 3 * rng.random((c.height, c.width))).astype(np.float32)) for c in cams]
    return w.gaussians, cams, targets


@pytest.mark.parametrize("m,n,store_all", [(5, 2, False), (4, 1, True)])
def test_time_steps_as_captured_iterations(R, m, n, store_all):
    g, cams, targets = frames()
    tg = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in targets]
    counts = [120, 10, 80, 5, 3, 200]          # Gaussians each frame's seeding added
    s = R.Settings()
    params = to_dev(g)
    start = [p.clone() for p in params]
    opt = R.Adam(*params)
    steps = R.KeyframeSteps(*params, cams, tg, opt, R.Schedule(m, n, threshold=50, store_all=store_all, seed=7), s)
    ref = K.Schedule(m, n, 50, store_all=store_all, seed=7)
    for f, c in enumerate(counts):
        kf, iters = steps.step(f, c)
        rkf, riters = ref.step(f, c)
        assert (kf, iters) == (rkf, riters), f
    steps.sync()
    say("iterations", steps.iterations, "graphs", sorted(steps.graphs))
    assert opt.steps == len(steps.iterations)
    assert sorted(steps.graphs) == sorted(set(steps.iterations))
    # the same iterations, eager
    eparams = [p.clone() for p in start]
    eopt = R.Adam(*eparams)
    for f in steps.iterations:
        images, saved = R.forward(*eparams, [cams[f]], s)
        _, gc, gd = R.loss_l1(saved, images, [tg[f]], 0.1)
        R.backward_adam(saved, eopt, gc, gd)
        saved.free()
    torch.cuda.synchronize()
    assert eopt.steps == opt.steps
    for k, a, b, s0 in zip(GROUPS, params, eparams, start):
        moved = (b - s0).abs()
        assert float(moved.max()) > 0.0, k
        diff = (a - b).abs()
        assert bool((diff <= 1e-3 * moved + 1e-6 * b.abs() + 1e-7).all()), (k, float((diff - 1e-3 * moved).max()))
    steps.free()
