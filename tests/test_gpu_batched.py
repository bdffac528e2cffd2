"""Batched keyframes (several views in one captured step) and the launch-shape autotuner.

* batched forward == per-view forward bitwise; batched gradients == sum of per-view
  gradients (float atomics reorder sums: relative 1e-5);
* graph replays == the eager step (images bitwise, gradients relative 1e-5), replayed
  several times with eager work and synchronisations in between;
* the batched step matches the oracle (bit-exact keys, images 1e-4, gradients 1e-3);
* a capacity overflow is reported as GSR_ECAPACITY and every kernel still exits normally;
* the autotuner picks one of the six launch shapes and caches it.
"""
import os
import sys

import numpy as np
import pytest

import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from parity_util import (check_grads, check_images, check_keys, check_loss_grads, oracle_for,  # noqa: E402
                         oracle_loss, settings, to_dev)

NAMES = ("means", "scales", "quats", "opacities", "sh")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_12677_amd import rasterize
    return rasterize


def small_views():
    """cfg1's Gaussians seen by three cameras of uneven size, with seeded targets."""
    w = scenes.make_cfg1()
    c = w.cameras[0]
    R1, t1 = scenes.look_at([0.2, 0.1, -0.3], [0.0, 0.0, 3.0], up=(0, -1, 0))
    cams = [c, scenes.Camera(100, 75, 90.0, 90.0, 50.3, 37.6, R1, t1), c.crop(13, 7, 37, 29)]
    rng = np.random.default_rng(8)
    targets = [(rng.random((3, k.height, k.width)).astype(np.float32),
                (1 + 3 * rng.random((k.height, k.width))).astype(np.float32)) for k in cams]
    return w.gaussians, cams, targets


def dev_targets(targets):
    return [(torch.from_numpy(tc).cuda(), torch.from_numpy(td).cuda()) for tc, td in targets]


def eager_step(R, params, cams, targets, s):
    images, saved = R.forward(*params, cams, s)
    loss, gc, gd = R.loss_l1(saved, images, targets, 0.1)
    grads = R.backward(saved, gc, gd)
    torch.cuda.synchronize()
    return images, loss, grads, saved


def close(ga, gb, tol=1e-5):
    """Per group ||a - b|| <= tol * max(||b||, 1e-2 ||b over all groups||): a group that is
    negligible in the whole gradient (the rotation gradient of isotropic Gaussians is zero
    analytically, so two atomic orders give different noise) is judged on the whole scale."""
    to = lambda t: t.detach().cpu().numpy().astype(np.float64)
    allb = np.sqrt(sum(np.linalg.norm(to(gb[k])) ** 2 for k in NAMES))
    for k in NAMES:
        a, b = to(ga[k]), to(gb[k])
        r = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-2 * allb, 1e-30)
        assert r <= tol, (k, r)


def _shifted(t):
    """A copy of t whose data starts one float past a 16-byte boundary."""
    buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
    out = buf[1:].view(t.shape)
    out.copy_(t)
    return out


def test_misaligned_sh_arrays_take_the_scalar_paths(R):
    """SH coefficients and an SH gradient output one float off a 16-byte boundary go
    through the kernels' scalar paths (the projection's coefficient loads, the backward's
    staging and gradient stores): the same images bit for bit and the same gradients up to
    the backward's atomic summation order as with aligned arrays."""
    g, cams, targets = small_views()
    params = to_dev(g)
    tg = dev_targets(targets)
    s = settings()
    a_images, _, a_grads, _ = eager_step(R, params, cams, tg, s)
    shifted = list(params[:4]) + [_shifted(params[4])]
    images, saved = R.forward(*shifted, cams, s)
    _, gc, gd = R.loss_l1(saved, images, tg, 0.1)
    grads = {k: torch.empty_like(p) for k, p in zip(NAMES, params)}
    grads["sh"] = _shifted(torch.zeros_like(params[4]))
    R.backward(saved, gc, gd, grads=grads)
    torch.cuda.synchronize()
    for a, b in zip(a_images, images):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    close(grads, a_grads)


def test_batched_equals_per_view(R):
    g, cams, targets = small_views()
    params = to_dev(g)
    tg = dev_targets(targets)
    s = settings()
    images, loss, grads, _ = eager_step(R, params, cams, tg, s)
    acc = None
    for i, c in enumerate(cams):
        im1, l1, g1, _ = eager_step(R, params, [c], [tg[i]], s)
        for a, b in zip(images[i], im1[0]):
            assert torch.equal(a, b)
        acc = g1 if acc is None else {k: acc[k] + g1[k] for k in acc}
    close(grads, acc)


def test_batched_step_matches_oracle(R):
    g, cams, targets = small_views()
    params = to_dev(g)
    s = settings()
    images, loss, grads, saved = eager_step(R, params, cams, dev_targets(targets), s)
    orc = oracle_for(g, cams, s)
    check_keys(saved.debug_export(), orc)
    outs = orc.forward()
    check_images(images, outs)
    _, gc, gd = R.loss_l1(saved, images, dev_targets(targets), 0.1)
    L, ref_gc, ref_gd, amb = oracle_loss(outs, targets, 0.1)
    check_loss_grads(gc, gd, ref_gc, ref_gd, amb)
    ref = orc.backward(ref_gc, ref_gd, None, ambiguous_pixels=amb)
    check_grads(grads, ref)


def test_graph_replays_match_eager(R):
    g, cams, targets = small_views()
    params = to_dev(g)
    tg = dev_targets(targets)
    s = settings()
    e_images, e_loss, e_grads, _ = eager_step(R, params, cams, tg, s)
    graph = R.Graph(*params, cams, tg, s)
    say("graph info", graph.info())
    for rep in range(4):
        graph.launch()
        graph.sync()
        for a, b in zip(graph.images, e_images):
            for x, y in zip(a, b):
                assert torch.equal(x, y), f"replay {rep}"
        close(graph.grads, e_grads)
        assert float(graph.loss) == pytest.approx(float(e_loss), rel=1e-5)
        eager_step(R, params, cams[:1], tg[:1], s)   # unrelated eager work between replays
    graph.free()


def test_graph_follows_parameter_updates(R):
    g, cams, targets = small_views()
    params = to_dev(g)
    tg = dev_targets(targets)
    s = settings()
    graph = R.Graph(*params, cams, tg, s)
    graph.launch()
    graph.sync()
    with torch.no_grad():       # a gradient-descent step in place, then replay
        params[0].add_(graph.grads["means"], alpha=-1e-3)
        params[4].add_(graph.grads["sh"], alpha=-1e-1)
    graph.launch()
    graph.sync()
    e_images, e_loss, e_grads, _ = eager_step(R, params, cams, tg, s)
    for a, b in zip(graph.images, e_images):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    close(graph.grads, e_grads)
    graph.free()


def test_graph_capacity_overflow_is_reported(R):
    # capture with capacities sized for tiny splats, then grow every splat 2000x in place:
    # the step needs ~108k keys against ~9k of capacity (oracle counts: 5,355 at scale
    # 0.01, 108,512 at 20); kernels stop at the capacity, the flag is raised and read back
    from paper_2408_12677_amd._native import GsrError, ECAPACITY
    g, cams, targets = small_views()
    params = to_dev(g)
    tg = dev_targets(targets)
    s = settings()
    with torch.no_grad():
        params[1].mul_(0.01)
    graph = R.Graph(*params, cams, tg, s, headroom=0.0)
    info = graph.info()
    assert info["capacity_keys"] < 20000
    with torch.no_grad():
        params[1].mul_(2000.0)
    graph.launch()
    with pytest.raises(GsrError) as ei:
        graph.sync()
    assert ei.value.status == ECAPACITY
    with pytest.raises(GsrError):
        graph.launch()
    graph.free()
    torch.cuda.synchronize()
    # the device is still healthy: an eager step right after works and matches the oracle keys
    images, loss, grads, saved = eager_step(R, params, cams, tg, s)
    assert saved.info()["num_keys"] > 100000
    say("overflow test capacities", info)


def test_graph_overflow_with_fused_adam_leaves_parameters_unchanged(R):
    # the same forced overflow, with the optimiser step fused into the captured step and two
    # launches queued back to back: both are reported, and neither moves a parameter, a
    # moment or the step counter (the overflow word is sticky across launches)
    from paper_2408_12677_amd._native import GsrError, ECAPACITY
    g, cams, targets = small_views()
    params = to_dev(g)
    tg = dev_targets(targets)
    with torch.no_grad():
        params[1].mul_(0.01)
    opt = R.Adam(*params)
    graph = R.Graph(*params, cams, tg, settings(), headroom=0.0, optimizer=opt)
    with torch.no_grad():
        params[1].mul_(2000.0)
    before = [p.clone() for p in params]
    graph.launch()
    try:
        graph.launch()      # may already see the first launch's overflow
    except GsrError as e:
        assert e.status == ECAPACITY
    with pytest.raises(GsrError) as ei:
        graph.sync()
    assert ei.value.status == ECAPACITY
    for a, b in zip(params, before):
        assert torch.equal(a, b)
    assert opt.steps == 0
    for k in NAMES:
        assert not opt.m[k].any() and not opt.v[k].any()
    graph.free()
    torch.cuda.synchronize()


def test_autotune_picks_a_launch_shape_and_caches_it(R, tmp_path, monkeypatch):
    monkeypatch.setenv("GSR_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    g, cams, _ = small_views()
    params = to_dev(g)
    s, ms = R.autotune(*params, cams)
    assert (s.tile, s.batch) in [(t, b) for t in (8, 16, 32) for b in (128, 256)]
    assert ms > 0
    text = (tmp_path / "tune.txt").read_text()
    assert f" {s.tile} {s.batch} " in text
    s2, ms2 = R.autotune(*params, cams)          # served from the cache
    assert (s2.tile, s2.batch) == (s.tile, s.batch) and ms2 == pytest.approx(ms, rel=1e-3)
    say("autotune", s.tile, s.batch, ms)


def test_cfg4_captured_8_view_step_matches_oracle(R):
    # the full-size batched step (8 views of uneven resolution, 4,348,800 pixels, one graph
    # launch) against the oracle's forward, L1 loss and backward of its own images
    w = scenes.make_cfg4()
    params = to_dev(w.gaussians)
    tg = dev_targets(w.targets)
    s = settings(exact_tiles=True)
    graph = R.Graph(*params, w.cameras, tg, s)
    graph.launch()
    graph.sync()
    say("cfg4 graph", graph.info())
    orc = oracle_for(w.gaussians, w.cameras, s, threads=8)
    outs = orc.forward()
    rep = check_images(graph.images, outs)
    L, ref_gc, ref_gd, amb = oracle_loss(outs, w.targets, 0.1)
    assert float(graph.loss) == pytest.approx(L, abs=1.1e-4 * len(w.cameras))
    ref = orc.backward(ref_gc, ref_gd, None, ambiguous_pixels=amb)
    grep = check_grads(graph.grads, ref)
    say("cfg4 8 views vs oracle", rep, grep)
    graph.free()


def test_cfg4_all_views_graph_vs_eager(R):
    w = scenes.make_cfg4()
    params = to_dev(w.gaussians)
    tg = dev_targets(w.targets)
    s = settings()
    say("cfg4 8 views", [(c.width, c.height) for c in w.cameras])
    e_images, e_loss, e_grads, saved = eager_step(R, params, w.cameras, tg, s)
    inf = saved.info()
    saved.free()
    graph = R.Graph(*params, w.cameras, tg, s)
    for rep in range(2):
        graph.launch()
        graph.sync()
        for a, b in zip(graph.images, e_images):
            for x, y in zip(a, b):
                assert torch.equal(x, y)
        close(graph.grads, e_grads)
    say("cfg4 batched", inf, graph.info())
    graph.free()


def test_graph_with_exact_tiles_matches_eager(R):
    g, cams, targets = small_views()
    params = to_dev(g)
    tg = dev_targets(targets)
    s = settings(exact_tiles=True)
    e_images, e_loss, e_grads, _ = eager_step(R, params, cams, tg, s)
    b_images, _, _, _ = eager_step(R, params, cams, tg, settings())
    for a, b in zip(e_images, b_images):          # the same images as the rectangle lists
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    graph = R.Graph(*params, cams, tg, s)
    for rep in range(3):
        graph.launch()
        graph.sync()
        for a, b in zip(graph.images, e_images):
            for x, y in zip(a, b):
                assert torch.equal(x, y), f"replay {rep}"
        close(graph.grads, e_grads)
    graph.free()
