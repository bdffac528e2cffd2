"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances and the ambiguity rule are stated in parity_util.  Every input is a
seeded synthetic workload from ``scenes``.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from parity_util import (IMG_TOL, check_grads, check_images, check_keys, check_loss_grads,  # noqa: E402
                         check_records, oracle_for, oracle_loss, settings, to_dev)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_12677_amd import rasterize
    return rasterize


def run_fwd(R, g, cams, s, save=True):
    params = to_dev(g)
    images, saved = R.forward(*params, cams, s, save=save)
    torch.cuda.synchronize()
    return params, images, saved


def fwd_bwd_parity(R, g, cams, s, targets=None, threads=8, check_key=True):
    params, images, saved = run_fwd(R, g, cams, s)
    dbg = saved.debug_export()
    orc = oracle_for(g, cams, s, threads=threads)
    if check_key:
        check_keys(dbg, orc)
        check_records(dbg, orc, s.tile)
    outs = orc.forward()
    rep = check_images(images, outs, dbg, cams)
    # output gradients: each side's own L1 loss of its own images (when targets are
    # given), else the same seeded random arrays on both sides
    if targets is not None:
        tg = [(torch.from_numpy(tc).cuda(), torch.from_numpy(td).cuda()) for tc, td in targets]
        loss, gc, gd = R.loss_l1(saved, images, tg, 0.1)
        L, ref_gc, ref_gd, amb = oracle_loss(outs, targets, 0.1)
        check_loss_grads(gc, gd, ref_gc, ref_gd, amb)
        assert float(loss) == pytest.approx(L, abs=1.1 * IMG_TOL * len(cams))
        grads = R.backward(saved, gc, gd)
        ref = orc.backward(ref_gc, ref_gd, None, ambiguous_pixels=amb)
    else:
        rng = np.random.default_rng(7)
        hgc = [rng.standard_normal((3, c.height, c.width)).astype(np.float32) for c in cams]
        hgd = [rng.standard_normal((c.height, c.width)).astype(np.float32) for c in cams]
        hga = [rng.standard_normal((c.height, c.width)).astype(np.float32) for c in cams]
        dev = lambda lst: [torch.from_numpy(a).cuda() for a in lst]
        grads = R.backward(saved, dev(hgc), dev(hgd), dev(hga))
        ref = orc.backward(hgc, hgd, hga)
    torch.cuda.synchronize()
    grep = check_grads(grads, ref)
    saved.free()
    return rep, grep


# ---------------------------------------------------------------------------------------
# forward: keys, order, ranges bit-exact; images within 1e-4
# ---------------------------------------------------------------------------------------

def test_cfg1_forward_parity(R):
    w = scenes.make_cfg1()
    s = settings()
    say("cfg1 forward", w.gaussians.n)
    params, images, saved = run_fwd(R, w.gaussians, w.cameras, s)
    dbg = saved.debug_export()
    orc = oracle_for(w.gaussians, w.cameras, s)
    check_keys(dbg, orc)
    check_records(dbg, orc, s.tile)
    rep = check_images(images, orc.forward(), dbg, w.cameras)
    assert dbg["keys"].size > 1000
    say("cfg1", rep, saved.info())


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_keys_bitexact_every_tile_size(R, tile, exact):
    w = scenes.make_cfg1()
    s = settings(tile=tile, exact_tiles=exact)
    say("keys tile", tile, "exact", exact)
    _, _, saved = run_fwd(R, w.gaussians, w.cameras, s)
    dbg = saved.debug_export()
    check_keys(dbg, oracle_for(w.gaussians, w.cameras, s))


def test_forward_bitwise_invariant_across_autotune_points(R):
    w = scenes.make_cfg1()
    cams = w.cameras + [w.cameras[0].crop(5, 3, 77, 61)]
    say("autotune invariance")
    ref = None
    for tile in (8, 16, 32):
        for batch, exact in ((128, False), (256, False), (128, True), (256, True)):
            _, images, _ = run_fwd(R, w.gaussians, cams, settings(tile=tile, batch=batch, exact_tiles=exact),
                                   save=False)
            cur = [t.cpu().numpy() for img in images for t in img]
            if ref is None:
                ref = cur
            else:
                for a, b in zip(ref, cur):
                    np.testing.assert_array_equal(a, b)


def test_forward_is_deterministic(R):
    w = scenes.make_cfg1()
    s = settings()
    _, a, _ = run_fwd(R, w.gaussians, w.cameras, s, save=False)
    _, b, _ = run_fwd(R, w.gaussians, w.cameras, s, save=False)
    for x, y in zip(a[0], b[0]):
        assert torch.equal(x, y)


def test_work_ordered_queue_leaves_results_unchanged(R):
    """A forward over the same tiles as an earlier one orders its tile queue by the earlier
    one's per-tile work and raises the heaviest tiles' wave priority: scheduling only, so
    the images and every per-pixel count are bit-identical to a forward without that
    order (the first one over a tile grid no other test uses)."""
    w = scenes.make_cfg1()
    cam = w.cameras[0].crop(5, 3, 117, 89)   # a grid of its own: the first forward has no order hint
    s = settings(tile=8)
    _, a, sa = run_fwd(R, w.gaussians, [cam], s)
    da = sa.debug_export()
    _, b, sb = run_fwd(R, w.gaussians, [cam], s)
    db = sb.debug_export()
    for x, y in zip(a[0], b[0]):
        assert torch.equal(x, y)
    for k in ("n_contrib", "n_used", "T_final", "ranges", "values"):
        np.testing.assert_array_equal(da[k], db[k], err_msg=k)
    sa.free()
    sb.free()


# ---------------------------------------------------------------------------------------
# forward + backward
# ---------------------------------------------------------------------------------------

def test_cfg1_fwd_bwd_random_output_grads(R):
    w = scenes.make_cfg1()
    say("cfg1 fwd+bwd")
    rep, grep = fwd_bwd_parity(R, w.gaussians, w.cameras, settings(bg=(0.1, 0.3, 0.2)))
    say("cfg1 bwd", rep, grep)


def test_multiview_uneven_ragged(R):
    w = scenes.make_cfg1()
    c = w.cameras[0]
    R1, t1 = scenes.look_at([0.2, 0.1, -0.3], [0.0, 0.0, 3.0], up=(0, -1, 0))
    cams = [c, scenes.Camera(100, 75, 90.0, 90.0, 50.3, 37.6, R1, t1), c.crop(13, 7, 37, 29)]
    say("multiview ragged")
    rep, grep = fwd_bwd_parity(R, w.gaussians, cams, settings())
    say(rep, grep)


@pytest.mark.parametrize("tile,batch", [(8, 128), (32, 256)])
def test_multiview_other_launch_shapes(R, tile, batch):
    w = scenes.make_cfg1()
    c = w.cameras[0]
    cams = [c, c.crop(20, 10, 50, 40)]
    fwd_bwd_parity(R, w.gaussians, cams, settings(tile=tile, batch=batch))


LAUNCH_SHAPES = [(t, b, e) for t in (8, 16, 32) for b in (128, 256) for e in (False, True)]


@pytest.mark.parametrize("tile,batch,exact", LAUNCH_SHAPES)
def test_every_launch_shape_multiview(R, tile, batch, exact):
    # every (tile, batch, list kind) the autotuner can pick: each compositing kernel variant
    w = scenes.make_cfg1()
    c = w.cameras[0]
    R1, t1 = scenes.look_at([0.2, 0.1, -0.3], [0.0, 0.0, 3.0], up=(0, -1, 0))
    cams = [c, scenes.Camera(100, 75, 90.0, 90.0, 50.3, 37.6, R1, t1), c.crop(13, 7, 37, 29)]
    say("launch shape", tile, batch, exact)
    rep, grep = fwd_bwd_parity(R, w.gaussians, cams, settings(tile=tile, batch=batch, exact_tiles=exact))
    say(rep, grep)


@pytest.mark.parametrize("tile,batch,exact", LAUNCH_SHAPES)
def test_every_launch_shape_cfg2_with_loss(R, tile, batch, exact):
    w = scenes.make_cfg2()
    say("cfg2 launch shape", tile, batch, exact)
    rep, grep = fwd_bwd_parity(R, w.gaussians, w.cameras, settings(tile=tile, batch=batch, exact_tiles=exact),
                               targets=w.targets)
    say(rep, grep)


def test_cfg2_fwd_bwd_with_l1_loss(R):
    w = scenes.make_cfg2()
    say("cfg2", w.gaussians.n)
    rep, grep = fwd_bwd_parity(R, w.gaussians, w.cameras, settings(), targets=w.targets)
    say("cfg2", rep, grep)


def test_cfg3_crop_fwd_bwd(R):
    w = scenes.make_cfg3()
    rng = np.random.default_rng(33)
    cam = w.cameras[0]
    x0, y0 = int(rng.integers(0, cam.width - 64)), int(rng.integers(0, cam.height - 64))
    crop = cam.crop(x0, y0, 64, 64)
    rec = oracle.Oracle(w.gaussians.arrays(), 3, [crop], oracle.Settings(threads=8)).records()
    idx = np.nonzero(rec["visible"])[0]
    pick = np.sort(rng.choice(idx, size=min(2000, idx.size), replace=False))
    g = w.gaussians.subset(pick)
    say("cfg3 crop", x0, y0, g.n)
    rep, grep = fwd_bwd_parity(R, g, [crop], settings())
    say("cfg3", rep, grep)


def test_loss_kernel_matches_oracle(R):
    w = scenes.make_cfg1()
    s = settings()
    params, images, saved = run_fwd(R, w.gaussians, w.cameras, s)
    rng = np.random.default_rng(4)
    tc = rng.random((3, 96, 128)).astype(np.float32)
    td = (rng.random((96, 128)) * 5).astype(np.float32)
    td[:10] = 0.0
    loss, gc, gd = R.loss_l1(saved, images, [(torch.from_numpy(tc).cuda(), torch.from_numpy(td).cuda())], 0.1)
    # the oracle's loss of the oracle's images: |dL| <= mean |dC| + 0.1 mean |dD|
    L, ref_gc, ref_gd, amb = oracle_loss(oracle_for(w.gaussians, w.cameras, s).forward(), [(tc, td)], 0.1)
    assert float(loss) == pytest.approx(L, abs=1.1 * IMG_TOL)
    check_loss_grads(gc, gd, ref_gc, ref_gd, amb)
    assert not (gd[0][:10] != 0).any()       # rows without a target depth


def test_autograd_function_matches_direct_backward(R):
    w = scenes.make_cfg1()
    s = settings()
    params = [p.clone().requires_grad_(True) for p in to_dev(w.gaussians)]
    out = R.render(*params, w.cameras, s)
    col, dep, alp = out[0]
    loss = col.square().mean() + 0.3 * dep.mean() + 0.2 * alp.sum()
    loss.backward()
    P = col.shape[1] * col.shape[2]
    gc = [2 * col.detach() / (3 * P)]
    gd = [torch.full_like(dep, 0.3 / P)]
    ga = [torch.full_like(alp, 0.2)]
    _, _, saved = run_fwd(R, w.gaussians, w.cameras, s)
    direct = R.backward(saved, gc, gd, ga)
    for name, p in zip(("means", "scales", "quats", "opacities", "sh"), params):
        a, b = p.grad.cpu().numpy(), direct[name].cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b) + 1e-12, name


def test_backward_accumulate_flag(R):
    w = scenes.make_cfg1()
    _, images, saved = run_fwd(R, w.gaussians, w.cameras, settings())
    gc = [torch.ones_like(images[0][0])]
    a = R.backward(saved, gc)
    b = {k: v.clone() for k, v in a.items()}
    R.backward(saved, gc, grads=b, accumulate=True)
    # the two backward runs add their float atomics in different orders, so an element
    # made of cancelling terms can differ in its last bits: the floor scales with the array
    for k in a:
        ak = a[k].cpu().numpy()
        np.testing.assert_allclose(b[k].cpu().numpy(), 2 * ak, rtol=1e-4, atol=1e-6 * float(np.abs(ak).max()) + 1e-9)


# ---------------------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------------------

def _one(R, g, cams, s):
    params, images, saved = run_fwd(R, g, cams, s)
    return params, images, saved


def test_empty_map(R):
    g = scenes.random_gaussians(np.random.default_rng(0), np.zeros((0, 3)), 0)
    cam = scenes.Camera(40, 30, 30.0, 30.0, 20.0, 15.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))
    s = settings(bg=(0.25, 0.5, 0.75))
    _, images, saved = _one(R, g, [cam], s)
    col, dep, alp = (t.cpu().numpy() for t in images[0])
    assert np.all(col[0] == 0.25) and np.all(col[2] == 0.75) and np.all(dep == 0) and np.all(alp == 0)
    assert saved.info()["num_keys"] == 0
    grads = R.backward(saved, [torch.ones(3, 30, 40, device="cuda")])
    assert grads["means"].numel() == 0


def test_everything_culled(R):
    rng = np.random.default_rng(1)
    g = scenes.random_gaussians(rng, np.stack([rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50), -rng.uniform(1, 3, 50)], 1), 3)
    cam = scenes.Camera(33, 17, 30.0, 30.0, 16.0, 8.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))
    _, images, saved = _one(R, g, [cam], settings())
    assert saved.info()["num_keys"] == 0
    assert float(images[0][2].abs().max()) == 0.0
    grads = R.backward(saved, [torch.ones(3, 17, 33, device="cuda")], [torch.ones(17, 33, device="cuda")])
    for k, v in grads.items():
        assert float(v.abs().max()) == 0.0, k


def test_single_pixel_and_huge_splat(R):
    # one Gaussian much larger than the image plus a tiny camera, with opacity above the clamp
    means = np.array([[0.0, 0.0, 2.0], [0.01, 0.0, 3.0]])
    g = scenes.random_gaussians(np.random.default_rng(2), means, 1)
    g.scales[:] = np.array([[2.0, 1.5, 1.0], [0.01, 0.01, 0.01]], np.float32)
    g.opacities[:] = np.array([0.999, 0.5], np.float32)
    for W, H in ((1, 1), (17, 9), (64, 48)):
        cam = scenes.Camera(W, H, 40.0, 40.0, W / 2, H / 2, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))
        fwd_bwd_parity(R, g, [cam], settings())


def test_lists_past_the_last_checkpoint(R):
    # 2,000 faint splats over the whole image: every pixel takes some 1,500 of them before
    # its transmittance stops, so the backward's items past the forward's last checkpoint
    # (list entry 1,024 on) walk several staged strides back from the final state
    rng = np.random.default_rng(11)
    n = 2000
    means = np.stack([rng.uniform(-0.2, 0.2, n), rng.uniform(-0.1, 0.1, n), rng.uniform(2.0, 6.0, n)], 1)
    g = scenes.random_gaussians(rng, means, 1)
    g.scales[:] = rng.uniform(8.0, 12.0, (n, 3)).astype(np.float32)
    g.opacities[:] = rng.uniform(0.0055, 0.0065, n).astype(np.float32)
    cam = scenes.Camera(40, 24, 30.0, 30.0, 20.0, 12.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))
    for tile, exact in ((16, False), (16, True), (8, False), (32, True)):
        s = settings(tile=tile, exact_tiles=exact)
        _, _, saved = run_fwd(R, g, [cam], s)
        longest = int(np.asarray(saved.debug_export()["n_contrib"]).max())
        saved.free()
        say("tile", tile, "exact", exact, "longest contributor list", longest)
        assert longest > 1100
        fwd_bwd_parity(R, g, [cam], s)


def test_invalid_arguments_raise(R):
    w = scenes.make_cfg1()
    params = to_dev(w.gaussians)
    with pytest.raises(ValueError):
        R.forward(params[0].double(), *params[1:], w.cameras)
    from paper_2408_12677_amd._native import GsrError
    with pytest.raises(GsrError):
        R.forward(*params, w.cameras, settings(tile=12))
    bad = scenes.Camera(0, 10, 1.0, 1.0, 0.0, 0.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))
    with pytest.raises(GsrError):
        R.forward(*params, [bad])


def test_check_finite_names_the_first_bad_gaussian(R):
    w = scenes.make_cfg1()
    base = to_dev(w.gaussians)
    s = settings(check_finite=True)
    _, saved = R.forward(*base, w.cameras, s)     # all finite: renders as usual
    saved.free()
    from paper_2408_12677_amd._native import GsrError
    for group, idx, val in ((0, (1234, 2), float("nan")), (4, (17, 0, 1), float("inf")), (3, (1999,), float("-inf"))):
        params = [p.clone() for p in base]
        params[group][idx] = val
        params[4][1500, 0, 0] = float("nan")   # a later bad Gaussian
        with pytest.raises(GsrError, match=f"Gaussian {min(idx[0], 1500)} has a NaN"):
            R.forward(*params, w.cameras, s)
        # without the check the values propagate and the call succeeds
        _, saved = R.forward(*params, w.cameras, settings())
        saved.free()
    # the context stays usable
    images, saved = R.forward(*base, w.cameras, s)
    torch.cuda.synchronize()
    assert all(torch.isfinite(t).all() for t in images[0])
    saved.free()


# ---------------------------------------------------------------------------------------
# full size: the headline 640x480 view of the 500k-Gaussian map, in the bench launch shape
# ---------------------------------------------------------------------------------------

def test_headline_view_full_size(R):
    w = scenes.make_cfg4()
    v = scenes.HEADLINE_VIEW
    cam = w.cameras[v]
    say("headline", w.gaussians.n, cam.width, cam.height)
    rep, grep = fwd_bwd_parity(R, w.gaussians, [cam], settings(), targets=[w.targets[v]], threads=8)
    say("headline", rep, grep)


def test_cfg5_full_view_checked_on_a_window(R):
    # one 1752x1168 view of the 3M-Gaussian map rendered whole; keys bit-exact over the whole
    # view, images and gradients against the oracle on a 256x192 window (output gradients
    # vanish outside it, so the GPU's full backward is the window's)
    w = scenes.make_cfg5()
    cam = w.cameras[0]
    s = settings(exact_tiles=True)
    say("cfg5 view", w.gaussians.n, cam.width, cam.height)
    params, images, saved = run_fwd(R, w.gaussians, [cam], s)
    dbg = saved.debug_export()
    rng = np.random.default_rng(55)
    x0, y0 = int(rng.integers(0, cam.width - 256)), int(rng.integers(0, cam.height - 192))
    win = (x0, y0, x0 + 256, y0 + 192)
    os_ = oracle.Settings(tile=s.tile, mu_fp32=True, threads=8, exact_tiles=True, window=win)
    orc = oracle.Oracle(w.gaussians.arrays(), w.gaussians.sh_degree, [cam], os_)
    check_keys(dbg, orc)
    o = orc.forward()[0]
    sl = (slice(y0, y0 + 192), slice(x0, x0 + 256))
    cut = lambda a: {k: (v[(slice(None),) + sl] if k in ("color", "lo", "hi") else v[sl])
                     for k, v in a.items() if isinstance(v, np.ndarray)}
    oc = cut(o)
    col, dep, alp = images[0]
    crop_imgs = [(col[:, sl[0], sl[1]], dep[sl], alp[sl])]
    rep = check_images(crop_imgs, [oc])
    H, W = cam.height, cam.width
    lengths = np.diff(dbg["ranges"].astype(np.int64), axis=1)[:, 0]
    say("cfg5 window", win, rep, "list length p50/p99", np.percentile(lengths, 50), np.percentile(lengths, 99))
    gC = np.zeros((3, H, W), np.float32)
    gD = np.zeros((H, W), np.float32)
    gC[(slice(None),) + sl] = rng.standard_normal((3, 192, 256))
    gD[sl] = rng.standard_normal((192, 256))
    grads = R.backward(saved, [torch.from_numpy(gC).cuda()], [torch.from_numpy(gD).cuda()])
    torch.cuda.synchronize()
    ref = orc.backward([gC], [gD], None)
    grep = check_grads(grads, ref)
    say("cfg5 window grads", grep)
    saved.free()


# ---------------------------------------------------------------------------------------
# exact ellipse-tile culling: shorter lists, the same images and gradients
# ---------------------------------------------------------------------------------------

def test_exact_tiles_multiview_fwd_bwd(R):
    w = scenes.make_cfg1()
    c = w.cameras[0]
    R1, t1 = scenes.look_at([0.2, 0.1, -0.3], [0.0, 0.0, 3.0], up=(0, -1, 0))
    cams = [c, scenes.Camera(100, 75, 90.0, 90.0, 50.3, 37.6, R1, t1), c.crop(13, 7, 37, 29)]
    for tile in (8, 16):
        say("exact tiles multiview, tile", tile)
        rep, grep = fwd_bwd_parity(R, w.gaussians, cams, settings(tile=tile, exact_tiles=True))
        say(rep, grep)


def test_exact_tiles_cfg2_with_loss(R):
    w = scenes.make_cfg2()
    s = settings(exact_tiles=True)
    rep, grep = fwd_bwd_parity(R, w.gaussians, w.cameras, s, targets=w.targets)
    _, _, box = run_fwd(R, w.gaussians, w.cameras, settings())
    _, _, ex = run_fwd(R, w.gaussians, w.cameras, s)
    nb, ne = len(box.debug_export()["keys"]), len(ex.debug_export()["keys"])
    say("cfg2 exact tiles", rep, grep, "pairs", nb, "->", ne)
    assert ne < nb


def test_headline_view_full_size_exact_tiles(R):
    w = scenes.make_cfg4()
    v = scenes.HEADLINE_VIEW
    cam = w.cameras[v]
    rep, grep = fwd_bwd_parity(R, w.gaussians, [cam], settings(exact_tiles=True), targets=[w.targets[v]],
                               threads=8)
    say("headline exact tiles", rep, grep)


# ---------------------------------------------------------------------------------------
# the guard-band clamp of the projection's Jacobian on off-centre cameras
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("tile,exact", [(8, False), (16, True)])
def test_jacobian_clamp_offcentre_crops(R, tile, exact):
    # crops whose principal points lie far from their centres (one outside the image): the
    # clamp at 1.3 half fields of view acts on many rendered splats
    w = scenes.make_cfg1()
    c = w.cameras[0]
    cams = [c.crop(0, 0, 40, 30), c.crop(80, 60, 48, 36), c.crop(88, 8, 40, 44)]
    s = settings(tile=tile, exact_tiles=exact, jclamp=1.3)
    plain = oracle_for(w.gaussians, cams, settings(tile=tile, exact_tiles=exact)).forward()
    clamped = oracle_for(w.gaussians, cams, s).forward()
    moved = max(float(np.abs(a["color"] - b["color"]).max()) for a, b in zip(plain, clamped))
    say("clamp", tile, exact, "largest image change by the clamp", moved)
    assert moved > 1e-3
    rep, grep = fwd_bwd_parity(R, w.gaussians, cams, s)
    say(rep, grep)


def test_jacobian_clamp_cfg3_crop_with_loss(R):
    w = scenes.make_cfg3()
    cam = w.cameras[0]
    crop = cam.crop(1100, 560, 64, 64)   # near the corner: x/z, y/z beyond the crop's limits
    rec = oracle.Oracle(w.gaussians.arrays(), 3, [crop], oracle.Settings(threads=8, jclamp=1.3)).records()
    idx = np.nonzero(rec["visible"])[0]
    pick = np.sort(np.random.default_rng(34).choice(idx, size=min(2000, idx.size), replace=False))
    g = w.gaussians.subset(pick)
    rng = np.random.default_rng(35)
    targets = [(rng.random((3, 64, 64)).astype(np.float32), (1 + 4 * rng.random((64, 64))).astype(np.float32))]
    rep, grep = fwd_bwd_parity(R, g, [crop], settings(jclamp=1.3), targets=targets)
    say("cfg3 clamp crop", g.n, rep, grep)


# ---------------------------------------------------------------------------------------
# variants: normalised depth output, a 3-sigma (lossy) splat extent
# ---------------------------------------------------------------------------------------

def test_normalized_depth_fwd_bwd(R):
    w = scenes.make_cfg1()
    c = w.cameras[0]
    cams = [c, c.crop(9, 5, 61, 47)]
    say("normalised depth, random output gradients")
    rep, grep = fwd_bwd_parity(R, w.gaussians, cams, settings(normalized_depth=True, bg=(0.2, 0.1, 0.0)))
    say(rep, grep)
    w2 = scenes.make_cfg2()
    say("normalised depth, cfg2 with loss")
    rep, grep = fwd_bwd_parity(R, w2.gaussians, w2.cameras, settings(normalized_depth=True, exact_tiles=True),
                               targets=w2.targets)
    say(rep, grep)


def test_lossy_extent_three_sigma(R):
    # extent k = 3 < sqrt(2 ln 255): rectangles cut splat tails that would pass the skip
    # rule, so the images depend on the tiles; the oracle follows the same rectangles
    w = scenes.make_cfg1()
    for tile in (8, 16):
        s = settings(tile=tile, extent_k=3.0)
        say("extent 3, tile", tile)
        rep, grep = fwd_bwd_parity(R, w.gaussians, w.cameras, s)
        say(rep, grep)
