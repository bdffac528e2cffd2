"""GPU optimiser step (gsr_adam_step, gsr_backward_adam, a graph with the optimiser)
against the FP64 optimiser oracle (oracle/adam.py) on seeded inputs.

Tolerances:
  * standalone step, same seeded gradients on both sides: per element
    |x - x_ref| <= 2e-5 |x_ref| + 1e-4 lr (binary32 arithmetic of a few steps, log/exp of
    the activated groups), moments within 2e-5 relative of their group's scale;
  * fused with the backward: the parameter gradient itself carries the backward's
    tolerance (parity_util: 1e-3 relative, Gaussians near a discrete decision excepted),
    so each element may differ by that gradient error carried through one Adam step
    (its derivative with respect to the gradient, bounded from the oracle's own values)
    plus the rounding above.
"""
import sys

import numpy as np
import pytest

import scenes
from oracle import adam as A

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from parity_util import GRAD_REL, oracle_for, settings, to_dev  # noqa: E402

GROUPS = A.GROUPS


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_12677_amd import rasterize
    return rasterize


def _params(rng, n, deg):
    K = (deg + 1) ** 2
    return dict(means=rng.standard_normal((n, 3)).astype(np.float32),
                scales=np.exp(rng.uniform(-5, -1, (n, 3))).astype(np.float32),
                quats=rng.standard_normal((n, 4)).astype(np.float32),
                opacities=rng.uniform(0.05, 0.95, n).astype(np.float32),
                sh=(rng.standard_normal((n, K, 3)) * 0.3).astype(np.float32))


def _grads(rng, p):
    g = {}
    for k in GROUPS:
        a = rng.standard_normal(p[k].shape) * 10.0 ** rng.uniform(-6, 0, p[k].shape)
        a[rng.random(p[k].shape) < 0.05] = 0.0
        g[k] = a.astype(np.float32)
    return g


def _dev(d, keys=GROUPS):
    return {k: torch.from_numpy(np.ascontiguousarray(d[k])).cuda() for k in keys}


def _rates(shape_sh, name):
    d = A.DEFAULTS
    if name != "sh":
        return d["lr_" + name]
    return d["lr_sh_dc"] if shape_sh[1] == 1 else max(d["lr_sh_dc"], d["lr_sh_rest"])


def _check_standalone(got, ref, T, name):
    lr = _rates(ref.shape, name)
    err = np.abs(got.astype(np.float64) - ref)
    tol = 2e-5 * np.abs(ref) + 1e-4 * lr * T
    assert (err <= tol).all(), f"{name}: worst {(err / tol).max():.3g}x of the tolerance"


@pytest.mark.parametrize("n,deg", [(1, 0), (3, 1), (1031, 3), (4099, 2)])
def test_adam_steps_match_oracle(R, n, deg):
    rng = np.random.default_rng(100 * n + deg)
    p = _params(rng, n, deg)
    dp = _dev(p)
    params = tuple(dp[k] for k in GROUPS)
    opt = R.Adam(*params)
    ref, m, v = {k: p[k].astype(np.float64) for k in GROUPS}, A.zeros_like(p), A.zeros_like(p)
    T = 4
    for t in range(1, T + 1):
        g = _grads(rng, p)
        opt.step(params, _dev(g))
        ref, m, v = A.step(ref, g, m, v, t)
    torch.cuda.synchronize()
    assert opt.steps == T
    for k in GROUPS:
        _check_standalone(dp[k].cpu().numpy(), ref[k], T, k)
        for mom, r in ((opt.m[k], m[k]), (opt.v[k], v[k])):
            scale = np.abs(r).max(initial=0)
            np.testing.assert_allclose(mom.cpu().numpy(), r, rtol=2e-5, atol=2e-5 * scale + 1e-30, err_msg=k)
    say("adam", n, deg, "ok")


def test_adam_unaligned_arrays_take_the_scalar_path(R):
    # arrays offset by one float from a 16-byte boundary: same results as aligned ones
    rng = np.random.default_rng(5)
    n, deg = 517, 3
    p = _params(rng, n, deg)
    g = _grads(rng, p)
    aligned = _dev(p)
    shifted = {}
    for k in GROUPS:
        buf = torch.empty(p[k].size + 1, dtype=torch.float32, device="cuda")
        t = buf[1:].view(p[k].shape)
        t.copy_(aligned[k])
        shifted[k] = t
    shifted["quats"] = aligned["quats"].clone()     # quaternions must stay 16-byte aligned
    oa = R.Adam(*(aligned[k] for k in GROUPS))
    os_ = R.Adam(*(shifted[k] for k in GROUPS))
    gd = _dev(g)
    for _ in range(2):
        oa.step(tuple(aligned[k] for k in GROUPS), gd)
        os_.step(tuple(shifted[k] for k in GROUPS), gd)
    torch.cuda.synchronize()
    for k in GROUPS:
        assert torch.equal(aligned[k], shifted[k]), k
    ref, m, v = {k: p[k].astype(np.float64) for k in GROUPS}, A.zeros_like(p), A.zeros_like(p)
    for t in (1, 2):
        ref, m, v = A.step(ref, g, m, v, t)
    for k in GROUPS:
        _check_standalone(shifted[k].cpu().numpy(), ref[k], 2, k)


def test_adam_rejects_bad_settings(R):
    rng = np.random.default_rng(6)
    p = _params(rng, 8, 0)
    d = _dev(p)
    params = tuple(d[k] for k in GROUPS)
    from paper_2408_12677_amd import _native as N
    for bad in (dict(beta1=1.0), dict(beta2=-0.1), dict(lr_means=-1.0), dict(eps=float("inf"))):
        opt = R.Adam(*params, **bad)
        with pytest.raises(N.GsrError):
            opt.step(params, _dev(_grads(rng, p)))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(d["means"].cpu().numpy(), p["means"])   # nothing ran


# ---------------------------------------------------------------------------------------
# fused with the backward
# ---------------------------------------------------------------------------------------

def _seeded_moments(rng, ref_g):
    """First and second moments of the size of the oracle gradients (so one step is a
    smooth function of the gradient)."""
    m0, v0 = {}, {}
    for k in GROUPS:
        sig = float(np.sqrt(np.mean(ref_g[k] ** 2))) or 1e-6
        shape = ref_g[k].shape
        m0[k] = (rng.standard_normal(shape) * sig).astype(np.float32)
        v0[k] = ((sig * rng.uniform(1.0, 3.0, shape)) ** 2).astype(np.float32)
    return m0, v0


def _fused_tolerance(p0, g, m0, v0, t, flagged, all_max):
    """Per-element bounds for params, m, v after one fused step, from oracle values only."""
    d = A.DEFAULTS
    b1, b2, eps = d["beta1"], d["beta2"], d["eps"]
    bc1, bc2 = A.bias_corrections(t, b1, b2)
    new_p, new_m, new_v = A.step(p0, g, m0, v0, t)
    tol = {}
    for k in GROUPS:
        x, gk = p0[k].astype(np.float64), g[k]
        gmax = np.abs(gk).max(initial=0)
        # the gradient bar of the parity tests, widened by the oracle's bound of the other
        # correct gradients (decisions inside their margins, non-unique loss signs)
        dg = GRAD_REL * np.maximum(np.maximum(np.abs(gk), 1e-2 * gmax), 1e-4 * all_max) + g["envelope"][k]
        if k == "scales":
            c = x
        elif k == "opacities":
            c = x * (1 - x)
        else:
            c = np.ones_like(x)
        gv, dgv = gk * c, dg * c
        mn = b1 * m0[k] + (1 - b1) * gv
        vn = b2 * v0[k] + (1 - b2) * gv * gv
        mh, vh = mn / bc1, vn / bc2
        D = np.sqrt(vh) + eps
        lr = A.DEFAULTS["lr_" + k] if k != "sh" else A._sh_rates(x.shape, d["lr_sh_dc"], d["lr_sh_rest"])
        dstep = lr * ((1 - b1) / (bc1 * D) + np.abs(mh) * (1 - b2) * np.abs(gv) / (bc2 * np.sqrt(vh) * D * D))
        dvar = 2 * dstep * dgv
        xn = new_p[k]
        if k == "scales":
            dx = xn * dvar
        elif k == "opacities":
            dx = xn * (1 - xn) * dvar
        else:
            dx = dvar
        rows = flagged.reshape((-1,) + (1,) * (x.ndim - 1))
        big = np.broadcast_to(rows, x.shape)
        tol[k] = dict(p=np.where(big, np.inf, dx + 4e-6 * np.abs(xn) + 1e-5 * np.max(lr)),
                      m=np.where(big, np.inf, 2 * (1 - b1) * dgv + 2e-6 * np.abs(new_m[k]) + 1e-30),
                      v=np.where(big, np.inf, 2 * (1 - b2) * (2 * np.abs(gv) * dgv + dgv ** 2)
                                 + 2e-6 * np.abs(new_v[k]) + 1e-37))
    return new_p, new_m, new_v, tol


def _check_fused(dev_params, opt, ref, tol, label):
    new_p, new_m, new_v = ref
    for k in GROUPS:
        for name, got, want in (("p", dev_params[k], new_p[k]), ("m", opt.m[k], new_m[k]), ("v", opt.v[k], new_v[k])):
            a = got.detach().cpu().numpy().astype(np.float64)
            assert np.isfinite(a).all(), f"{label} {k}.{name}"
            err = np.abs(a - want)
            bad = err > tol[k][name]
            assert not bad.any(), f"{label} {k}.{name}: {bad.sum()} elements, worst " \
                                  f"{(err / np.maximum(tol[k][name], 1e-300)).max():.3g}x"


def _fused_case(rng, w_gauss, cams):
    g = w_gauss
    orc = oracle_for(g, cams, settings())
    hgc = [rng.standard_normal((3, c.height, c.width)).astype(np.float32) for c in cams]
    hgd = [rng.standard_normal((c.height, c.width)).astype(np.float32) for c in cams]
    ref_g = orc.backward(hgc, hgd, None)
    m0, v0 = _seeded_moments(rng, ref_g)
    return orc, hgc, hgd, ref_g, m0, v0


def _load_opt(opt, m0, v0, t0):
    for k in GROUPS:
        opt.m[k].copy_(torch.from_numpy(m0[k]))
        opt.v[k].copy_(torch.from_numpy(v0[k]))
    opt.state.zero_()
    opt.state[0] = t0


def test_backward_fused_with_adam_matches_oracle(R):
    w = scenes.make_cfg1()
    rng = np.random.default_rng(21)
    orc, hgc, hgd, ref_g, m0, v0 = _fused_case(rng, w.gaussians, w.cameras)
    params = to_dev(w.gaussians)
    dp = dict(zip(GROUPS, params))
    opt = R.Adam(*params)
    t0 = 5
    _load_opt(opt, m0, v0, t0)
    images, saved = R.forward(*params, w.cameras, settings())
    R.backward_adam(saved, opt, [torch.from_numpy(a).cuda() for a in hgc], [torch.from_numpy(a).cuda() for a in hgd])
    torch.cuda.synchronize()
    saved.free()
    assert opt.steps == t0 + 1
    p0 = dict(zip(GROUPS, w.gaussians.arrays()))
    all_max = max(np.abs(ref_g[k]).max(initial=0) for k in GROUPS)
    *ref, tol = _fused_tolerance(p0, ref_g, m0, v0, t0 + 1, ref_g["flagged"], all_max)
    _check_fused(dp, opt, ref, tol, "fused")
    say("fused adam ok; flagged", int(ref_g["flagged"].sum()), "of", len(ref_g["flagged"]))


def test_graph_with_adam_matches_oracle_then_eager(R):
    # three cameras of uneven size; the captured step ends with the fused Adam step
    w = scenes.make_cfg1()
    c = w.cameras[0]
    R1, t1 = scenes.look_at([0.2, 0.1, -0.3], [0.0, 0.0, 3.0], up=(0, -1, 0))
    cams = [c, scenes.Camera(100, 75, 90.0, 90.0, 50.3, 37.6, R1, t1), c.crop(13, 7, 37, 29)]
    rng = np.random.default_rng(8)
    targets = [(rng.random((3, k.height, k.width)).astype(np.float32),
                (1 + 3 * rng.random((k.height, k.width))).astype(np.float32)) for k in cams]
    tg = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in targets]
    s = settings()
    # the oracle's step: its own images, its own L1 gradients
    orc = oracle_for(w.gaussians, cams, s)
    from parity_util import oracle_loss
    L, ref_gc, ref_gd, amb = oracle_loss(orc.forward(), targets, 0.1)
    ref_g = orc.backward(ref_gc, ref_gd, None, ambiguous_pixels=amb)
    m0, v0 = _seeded_moments(rng, ref_g)
    t0 = 3
    # graph path
    params = to_dev(w.gaussians)
    opt = R.Adam(*params)
    _load_opt(opt, m0, v0, t0)
    graph = R.Graph(*params, cams, tg, s, optimizer=opt)
    graph.launch()
    graph.sync()
    assert opt.steps == t0 + 1 and graph.grads is None
    p0 = dict(zip(GROUPS, w.gaussians.arrays()))
    all_max = max(np.abs(ref_g[k]).max(initial=0) for k in GROUPS)
    *ref, tol = _fused_tolerance(p0, ref_g, m0, v0, t0 + 1, ref_g["flagged"], all_max)
    _check_fused(dict(zip(GROUPS, params)), opt, ref, tol, "graph replay 1")
    # two more replays against two eager fused iterations from the same state
    eparams = [p.clone() for p in params]
    eopt = R.Adam(*eparams)
    for k in GROUPS:
        eopt.m[k].copy_(opt.m[k])
        eopt.v[k].copy_(opt.v[k])
    eopt.state.copy_(opt.state)
    start = [p.clone() for p in params]
    for _ in range(2):
        graph.launch()
        graph.sync()
        images, saved = R.forward(*eparams, cams, s)
        _, gc, gd = R.loss_l1(saved, images, tg, 0.1)
        R.backward_adam(saved, eopt, gc, gd)
        saved.free()
    torch.cuda.synchronize()
    assert opt.steps == eopt.steps == t0 + 3
    for k, a, b, s0 in zip(GROUPS, params, eparams, start):
        moved = (b - s0).abs()
        diff = (a - b).abs()
        assert bool((diff <= 1e-3 * moved + 1e-6 * b.abs() + 1e-7).all()), k
    graph.free()
