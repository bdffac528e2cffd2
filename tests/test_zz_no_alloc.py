"""The allocation-free backward (gsr_backward_noalloc) against gsr_backward.

Both run the same kernels on the same saved forward; only where the per-record gradient
rows live differs (the library's fixed device array instead of pool memory), so the
gradients must agree to the gradient bar of the oracle parity tests (per group
||g - g_ref|| <= 1e-3 ||g_ref||, per element 1e-3 relative above 1e-2 of the group's
largest; float atomics reorder the sums).  Two calls in a row, the second on a smaller
saved state, check that each call clears what it uses; a saved state larger than the
array is refused before any device work and the context stays usable.
"""
import sys

import numpy as np
import pytest

import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from parity_util import to_dev  # noqa: E402

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


def output_grads(cams, seed):
    rng = np.random.default_rng(seed)
    dev = lambda a: torch.from_numpy(a).cuda()
    gc = [dev(rng.standard_normal((3, c.height, c.width)).astype(np.float32)) for c in cams]
    gd = [dev(rng.standard_normal((c.height, c.width)).astype(np.float32)) for c in cams]
    ga = [dev(rng.standard_normal((c.height, c.width)).astype(np.float32)) for c in cams]
    return gc, gd, ga


def same_grads(a, b, what):
    """The oracle tests' gradient bar; a group negligible next to the whole gradient (the
    rotation gradient of isotropic Gaussians is 0 analytically) is measured on the whole
    gradient's scale."""
    ys = {k: b[k].double().cpu().numpy().reshape(-1) for k in NAMES}
    all_norm = np.sqrt(sum(np.linalg.norm(y) ** 2 for y in ys.values()))
    all_max = max(np.abs(y).max(initial=0) for y in ys.values())
    for k in NAMES:
        x = a[k].double().cpu().numpy().reshape(-1)
        y = ys[k]
        assert np.isfinite(x).all(), f"{what}: {k} not finite"
        ny = max(np.linalg.norm(y), 1e-3 * all_norm)
        assert np.linalg.norm(x - y) <= 1e-3 * ny, f"{what}: {k} norm"
        thr = 1e-3 * np.maximum(np.maximum(np.abs(y), 1e-2 * np.abs(y).max(initial=0)), 1e-4 * all_max)
        assert (np.abs(x - y) <= thr).all(), f"{what}: {k} elements"


def both_backwards(R, g, cams, s, seed):
    params = to_dev(g)
    images, saved = R.forward(*params, cams, s)
    gc, gd, ga = output_grads(cams, seed)
    ref = R.backward(saved, gc, gd, ga)
    # preallocated outputs filled with garbage: the call must overwrite every element
    out = {k: torch.full_like(p, float("nan")) for k, p in zip(NAMES, params)}
    R.backward(saved, gc, gd, ga, grads=out, noalloc=True)
    torch.cuda.synchronize()
    same_grads(out, ref, f"{g.n} Gaussians x {len(cams)} views")
    # accumulate: a second call adds the same gradient again
    R.backward(saved, gc, gd, ga, grads=out, accumulate=True, noalloc=True)
    torch.cuda.synchronize()
    same_grads(out, {k: 2 * v for k, v in ref.items()}, "accumulated")
    saved.free()
    return ref


def test_noalloc_backward_two_calls_second_smaller(R):
    big = scenes.make_cfg2()
    say("noalloc: cfg2", big.gaussians.n, "Gaussians, then cfg1")
    both_backwards(R, big.gaussians, big.cameras, R.Settings(), seed=3)
    small = scenes.make_cfg1()
    c = small.cameras[0]
    cams = [c, c.crop(9, 5, 61, 47)]
    both_backwards(R, small.gaussians, cams, R.Settings(tile=8, batch=128), seed=4)


def test_noalloc_backward_rejects_too_large_saved_state(R):
    from paper_2408_12677_amd._native import NOALLOC_SCRATCH_BYTES, GsrError
    rng = np.random.default_rng(5)
    n = 100_000
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 4, n)], 1)
    g = scenes.random_gaussians(rng, means, 0)
    V = 16
    assert V * n * 48 + n * 12 > NOALLOC_SCRATCH_BYTES
    cam = scenes.Camera(16, 16, 10.0, 10.0, 8.0, 8.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))
    params = to_dev(g)
    say("noalloc: refusal at", V, "views x", n)
    images, saved = R.forward(*params, [cam] * V, R.Settings())
    gc, gd, ga = output_grads([cam] * V, 6)
    out = {k: torch.zeros_like(p) for k, p in zip(NAMES, params)}
    with pytest.raises(GsrError, match="EINVAL"):
        R.backward(saved, gc, gd, ga, grads=out, noalloc=True)
    for k in NAMES:
        assert float(out[k].abs().max()) == 0.0, k  # nothing was launched
    ref = R.backward(saved, gc, gd, ga)  # the context is still usable
    torch.cuda.synchronize()
    assert all(torch.isfinite(v).all() for v in ref.values())
    saved.free()
