"""Helpers of the GPU-vs-oracle parity tests (not collected as tests).

Tolerances (FP32 kernels against the FP64 oracle):
  * tile keys, sorted record order and tile ranges: bit-exact;
  * splat centre, depth bits and tile rectangles: bit-exact (same binary32 op sequence);
  * images: max |diff| <= 1e-4 on every pixel whose per-pixel decisions are unique.  A
    decision is ambiguous when its operands lie within a relative margin of the threshold
    (a skip value a within 1e-5 of 1/255, a transmittance within 1e-4 of 1e-4: about ten
    times the binary32 error of each), and then either outcome is correct: the oracle
    enumerates every combination of a pixel's ambiguous decisions and the GPU value must
    lie within 1e-4 of the range they span.  The number of ambiguous pixels is held to what
    the margins predict: the oracle counts the values within 100 times the margins, a
    window 100 times wider, so lambda = that count / 100 decisions are expected and at most
    lambda + 4 sqrt(lambda) + 5 pixels may be ambiguous (a Poisson count's upper tail);
  * loss and its output gradients: the oracle's L1 loss of the oracle's own images; the
    sign must agree wherever the target lies more than LOSS_MARGIN outside the range of
    the pixel's correct outcomes;
  * gradients: per parameter group ||g - g_ref||_2 <= 1e-3 ||g_ref||_2 + ||env||_2, and per
    element |g - g_ref| <= 1e-3 max(|g_ref|, 1e-2 max|g_ref|) + env, where env is the
    oracle's bound on how far a correct gradient can lie from g_ref over the correct
    outcomes of every ambiguous decision (skip, stop, opacity clamp) and every non-unique
    loss gradient.  Its norm is reported relative to the group's (at most 2%; 0.08% on the
    headline view), and so are the Gaussians with env above the 1e-3 term in some element
    ("widened").  At most 1% of the
    Gaussians with a gradient may contribute to a pixel with too many ambiguous decisions
    to enumerate (flagged: those are left out of the per-element check).
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2408_12677_amd import rasterize as R

IMG_TOL = 1e-4
GRAD_REL = 1e-3
# the L1 loss gradient (Eq. 12) is sign(rendered - target): where the oracle's rendered
# value lies within this margin of the target the sign is not unique (about five times
# the largest image difference measured between the two sides); depth uses it relative
# to max(1, |target|)
LOSS_MARGIN = 2e-5
FLAGGED_FRACTION = 0.01  # Gaussians at pixels whose outcomes were not enumerated
ENV_NORM_CAP = 0.02      # norm of the decision bound, relative to the group's gradient norm
NAMES = ("means", "scales", "quats", "opacities", "sh")


def to_dev(g, device="cuda"):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in g.arrays()]


def settings(**kw) -> R.Settings:
    return R.Settings(**kw)


def oracle_for(g, cams, s: R.Settings, threads=8):
    os_ = oracle.Settings(tile=s.tile, extent_k=s.extent_k, lowpass=s.lowpass, alpha_min=s.alpha_min,
                          alpha_max=s.alpha_max, T_min=s.T_min, guard=s.guard, bg=tuple(s.bg), mu_fp32=True,
                          threads=threads, exact_tiles=s.exact_tiles, normalized_depth=s.normalized_depth,
                          jclamp=s.jclamp)
    return oracle.Oracle(g.arrays(), g.sh_degree, cams, os_)


def check_keys(dbg, orc):
    k, v, r = orc.keys()
    assert dbg["keys"].shape == k.shape, (dbg["keys"].shape, k.shape)
    np.testing.assert_array_equal(dbg["keys"], k)
    np.testing.assert_array_equal(dbg["values"], v)
    np.testing.assert_array_equal(dbg["ranges"], r)


def check_records(dbg, orc, tile):
    rec = orc.records()
    vis = rec["visible"]
    np.testing.assert_array_equal(dbg["tiles_touched"] > 0, vis)
    np.testing.assert_array_equal(dbg["mu"][vis].view(np.uint32), rec["mu"][vis].view(np.uint32))
    np.testing.assert_array_equal(dbg["depth"][vis].view(np.uint32), rec["z"][vis].view(np.uint32))
    np.testing.assert_array_equal(dbg["rect"][vis][:, [0, 1]], rec["rect"][vis][:, [0, 1]] // tile)
    np.testing.assert_array_equal(dbg["rect"][vis][:, [2, 3]], rec["rect"][vis][:, [2, 3]] // tile)
    # conic: bit-exact against the binary32 formula (det = a*c - b*b, inv = 1/det,
    # (A, B, C) = (c, -b, a) * inv) applied to the oracle's binary32 covariance ...
    a, b, c = (rec["cov"][vis][:, i].astype(np.float32) for i in range(3))
    with np.errstate(all="ignore"):
        det = (a * c - b * b).astype(np.float32)
        inv = (np.float32(1) / det).astype(np.float32)
    c32 = np.stack([c * inv, -b * inv, a * inv], 1).astype(np.float32)
    np.testing.assert_array_equal(dbg["conic"][vis].view(np.uint32), c32.view(np.uint32))
    # ... and close to the FP64 conic wherever binary32 can represent it well (a covariance
    # with det >= 1e-2 a c; near-plane splats can have det/(a c) ~ 1e-4)
    conic_ref = rec["conic"][vis]
    well = (det.astype(np.float64) >= 1e-2 * a.astype(np.float64) * c.astype(np.float64))
    scale = np.abs(conic_ref).max(1, keepdims=True)
    assert np.all((np.abs(dbg["conic"][vis] - conic_ref) <= 1e-4 * scale + 1e-12)[well])
    np.testing.assert_allclose(dbg["color"][vis], rec["color"][vis], atol=1e-5)


def ambiguity_cap(outs):
    """(lambda, cap): the ambiguous decisions the margins predict and the Poisson cap."""
    lam = sum(float(o["near_a"].sum() + o["near_T"].sum()) for o in outs) / oracle.NEAR_WIDE
    return lam, lam + 4.0 * np.sqrt(lam) + 5.0


def check_images(images, outs, dbg=None, cams=None, tol=IMG_TOL):
    """Compare per-view GPU images with the oracle's; returns a small report dict."""
    report = dict(max_diff=0.0, ambiguous=0, unbounded=0, pixels=0)
    off = 0
    for v, ((col, dep, alp), o) in enumerate(zip(images, outs)):
        col, dep, alp = (t.detach().cpu().numpy().astype(np.float64) for t in (col, dep, alp))
        amb = o["ambiguous"]
        ok = ~amb
        dc = np.abs(col - o["color"]).max(0)
        dd = np.abs(dep - o["depth"])
        da = np.abs(alp - o["alpha"])
        worst = max(dc[ok].max(initial=0), dd[ok].max(initial=0), da[ok].max(initial=0))
        assert worst <= tol, f"view {v}: max diff {worst:.3g} > {tol} (colour {dc[ok].max(initial=0):.3g}, " \
                             f"depth {dd[ok].max(initial=0):.3g}, alpha {da[ok].max(initial=0):.3g})"
        if amb.any():
            # every ambiguous pixel lies within tol of the range of its correct outcomes ...
            gpu = np.concatenate([col, dep[None], alp[None]], 0)
            bounded = o["events"] >= 0
            out_of_range = np.maximum(o["lo"] - tol - gpu, gpu - o["hi"] - tol).max(0)
            bad = amb & bounded & (out_of_range > 0)
            assert not bad.any(), f"view {v}: {bad.sum()} ambiguous pixels outside their outcomes' range " \
                                  f"(worst {out_of_range[bad].max():.3g})"
            # ... and where they were too many to enumerate, within one skipped splat
            unb = amb & ~bounded
            if unb.any():
                assert dc[unb].max() <= 1 / 255 + tol and da[unb].max() <= 1 / 255 + tol
            report["unbounded"] += int(unb.sum())
        if dbg is not None:
            H, W = dep.shape
            nc = dbg["n_contrib"][off:off + H * W].reshape(H, W)
            np.testing.assert_array_equal(nc[ok], o["n_contrib"][ok])
            nu = dbg["n_used"][off:off + H * W].reshape(H, W)
            np.testing.assert_array_equal(nu[ok], o["n_used"][ok])
            tf = dbg["T_final"][off:off + H * W].reshape(H, W)
            assert np.abs(tf[ok] - o["T_final"][ok]).max(initial=0) <= tol
            off += H * W
        report["max_diff"] = max(report["max_diff"], float(worst))
        report["ambiguous"] += int(amb.sum())
        report["pixels"] += amb.size
    lam, cap = ambiguity_cap(outs)
    report["expected_ambiguous"] = round(lam, 1)
    assert report["ambiguous"] <= cap, f"{report['ambiguous']} ambiguous pixels, the margins predict {lam:.1f}"
    assert report["unbounded"] <= max(2, 1e-4 * report["pixels"]), report
    return report


def check_grads(gpu, ref, rel=GRAD_REL, names=NAMES):
    """gpu: dict of torch tensors, ref: oracle backward dict (with 'envelope', 'flagged').

    A group whose reference is negligible next to the whole gradient (||g_ref|| below
    1e-3 ||g_ref(all groups)||; e.g. the rotation gradient of isotropic Gaussians, zero
    analytically, which binary32 leaves as the residue of cancelling terms) is measured on
    the scale of the whole gradient: its norm floor is 1e-3 ||g_ref(all groups)|| and its
    element floor 1e-3 max|g_ref(all groups)|; other groups have the element floor
    1e-4 max|g_ref(all groups)|.
    """
    flagged = ref["flagged"]
    n = len(flagged)
    report = {}
    all_norm = np.sqrt(sum(np.linalg.norm(ref[k]) ** 2 for k in names))
    all_max = max(np.abs(ref[k]).max(initial=0) for k in names)
    widened = np.zeros(n, bool)
    has_grad = np.zeros(n, bool)
    for name in names:
        g = gpu[name].detach().cpu().numpy().astype(np.float64).reshape(n, -1)
        r = ref[name].reshape(n, -1)
        env = ref["envelope"][name].reshape(n, -1)
        d = g - r
        negligible = np.linalg.norm(r) < 1e-3 * all_norm
        nr = max(np.linalg.norm(r), 1e-3 * all_norm)
        norm_rel = np.linalg.norm(d) / max(nr, 1e-30)
        # the decision bound may loosen a few elements, not the check (a sanity bound: 2% of
        # the group's norm; the headline view's is 0.08%)
        assert np.linalg.norm(env) <= ENV_NORM_CAP * nr, f"{name}: decision bound ||env|| " \
                                                         f"{np.linalg.norm(env):.3g} vs ||g_ref|| {nr:.3g}"
        report.setdefault("env_norm_rel", {})[name] = float(np.linalg.norm(env) / max(nr, 1e-30))
        assert np.linalg.norm(d) <= rel * nr + np.linalg.norm(env), f"{name}: ||diff||/||ref|| = {norm_rel:.3g}"
        floor = (1e-3 if negligible else 1e-4) * all_max
        base = rel * np.maximum(np.maximum(np.abs(r), 1e-2 * np.abs(r).max(initial=0)), floor)
        keep = ~flagged
        thr = base[keep] + env[keep]
        bad = np.abs(d[keep]) > thr
        assert not bad.any(), f"{name}: {bad.sum()} elements outside tolerance, worst " \
                              f"{(np.abs(d[keep]) / np.maximum(thr, 1e-30)).max():.3g}x"
        widened |= (env > base).any(1)
        has_grad |= (r != 0).any(1)
        report[name] = norm_rel
    contributing = max(int(has_grad.sum()), 1)
    report["contributing"] = contributing
    report["widened"] = int((widened & has_grad).sum())
    report["flagged"] = int(flagged.sum())
    assert report["flagged"] <= FLAGGED_FRACTION * contributing, report
    return report


def oracle_loss(outs, targets, depth_weight=0.1):
    """The oracle's L1 loss of its own images (nothing from the GPU).

    Returns (loss, [dL/dC], [dL/dD], [pixel masks]) where a mask (uint8, bit k for colour
    channel k = 0..2, bit 3 for depth) marks the outputs whose loss gradient is not unique:
    a colour or valid target depth within LOSS_MARGIN of the range the pixel's correct
    outcomes span (just the value where its decisions are unique); every bit is set at a
    pixel whose outcomes were too many to enumerate."""
    L, gcs, gds, amb = 0.0, [], [], []
    for o, (tc, td) in zip(outs, targets):
        tc = np.asarray(tc, np.float64)
        td = np.asarray(td, np.float64)
        l, gC, gD = oracle.l1_loss(o["color"], o["depth"], tc, td, depth_weight)
        L += l
        gcs.append(gC)
        gds.append(gD)
        # a tie: the target within LOSS_MARGIN of the range of the pixel's correct outcomes
        lo, hi = o["lo"], o["hi"]
        near_c = (tc >= lo[:3] - LOSS_MARGIN) & (tc <= hi[:3] + LOSS_MARGIN)
        dm = LOSS_MARGIN * np.maximum(1.0, np.abs(td))
        near_d = (td > 0) & (td >= lo[3] - dm) & (td <= hi[3] + dm)
        m = near_c[0] * 1 + near_c[1] * 2 + near_c[2] * 4 + near_d * 8
        m = np.where(o["events"] < 0, 31, m)
        amb.append(m.astype(np.uint8))
    return L, gcs, gds, amb


def check_loss_grads(gc, gd, ref_gc, ref_gd, amb):
    """GPU loss gradients (per-view torch lists) against oracle_loss's: equal where unique,
    and no larger than the oracle's magnitude where not."""
    for v, (a, b, c, d, m) in enumerate(zip(gc, gd, ref_gc, ref_gd, amb)):
        a = a.detach().cpu().numpy().astype(np.float64)
        c = np.asarray(c)
        tied = np.stack([(m >> k) & 1 for k in range(3)]).astype(bool)
        ok = ~tied
        np.testing.assert_allclose(a[ok], c[ok], rtol=1e-6, atol=0, err_msg=f"view {v} colour")
        assert (np.abs(a[tied]) <= np.abs(c).max() * (1 + 1e-6)).all()
        if b is not None:
            b = b.detach().cpu().numpy().astype(np.float64)
            d = np.asarray(d)
            td = ((m >> 3) & 1).astype(bool)
            np.testing.assert_allclose(b[~td], d[~td], rtol=1e-6, atol=0, err_msg=f"view {v} depth")
            assert (np.abs(b[td]) <= np.abs(d).max() * (1 + 1e-6)).all()
