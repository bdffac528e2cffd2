"""Benchmark: forward + L1 loss + backward of the differentiable Gaussian-splatting
rasterizer on one MI355X.

Workload (seeded, synthetic): a 500k-Gaussian map (SH degree 3) seeded by the quadtree
rule on a synthetic room, observed by 8 orbit views of uneven resolution (2x 320x240,
3x 640x480, 2x 1280x960, 1x 1200x680).  The headline step renders the first 640x480
view, evaluates L1(colour) + 0.1 L1(depth) against its target, and back-propagates to
every Gaussian parameter.  A "step" is that whole path; ``value`` is Mpixel/s of it.

Also reported: the same 8 views as one batched call against 8 sequential per-view
steps; per-kernel device time from HIP events on the library's stream; the roofline
of the dominant kernel; the FP64 CPU oracle timed on this host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
HEADLINE_VIEW = 2              # first 640x480 view of the 8-view orbit
DEPTH_W = 0.1


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------------------------
# algorithmic work model (bytes each kernel must move at least once per launch)
# ------------------------------------------------------------------------------------
def kernel_bytes(name, st):
    """Algorithmic HBM bytes of one launch of kernel ``name`` given step statistics."""
    N, V, Nv, M, P, K = st["N"], st["V"], st["N_vis"], st["M"], st["P"], st["K"]
    pg = 4 * (3 + 3 + 4 + 1 + 3 * K)            # parameter bytes per Gaussian
    if name == "project":
        return N * pg + V * N * 4 + Nv * (16 * 3 + 8)
    if name == "duplicate":
        return V * N * 4 + Nv * (8 + 16) + M * 12
    if name == "radix_hist":
        return M * 8
    if name == "radix_scatter":
        return M * 12 * 2
    if name == "ranges":
        return M * 8 + st["tiles"] * 8
    if name == "blend_fwd":
        return st["loaded_fwd"] * (4 + 48) + P * 28
    if name == "blend_bwd":
        return st["loaded_bwd"] * (4 + 48) + P * 28 + st["wave_hits"] * 40
    if name == "project_bwd":
        return 2 * N * pg + V * N * 4 + Nv * 48
    if name == "loss_l1":
        return P * 4 * 4 * 2
    if name == "fill":
        return V * N * 48
    return 0


def step_stats(R, params, cams, targets, settings):
    """One untimed step that exports the counts the work model needs."""
    import torch
    images, saved = R.forward(*params, cams, settings)
    dbg = saved.debug_export()
    inf = saved.info()
    torch.cuda.synchronize()
    ts = settings.tile
    loaded_fwd = loaded_bwd = wave_hits = 0
    off = 0
    for v, c in enumerate(cams):
        tx, ty = -(-c.width // ts), -(-c.height // ts)
        H, W = c.height, c.width
        nc = dbg["n_contrib"][off:off + H * W].reshape(H, W).astype(np.int64)
        tf = dbg["T_final"][off:off + H * W].reshape(H, W)
        off += H * W
        t0 = sum(-(-cc.width // ts) * -(-cc.height // ts) for cc in cams[:v])
        rng = dbg["ranges"][t0:t0 + tx * ty].astype(np.int64)
        length = (rng[:, 1] - rng[:, 0]).reshape(ty, tx)
        pad = np.zeros((ty * ts, tx * ts), np.int64)
        done = np.zeros((ty * ts, tx * ts), bool)
        pad[:H, :W] = nc
        done[:H, :W] = tf < settings.T_min
        done[H:, :] = True
        done[:, W:] = True
        blk_n = pad.reshape(ty, ts, tx, ts).max(axis=(1, 3))
        blk_done = done.reshape(ty, ts, tx, ts).all(axis=(1, 3))
        # forward: a block stages records until every pixel has stopped, else the whole list
        fwd_need = np.where(blk_done, blk_n, length)
        loaded_fwd += int(np.minimum(length, -(-fwd_need // settings.batch) * settings.batch).sum())
        loaded_bwd += int(blk_n.sum())
        # backward: (wavefront, list entry) pairs, with the wavefront's longest contributor list
        wv = pad.reshape(ty, ts, tx, ts).transpose(0, 2, 1, 3).reshape(ty * tx, -1, 64).max(axis=2)
        wave_hits += int(wv.sum())
    st = dict(N=int(params[0].shape[0]), V=len(cams), N_vis=int((dbg["tiles_touched"] > 0).sum()),
              M=int(inf["num_keys"]), P=int(inf["num_pixels"]), K=int(params[4].shape[1]),
              tiles=int(inf["num_tiles"]), sort_passes=int(inf["sort_passes"]), loaded_fwd=loaded_fwd,
              loaded_bwd=loaded_bwd, wave_hits=wave_hits,
              E_bwd=int(dbg["n_contrib"].astype(np.int64).sum()))
    saved.free()
    return st


def timed_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); multi-GPU runs are "
              "not part of it.", file=sys.stderr)
        sys.exit(2)

    import torch
    import scenes
    from paper_2408_12677_amd import rasterize as R

    log("generating the 500k-Gaussian room map and its 8 orbit views")
    t0 = time.perf_counter()
    w = scenes.make_cfg4()
    log(f"  generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda", 0)
    params = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in w.gaussians.arrays()]
    targets = [(torch.from_numpy(tc).to(dev), torch.from_numpy(td).to(dev)) for tc, td in w.targets]
    s = R.Settings(tile=args.tile, batch=args.batch)
    grads = dict(means=torch.empty_like(params[0]), scales=torch.empty_like(params[1]),
                 quats=torch.empty_like(params[2]), opacities=torch.empty_like(params[3]),
                 sh=torch.empty_like(params[4]))
    ctx = R.context(dev)

    def step(views, accumulate=False):
        cams = [w.cameras[v] for v in views]
        tg = [targets[v] for v in views]
        images, saved = R.forward(*params, cams, s)
        _, gc, gd = R.loss_l1(saved, images, tg, DEPTH_W)
        R.backward(saved, gc, gd, None, grads=grads, accumulate=accumulate)
        saved.free()

    head = [HEADLINE_VIEW]
    cam = w.cameras[HEADLINE_VIEW]
    px_head = cam.width * cam.height
    stats = step_stats(R, params, [cam], [targets[HEADLINE_VIEW]], s)
    log("headline stats", stats)

    # headline: per-view fwd+loss+bwd, K timed steps
    log(f"timing {args.steps} headline steps ({args.warmup} warm-up)")
    ms = timed_steps(lambda: step(head), args.steps, args.warmup) * 1e3
    # the same steps again with the per-kernel event timer on (kernel durations)
    ctx.set_timing(True)
    ctx.timing(reset=True)
    ms_timed = timed_steps(lambda: step(head), args.steps, 0) * 1e3
    ktimes = ctx.timing(reset=True)
    ctx.set_timing(False)
    per_kernel = {k: dict(ms_per_step=t / args.steps, launches_per_step=n / args.steps, avg_launch_us=1e3 * t / n)
                  for k, (t, n) in ktimes.items() if n > 0}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_step"])
    alg = {k: kernel_bytes(k, stats) for k in per_kernel}
    step_bytes = sum(alg[k] * per_kernel[k]["launches_per_step"] for k in per_kernel)
    dk = per_kernel[dom]
    achieved = alg[dom] / (dk["avg_launch_us"] * 1e-6) / 1e9 if alg[dom] else 0.0
    traffic = None
    prof = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(prof):
        try:
            tj = json.load(open(prof))
            from paper_2408_12677_amd import build as B
            import hashlib
            src = hashlib.sha256(open(B.SOURCES[1], "rb").read()).hexdigest()[:16]
            if tj.get("kernel") == dom and tj.get("kernels_sha") == src:
                traffic = tj.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    alg_bytes_per_launch=int(alg[dom]), avg_launch_us=round(dk["avg_launch_us"], 2))

    out = {
        "metric": "fwd+bwd Mpixel/s at 500k Gaussians 640x480; batched vs per-view, HBM GB/s",
        "value": round(px_head / (ms * 1e-3) / 1e6, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "500k-Gaussian quadtree-seeded room map (SH3), one 640x480 view: "
                               "forward + L1(colour)+0.1 L1(depth) + backward",
                   "gaussians": stats["N"], "width": cam.width, "height": cam.height, "sh_degree": 3,
                   "tile": s.tile, "batch": s.batch, "path": "per-view"},
        "hbm": {"alg_bytes_per_step": int(step_bytes),
                "alg_GBps": round(step_bytes / (ms * 1e-3) / 1e9, 1),
                "frac_of_peak": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline": roofline,
        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in per_kernel.items()},
        "ms_per_step_with_event_timer": round(ms_timed, 4),
        "work": {k: stats[k] for k in ("N_vis", "M", "P", "tiles", "sort_passes", "E_bwd")},
    }

    if not args.no_batched:
        allv = list(range(len(w.cameras)))
        px_all = sum(c.width * c.height for c in w.cameras)
        k2 = max(3, args.steps // 3)
        log(f"timing batched (8 views, one call) and 8 sequential per-view steps, {k2} steps each")
        ms_b = timed_steps(lambda: step(allv), k2, 2) * 1e3

        def seq():
            for i, v in enumerate(allv):
                step([v], accumulate=i > 0)
        ms_s = timed_steps(seq, k2, 1) * 1e3
        out["batched"] = {"views": len(allv), "pixels": px_all,
                          "batched_ms": round(ms_b, 3), "batched_Mpixel_s": round(px_all / (ms_b * 1e-3) / 1e6, 2),
                          "per_view_ms": round(ms_s, 3), "per_view_Mpixel_s": round(px_all / (ms_s * 1e-3) / 1e6, 2),
                          "steps": k2}

    if not args.no_cpu_baseline:
        import oracle
        log("timing the FP64 CPU oracle on headline steps (single thread, >= 10 s)")
        tc, td = w.targets[HEADLINE_VIEW]
        total, reps = 0.0, 0
        while total < 10.0 and reps < 20:
            total += oracle.time_fwd_bwd(w.gaussians.arrays(), 3, [cam], [(tc, td)],
                                         oracle.Settings(tile=s.tile, threads=1), DEPTH_W)
            reps += 1
        sec = total / reps
        out["cpu_baseline"] = {"value": round(px_head / sec / 1e6, 5), "unit": "Mpixel/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{reps} full headline steps (500k Gaussians, 640x480 fwd+L1+bwd), "
                                         f"{sec:.2f} s each"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
