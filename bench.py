"""Benchmark: forward + L1 loss + backward of the differentiable Gaussian-splatting
rasterizer on one MI355X.

Workload (seeded, synthetic): a 500k-Gaussian map (SH degree 3) seeded by the quadtree
rule on a synthetic room, observed by 8 orbit views of uneven resolution (2x 320x240,
3x 640x480, 2x 1280x960, 1x 1200x680).  The headline step renders the first 640x480
view, evaluates L1(colour) + 0.1 L1(depth) against its target, and back-propagates to
every Gaussian parameter.  A "step" is that whole path; ``value`` is Mpixel/s of it.

Also reported: the same 8 views as one batched call against 8 sequential per-view
steps; per-kernel device time from HIP events on the library's stream; the roofline
of the dominant kernel; quadtree seeding of one frame (640x480 and 1752x1168); the
FP64 CPU oracle timed on this host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = "paper_2408_12677_amd/csrc/"
KERNEL_HEADERS = ("gsr_internal.h", "gsr_adam.h", "gsr_tsdf.h")


def kernel_source(name):
    """The source file that holds kernel ``name`` (short name, as short_kernel_name gives)."""
    if name.startswith("tsdf"):
        return "gsr_tsdf.hip"
    if name.startswith("adam"):
        return "gsr_optim.hip"
    if name.startswith("seed"):
        return "gsr_seed.hip"
    return "gsr_kernels.hip"
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
    if name == "project":                        # (+ the exact row runs of each visible record)
        # colour coefficients are read only for Gaussians some view sees
        sh = 4 * 3 * K
        return (N * (pg - sh) + st.get("N_any", N) * sh + V * N * 4 + Nv * (16 * 3 + 8)
                + Nv * st.get("row_run_bytes", 0))
    E1 = st["E_rows"]
    if name == "radix_hist":                     # depth digits of the visible records
        return Nv * 4
    if name == "radix_scatter":
        return Nv * 16
    if name == "bin_count":                      # mean of the row and the tile histogram launches
        return (Nv * 12 + E1 * 8) / 2
    if name == "bin_scatter":                    # mean of the row and the tile placement (+ ranges) launches
        return (Nv * 12 + E1 * 8 + E1 * 8 + st.get("M_listed", M) * 4 + st["tiles"] * 32) / 2
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


# ------------------------------------------------------------------------------------
# measured HBM traffic (rocprofv3 FETCH_SIZE / WRITE_SIZE, calibrated by a plain copy)
# ------------------------------------------------------------------------------------
def kernels_sha(name="blend_bwd"):
    """Digest of the sources of kernel ``name`` (its file and the internal headers); stored
    traffic is only reported for the same sources."""
    h = hashlib.sha256()
    for rel in (kernel_source(name),) + KERNEL_HEADERS:
        with open(os.path.join(ROOT, CSRC, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_kernel_name(full):
    """'void gsr::(anonymous namespace)::k_blend_bwd<16, 256>(...)' -> 'blend_bwd'."""
    n = full.split("(gsr::")[0] if full.startswith("void gsr::") else full
    n = n.replace("void ", "").replace("gsr::(anonymous namespace)::", "")
    n = n.split("(")[0].split("<")[0].strip()
    n = n[2:] if n.startswith("k_") else n
    # variants of one kernel (two pixels per lane, slots in registers) share its name
    if n.endswith("_r"):
        n = n[:-2]
    return "blend_bwd" if n == "blend_bwd2" else n


def shape_key(s):
    """The launch shape counters were taken at: tile, batch and list kind."""
    return f"tile{s.tile}_batch{s.batch}_{'exact' if s.exact_tiles else 'rect'}"


def traffic_from_counters(fetch_dir, write_dir, copy_mb, shape):
    """Per-kernel HBM bytes per dispatch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE; both count KiB per dispatch) of bench.py at launch shape ``shape``.  Each
    counter is scaled by the factor that makes it read the known size of the largest plain
    copy of ``copy_mb`` MiB in the run."""
    def load(d, counter):
        per = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    if row.get("Counter_Name") == counter:
                        per.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]) * 1024.0)
        return per
    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy_bytes = copy_mb << 20
    copies = [k for k in fetch if "copyBuffer" in k]
    if not copies:
        raise SystemExit("no copy kernel in the FETCH_SIZE run: profile bench.py --copy-probe MB")
    ck = max(copies, key=lambda k: max(fetch[k]))
    ff = copy_bytes / max(fetch[ck])
    fw = copy_bytes / max(write.get(ck, [copy_bytes]))
    kernels = {}
    for k in fetch:
        if "gsr::" not in k:
            continue
        fv, wv = fetch[k], write.get(k, [0.0])
        name = short_kernel_name(k)
        kernels[name] = dict(dispatches=len(fv), fetch_bytes=round(ff * sum(fv) / len(fv)),
                             write_bytes=round(fw * sum(wv) / len(wv)), sources_sha=kernels_sha(name))
    return dict(copy_kernel=ck, copy_bytes=copy_bytes, launch_shape=shape,
                fetch_factor=round(ff, 5), write_factor=round(fw, 5), kernels=kernels)


def stored_traffic(name, s=None):
    """Measured HBM bytes per launch of kernel ``name`` (fetch + write), or None unless the
    counters were taken for the current kernel sources (and, for the rasterizer's kernels,
    ``s`` given, at the launch shape of ``s``)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    k = t.get("kernels", {}).get(name)
    if k is None or k.get("sources_sha") != kernels_sha(name) or (s is not None and t.get("launch_shape") != shape_key(s)):
        return None
    return int(k["fetch_bytes"] + k["write_bytes"])


FP32_PEAK_TFLOPS = 157.3      # MI355X FP32 vector, published (packed FP32: two lanes' FMAs per issue)
FP32_UNPACKED_TFLOPS = 78.6   # 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-FMA/s, 2 flops each
# Algorithmic flops per unit (exp and divide counted as one each):
FLOPS_FWD_EVAL = 21           # forward, per evaluated (pixel, list entry): about 20 flops + 1 exp
FLOPS_BWD_EVAL = 62           # backward, per walked (pixel, list entry): about 60 + 1 exp + 1 divide
FLOPS_WAVE_SUM = 10 * 6       # per (wavefront, list entry) with a contributor: ten values x 6 steps


def kernel_roofline(name, st, alg_bytes, avg_us, s):
    """Roofline entry for kernel `name`: HBM for the data-movement kernels, FP32 ALU for
    the compositing kernels (algorithmic flops from the evaluated (pixel, splat) pairs)."""
    sec = avg_us * 1e-6
    if name in ("blend_fwd", "blend_bwd"):
        if name == "blend_fwd":
            flops = st["E_fwd"] * FLOPS_FWD_EVAL
        else:
            flops = st["E_bwd"] * FLOPS_BWD_EVAL + st["wave_hits"] * FLOPS_WAVE_SUM
        ach = flops / sec / 1e12
        return dict(bound="alu", kernel=name, achieved=round(ach, 2), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(ach / FP32_PEAK_TFLOPS, 4), traffic=stored_traffic(name, s),
                    frac_of_unpacked_peak=round(ach / FP32_UNPACKED_TFLOPS, 4),
                    alg_flops_per_launch=int(flops),
                    alg_bytes_per_launch=int(alg_bytes), avg_launch_us=round(avg_us, 2))
    ach = alg_bytes / sec / 1e9 if alg_bytes else 0.0
    return dict(bound="hbm", kernel=name, achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(ach / HBM_PEAK_GBS, 4), traffic=stored_traffic(name, s), alg_bytes_per_launch=int(alg_bytes),
                avg_launch_us=round(avg_us, 2))


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
    nc_all = dbg["n_contrib"].astype(np.int64)
    # evaluated pairs: the forward walks each pixel's list to its stop (T < T_min) or to the
    # end of the tile's list; contributors are the evaluated entries that passed the skip rule
    e_fwd = 0
    off = 0
    for v, c in enumerate(cams):
        H, W = c.height, c.width
        tx = -(-W // ts)
        t0 = sum(-(-cc.width // ts) * -(-cc.height // ts) for cc in cams[:v])
        rng = dbg["ranges"][t0:t0 + tx * -(-H // ts)].astype(np.int64)
        length = (rng[:, 1] - rng[:, 0]).reshape(-(-H // ts), tx)
        ys, xs = np.mgrid[0:H, 0:W]
        L = length[ys // ts, xs // ts]
        nc = nc_all[off:off + H * W].reshape(H, W)
        tf = dbg["T_final"][off:off + H * W].reshape(H, W)
        e_fwd += int(np.where(tf < settings.T_min, nc, L).sum())
        off += H * W
    e_used = int(dbg["n_used"].astype(np.int64).sum()) if "n_used" in dbg else int(nc_all.sum())
    vis = dbg["tiles_touched"] > 0
    e_rows = int((dbg["rect"][vis, 3] - dbg["rect"][vis, 2] + 1).astype(np.int64).sum())
    st = dict(N=int(params[0].shape[0]), V=len(cams), N_vis=int((dbg["tiles_touched"] > 0).sum()),
              M=int(inf["num_keys"]), P=int(inf["num_pixels"]), K=int(params[4].shape[1]),
              tiles=int(inf["num_tiles"]), sort_passes=int(inf["sort_passes"]), loaded_fwd=loaded_fwd,
              loaded_bwd=loaded_bwd, wave_hits=wave_hits, E_rows=e_rows,
              E_bwd=int(nc_all.sum()), E_fwd=e_fwd, E_used=e_used,
              row_run_bytes=32 if settings.exact_tiles else 0)
    n = (dbg["ranges"][:, 1].astype(np.int64) - dbg["ranges"][:, 0].astype(np.int64))
    st["M_listed"] = int(n.sum())  # pairs in the tile lists (fewer than M with exact tiles)
    st["N_any"] = int((dbg["tiles_touched"].reshape(len(cams), -1) > 0).any(axis=0).sum())  # seen by some view
    st["tile_list_length"] = {"p50": float(np.percentile(n, 50)), "p99": float(np.percentile(n, 99)),
                              "max": int(n.max(initial=0))}
    saved.free()
    return st


def seeding_leg(R, torch, dev, log):
    """Quadtree seeding + initialisation (gsr_seed) of ray-cast room frames at the headline
    and the paper's full resolution: Mpixel/s per frame (host-timed, the call synchronises
    once) and the algorithmic HBM rate of its two passes over the frame."""
    import scenes
    res = {}
    for W, H in ((640, 480), (1752, 1168)):
        room = scenes.Room(np.random.default_rng(21), (6.0, 5.0, 3.0), 20)
        cam = room.random_camera(np.random.default_rng(22), W, H)
        depth, rgb = room.raycast(cam, perturbed=True)
        rgb_d = torch.from_numpy(np.ascontiguousarray(rgb, np.float32)).to(dev)
        depth_d = torch.from_numpy(depth.astype(np.float32)).to(dev)
        for _ in range(3):
            g = R.seed(rgb_d, depth_d, cam, "contrast", 0.1, 4, 0.5, 3)
        torch.cuda.synchronize()
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            g = R.seed(rgb_d, depth_d, cam, "contrast", 0.1, 4, 0.5, 3)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        n = int(g["means"].shape[0])
        alg = W * H * 16 * 2 + n * (3 + 3 + 4 + 1 + 48 + 4) * 4   # two reads of rgb + depth; the Gaussians
        res[f"{W}x{H}"] = {"ms": round(sec * 1e3, 4), "Mpixel_s": round(W * H / sec / 1e6, 1), "gaussians": n,
                           "alg_GBps": round(alg / sec / 1e9, 1),
                           "frac_of_hbm_peak": round(alg / sec / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"seeding {W}x{H}: {res[f'{W}x{H}']}")
    res["workload"] = "ray-cast room frames, contrast threshold 0.1, min side 4, SH degree 3 outputs"
    return res


def optimiser_leg(R, torch, params, cam, target, s, steps, warmup, log):
    """Adam over the whole map (every parameter row, 28 HBM bytes per element: value,
    gradient and both moments read, value and moments written): the standalone step with
    its roofline, and one captured iteration with the step fused into the backward
    projection against the same iteration followed by the standalone step."""
    work = [p.clone() for p in params]
    opt = R.Adam(*work)
    gen = torch.Generator(device=work[0].device).manual_seed(5)
    grads = {k: torch.randn(p.shape, device=p.device, generator=gen) * 1e-3 for k, p in zip(R.GROUPS, work)}
    ctx = R.context(work[0].device)
    for _ in range(warmup):
        opt.step(work, grads)
    ctx.set_timing(True)
    ctx.timing(reset=True)
    sec = timed_steps(lambda: opt.step(work, grads), steps, 0)
    ms_k, n_k = ctx.timing(reset=True)["adam"]
    ctx.set_timing(False)
    avg_us = 1e3 * ms_k / max(n_k, 1)
    elems = sum(p.numel() for p in work)
    alg = elems * 28
    ach = alg / (avg_us * 1e-6) / 1e9
    roof = dict(bound="hbm", kernel="adam", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(ach / HBM_PEAK_GBS, 4), traffic=stored_traffic("adam"), alg_bytes_per_launch=int(alg),
                avg_launch_us=round(avg_us, 2))
    log(f"adam step over {elems} elements: {avg_us:.1f} us per launch, {ach:.0f} GB/s")
    px = cam.width * cam.height
    g_plain = R.Graph(*work, [cam], [target], s, depth_weight=DEPTH_W)

    def unfused():
        g_plain.launch()
        opt.step(work, g_plain.grads)
    ms_unfused = timed_steps(unfused, steps, warmup) * 1e3
    g_plain.sync()
    g_plain.free()
    g_fused = R.Graph(*work, [cam], [target], s, depth_weight=DEPTH_W, optimizer=opt)
    ms_fused = timed_steps(g_fused.launch, steps, warmup) * 1e3
    g_fused.sync()
    g_fused.free()
    log(f"iteration with Adam: fused {ms_fused:.3f} ms, graph + standalone step {ms_unfused:.3f} ms")
    return {"workload": "Adam (3D Gaussian splatting rates) over the headline map: every parameter row",
            "elements": elems, "standalone_step_ms": round(sec * 1e3, 4), "roofline": roof,
            "iteration_fused_ms": round(ms_fused, 4), "iteration_fused_Mpixel_s": round(px / ms_fused / 1e3, 3),
            "iteration_unfused_ms": round(ms_unfused, 4),
            "iteration_unfused_Mpixel_s": round(px / ms_unfused / 1e3, 3)}


def tsdf_leg(R, torch, dev, log):
    """TSDF fusion (Eq. 6-9) of ray-cast depth frames of the room at 1 cm voxels, at the
    headline and the paper's full resolution: ms and Mpixel/s per fused frame once the
    map holds the scene (host-timed), and the roofline of the per-voxel update kernel
    (16 bytes per voxel of a met block: distance and weight read and written, plus one
    depth read per pixel)."""
    import scenes
    res = {}
    for W, H in ((640, 480), (1752, 1168)):
        room = scenes.Room(np.random.default_rng(31), (6.0, 5.0, 3.0), 20)
        frames = []
        for k in range(8):
            cam = room.random_camera(np.random.default_rng(3100 + k), W, H)
            depth, _ = room.raycast(cam, with_color=False)
            frames.append((cam, torch.from_numpy(depth.astype(np.float32)).to(dev)))
        m = R.TsdfMap(dev, max_blocks=1 << 18)
        met = []
        for cam, d in frames:                     # first pass: allocation of the scene
            m.integrate(d, cam)
            met.append(m.info()["met_last"])
        reps = 5
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for cam, d in frames:
                m.integrate(d, cam)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / (reps * len(frames))
        ctx = R.context(dev)
        ctx.set_timing(True)
        ctx.timing(reset=True)
        for _ in range(reps):
            for cam, d in frames:
                m.integrate(d, cam)
        kt = ctx.timing(reset=True)
        ctx.set_timing(False)
        inf = m.info()
        m.free()
        fuse_us = 1e3 * kt["tsdf_fuse"][0] / max(kt["tsdf_fuse"][1], 1)
        alloc_us = 1e3 * kt["tsdf_alloc"][0] / max(kt["tsdf_alloc"][1], 1)
        alg = float(np.mean(met)) * 512 * 16 + W * H * 4
        ach = alg / (fuse_us * 1e-6) / 1e9
        key = f"{W}x{H}"
        res[key] = {"ms_per_frame": round(sec * 1e3, 4), "Mpixel_s": round(W * H / sec / 1e6, 1),
                    "blocks": inf["blocks"], "met_blocks_per_frame": int(np.mean(met)),
                    "alloc_us": round(alloc_us, 2), "fuse_us": round(fuse_us, 2),
                    "fuse_roofline": dict(bound="hbm", kernel="tsdf_fuse", achieved=round(ach, 1),
                                          peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4),
                                          traffic=stored_traffic("tsdf_integrate"),
                                          alg_bytes_per_launch=int(alg), avg_launch_us=round(fuse_us, 2))}
        log(f"tsdf {key}: {res[key]}")
    res["workload"] = "8 ray-cast depth frames of the room, 1 cm voxels, band 8 cm, 17 samples per pixel, each fused 5 more times"
    return res


def host_cpu():
    """The host CPU model (/proc/cpuinfo), as lscpu names it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def scale_leg(R, torch, w, views, s, steps, warmup, step_hbm, what):
    """One captured forward + L1 + backward of ``views`` (None: all) of workload ``w``:
    Mpixel/s, HBM fraction of the algorithmic bytes, sizes and per-tile list lengths."""
    dev = torch.device("cuda", 0)
    cams = w.cameras if views is None else [w.cameras[v] for v in views]
    tgs = w.targets if views is None else [w.targets[v] for v in views]
    params = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in w.gaussians.arrays()]
    targets = [(torch.from_numpy(tc).to(dev), torch.from_numpy(td).to(dev)) for tc, td in tgs]
    px = sum(c.width * c.height for c in cams)
    log(f"{w.name}: {w.gaussians.n} Gaussians, {len(cams)} views, {px} pixels")
    st = step_stats(R, params, cams, targets, s)
    g = R.Graph(*params, cams, targets, s, depth_weight=DEPTH_W)
    ms = timed_steps(g.launch, steps, warmup) * 1e3
    g.sync()
    g.free()
    res = {"workload": what, "gaussians": w.gaussians.n, "views": len(cams), "pixels": px,
           "ms_per_step": round(ms, 3), "Mpixel_s": round(px / (ms * 1e-3) / 1e6, 2), "hbm": step_hbm(st, ms),
           "work": {k: st[k] for k in ("N_vis", "M", "E_fwd", "E_bwd", "tiles")},
           "tile_list_length": st["tile_list_length"],
           "steps": steps}
    log(w.name, res)
    del params, targets
    torch.cuda.empty_cache()
    return res


def autograd_leg(R, torch, w, s, steps, log):
    """1M Gaussians at 1200x680 through the autograd Function: forward, an L1 colour loss
    in torch, backward to every parameter."""
    dev = torch.device("cuda", 0)
    cam = w.cameras[0]
    params = [torch.from_numpy(np.ascontiguousarray(a)).to(dev).requires_grad_(True) for a in w.gaussians.arrays()]
    gen = torch.Generator(device=dev).manual_seed(3)
    target = torch.rand((3, cam.height, cam.width), device=dev, generator=gen)

    def one():
        for p in params:
            p.grad = None
        col, dep, alp = R.GSRasterize.apply(*params, [cam], s)
        loss = (col - target).abs().mean()
        loss.backward()
    ms = timed_steps(one, steps, 2) * 1e3
    px = cam.width * cam.height
    res = {"workload": f"{w.gaussians.n} Gaussians on 50 planes, one 1200x680 view, torch.autograd.Function "
                       f"forward + L1 (torch) + backward", "ms_per_step": round(ms, 3),
           "Mpixel_s": round(px / (ms * 1e-3) / 1e6, 2), "steps": steps}
    log("cfg3 autograd", res)
    del params
    torch.cuda.empty_cache()
    return res


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
    ap.add_argument("--rect-tiles", action="store_true", help="full tile rectangles instead of exact tile lists")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-seed", action="store_true", help="skip the quadtree seeding measurement")
    ap.add_argument("--no-optim", action="store_true", help="skip the optimiser-step measurement")
    ap.add_argument("--no-tsdf", action="store_true", help="skip the TSDF fusion measurement")
    ap.add_argument("--autotune", type=int, default=0,
                    help="1: time the headline at the autotuner's pick instead of the given launch shape "
                         "(the pick is reported either way)")
    ap.add_argument("--no-scale", action="store_true", help="skip the 1M (1200x680) and 3M (16 x 1752x1168) legs")
    ap.add_argument("--only-headline", action="store_true",
                    help="profiling runs: the headline launch shape only (no autotuner sweep, no other "
                         "tile-list kind, no batched, scale or CPU legs), so that per-kernel counters "
                         "and durations average one shape")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="first run a plain device copy of this many MiB (counter calibration under rocprofv3)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU: turn two rocprofv3 --pmc runs of bench.py --copy-probe MB into "
                         "profiles/traffic.json and exit")
    args = ap.parse_args()
    if args.traffic_from:
        from types import SimpleNamespace
        shape = shape_key(SimpleNamespace(tile=args.tile, batch=args.batch, exact_tiles=not args.rect_tiles))
        t = traffic_from_counters(args.traffic_from[0], args.traffic_from[1], args.copy_probe or 256, shape)
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(t, f, indent=1)
            f.write("\n")
        for k, v in sorted(t["kernels"].items(), key=lambda kv: -kv[1]["fetch_bytes"] - kv[1]["write_bytes"]):
            print(f"{k:16s} x{v['dispatches']:4d}  fetch {v['fetch_bytes'] / 1e6:9.2f} MB  "
                  f"write {v['write_bytes'] / 1e6:9.2f} MB")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); multi-GPU runs are "
              "not part of it.", file=sys.stderr)
        sys.exit(2)

    import torch
    import scenes
    from paper_2408_12677_amd import rasterize as R

    if args.copy_probe:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters give the
        # scale that turns the counters of the rasterizer kernels into HBM bytes
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 3 copies of {nbytes} bytes")
        del src, dst
    log("generating the 500k-Gaussian room map and its 8 orbit views")
    t0 = time.perf_counter()
    w = scenes.make_cfg4()
    log(f"  generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda", 0)
    params = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in w.gaussians.arrays()]
    targets = [(torch.from_numpy(tc).to(dev), torch.from_numpy(td).to(dev)) for tc, td in w.targets]
    # the headline launch shape: fixed (tile 16, batch 256, exact tile lists: the autotuner's
    # usual pick on MI355X) so the timing and the stored counters describe the same kernels
    s = R.Settings(tile=args.tile, batch=args.batch, exact_tiles=not args.rect_tiles)
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
    os.environ.setdefault("GSR_AUTOTUNE_CACHE", os.path.join("/tmp", "gsr_bench_autotune.txt"))
    if args.only_headline:
        args.no_batched = args.no_scale = args.no_cpu_baseline = True
        s_tuned, tune_ms = None, None
    else:
        s_tuned, tune_ms = R.autotune(*params, [cam], s, use_cache=False)
        log(f"autotuner's pick: tile {s_tuned.tile}, batch {s_tuned.batch}, exact tiles {s_tuned.exact_tiles} "
            f"({tune_ms:.3f} ms/step of kernel time)")
        if args.autotune:
            s = s_tuned
    stats = step_stats(R, params, [cam], [targets[HEADLINE_VIEW]], s)
    log("headline stats", stats)

    # headline, eager per-view calls (forward, loss, backward; one host read-back)
    log(f"timing {args.steps} eager headline steps ({args.warmup} warm-up)")
    ms_eager = timed_steps(lambda: step(head), args.steps, args.warmup) * 1e3
    # the same steps with the per-kernel event timer on (kernel durations)
    ctx.set_timing(True)
    ctx.timing(reset=True)
    ms_timed = timed_steps(lambda: step(head), args.steps, 0) * 1e3
    ktimes = ctx.timing(reset=True)
    ctx.set_timing(False)
    # headline, captured step replayed (the repeated iterations of one keyframe)
    g1 = R.Graph(*params, [cam], [targets[HEADLINE_VIEW]], s, depth_weight=DEPTH_W)
    log(f"timing {args.steps} graph-replayed headline steps")
    ms = timed_steps(g1.launch, args.steps, args.warmup) * 1e3
    g1.sync()
    g1.free()
    # the same step with the other kind of tile list (rectangles / exact ellipse-tile
    # lists: the same images, different list lengths)
    import dataclasses
    sx = dataclasses.replace(s, exact_tiles=not s.exact_tiles)
    kinds = (s,) if args.only_headline else (s, sx)
    ms_kind = {s.exact_tiles: ms}
    if not args.only_headline:
        gx = R.Graph(*params, [cam], [targets[HEADLINE_VIEW]], sx, depth_weight=DEPTH_W)
        log(f"timing {args.steps} graph-replayed headline steps with exact tile lists {sx.exact_tiles}")
        ms_kind[sx.exact_tiles] = timed_steps(gx.launch, args.steps, args.warmup) * 1e3
        gx.sync()
        gx.free()
    pairs = {}
    for kind in kinds:
        _, sv = R.forward(*params, [cam], kind)
        pairs[kind.exact_tiles] = int(sv.debug_export()["ranges"][:, 1].max(initial=0))
        sv.free()

    per_kernel = {k: dict(ms_per_step=t / args.steps, launches_per_step=n / args.steps, avg_launch_us=1e3 * t / n)
                  for k, (t, n) in ktimes.items() if n > 0}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_step"])
    alg = {k: kernel_bytes(k, stats) for k in per_kernel}
    step_bytes = sum(alg[k] * per_kernel[k]["launches_per_step"] for k in per_kernel)
    dk = per_kernel[dom]
    roofline = kernel_roofline(dom, stats, alg[dom], dk["avg_launch_us"], s)

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
                               "forward + L1(colour)+0.1 L1(depth) + backward, captured step replayed",
                   "gaussians": stats["N"], "width": cam.width, "height": cam.height, "sh_degree": 3,
                   "tile": s.tile, "batch": s.batch, "exact_tiles": s.exact_tiles, "path": "hipGraph, one view"},
        "autotune": None if s_tuned is None else {
            "tile": s_tuned.tile, "batch": s_tuned.batch, "exact_tiles": s_tuned.exact_tiles,
            "kernel_ms_per_step": round(tune_ms, 4), "used": bool(args.autotune)},
        "tile_lists": {("exact" if k else "rectangles"): {"ms_per_step": round(v, 4),
                                                         "Mpixel_s": round(px_head / (v * 1e-3) / 1e6, 3),
                                                         "pairs": pairs[k]} for k, v in ms_kind.items()},
        "eager_per_view": {"ms_per_step": round(ms_eager, 4),
                           "Mpixel_s": round(px_head / (ms_eager * 1e-3) / 1e6, 3)},
        "hbm": {"alg_bytes_per_step": int(step_bytes),
                "alg_GBps": round(step_bytes / (ms * 1e-3) / 1e9, 1),
                "frac_of_peak": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline": roofline,
        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in per_kernel.items()},
        "ms_per_step_with_event_timer": round(ms_timed, 4),
        "work": {k: stats[k] for k in ("N_vis", "M", "E_rows", "P", "tiles", "sort_passes", "E_fwd", "E_bwd",
                                       "E_used", "wave_hits", "tile_list_length")},
    }
    out["roofline_all"] = {k: kernel_roofline(k, stats, alg[k], per_kernel[k]["avg_launch_us"], s)
                           for k in per_kernel if alg.get(k)}

    def step_hbm(st, ms_step):
        """Algorithmic bytes of one step (the headline's launches per step, ``st``'s sizes)."""
        b = sum(kernel_bytes(k, st) * per_kernel[k]["launches_per_step"] for k in per_kernel)
        return {"alg_bytes_per_step": int(b), "alg_GBps": round(b / (ms_step * 1e-3) / 1e9, 1),
                "frac_of_peak": round(b / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


    if not args.no_batched:
        allv = list(range(len(w.cameras)))
        px_all = sum(c.width * c.height for c in w.cameras)
        k2 = max(3, args.steps // 3)
        log(f"timing the 8 views: one captured batched step vs 8 eager per-view steps, {k2} steps each")
        gb = R.Graph(*params, w.cameras, targets, s, depth_weight=DEPTH_W)
        ms_b = timed_steps(gb.launch, k2, 2) * 1e3
        gb.sync()
        binfo = gb.info()
        gb.free()

        def seq():
            for i, v in enumerate(allv):
                step([v], accumulate=i > 0)
        ms_s = timed_steps(seq, k2, 1) * 1e3
        # the same 8 per-view steps, each captured in a graph of its own (launch overhead and
        # host read-backs removed, no batching): separates the gain of capture from that of
        # batching
        gvs = [R.Graph(*params, [w.cameras[v]], [targets[v]], s, depth_weight=DEPTH_W) for v in allv]

        def seq_graphs():
            for gv in gvs:
                gv.launch()
        ms_sg = timed_steps(seq_graphs, k2, 1) * 1e3
        for gv in gvs:
            gv.sync()
            gv.free()
        bst = step_stats(R, params, w.cameras, targets, s)
        out["batched"] = {"views": len(allv), "pixels": px_all, "keys": binfo["num_keys"],
                          "batched_graph_ms": round(ms_b, 3),
                          "batched_graph_Mpixel_s": round(px_all / (ms_b * 1e-3) / 1e6, 2),
                          "per_view_graphs_ms": round(ms_sg, 3),
                          "per_view_graphs_Mpixel_s": round(px_all / (ms_sg * 1e-3) / 1e6, 2),
                          "per_view_eager_ms": round(ms_s, 3),
                          "per_view_eager_Mpixel_s": round(px_all / (ms_s * 1e-3) / 1e6, 2),
                          "hbm": step_hbm(bst, ms_b),
                          "work": {k: bst[k] for k in ("N_vis", "M", "E_fwd", "E_bwd", "tiles")},
                          "tile_list_length": bst["tile_list_length"],
                          "steps": k2}
        log("batched", out["batched"])

    if not args.no_scale:
        out["cfg2"] = scale_leg(R, torch, scenes.make_cfg2(), [0], s, args.steps, args.warmup, step_hbm,
                                "200k-Gaussian room map seeded from 640x480 views, view 0 "
                                              "(640x480), forward + L1 + backward, captured step")
        out["cfg3_autograd"] = autograd_leg(R, torch, scenes.make_cfg3(), s, max(3, args.steps // 3), log)
        out["cfg5"] = scale_leg(R, torch, scenes.make_cfg5(), None, s, max(3, args.steps // 6), 1, step_hbm,
                                "3M Gaussians seeded on a 10x8x3 m room with 200 boxes, 16 views "
                                              "1752x1168 in one captured step (forward + L1 + backward)")

    if not args.no_optim:
        out["optimiser"] = optimiser_leg(R, torch, params, cam, targets[HEADLINE_VIEW], s, args.steps,
                                         args.warmup, log)

    if not args.no_seed:
        out["seeding"] = seeding_leg(R, torch, dev, log)

    if not args.no_tsdf:
        out["tsdf"] = tsdf_leg(R, torch, dev, log)

    if not args.no_cpu_baseline:
        import oracle
        tc, td = w.targets[HEADLINE_VIEW]
        # this process's CPU share (a GPU machine gives each GPU 16 CPUs, whatever nproc shows)
        threads = max(1, min(16, len(os.sched_getaffinity(0))))

        def oracle_rate(th, budget):
            total, reps = 0.0, 0
            while total < budget and reps < 20:
                total += oracle.time_fwd_bwd(w.gaussians.arrays(), 3, [cam], [(tc, td)],
                                             oracle.Settings(tile=s.tile, threads=th, exact_tiles=s.exact_tiles),
                                             DEPTH_W)
                reps += 1
            return total / reps, reps
        log(f"timing the FP64 CPU oracle on headline steps ({threads} threads, >= 10 s, then 1 thread, >= 8 s)")
        sec, reps = oracle_rate(threads, 10.0)
        sec1, reps1 = oracle_rate(1, 8.0)
        out["cpu_baseline"] = {"value": round(px_head / sec / 1e6, 5), "unit": "Mpixel/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{reps} full headline steps (500k Gaussians, 640x480 fwd+L1+bwd) on "
                                         f"{threads} threads (tile-parallel, per-thread gradient buffers summed "
                                         f"in thread order), {sec:.2f} s each",
                               "host": host_cpu(), "nproc": os.cpu_count(),
                               "single_thread": {"value": round(px_head / sec1 / 1e6, 5), "sample":
                                                 f"{reps1} steps, {sec1:.2f} s each"}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
