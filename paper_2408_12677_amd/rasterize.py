"""PyTorch-facing API of libgsr: device memory and streams come from torch, every
computation runs in the HIP library (argument marshalling only here).

    images, saved = forward(means, scales, quats, opacities, sh, cameras)
    loss, gC, gD  = loss_l1(saved, images, targets, depth_weight=0.1)
    grads         = backward(saved, gC, gD)

``GSRasterize`` wraps forward/backward as a ``torch.autograd.Function``; the backward
recomputes per-pixel transmittance from the saved final value instead of storing
per-(pixel, Gaussian) state.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _native as N


@dataclass
class Settings:
    """Rendering rules; defaults: 16 px tiles, 256-record LDS batches, extent 3.33 sigma,
    low-pass 0.3 px^2, skip a < 1/255, clamp alpha at 0.99, stop at T < 1e-4, frustum
    guard band 0.15 x the image size per side, black bg."""
    tile: int = 16
    batch: int = 256
    extent_k: float = 3.33
    lowpass: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    guard: float = 0.15
    bg: tuple = (0.0, 0.0, 0.0)
    exact_tiles: bool = False   # GSR_EXACT_TILES: per tile row, only the columns the ellipse reaches
    normalized_depth: bool = False   # GSR_NORMALIZED_DEPTH: depth output D / (1 - T_final)
    check_finite: bool = False   # GSR_CHECK_FINITE: eager forwards reject NaN/Inf parameters
    jclamp: float = 0.0     # > 0: x/z, y/z clamped inside the projection's Jacobian (guard band)

    def c(self) -> N.Settings:
        return N.Settings(self.tile, self.batch, self.extent_k, self.lowpass, self.alpha_min, self.alpha_max,
                          self.T_min, self.guard, (ctypes.c_float * 3)(*self.bg),
                          (N.EXACT_TILES if self.exact_tiles else 0) | (N.NORMALIZED_DEPTH if self.normalized_depth else 0)
                          | (N.CHECK_FINITE if self.check_finite else 0), self.jclamp)


@dataclass
class Camera:
    """OpenCV pinhole camera; R (3x3) and t (3,) map world to camera: x_c = R x_w + t."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray = field(default_factory=lambda: np.eye(3, dtype=np.float32))
    t: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))
    znear: float = 0.01


def _cams(cameras):
    if not 1 <= len(cameras) <= N.MAX_VIEWS:
        raise ValueError(f"need 1..{N.MAX_VIEWS} cameras")
    arr = (N.Camera * len(cameras))()
    for i, c in enumerate(cameras):
        a = arr[i]
        a.width, a.height = int(c.width), int(c.height)
        a.fx, a.fy, a.cx, a.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        a.R[:] = [float(v) for v in np.asarray(c.R, np.float32).reshape(9)]
        a.t[:] = [float(v) for v in np.asarray(c.t, np.float32).reshape(3)]
        a.znear = float(getattr(c, "znear", 0.01))
    return arr


class Context:
    """A gsr_ctx bound to one device and one HIP stream.

    allocator (optional): an object with ``alloc(nbytes, stream) -> int`` (a device address,
    0 when it cannot) and ``free(ptr, stream)``, given to the library as its gsr_alloc; by
    default the library uses the device's stream-ordered pool."""

    def __init__(self, device: int, stream: int, allocator=None):
        lib = N.load()
        self.lib = lib
        self.device = device
        self.stream = stream
        self._alloc = None
        if allocator is not None:
            def _a(user, nbytes, strm):
                try:
                    return int(allocator.alloc(int(nbytes), strm or 0)) or None
                except Exception:  # noqa: BLE001 -- the library sees an allocation failure
                    return None

            def _f(user, ptr, strm):
                allocator.free(int(ptr), strm or 0)
            self._alloc = N.Alloc(N.ALLOC_FN(_a), N.FREE_FN(_f), None)
        h = ctypes.c_void_p()
        N.check(lib.gsr_ctx_create(device, ctypes.c_void_p(stream),
                                   ctypes.byref(self._alloc) if self._alloc is not None else None, ctypes.byref(h)))
        self.h = h

    def set_timing(self, on: bool):
        N.check(self.lib.gsr_ctx_set_timing(self.h, int(bool(on))), self.h)

    def timing(self, reset: bool = True) -> dict:
        """{kernel name: (total ms, launches)} accumulated since the last reset (synchronises)."""
        t = N.Timing()
        N.check(self.lib.gsr_ctx_get_timing(self.h, ctypes.byref(t), int(reset)), self.h)
        return {self.lib.gsr_kernel_name(i).decode(): (t.ms[i], t.launches[i]) for i in range(t.count)}

    def __del__(self):
        h = getattr(self, "h", None)
        if h and h.value:
            self.lib.gsr_ctx_destroy(h)
            self.h = None


_contexts: dict = {}
_active: list = []


class using:
    """Inside ``with using(ctx):`` every call of this module runs on ``ctx`` (for example a
    context with a caller's allocator) instead of the cached per-stream context."""

    def __init__(self, ctx: Context):
        self.ctx = ctx

    def __enter__(self):
        _active.append(self.ctx)
        return self.ctx

    def __exit__(self, *exc):
        _active.pop()


def context(device: torch.device | int | None = None) -> Context:
    """The cached context of ``device`` bound to torch's current stream there (or the one
    a ``using`` block selects)."""
    if _active:
        return _active[-1]
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(idx).cuda_stream
    key = (idx, stream)
    ctx = _contexts.get(key)
    if ctx is None:
        ctx = _contexts[key] = Context(idx, stream)
    return ctx


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, name, shape, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32 or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Saved:
    """Owner of a gsr_saved handle plus references that keep its inputs alive."""

    def __init__(self, ctx: Context, handle, keep, cameras, n, sh_degree):
        self.ctx = ctx
        self.h = handle
        self.keep = keep
        self.cameras = list(cameras)
        self.n = n
        self.sh_degree = sh_degree

    def info(self) -> dict:
        inf = N.Info()
        N.check(self.ctx.lib.gsr_saved_info(self.h, ctypes.byref(inf)), self.ctx.h)
        return {k: getattr(inf, k) for k, _ in N.Info._fields_}

    def debug_export(self) -> dict:
        inf = self.info()
        M, T, P, R = inf["num_keys"], inf["num_tiles"], inf["num_pixels"], inf["num_records"]
        out = dict(keys=np.zeros(M, np.uint64), values=np.zeros(M, np.uint32), ranges=np.zeros((T, 2), np.uint32),
                   T_final=np.zeros(P, np.float32), n_contrib=np.zeros(P, np.uint32),
                   tiles_touched=np.zeros(R, np.uint32), mu=np.zeros((R, 2), np.float32),
                   depth=np.zeros(R, np.float32), conic=np.zeros((R, 3), np.float32),
                   color=np.zeros((R, 3), np.float32), rect=np.zeros((R, 4), np.int32),
                   n_used=np.zeros(P, np.uint32))
        d = N.Debug(*(ctypes.c_void_p(out[k].ctypes.data) for k, _ in N.Debug._fields_))
        N.check(self.ctx.lib.gsr_debug_export(self.ctx.h, self.h, ctypes.byref(d)), self.ctx.h)
        used = int(out["ranges"][:, 1].max(initial=0))   # pairs in use (fewer with exact tiles)
        out["keys"], out["values"] = out["keys"][:used], out["values"][:used]
        return out

    def free(self):
        if self.h is not None and self.h.value:
            self.ctx.lib.gsr_saved_free(self.h)
        self.h = None
        self.keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _sh_degree(sh):
    K = sh.shape[1]
    deg = int(round(math.sqrt(K))) - 1
    if (deg + 1) ** 2 != K or not 0 <= deg <= 3:
        raise ValueError("sh must have shape [N, (deg+1)^2, 3] with deg in 0..3")
    return deg


def forward(means, scales, quats, opacities, sh, cameras, settings: Settings | None = None, save: bool = True):
    """Render every camera.  Returns ([(color[3,H,W], depth[H,W], alpha[H,W]) per view], Saved|None)."""
    settings = settings or Settings()
    dev = means.device
    n = means.shape[0]
    deg = _sh_degree(sh)
    _need(means, "means", (n, 3), dev)
    _need(scales, "scales", (n, 3), dev)
    _need(quats, "quats", (n, 4), dev)
    _need(opacities, "opacities", (n,), dev)
    _need(sh, "sh", (n, (deg + 1) ** 2, 3), dev)
    if n and quats.data_ptr() % 16:
        raise ValueError("quats must be 16-byte aligned")
    ctx = context(dev)
    cams = _cams(cameras)
    images = []
    outs = (N.ViewOut * len(cameras))()
    for i, c in enumerate(cameras):
        H, W = int(c.height), int(c.width)
        col = torch.empty((3, H, W), dtype=torch.float32, device=dev)
        dep = torch.empty((H, W), dtype=torch.float32, device=dev)
        alp = torch.empty((H, W), dtype=torch.float32, device=dev)
        images.append((col, dep, alp))
        outs[i] = N.ViewOut(col.data_ptr(), dep.data_ptr(), alp.data_ptr())
    g = N.Gaussians(n, deg, means.data_ptr(), scales.data_ptr(), quats.data_ptr(), opacities.data_ptr(),
                    sh.data_ptr())
    s = settings.c()
    h = ctypes.c_void_p()
    N.check(ctx.lib.gsr_forward(ctx.h, ctypes.byref(g), cams, len(cameras), ctypes.byref(s), outs,
                                ctypes.byref(h) if save else None), ctx.h)
    saved = Saved(ctx, h, (means, scales, quats, opacities, sh), cameras, n, deg) if save else None
    return images, saved


def loss_l1(saved: Saved, images, targets, depth_weight: float = 0.1):
    """Eq. 12 as a mean L1 colour error plus depth_weight x mean L1 depth error over valid target
    depths, summed over views.  Returns (loss[()], [dL/dcolor], [dL/ddepth])."""
    ctx = saved.ctx
    V = len(saved.cameras)
    dev = images[0][0].device
    outs = (N.ViewOut * V)()
    tg = (N.Target * V)()
    gcs, gds = [], []
    gcp = (ctypes.c_void_p * V)()
    gdp = (ctypes.c_void_p * V)()
    for i, ((col, dep, alp), (tc, td)) in enumerate(zip(images, targets)):
        _need(tc, "target color", col.shape, dev)
        if td is not None:
            _need(td, "target depth", dep.shape, dev)
        outs[i] = N.ViewOut(col.data_ptr(), dep.data_ptr(), alp.data_ptr())
        tg[i] = N.Target(tc.data_ptr(), None if td is None else td.data_ptr())
        gc = torch.empty_like(col)
        gd = torch.empty_like(dep)
        gcs.append(gc)
        gds.append(gd)
        gcp[i] = gc.data_ptr()
        gdp[i] = gd.data_ptr()
    loss = torch.empty((), dtype=torch.float32, device=dev)
    N.check(ctx.lib.gsr_loss_l1(ctx.h, saved.h, outs, tg, float(depth_weight), gcp, gdp,
                                ctypes.c_void_p(loss.data_ptr())), ctx.h)
    return loss, gcs, gds


def _view_grads(saved: Saved, g_color, g_depth, g_alpha, keep: list):
    """The per-view dL/d(outputs) as a gsr_view_grad array; every given tensor must have its
    view's image shape ([3,H,W] colour, [H,W] depth and alpha) on the parameters' device."""
    V = len(saved.cameras)
    dev = saved.keep[0].device
    gv = (N.ViewGrad * V)()
    for i, cam in enumerate(saved.cameras):
        H, W = int(cam.height), int(cam.width)

        def p(lst, name, shape):
            if lst is None or lst[i] is None:
                return None
            t = lst[i]
            if not isinstance(t, torch.Tensor):
                raise TypeError(f"{name}[{i}] must be a torch.Tensor")
            if tuple(t.shape) != shape or t.device != dev:
                raise ValueError(f"{name}[{i}] must have shape {shape} on {dev}, got {tuple(t.shape)} on {t.device}")
            t = t.contiguous().float()
            keep.append(t)
            return t.data_ptr()
        gv[i] = N.ViewGrad(p(g_color, "g_color", (3, H, W)), p(g_depth, "g_depth", (H, W)),
                           p(g_alpha, "g_alpha", (H, W)))
    return gv


def backward(saved: Saved, g_color, g_depth=None, g_alpha=None, grads=None, accumulate: bool = False,
             noalloc: bool = False):
    """dL/d(means, scales, quats, opacities, sh) for dL/d(outputs) given per view (None = 0).

    noalloc: run gsr_backward_noalloc (the library's fixed device scratch array instead of
    pool memory; pass `grads` too for a call that allocates nothing)."""
    ctx = saved.ctx
    means, scales, quats, opacities, sh = saved.keep
    keep = []
    gv = _view_grads(saved, g_color, g_depth, g_alpha, keep)
    if grads is None:
        grads = dict(means=torch.empty_like(means), scales=torch.empty_like(scales), quats=torch.empty_like(quats),
                     opacities=torch.empty_like(opacities), sh=torch.empty_like(sh))
        accumulate = False
    for k, ref in zip(GROUPS, saved.keep):
        if grads.get(k) is not None:
            _need(grads[k], f"grads[{k!r}]", ref.shape, ref.device)
    go = N.GaussianGrads(*(None if grads.get(k) is None else grads[k].data_ptr()
                           for k in ("means", "scales", "quats", "opacities", "sh")))
    fn = ctx.lib.gsr_backward_noalloc if noalloc else ctx.lib.gsr_backward
    N.check(fn(ctx.h, saved.h, gv, ctypes.byref(go), N.ACCUMULATE if accumulate else 0), ctx.h)
    return grads


class GSRasterize(torch.autograd.Function):
    """Differentiable render of V views; outputs (color_0, depth_0, alpha_0, color_1, ...)."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, cameras, settings):
        images, saved = forward(means, scales, quats, opacities, sh, cameras, settings, save=True)
        ctx.saved_handle = saved
        ctx.views = len(cameras)
        return tuple(t for img in images for t in img)

    @staticmethod
    def backward(ctx, *grads):
        saved = ctx.saved_handle
        V = ctx.views
        gc = [grads[3 * i] for i in range(V)]
        gd = [grads[3 * i + 1] for i in range(V)]
        ga = [grads[3 * i + 2] for i in range(V)]
        out = backward(saved, gc, gd, ga)
        saved.free()
        ctx.saved_handle = None
        return out["means"], out["scales"], out["quats"], out["opacities"], out["sh"], None, None


def render(means, scales, quats, opacities, sh, cameras, settings: Settings | None = None):
    """Autograd-enabled render; returns [(color, depth, alpha)] per camera."""
    flat = GSRasterize.apply(means, scales, quats, opacities, sh, list(cameras), settings or Settings())
    return [tuple(flat[3 * i:3 * i + 3]) for i in range(len(cameras))]


def _param_checks(means, scales, quats, opacities, sh):
    dev = means.device
    n = means.shape[0]
    deg = _sh_degree(sh)
    _need(means, "means", (n, 3), dev)
    _need(scales, "scales", (n, 3), dev)
    _need(quats, "quats", (n, 4), dev)
    _need(opacities, "opacities", (n,), dev)
    _need(sh, "sh", (n, (deg + 1) ** 2, 3), dev)
    if n and quats.data_ptr() % 16:
        raise ValueError("quats must be 16-byte aligned")
    return dev, n, deg


class Graph:
    """One forward + L1 loss + backward step of several views, captured in a hipGraph.

    The parameter tensors, targets and the output buffers created here are bound at
    capture; ``launch()`` re-runs the step on their current contents (update the
    parameters in place between launches).  ``images``, ``grad_color``/``grad_depth``,
    ``grads`` and ``loss`` hold the latest step's results once the stream reaches it.
    """

    def __init__(self, means, scales, quats, opacities, sh, cameras, targets, settings: Settings | None = None,
                 depth_weight: float = 0.1, headroom: float = 0.25, optimizer: "Adam | None" = None):
        settings = settings or Settings()
        dev, n, deg = _param_checks(means, scales, quats, opacities, sh)
        self.ctx = context(dev)
        lib = self.ctx.lib
        self.cameras = list(cameras)
        V = len(self.cameras)
        self.params = (means, scales, quats, opacities, sh)
        self.targets = [(tc, td) for tc, td in targets]
        self.images, outs = [], (N.ViewOut * V)()
        tg = (N.Target * V)()
        self.grad_color, self.grad_depth = [], []
        gcp, gdp = (ctypes.c_void_p * V)(), (ctypes.c_void_p * V)()
        for i, c in enumerate(self.cameras):
            H, W = int(c.height), int(c.width)
            col = torch.empty((3, H, W), dtype=torch.float32, device=dev)
            dep = torch.empty((H, W), dtype=torch.float32, device=dev)
            alp = torch.empty((H, W), dtype=torch.float32, device=dev)
            self.images.append((col, dep, alp))
            outs[i] = N.ViewOut(col.data_ptr(), dep.data_ptr(), alp.data_ptr())
            tc, td = self.targets[i]
            _need(tc, "target color", col.shape, dev)
            if td is not None:
                _need(td, "target depth", dep.shape, dev)
            tg[i] = N.Target(tc.data_ptr(), None if td is None else td.data_ptr())
            gc, gd = torch.empty_like(col), torch.empty_like(dep)
            self.grad_color.append(gc)
            self.grad_depth.append(gd)
            gcp[i], gdp[i] = gc.data_ptr(), gd.data_ptr()
        self.optimizer = optimizer
        if optimizer is None:
            self.grads = dict(means=torch.empty_like(means), scales=torch.empty_like(scales),
                              quats=torch.empty_like(quats), opacities=torch.empty_like(opacities),
                              sh=torch.empty_like(sh))
            gg = ctypes.byref(N.GaussianGrads(*(self.grads[k].data_ptr() for k in GROUPS)))
        else:   # each launch ends with one Adam step applied to the parameters in place
            optimizer._check(self.params)
            self.grads = None
            gg = None
        self.loss = torch.zeros((), dtype=torch.float32, device=dev)
        g = N.Gaussians(n, deg, means.data_ptr(), scales.data_ptr(), quats.data_ptr(), opacities.data_ptr(),
                        sh.data_ptr())
        s = settings.c()
        self.settings = settings
        h = ctypes.c_void_p()
        N.check(lib.gsr_graph_create(self.ctx.h, ctypes.byref(g), _cams(self.cameras), V, ctypes.byref(s), outs, tg,
                                     float(depth_weight), gcp, gdp, gg,
                                     ctypes.c_void_p(self.loss.data_ptr()), float(headroom),
                                     None if optimizer is None else ctypes.byref(optimizer.c),
                                     ctypes.byref(h)),
                self.ctx.h)
        self.h = h

    def launch(self):
        N.check(self.ctx.lib.gsr_graph_launch(self.h), self.ctx.h)

    def sync(self):
        N.check(self.ctx.lib.gsr_graph_sync(self.h), self.ctx.h)

    def info(self) -> dict:
        inf = N.Info()
        ck, cv = ctypes.c_int64(), ctypes.c_int64()
        N.check(self.ctx.lib.gsr_graph_info(self.h, ctypes.byref(inf), ctypes.byref(ck), ctypes.byref(cv)),
                self.ctx.h)
        d = {k: getattr(inf, k) for k, _ in N.Info._fields_}
        d.update(capacity_keys=ck.value, capacity_visible=cv.value)
        return d

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.ctx.lib.gsr_graph_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def autotune(means, scales, quats, opacities, sh, cameras, settings: Settings | None = None,
             use_cache: bool = True):
    """Pick (tile, batch, exact tile lists or not) for this workload by timing forward +
    backward at every choice (or from the cache).  Returns (settings, step ms)."""
    import dataclasses
    settings = settings or Settings()
    dev, n, deg = _param_checks(means, scales, quats, opacities, sh)
    ctx = context(dev)
    g = N.Gaussians(n, deg, means.data_ptr(), scales.data_ptr(), quats.data_ptr(), opacities.data_ptr(),
                    sh.data_ptr())
    s = settings.c()
    ms = ctypes.c_float()
    N.check(ctx.lib.gsr_autotune(ctx.h, ctypes.byref(g), _cams(cameras), len(cameras), ctypes.byref(s),
                                 0 if use_cache else N.AUTOTUNE_NO_CACHE, ctypes.byref(ms)), ctx.h)
    return (dataclasses.replace(settings, tile=int(s.tile), batch=int(s.batch),
                                exact_tiles=bool(s.flags & N.EXACT_TILES)), float(ms.value))


def seed(rgb, depth, camera, measure: str = "contrast", threshold: float = 0.1, min_side: int = 4,
         opacity: float = 0.5, sh_degree: int = 0, tsdf: "TsdfMap | None" = None):
    """Quadtree seeding and Gaussian initialisation of one RGB-D frame (gsr_seed).

    rgb [3,H,W] and depth [H,W] are float32 device tensors of the camera's size.  With a
    TSDF map (that has fused this frame) a leaf is kept only where the voxel at its mean
    has weight 1.  Returns a dict of means [n,3], scales [n,3], quats [n,4], opacities
    [n], sh [n,K,3] and the cells' leaves [n,4] (x0, y0, w, h)."""
    H, W = int(camera.height), int(camera.width)
    dev = rgb.device
    _need(rgb, "rgb", (3, H, W), dev)
    _need(depth, "depth", (H, W), dev)
    m = {"contrast": N.SEED_CONTRAST, "depth_variance": N.SEED_DEPTH_VARIANCE}[measure]
    s = N.SeedSettings(m, float(threshold), int(min_side), float(opacity), int(sh_degree))
    cap = (-(-W // int(min_side))) * (-(-H // int(min_side)))
    K = (int(sh_degree) + 1) ** 2
    f = dict(device=dev, dtype=torch.float32)
    out = dict(means=torch.empty((cap, 3), **f), scales=torch.empty((cap, 3), **f), quats=torch.empty((cap, 4), **f),
               opacities=torch.empty(cap, **f), sh=torch.empty((cap, K, 3), **f),
               leaves=torch.empty((cap, 4), dtype=torch.int32, device=dev))
    so = N.SeedOut(*(out[k].data_ptr() for k in ("means", "scales", "quats", "opacities", "sh", "leaves")))
    ctx = context(dev)
    n = ctypes.c_int64()
    N.check(ctx.lib.gsr_seed(ctx.h, ctypes.byref(_cams([camera])[0]), _ptr(rgb), _ptr(depth), ctypes.byref(s),
                             None if tsdf is None else tsdf.h, ctypes.byref(so), cap, ctypes.byref(n)), ctx.h)
    return {k: v[:n.value] for k, v in out.items()}


GROUPS = ("means", "scales", "quats", "opacities", "sh")


class Adam:
    """Adam over one Gaussian map (gsr_adam): the moments, in the parameter layouts, and
    the device step counter live here.  Rates and betas default to gsr_adam_default's
    (keyword arguments lr_means, lr_scales, lr_quats, lr_opacities, lr_sh_dc, lr_sh_rest,
    beta1, beta2, eps override them)."""

    def __init__(self, means, scales, quats, opacities, sh, **hyper):
        dev, n, deg = _param_checks(means, scales, quats, opacities, sh)
        self.device, self.n, self.sh_degree = dev, n, deg
        params = (means, scales, quats, opacities, sh)
        self.shapes = tuple(p.shape for p in params)
        self.m = {k: torch.zeros_like(p) for k, p in zip(GROUPS, params)}
        self.v = {k: torch.zeros_like(p) for k, p in zip(GROUPS, params)}
        self.state = torch.zeros(4, dtype=torch.int32, device=dev)
        self.ctx = context(dev)
        c = N.Adam()
        N.check(self.ctx.lib.gsr_adam_default(ctypes.byref(c)))
        for k, val in hyper.items():
            if k not in {f for f, _ in N.Adam._fields_[:9]}:
                raise TypeError(f"unknown Adam setting {k!r}")
            setattr(c, k, float(val))
        c.m = N.GaussianGrads(*(self.m[k].data_ptr() for k in GROUPS))
        c.v = N.GaussianGrads(*(self.v[k].data_ptr() for k in GROUPS))
        c.state = self.state.data_ptr()
        self.c = c

    def _check(self, params):
        if tuple(p.shape for p in params) != self.shapes:
            raise ValueError("parameter shapes differ from the optimiser's")

    @property
    def steps(self) -> int:
        return int(self.state[0].item())

    def step(self, params, grads: dict):
        """One Adam step of params (means, scales, quats, opacities, sh; updated in place)
        from grads (dict of the same layouts)."""
        self._check(params)
        for k, p in zip(GROUPS, params):
            _need(grads[k], f"grad {k}", p.shape, self.device)
        pp = N.GaussianGrads(*(p.data_ptr() for p in params))
        gg = N.GaussianGrads(*(grads[k].data_ptr() for k in GROUPS))
        N.check(self.ctx.lib.gsr_adam_step(self.ctx.h, self.n, self.sh_degree, ctypes.byref(pp), ctypes.byref(gg),
                                           ctypes.byref(self.c)), self.ctx.h)


def backward_adam(saved: Saved, opt: Adam, g_color, g_depth=None, g_alpha=None):
    """gsr_backward_adam: the backward of `saved` with one Adam step applied at once to
    the parameter tensors given to forward (updated in place; no gradients are written)."""
    ctx = saved.ctx
    opt._check(saved.keep)
    keep = []
    gv = _view_grads(saved, g_color, g_depth, g_alpha, keep)
    N.check(ctx.lib.gsr_backward_adam(ctx.h, saved.h, gv, ctypes.byref(opt.c)), ctx.h)


class Schedule:
    """The keyframe-list optimisation schedule (gsr_schedule): step(frame, new_gaussians)
    returns (is_keyframe, [frame rendered by each iteration])."""

    def __init__(self, m: int, n: int, threshold: int = 50, store_all: bool = False, seed: int = 0):
        self.lib = N.load()
        s = N.ScheduleSettings(int(m), int(n), int(threshold), int(bool(store_all)), int(seed) & (2 ** 64 - 1))
        h = ctypes.c_void_p()
        N.check(self.lib.gsr_schedule_create(ctypes.byref(s), ctypes.byref(h)))
        self.h, self.m = h, int(m)
        self._buf = (ctypes.c_int64 * max(1, self.m))()

    def step(self, frame: int, new_gaussians: int):
        cnt, kf = ctypes.c_int32(), ctypes.c_int32()
        N.check(self.lib.gsr_schedule_step(self.h, int(frame), int(new_gaussians), self._buf, max(1, self.m),
                                           ctypes.byref(cnt), ctypes.byref(kf)))
        return bool(kf.value), [int(self._buf[i]) for i in range(cnt.value)]

    @property
    def keyframes(self) -> list:
        cnt = ctypes.c_int64()
        N.check(self.lib.gsr_schedule_keyframes(self.h, None, 0, ctypes.byref(cnt)))
        buf = (ctypes.c_int64 * max(1, cnt.value))()
        N.check(self.lib.gsr_schedule_keyframes(self.h, buf, cnt.value, ctypes.byref(cnt)))
        return [int(buf[i]) for i in range(cnt.value)]

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.gsr_schedule_free(h)
            self.h = None


class KeyframeSteps:
    """Time steps of the keyframe-list optimisation (Sec. III-B-3; the m / n settings of
    Sec. IV-A) run as captured iterations.  ``step(frame, new_gaussians)`` asks the schedule
    (gsr_schedule) which view each iteration of the time step renders, then replays, per
    iteration, the captured optimisation iteration of that view: forward, L1 loss and
    backward with the fused Adam step (gsr_graph_create with an optimiser).  Each view's
    graph is captured on its first use and replayed afterwards, so a time step is a run of
    graph launches with no host read-back; ``sync()`` waits for them and reports a capacity
    overflow (re-create the object then).

    cameras and targets are indexed by frame; the parameters are updated in place."""

    def __init__(self, means, scales, quats, opacities, sh, cameras, targets, optimizer: "Adam",
                 schedule: Schedule, settings: Settings | None = None, depth_weight: float = 0.1,
                 headroom: float = 0.25):
        self.params = (means, scales, quats, opacities, sh)
        self.cameras, self.targets = cameras, targets
        self.optimizer, self.schedule = optimizer, schedule
        self.settings = settings or Settings()
        self.depth_weight, self.headroom = float(depth_weight), float(headroom)
        self.graphs: dict = {}
        self.iterations: list = []   # the frame rendered by every iteration so far

    def graph(self, frame: int) -> Graph:
        g = self.graphs.get(frame)
        if g is None:
            g = self.graphs[frame] = Graph(*self.params, [self.cameras[frame]], [self.targets[frame]], self.settings,
                                           self.depth_weight, self.headroom, optimizer=self.optimizer)
        return g

    def step(self, frame: int, new_gaussians: int):
        """Run one time step; returns (is_keyframe, [frame of each iteration])."""
        kf, iters = self.schedule.step(frame, new_gaussians)
        for f in iters:
            self.graph(f).launch()
        self.iterations.extend(iters)
        return kf, iters

    def sync(self):
        for g in self.graphs.values():
            g.sync()

    def free(self):
        for g in self.graphs.values():
            g.free()
        self.graphs.clear()


class TsdfMap:
    """A TSDF voxel-block map on one device (gsr_tsdf_*).  integrate(depth, camera) fuses a
    depth frame; export() copies the allocated blocks to the host."""

    def __init__(self, device=None, voxel: float = 0.01, trunc: float = 0.08, w_max: float = 100.0,
                 step: float = 0.01, weighting: str = "eq9", max_blocks: int = 1 << 16):
        self.ctx = context(device)
        s = N.TsdfSettings(float(voxel), float(trunc), float(w_max), float(step),
                           {"eq9": N.TSDF_EQ9, "unit": N.TSDF_UNIT_WEIGHT}[weighting])
        h = ctypes.c_void_p()
        N.check(self.ctx.lib.gsr_tsdf_create(self.ctx.h, ctypes.byref(s), int(max_blocks), ctypes.byref(h)),
                self.ctx.h)
        self.h = h
        self.max_blocks = int(max_blocks)

    def integrate(self, depth, camera):
        H, W = int(camera.height), int(camera.width)
        _need(depth, "depth", (H, W), depth.device)
        N.check(self.ctx.lib.gsr_tsdf_integrate(self.ctx.h, self.h, ctypes.byref(_cams([camera])[0]), _ptr(depth)),
                self.ctx.h)

    def info(self) -> dict:
        b, m, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint32()
        N.check(self.ctx.lib.gsr_tsdf_info(self.ctx.h, self.h, ctypes.byref(b), ctypes.byref(m), ctypes.byref(f)),
                self.ctx.h)
        return dict(blocks=b.value, met_last=m.value, flags=f.value)

    def export(self):
        """(coords [n,3] int32, tsdf [n,8,8,8], weight [n,8,8,8]) as numpy arrays, voxels
        indexed [z, y, x] within a block."""
        import numpy as np
        n = self.info()["blocks"]
        c = np.zeros((n, 3), np.int32)
        t = np.zeros((n, 8, 8, 8), np.float32)
        w = np.zeros((n, 8, 8, 8), np.float32)
        cnt = ctypes.c_int64()
        N.check(self.ctx.lib.gsr_tsdf_export(self.ctx.h, self.h, c.ctypes.data_as(ctypes.c_void_p),
                                             t.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
                                             n, ctypes.byref(cnt)), self.ctx.h)
        return c, t, w

    def weights(self, points):
        """Weight of the voxel holding each point (points: float32 device tensor [n,3])."""
        _need(points, "points", (points.shape[0], 3), points.device)
        out = torch.empty(points.shape[0], dtype=torch.float32, device=points.device)
        N.check(self.ctx.lib.gsr_tsdf_weights(self.ctx.h, self.h, _ptr(points), int(points.shape[0]), _ptr(out)),
                self.ctx.h)
        return out

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.ctx.lib.gsr_tsdf_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
