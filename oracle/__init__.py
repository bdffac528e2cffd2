"""Plain FP64 CPU oracle of the differentiable tile-based Gaussian-splatting rasterizer.

TEST INFRASTRUCTURE ONLY: the product library never imports, links or calls
anything here.  Only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP path; the two meet only
in the seeded input generators of ``scenes``.

What it computes (GSFusion, Sec. III-A-2 and III-B-3):

* the 3D Gaussian covariance Sigma = R S S^T R^T (Eq. 2), its perspective
  projection mu = pi(T^-1 p) (Eq. 4) and EWA covariance J W Sigma W^T J^T
  (Eq. 5) plus a screen-space low-pass, the conic of the 2D splat (Eq. 3);
* SH colour: 0.5 + sum_k sh_k Y_k(view direction), clamped at zero;
* tile keys (tile id << 32 | binary32 depth bits), a stable sort and tile
  ranges, with the discrete stage as an exact binary32 operation sequence;
* front-to-back alpha compositing (Eq. 11) of colour, depth and alpha with an
  opacity clamp, a skip rule for faint splats and early termination;
* the L1 loss (Eq. 12) plus a weighted L1 depth term, and the exact reverse-mode
  gradients to means, scales, rotations, opacities and SH coefficients.

``brute.py`` is an independent NumPy/SciPy implementation of the same per-pixel
definition without tiles, used to pin this one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

# near_a / near_T count values within this many times the ambiguity margins (kWide in
# oracle.cpp): a window this much narrower holds 1/NEAR_WIDE of them on average
NEAR_WIDE = 100.0

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

BUILD_CMD = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
             "-o", _LIB, _SRC, "-lpthread"]


def build(force: bool = False) -> str:
    """Compile liboracle.so (host C++ only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(BUILD_CMD)
    return _LIB


class _Cam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("znear", ctypes.c_float)]


class _Set(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("extent_k", ctypes.c_float), ("lowpass", ctypes.c_float),
                ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float), ("T_min", ctypes.c_float),
                ("guard", ctypes.c_float), ("bg", ctypes.c_float * 3), ("mu_fp32", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("amb_rel_a", ctypes.c_float), ("amb_rel_T", ctypes.c_float),
                ("exact_tiles", ctypes.c_int32), ("normalized_depth", ctypes.c_int32),
                ("window", ctypes.c_int32 * 4), ("jclamp", ctypes.c_float)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        lib.or_create.restype = P
        lib.or_create.argtypes = [P, P, P, P, P, ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int32, P]
        lib.or_destroy.argtypes = [P]
        lib.or_num_keys.restype = ctypes.c_int64
        lib.or_num_keys.argtypes = [P]
        lib.or_num_tiles.restype = ctypes.c_int64
        lib.or_num_tiles.argtypes = [P]
        lib.or_get_keys.argtypes = [P, P, P, P]
        lib.or_get_records.argtypes = [P] * 8
        lib.or_forward.argtypes = [P] * 12
        lib.or_backward.argtypes = [P] * 16
        lib.or_sh_eval.argtypes = [ctypes.c_int32, P, ctypes.c_int64, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Settings:
    """Rendering rules (paper readings: clamp 0.99, skip < 1/255, stop at T < 1e-4; only
    Gaussians whose centre lies in the view frustum, widened by ``guard`` x the image
    size on each side, are rendered)."""
    tile: int = 16
    extent_k: float = 3.33
    lowpass: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    guard: float = 0.15
    bg: tuple = (0.0, 0.0, 0.0)
    mu_fp32: bool = True
    threads: int = 1
    amb_rel_a: float = 1e-5     # binary32 a = o exp(-q/2) is good to ~5e-6 relative
    amb_rel_T: float = 1e-4     # binary32 T accumulates ~100 rounded products
    exact_tiles: bool = False   # per tile row, only the columns the ellipse can reach
    normalized_depth: bool = False   # depth output D / (1 - T_final)
    # (x0, y0, x1, y1): only pixels x0 <= x < x1, y0 <= y < y1 of every view are rendered and
    # differentiated (outputs elsewhere stay 0); None: every pixel
    window: tuple | None = None
    # > 0: x/z and y/z clamped inside the projection's Jacobian to +-jclamp W / (2 fx) and
    # +-jclamp H / (2 fy) (a guard band; 0: Eq. 5 as printed)
    jclamp: float = 0.0

    def _c(self):
        w = (0, 0, 0, 0) if self.window is None else tuple(int(x) for x in self.window)
        return _Set(self.tile, self.extent_k, self.lowpass, self.alpha_min, self.alpha_max, self.T_min, self.guard,
                    (ctypes.c_float * 3)(*self.bg), int(self.mu_fp32), int(self.threads), self.amb_rel_a,
                    self.amb_rel_T, int(self.exact_tiles), int(self.normalized_depth), (ctypes.c_int32 * 4)(*w),
                    float(self.jclamp))


def _cams(cameras):
    arr = (_Cam * len(cameras))()
    for i, c in enumerate(cameras):
        arr[i].width, arr[i].height = int(c.width), int(c.height)
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = c.fx, c.fy, c.cx, c.cy
        arr[i].R[:] = [float(v) for v in np.asarray(c.R, np.float32).ravel()]
        arr[i].t[:] = [float(v) for v in np.asarray(c.t, np.float32).ravel()]
        arr[i].znear = c.znear
    return arr


class Oracle:
    """One oracle evaluation of a Gaussian map seen by one or more cameras.

    ``params`` is (means, scales, quats, opacities, sh) in any float dtype; they
    are promoted to float64 (exact for float32 input).
    """

    def __init__(self, params, sh_degree, cameras, settings: Settings | None = None):
        self.lib = _load()
        self.settings = settings or Settings()
        self.params = [np.ascontiguousarray(np.asarray(a, np.float64)) for a in params]
        self.n = self.params[0].shape[0]
        self.sh_degree = int(sh_degree)
        self.K = (self.sh_degree + 1) ** 2
        self.cameras = list(cameras)
        self._cam = _cams(self.cameras)
        self._set = self.settings._c()
        m, s, q, o, sh = self.params
        self.h = self.lib.or_create(_ptr(m), _ptr(s), _ptr(q), _ptr(o), _ptr(sh), self.n, self.sh_degree,
                                    ctypes.byref(self._cam), len(self.cameras), ctypes.byref(self._set))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.or_destroy(h)
            self.h = None

    @property
    def num_keys(self) -> int:
        return int(self.lib.or_num_keys(self.h))

    @property
    def num_tiles(self) -> int:
        return int(self.lib.or_num_tiles(self.h))

    def keys(self):
        M, T = self.num_keys, self.num_tiles
        keys = np.zeros(M, np.uint64)
        vals = np.zeros(M, np.uint32)
        ranges = np.zeros((T, 2), np.uint32)
        self.lib.or_get_keys(self.h, _ptr(keys), _ptr(vals), _ptr(ranges))
        return keys, vals, ranges

    def records(self):
        VN = len(self.cameras) * self.n
        out = dict(visible=np.zeros(VN, np.uint8), mu=np.zeros((VN, 2), np.float32),
                   z=np.zeros(VN, np.float32), cov=np.zeros((VN, 3), np.float32),
                   rect=np.zeros((VN, 4), np.int32), conic=np.zeros((VN, 3)), color=np.zeros((VN, 3)))
        self.lib.or_get_records(self.h, *(_ptr(out[k]) for k in
                                          ("visible", "mu", "z", "cov", "rect", "conic", "color")))
        out["visible"] = out["visible"].astype(bool)
        return out

    def _split(self, flat, per_pixel_channels):
        res, off = [], 0
        for c in self.cameras:
            P = c.width * c.height * per_pixel_channels
            a = flat[off:off + P]
            res.append(a.reshape((per_pixel_channels, c.height, c.width)) if per_pixel_channels > 1
                       else a.reshape((c.height, c.width)))
            off += P
        return res

    def forward(self):
        """Per view: dict(color[3,H,W], depth, alpha, T_final, n_contrib, n_used, ambiguous,
        lo[5,H,W], hi[5,H,W], events, near_a, near_T).

        ``ambiguous`` marks pixels with a skip or stop decision inside its margin; lo/hi bound
        (colour 3, depth, alpha) over every correct outcome of those decisions (equal to the
        values elsewhere); ``events`` counts such decisions (-1: too many to enumerate, the
        bounds then hold the reference outcome only); near_a / near_T count the values within
        ``NEAR_WIDE`` times the margins."""
        P = sum(c.width * c.height for c in self.cameras)
        color = np.zeros(3 * P)
        depth, alpha, T = np.zeros(P), np.zeros(P), np.zeros(P)
        nc = np.zeros(P, np.int32)
        nu = np.zeros(P, np.int32)
        amb = np.zeros(P, np.uint8)
        lo, hi = np.zeros((P, 5)), np.zeros((P, 5))
        ev = np.zeros(P, np.int32)
        near = np.zeros((P, 2), np.int32)
        self.lib.or_forward(self.h, _ptr(color), _ptr(depth), _ptr(alpha), _ptr(T), _ptr(nc), _ptr(nu), _ptr(amb),
                            _ptr(lo), _ptr(hi), _ptr(ev), _ptr(near))
        cols = self._split(color, 3)
        outs = []
        off = 0
        split = [self._split(x, 1) for x in (depth, alpha, T, nc, nu, amb, ev)]
        for v, (d, a, t, n, u, m, e) in enumerate(zip(*split)):
            H, W = d.shape
            sl = slice(off, off + H * W)
            off += H * W
            outs.append(dict(color=cols[v], depth=d, alpha=a, T_final=t, n_contrib=n, n_used=u,
                             ambiguous=m.astype(bool), events=e,
                             lo=lo[sl].T.reshape(5, H, W), hi=hi[sl].T.reshape(5, H, W),
                             near_a=near[sl, 0].reshape(H, W), near_T=near[sl, 1].reshape(H, W)))
        return outs

    def backward(self, g_color=None, g_depth=None, g_alpha=None, ambiguous_pixels=None):
        """Gradients of sum over views of <g, outputs>; inputs are per-view lists (None = 0).

        ambiguous_pixels: optional per-view [H,W] masks of pixels whose output gradient is
        not unique (an L1 sign at a tie: such an output gradient may change by up to twice
        its value): uint8 bit k set for output k (colour 0-2, depth 3, alpha 4), or boolean
        (every output of a marked pixel).  Returns the gradients, ``envelope`` (same layouts: how far
        any correct gradient can lie from these, over the correct outcomes of every decision
        inside its margin and the non-unique output gradients) and ``flagged`` (Gaussians
        contributing to a pixel whose outcomes were too many to enumerate)."""
        def cat(lst, ch):
            if lst is None:
                return None
            return np.ascontiguousarray(np.concatenate([np.asarray(x, np.float64).reshape(-1) for x in lst]))
        gc, gd, ga = cat(g_color, 3), cat(g_depth, 1), cat(g_alpha, 1)
        n, K = self.n, self.K
        shapes = dict(means=(n, 3), scales=(n, 3), quats=(n, 4), opacities=(n,), sh=(n, K, 3))
        d = {k: np.zeros(s) for k, s in shapes.items()}
        env = {k: np.zeros(s) for k, s in shapes.items()}
        flagged = np.zeros(n, np.uint8)
        pa = None
        if ambiguous_pixels is not None:
            def bits(m):
                m = np.asarray(m)
                return np.where(m, 31, 0).astype(np.uint8) if m.dtype == bool else m.astype(np.uint8)
            pa = np.ascontiguousarray(np.concatenate([bits(m).reshape(-1) for m in ambiguous_pixels]), np.uint8)
        self.lib.or_backward(self.h, _ptr(gc), _ptr(gd), _ptr(ga), _ptr(pa), _ptr(d["means"]), _ptr(d["scales"]),
                             _ptr(d["quats"]), _ptr(d["opacities"]), _ptr(d["sh"]), _ptr(flagged),
                             _ptr(env["means"]), _ptr(env["scales"]), _ptr(env["quats"]), _ptr(env["opacities"]),
                             _ptr(env["sh"]))
        d["flagged"] = flagged.astype(bool)
        d["envelope"] = env
        return d


def l1_loss(color, depth, target_color, target_depth, depth_weight=0.1):
    """Eq. 12 as a mean plus a weighted mean L1 depth term over valid target depths.

    L = mean_{3P} |C - C*| + w * (1/P) sum_{D*>0} |D - D*|;  returns (L, dL/dC, dL/dD)
    with sign(0) = 0.
    """
    color = np.asarray(color, np.float64)
    depth = np.asarray(depth, np.float64)
    tc = np.asarray(target_color, np.float64)
    td = np.asarray(target_depth, np.float64)
    P = depth.size
    valid = td > 0
    L = np.abs(color - tc).sum() / (3 * P) + depth_weight * np.abs(depth - td)[valid].sum() / P
    gC = np.sign(color - tc) / (3 * P)
    gD = np.where(valid, np.sign(depth - td), 0.0) * (depth_weight / P)
    return L, gC, gD


def sh_eval(degree, dirs, grad=False):
    """Real SH basis Y[n,K] (and polynomial-extension gradients [n,K,3]) at unit dirs."""
    lib = _load()
    dirs = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 3))
    K = (degree + 1) ** 2
    Y = np.zeros((dirs.shape[0], K))
    dY = np.zeros((dirs.shape[0], K, 3)) if grad else None
    lib.or_sh_eval(degree, _ptr(dirs), dirs.shape[0], _ptr(Y), _ptr(dY))
    return (Y, dY) if grad else Y


def time_fwd_bwd(params, sh_degree, cameras, targets, settings: Settings, depth_weight=0.1):
    """One oracle step (build + forward + L1 loss + backward); returns seconds."""
    import time
    t0 = time.perf_counter()
    o = Oracle(params, sh_degree, cameras, settings)
    outs = o.forward()
    gcs, gds = [], []
    for out, (tc, td) in zip(outs, targets):
        _, gC, gD = l1_loss(out["color"], out["depth"], tc, td, depth_weight)
        gcs.append(gC)
        gds.append(gD)
    o.backward(gcs, gds, None)
    return time.perf_counter() - t0
