"""ctypes mirror of include/gsr.h.  Argument marshalling only: every step runs in libgsr.so."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgsr.so")

P = ctypes.c_void_p
MAX_VIEWS = 16
MAX_KERNELS = 32

OK, EINVAL, ENOMEM, EDEVICE, ECAPACITY, EINTERNAL = range(6)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ECAPACITY", 5: "EINTERNAL"}
ACCUMULATE = 1
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024  # GSR_NOALLOC_SCRATCH_BYTES
EXACT_TILES = 1
NORMALIZED_DEPTH = 2
CHECK_FINITE = 4


class GsrError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"gsr {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


# gsr_alloc: a caller's device allocator (see include/gsr.h)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Alloc(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", P)]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("means", P), ("scales", P),
                ("quats", P), ("opacities", P), ("sh", P)]


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("znear", ctypes.c_float)]


class Settings(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("batch", ctypes.c_int32), ("extent_k", ctypes.c_float),
                ("lowpass", ctypes.c_float), ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("T_min", ctypes.c_float), ("guard", ctypes.c_float), ("bg", ctypes.c_float * 3),
                ("flags", ctypes.c_uint32), ("jclamp", ctypes.c_float)]


class ViewOut(ctypes.Structure):
    _fields_ = [("color", P), ("depth", P), ("alpha", P)]


class ViewGrad(ctypes.Structure):
    _fields_ = [("color", P), ("depth", P), ("alpha", P)]


class Target(ctypes.Structure):
    _fields_ = [("color", P), ("depth", P)]


class GaussianGrads(ctypes.Structure):
    _fields_ = [("means", P), ("scales", P), ("quats", P), ("opacities", P), ("sh", P)]


class Info(ctypes.Structure):
    _fields_ = [("num_keys", ctypes.c_int64), ("num_tiles", ctypes.c_int64), ("num_pixels", ctypes.c_int64),
                ("num_records", ctypes.c_int64), ("views", ctypes.c_int32), ("sort_passes", ctypes.c_int32)]


class Timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * MAX_KERNELS), ("launches", ctypes.c_int64 * MAX_KERNELS),
                ("count", ctypes.c_int32)]


class Debug(ctypes.Structure):
    _fields_ = [("keys", P), ("values", P), ("ranges", P), ("T_final", P), ("n_contrib", P),
                ("tiles_touched", P), ("mu", P), ("depth", P), ("conic", P), ("color", P), ("rect", P),
                ("n_used", P)]


class SeedSettings(ctypes.Structure):
    _fields_ = [("measure", ctypes.c_int32), ("threshold", ctypes.c_float), ("min_side", ctypes.c_int32),
                ("opacity", ctypes.c_float), ("sh_degree", ctypes.c_int32)]


class SeedOut(ctypes.Structure):
    _fields_ = [("means", P), ("scales", P), ("quats", P), ("opacities", P), ("sh", P), ("leaves", P)]


class Adam(ctypes.Structure):
    _fields_ = [("lr_means", ctypes.c_float), ("lr_scales", ctypes.c_float), ("lr_quats", ctypes.c_float),
                ("lr_opacities", ctypes.c_float), ("lr_sh_dc", ctypes.c_float), ("lr_sh_rest", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("m", GaussianGrads), ("v", GaussianGrads), ("state", P)]


class ScheduleSettings(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("threshold", ctypes.c_int64),
                ("store_all", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class TsdfSettings(ctypes.Structure):
    _fields_ = [("voxel", ctypes.c_float), ("trunc", ctypes.c_float), ("w_max", ctypes.c_float),
                ("step", ctypes.c_float), ("weighting", ctypes.c_int32)]


TSDF_EQ9, TSDF_UNIT_WEIGHT = 0, 1
SEED_CONTRAST, SEED_DEPTH_VARIANCE = 0, 1

# every symbol include/gsr.h declares, with its ctypes signature
SIGNATURES = {
    "gsr_abi_version": (ctypes.c_int32, []),
    "gsr_settings_default": (ctypes.c_int, [P]),
    "gsr_ctx_create": (ctypes.c_int, [ctypes.c_int32, P, P, P]),
    "gsr_ctx_destroy": (ctypes.c_int, [P]),
    "gsr_ctx_set_stream": (ctypes.c_int, [P, P]),
    "gsr_ctx_set_timing": (ctypes.c_int, [P, ctypes.c_int32]),
    "gsr_ctx_get_timing": (ctypes.c_int, [P, P, ctypes.c_int32]),
    "gsr_kernel_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "gsr_forward": (ctypes.c_int, [P, P, P, ctypes.c_int32, P, P, P]),
    "gsr_loss_l1": (ctypes.c_int, [P, P, P, P, ctypes.c_float, P, P, P]),
    "gsr_backward": (ctypes.c_int, [P, P, P, P, ctypes.c_uint32]),
    "gsr_backward_noalloc": (ctypes.c_int, [P, P, P, P, ctypes.c_uint32]),
    "gsr_saved_info": (ctypes.c_int, [P, P]),
    "gsr_saved_free": (ctypes.c_int, [P]),
    "gsr_debug_export": (ctypes.c_int, [P, P, P]),
    "gsr_last_error": (ctypes.c_char_p, [P]),
    "gsr_graph_create": (ctypes.c_int, [P, P, P, ctypes.c_int32, P, P, P, ctypes.c_float, P, P, P, P,
                                        ctypes.c_float, P, P]),
    "gsr_graph_launch": (ctypes.c_int, [P]),
    "gsr_graph_sync": (ctypes.c_int, [P]),
    "gsr_graph_info": (ctypes.c_int, [P, P, P, P]),
    "gsr_graph_free": (ctypes.c_int, [P]),
    "gsr_autotune": (ctypes.c_int, [P, P, P, ctypes.c_int32, P, ctypes.c_uint32, P]),
    "gsr_seed_settings_default": (ctypes.c_int, [P]),
    "gsr_seed": (ctypes.c_int, [P, P, P, P, P, P, P, ctypes.c_int64, P]),
    "gsr_tsdf_settings_default": (ctypes.c_int, [P]),
    "gsr_tsdf_create": (ctypes.c_int, [P, P, ctypes.c_int64, P]),
    "gsr_tsdf_free": (ctypes.c_int, [P]),
    "gsr_tsdf_integrate": (ctypes.c_int, [P, P, P, P]),
    "gsr_tsdf_info": (ctypes.c_int, [P, P, P, P, P]),
    "gsr_tsdf_export": (ctypes.c_int, [P, P, P, P, P, ctypes.c_int64, P]),
    "gsr_tsdf_weights": (ctypes.c_int, [P, P, P, ctypes.c_int64, P]),
    "gsr_adam_default": (ctypes.c_int, [P]),
    "gsr_adam_step": (ctypes.c_int, [P, ctypes.c_int64, ctypes.c_int32, P, P, P]),
    "gsr_backward_adam": (ctypes.c_int, [P, P, P, P]),
    "gsr_schedule_create": (ctypes.c_int, [P, P]),
    "gsr_schedule_free": (ctypes.c_int, [P]),
    "gsr_schedule_step": (ctypes.c_int, [P, ctypes.c_int64, ctypes.c_int64, P, ctypes.c_int32, P, P]),
    "gsr_schedule_keyframes": (ctypes.c_int, [P, P, ctypes.c_int64, P]),
}
AUTOTUNE_NO_CACHE = 1

_lib = None


def load():
    """Load the in-tree libgsr.so; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2408_12677_amd.build` "
                              "(there is no fallback implementation)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if lib.gsr_abi_version() != 1:
            raise ImportError("libgsr.so ABI version mismatch")
        _lib = lib
    return _lib


def check(status, ctx=None):
    if status != OK:
        msg = load().gsr_last_error(ctx)
        raise GsrError(status, msg.decode() if msg else "")
