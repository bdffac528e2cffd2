"""Build libgsr.so (the HIP kernels and C ABI) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libgsr.so")
SOURCES = [os.path.join(CSRC, f) for f in ("gsr_host.hip", "gsr_kernels.hip", "gsr_seed.hip", "gsr_optim.hip", "gsr_tsdf.hip",
                                           "gsr_schedule.cpp", "gsr_validate.cpp")]
HEADERS = [os.path.join(ROOT, "include", "gsr.h"), os.path.join(CSRC, "gsr_internal.h"), os.path.join(CSRC, "gsr_adam.h"),
           os.path.join(CSRC, "gsr_tsdf.h"), os.path.join(CSRC, "gsr_validate.h")]
ARCH = os.environ.get("GSR_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def command(out: str = LIB) -> list:
    return [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-I", os.path.join(ROOT, "include"),
        # correctly rounded binary32 divide/sqrt for the exact discrete stage
        "-fhip-fp32-correctly-rounded-divide-sqrt",
        # hardware float atomics (global_atomic_add_f32) for the backward reductions
        "-munsafe-fp-atomics",
        # no packed-FP32 (v_pk_*_f32) instruction selection
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        "-o", out, *SOURCES,
    ]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every HIP source into libgsr.so (always recompiles when force)."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in SOURCES + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
