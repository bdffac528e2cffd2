"""The C-ABI library builds, loads and exports every symbol include/gsr.h declares.

CPU only: no device work is started; only calls that validate their arguments
before touching HIP are made.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2408_12677_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2408_12677_amd import build
        build.build(force=True)
    return _native.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gsr_forward", "gsr_backward", "gsr_loss_l1", "gsr_ctx_create", "gsr_debug_export"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2408_12677_amd import _native
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _native.SIGNATURES, f"binding lacks {name}"


def test_abi_version_and_defaults(lib):
    from paper_2408_12677_amd import _native as N
    assert lib.gsr_abi_version() == 1
    s = N.Settings()
    assert lib.gsr_settings_default(ctypes.byref(s)) == N.OK
    assert (s.tile, s.batch) == (16, 256)
    assert s.extent_k == pytest.approx(3.33) and s.lowpass == pytest.approx(0.3)
    assert s.alpha_min == pytest.approx(1 / 255) and s.alpha_max == pytest.approx(0.99)
    assert s.T_min == pytest.approx(1e-4) and list(s.bg) == [0, 0, 0] and s.flags == 0
    # the default extent keeps every splat value >= alpha_min inside its rectangle
    import math
    assert s.extent_k >= math.sqrt(2 * math.log(255))


def test_null_arguments_are_rejected_before_device_work(lib):
    from paper_2408_12677_amd import _native as N
    assert lib.gsr_settings_default(None) == N.EINVAL
    assert lib.gsr_forward(None, None, None, 1, None, None, None) == N.EINVAL
    assert lib.gsr_backward(None, None, None, None, 0) == N.EINVAL
    assert lib.gsr_loss_l1(None, None, None, None, 0.1, None, None, None) == N.EINVAL
    assert lib.gsr_saved_free(None) == N.EINVAL
    assert lib.gsr_saved_info(None, None) == N.EINVAL
    assert lib.gsr_ctx_destroy(None) == N.EINVAL
    assert lib.gsr_ctx_create(0, None, None, None) == N.EINVAL
    assert b"NULL" in lib.gsr_last_error(None)
    # a caller's allocator needs both functions (checked before any device call)
    half = N.Alloc(N.ALLOC_FN(lambda user, n, s: None), N.FREE_FN(), None)
    h = ctypes.c_void_p()
    assert lib.gsr_ctx_create(0, None, ctypes.byref(half), ctypes.byref(h)) == N.EINVAL
    assert b"alloc and free" in lib.gsr_last_error(None)
    assert not h.value


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2408_12677_amd import _native as N
    monkeypatch.setattr(N, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(N, "_lib", None)
    with pytest.raises(ImportError):
        N.load()


def test_binding_does_not_import_the_oracle():
    import ast
    pkg = os.path.join(ROOT, "paper_2408_12677_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                tree = ast.parse(open(os.path.join(dirpath, f)).read())
                for node in ast.walk(tree):
                    if isinstance(node, ast.Import):
                        assert not any(a.name.split(".")[0] in ("oracle", "scenes") for a in node.names), f
                    if isinstance(node, ast.ImportFrom) and node.module:
                        assert node.module.split(".")[0] not in ("oracle", "scenes"), f
