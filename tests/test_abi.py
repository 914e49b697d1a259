"""The C ABI library loads and exports what include/fill.h declares (CPU only).

No compute call is made here: these run without a GPU.
"""

from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fill.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fill_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("fill_plan_create", "fill_realize", "fill_mean", "fill_plan_destroy", "fill_get_stats"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1109_0286_amd as F
    lib = ctypes.CDLL(F.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(F.EXPORTS) == declared_functions()


def test_host_only_calls():
    import paper_1109_0286_amd as F
    for n in (16, 32, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096):
        assert F.fill_supported_size(n)
    for n in (0, 8, 48, 100, 1000, 6144, 8192, -1):
        assert not F.fill_supported_size(n)
    assert F.fill_strerror(F.FILL_OK) == "ok"
    assert "converge" in F.fill_strerror(F.FILL_ENOCONV)
    assert F.fill_strerror(12345) == "unknown error"


def test_plan_create_rejects_bad_arguments_before_touching_the_gpu():
    import numpy as np
    import paper_1109_0286_amd as F
    P = np.ones((64, 33))
    m = np.zeros((64, 64), np.uint8)
    with pytest.raises(F.FillError) as e:
        F.fill_plan_create(100, 64, np.zeros((64, 100), np.uint8), np.ones((64, 51)), 0, None)
    assert e.value.code == F.FILL_EUNSUPPORTED_SIZE
    with pytest.raises(F.FillError) as e:
        F.fill_plan_create(64, 64, m, P, 7, None)
    assert e.value.code == F.FILL_EINVAL
    with pytest.raises(ValueError):
        F.fill_plan_create(64, 64, m, np.ones((64, 64)), 0, None)


def test_build_sources_are_gfx950_only():
    src = os.path.join(ROOT, "paper_1109_0286_amd", "csrc")
    for f in os.listdir(src):
        txt = open(os.path.join(src, f)).read()
        assert "__CUDA" not in txt and "__HIP_PLATFORM" not in txt, f


def test_strips_create_rejects_bad_arguments_before_touching_the_gpu():
    import numpy as np
    import paper_1109_0286_amd as F
    lib = F.fill._lib
    m = np.zeros((64, 64), np.uint8)
    P = np.ones((64, 33))
    h = ctypes.c_void_p()

    def create(nstrips, betas, widths, threshold=0.03, iters=20, prec=0, noise=1e-3):
        b = np.asarray(betas, dtype=np.float64)
        w = np.asarray(widths, dtype=np.float64)
        return lib.fill_strips_create(64, 64, m.ctypes.data, P.ctypes.data, noise, nstrips, b.ctypes.data,
                                      w.ctypes.data, threshold, iters, prec, None, ctypes.byref(h))

    assert create(0, [1.0], [4.0]) == F.FILL_EINVAL
    assert create(1, [1.0], [32.0]) == F.FILL_EINVAL      # disk of 65 px does not fit 64
    assert create(1, [1.0], [0.5]) == F.FILL_EINVAL
    assert create(1, [0.0], [4.0]) == F.FILL_EINVAL
    assert create(1, [1.0], [4.0], threshold=1.0) == F.FILL_EINVAL
    assert create(1, [1.0], [4.0], iters=0) == F.FILL_EINVAL
    assert create(1, [1.0], [4.0], prec=5) == F.FILL_EINVAL
    assert create(1, [1.0], [4.0], noise=-1.0) == F.FILL_EINVAL
    assert create(1, [1.0], [40.0]) == F.FILL_EINVAL
    assert b"disk" in lib.fill_strips_last_error()
    assert h.value is None
