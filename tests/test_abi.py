"""The C-ABI library builds, loads and exports every entry point declared in
include/yy.h; argument and geometry errors are reported before any device
work (these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1905_02300_amd import yy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "yy.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(yy_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(yy.LIB_PATH):
        from paper_1905_02300_amd import build
        build.build()
    return yy.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(yy.EXPORTS)


def test_workspace_bytes_and_argument_errors(lib):
    b = yy.workspace_bytes(16, 24, 72)
    assert b > 2 * 18 * 26 * 74 * 8 * 30
    assert yy.workspace_bytes(16, 24, 72, prec=yy.YY_FP32_MIXED) < b
    for bad in [(1, 24, 72), (16, 5, 72), (16, 24, 5)]:
        with pytest.raises(yy.YYError) as e:
            yy.workspace_bytes(*bad)
        assert e.value.status == yy.YY_ERR_ARG
    with pytest.raises(yy.YYError):
        yy.workspace_bytes(16, 24, 72, r1=1.0, r2=0.5)
    with pytest.raises(yy.YYError):
        yy.workspace_bytes(16, 24, 72, prec=7)


def test_field_size_limit(lib):
    # one FP64 field (2 patches, ghosts, k = 0 at row element 16, rows padded
    # to 16 elements) must stay below 4 GiB, since kernels address fields by
    # 32-bit byte offsets
    assert yy.workspace_bytes(128, 384, 1152) > 0
    assert yy.workspace_bytes(254, 766, 1342) > 0        # 2*256*768*1360*8 < 2^32
    with pytest.raises(yy.YYError) as e:
        yy.workspace_bytes(256, 768, 1360)               # 2*258*770*1392*8 > 2^32
    assert e.value.status == yy.YY_ERR_ARG


def _create(lib, g, ptr, nbytes):
    h = ctypes.c_void_p()
    st = lib.yy_create(ctypes.byref(g), 0, ctypes.c_void_p(ptr), nbytes, ctypes.byref(h))
    return st, h


def test_create_rejects_before_touching_the_device(lib):
    g = yy.Grid(8, 12, 36, 0.5, 1.0, 0.0)
    need = yy.workspace_bytes(8, 12, 36)
    st, h = _create(lib, g, 0, need)
    assert st == yy.YY_ERR_ARG and not h.value
    st, h = _create(lib, g, 256, need - 256)
    assert st == yy.YY_ERR_WORKSPACE and not h.value
    st, h = _create(lib, g, 257, need)
    assert st == yy.YY_ERR_WORKSPACE
    # overlap far below one cell: ghost targets fall outside every donor window
    g2 = yy.Grid(8, 12, 36, 0.5, 1.0, 1e-9)
    st, h = _create(lib, g2, 256, yy.workspace_bytes(8, 12, 36, delta=1e-9))
    assert st == yy.YY_ERR_GEOMETRY and not h.value


def test_null_handle_errors(lib):
    assert lib.yy_step(None, 2, None) == yy.YY_ERR_ARG
    k = ctypes.c_int32(-1)
    assert lib.yy_step_tol(None, 4, ctypes.c_double(1e-6), ctypes.byref(k), None) == yy.YY_ERR_ARG
    assert lib.yy_set_params(None, None) == yy.YY_ERR_ARG
    assert lib.yy_destroy(None) == yy.YY_ERR_ARG
    assert lib.yy_strerror(yy.YY_ERR_GEOMETRY).decode().startswith("overlap")
