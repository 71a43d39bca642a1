"""CPU-side checks of the C ABI: the library loads, exports every entry point
that include/swalign.h declares, the ctypes layouts match the C structs, and
argument validation fails cleanly before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swalign.h")


def declared_entry_points():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2503_13756_amd import _abi

    if not os.path.exists(_abi.LIB_PATH):
        from paper_2503_13756_amd import build

        build.build()
    return _abi.load()


def test_header_declares_the_boundary():
    names = declared_entry_points()
    for need in ("sw_project", "sw_quantiles", "sw_align_batch", "sw_ctx_create",
                 "sw_ctx_destroy", "sw_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2503_13756_amd import _abi

    names = declared_entry_points()
    for name in names:
        assert hasattr(lib, name), name
    bound = {s[0] for s in _abi.SIGNATURES}
    assert set(names) <= bound, set(names) - bound


def test_struct_layouts():
    from paper_2503_13756_amd import _abi

    assert ctypes.sizeof(_abi.sw_geom) == 16
    assert ctypes.sizeof(_abi.sw_result) == 24
    assert _abi.sw_batch.geom.offset == 64
    assert _abi.sw_batch.filter.offset == 92
    assert ctypes.sizeof(_abi.sw_batch) == 96


@pytest.mark.parametrize("L,n,Q", [(4, 64, 64), (300, 64, 64), (64, 60, 64), (64, 40, 64),
                                   (64, 1024, 64), (64, 64, 6), (64, 64, 30)])
def test_invalid_geometry_rejected_before_device_work(lib, L, n, Q):
    from paper_2503_13756_amd import _abi

    g = _abi.sw_geom(L, n, Q, 0)
    fake_ctx = ctypes.c_void_p(1)  # never dereferenced: validation comes first
    st = lib.sw_project(fake_ctx, ctypes.c_void_p(8), 1, ctypes.byref(g), ctypes.c_void_p(8), None)
    assert st == _abi.SW_E_INVALID
    assert lib.sw_last_error()


def test_null_arguments_rejected(lib):
    from paper_2503_13756_amd import _abi

    g = _abi.sw_geom(64, 64, 64, 0)
    assert lib.sw_project(None, None, 1, ctypes.byref(g), None, None) == _abi.SW_E_INVALID
    fake_ctx = ctypes.c_void_p(1)
    assert lib.sw_quantiles(fake_ctx, None, 1, ctypes.byref(g), None, None, None) == _abi.SW_E_INVALID
    b = _abi.sw_batch()
    b.geom = g
    b.n_ref, b.n_img = 1, 1
    assert lib.sw_align_batch(fake_ctx, ctypes.byref(b), None, None, None) == _abi.SW_E_INVALID
    b.geom = _abi.sw_geom(64, 64, 64, 7)
    assert lib.sw_align_batch(fake_ctx, ctypes.byref(b), None, None, None) == _abi.SW_E_INVALID


def test_empty_batch_is_a_no_op(lib):
    from paper_2503_13756_amd import _abi

    g = _abi.sw_geom(64, 64, 64, 0)
    fake_ctx = ctypes.c_void_p(1)
    assert lib.sw_project(fake_ctx, None, 0, ctypes.byref(g), None, None) == _abi.SW_OK
    assert lib.sw_tables(fake_ctx, None, 0, ctypes.byref(g), None, None, None) == _abi.SW_OK
