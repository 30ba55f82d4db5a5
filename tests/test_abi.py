"""The C-ABI library loads without a GPU and exports every declared symbol."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "wl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wl_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    from paper_2304_08159_amd import _lib
    assert set(_declared()) == set(_lib.EXPORTS)


def test_library_loads_and_exports_every_symbol():
    from paper_2304_08159_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwl.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    lib.wl_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.wl_version()


def test_host_side_validation_without_gpu():
    """Footprint calls are host-only: check argument validation and exact sizes."""
    from paper_2304_08159_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwl.so not built")
    lib = _lib.load()
    d = _lib.SimDesc()
    d.ndim = 3
    for i in range(3):
        d.n[i] = 64
    d.nu, d.tol = 0.01, 1e-5
    sz = ctypes.c_size_t()
    assert lib.wl_sim_footprint(ctypes.byref(d), ctypes.byref(sz)) == 0
    cells = 64 ** 3
    # 9 velocity + p + sigma + 12 BDIM fields + fine level (3 L, x1, b) at 4 B each
    assert sz.value >= (9 + 2 + 12 + 5) * 4 * cells
    assert sz.value <= (9 + 2 + 12 + 6) * 4 * cells * 8 // 7 + (1 << 22)
    d.prec = 1
    sz64 = ctypes.c_size_t()
    assert lib.wl_sim_footprint(ctypes.byref(d), ctypes.byref(sz64)) == 0
    assert sz64.value > 1.9 * sz.value
    d.ndim = 2                                   # 2D needs n[2] == 1
    assert lib.wl_sim_footprint(ctypes.byref(d), ctypes.byref(sz)) == -1
    assert b"n[2]" in lib.wl_last_error()
    d.n[2] = 1
    d.bc_lo[0], d.bc_hi[0] = 0, 2                # periodic paired with outflow
    assert lib.wl_sim_footprint(ctypes.byref(d), ctypes.byref(sz)) == -1
    n = (ctypes.c_int * 3)(16, 16, 3)
    per = (ctypes.c_int * 3)(1, 1, 1)
    assert lib.wl_poisson_footprint(3, n, per, 0, 2, ctypes.byref(sz)) == -1   # 3 is odd
    n = (ctypes.c_int * 3)(64, 64, 3)
    assert lib.wl_poisson_footprint(3, n, per, 0, 0, ctypes.byref(sz)) == -1   # coarsest > 1024
    assert b"1024" in lib.wl_last_error()
    n = (ctypes.c_int * 3)(256, 256, 256)
    assert lib.wl_poisson_footprint(3, n, per, 2, 0, ctypes.byref(sz)) == 0
    assert sz.value > 3 * 8 * 256 ** 3
