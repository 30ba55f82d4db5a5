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


def test_batch_footprint_validates_requests_without_a_gpu():
    from paper_2304_08159_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwl.so not built")
    lib = _lib.load()

    def req(ndim, n, per=(0, 0, 0)):
        r = _lib.BatchRequest()
        r.ndim = ndim
        for i in range(3):
            r.n[i] = n[i]
            r.periodic[i] = per[i]
        r.tol = 1e-8
        r.max_vcycles = 50
        return r
    sz = ctypes.c_size_t()
    ok = (_lib.BatchRequest * 2)(req(2, (64, 48, 1)), req(3, (32, 32, 16)))
    assert lib.wl_poisson_batch_footprint(ok, 2, ctypes.byref(sz)) == _lib.WL_OK
    # level arrays of both requests plus the request table
    assert sz.value > 8 * (2 * 64 * 48 + 2 * 32 * 32 * 16)
    one = ctypes.c_size_t()
    assert lib.wl_poisson_batch_footprint(ok, 1, ctypes.byref(one)) == _lib.WL_OK
    assert one.value < sz.value
    for bad in (req(3, (128, 64, 64)),      # more than 262144 cells
                req(2, (64, 48, 2)),        # 2D with n[2] != 1
                req(4, (8, 8, 8)),          # ndim
                req(2, (66, 66, 1))):       # coarsest level 33 x 33 > 1024 cells
        arr = (_lib.BatchRequest * 2)(ok[0], bad)
        st = lib.wl_poisson_batch_footprint(arr, 2, ctypes.byref(sz))
        assert st == _lib.WL_ERR_INVALID_ARG
        assert b"request 1" in lib.wl_last_error()


def test_fused_sweep_mode_is_validated_without_a_gpu():
    from paper_2304_08159_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwl.so not built")
    lib = _lib.load()
    assert lib.wl_set_fused_sweeps(3) == -1
    assert b"mode" in lib.wl_last_error()
    assert lib.wl_set_fused_sweeps(-1) == -1
    for mode in (0, 2, 1):
        assert lib.wl_set_fused_sweeps(mode) == 0


def test_run_validates_arguments_without_a_gpu():
    import ctypes as C
    from paper_2304_08159_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwl.so not built")
    lib = _lib.load()
    taken = C.c_int(7)
    assert lib.wl_run(None, 3, 0.0, None, C.byref(taken)) == -1
    assert taken.value == 0 and b"sim" in lib.wl_last_error()


def test_stop_rule_and_state_calls_validate_without_a_gpu():
    from paper_2304_08159_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwl.so not built")
    lib = _lib.load()
    d = _lib.SimDesc()
    d.ndim = 3
    for i in range(3):
        d.n[i] = 16
    d.nu, d.tol = 0.01, 1e-8
    sz = ctypes.c_size_t()
    for rule in (_lib.STOP_DIVERGENCE, _lib.STOP_RELATIVE):
        d.stop_rule = rule
        assert lib.wl_sim_footprint(ctypes.byref(d), ctypes.byref(sz)) == 0
    d.stop_rule = 2
    assert lib.wl_sim_footprint(ctypes.byref(d), ctypes.byref(sz)) == -1
    assert b"stop_rule" in lib.wl_last_error()
    assert lib.wl_state_size(None, ctypes.byref(sz)) == -1
    assert lib.wl_get_state(None, None) == -1
    assert lib.wl_set_state(None, None) == -1


def test_smoother_switch_is_validated_without_a_gpu():
    from paper_2304_08159_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwl.so not built")
    lib = _lib.load()
    assert lib.wl_set_smoother(2) == -1 and b"kind" in lib.wl_last_error()
    d = _lib.SimDesc()
    d.ndim = 3
    for i in range(3):
        d.n[i] = 32
    d.nu, d.tol = 0.01, 1e-5
    sizes = {}
    for kind in (_lib.SMOOTH_CG, _lib.SMOOTH_JACOBI):
        assert lib.wl_set_smoother(kind) == 0
        sz = ctypes.c_size_t()
        assert lib.wl_sim_footprint(ctypes.byref(d), ctypes.byref(sz)) == 0
        sizes[kind] = sz.value
    # CG smoothing carves four more arrays per level (residual, direction,
    # M p, inverse diagonal): at least 4 fine-level FP32 fields
    assert sizes[_lib.SMOOTH_CG] - sizes[_lib.SMOOTH_JACOBI] >= 4 * 4 * 32 ** 3
