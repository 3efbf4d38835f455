"""The C ABI without a GPU: the library loads, exports what include/wsimg.h declares, and
rejects invalid arguments on the host before any HIP call."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wsimg.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2601_19714_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2601_19714_amd import build
        build.build()
    return _lib.load(), _lib


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wsimg_[a-z_]+)\s*\(", text)))


def test_header_declares_exactly_the_binding_list(lib):
    _, mod = lib
    assert _declared_functions() == sorted(mod.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    L, _ = lib
    cdll = ctypes.CDLL(L._name)
    for name in _declared_functions():
        assert hasattr(cdll, name), name


def test_status_strings_and_version(lib):
    L, mod = lib
    assert L.wsimg_version() >= 1
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.wsimg_status_string(code)
    names = [L.wsimg_stage_name(i) for i in range(mod.WSIMG_N_KERNELS)]
    assert all(names) and L.wsimg_stage_name(mod.WSIMG_N_KERNELS) is None


def _params(mod, **kw):
    p = mod.Params()
    p.n, p.n_wplanes, p.support, p.precision = 256, 8, 7, mod.WSIMG_F32
    p.pixel_rad, p.beta = 1e-5, 0.0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("field,value", [
    ("n", 100), ("n", 8), ("n", 32768), ("n_wplanes", 0), ("n_wplanes", 5000),
    ("support", 8), ("support", 1), ("support", 17), ("precision", 3),
    ("pixel_rad", 0.0), ("pixel_rad", float("nan")), ("pixel_rad", 0.01),
    ("beta", float("inf")), ("w_support", 1), ("w_support", 4), ("w_support", 17), ("w_support", 9),
    ("flags", 0x20),
])
def test_invalid_params_rejected_on_host(lib, field, value):
    L, mod = lib
    h = ctypes.c_void_p(1234)
    p = _params(mod, **{field: value})
    st = L.wsimg_plan_create(ctypes.byref(h), ctypes.byref(p), 100, None)
    assert st == mod.WSIMG_E_INVALID, (field, value, st)
    assert h.value is None
    assert L.wsimg_last_error()


def test_every_declared_flag_is_accepted_on_host(lib):
    """Each flag the header declares passes the host checks (plan_query: no GPU needed)."""
    L, mod = lib
    for flag in (mod.WSIMG_FIXED_WRANGE, mod.WSIMG_UNNORMALIZED, mod.WSIMG_FOLD_W, mod.WSIMG_PAD2,
                 mod.WSIMG_COMPLEX_OUT):
        p = _params(mod, flags=flag, w_lo=-1.0, w_hi=1.0)
        info = mod.PlanInfo()
        assert L.wsimg_plan_query(ctypes.byref(p), 100, 1, ctypes.byref(info)) == mod.WSIMG_OK, flag


def test_noalloc_capacity_checked_on_host(lib):
    """wsimg_image_noalloc refuses a geometry whose scratch exceeds its static array before
    any device work (no GPU here), and checks parameters like wsimg_plan_create."""
    L, mod = lib
    p = _params(mod, n=4096, n_wplanes=32)
    st = L.wsimg_image_noalloc(ctypes.byref(p), 7_000_000, None, None, None, 1.4e9, None, None, None)
    assert st == mod.WSIMG_E_CAPACITY
    assert b"static scratch" in L.wsimg_last_error()
    p = _params(mod, support=8)
    assert L.wsimg_image_noalloc(ctypes.byref(p), 10, None, None, None, 1e9, None, None, None) == mod.WSIMG_E_INVALID
    p = _params(mod)
    assert L.wsimg_image_noalloc(ctypes.byref(p), -1, None, None, None, 1e9, None, None, None) == mod.WSIMG_E_INVALID
    # within the array, a missing output is an argument error (still before any device work)
    assert L.wsimg_image_noalloc(ctypes.byref(p), 0, None, None, None, 1e9, None, None, None) == mod.WSIMG_E_INVALID


def test_w_support_accepted_below_the_plane_count(lib):
    """The w-kernel needs an odd support below n_wplanes (8 planes here): 3..7 pass the host
    checks, 9 does not (the invalid-parameter test above)."""
    L, mod = lib
    for ws in (3, 5, 7):
        p = _params(mod, w_support=ws)
        info = mod.PlanInfo()
        assert L.wsimg_plan_query(ctypes.byref(p), 100, 1, ctypes.byref(info)) == mod.WSIMG_OK, ws


def test_fixed_range_and_capacity_rules(lib):
    L, mod = lib
    h = ctypes.c_void_p()
    p = _params(mod, flags=mod.WSIMG_FIXED_WRANGE, w_lo=5.0, w_hi=-5.0)
    assert L.wsimg_plan_create(ctypes.byref(h), ctypes.byref(p), 10, None) == mod.WSIMG_E_INVALID
    p = _params(mod)
    assert L.wsimg_plan_create(ctypes.byref(h), ctypes.byref(p), -1, None) == mod.WSIMG_E_INVALID
    assert L.wsimg_plan_create(ctypes.byref(h), ctypes.byref(p), 1 << 40, None) == mod.WSIMG_E_INVALID
    assert L.wsimg_plan_create(None, ctypes.byref(p), 10, None) == mod.WSIMG_E_INVALID
    assert L.wsimg_plan_create(ctypes.byref(h), None, 10, None) == mod.WSIMG_E_INVALID
    p = _params(mod, n=16384)
    assert L.wsimg_plan_create(ctypes.byref(h), ctypes.byref(p), 10, None) == mod.WSIMG_E_UNSUPPORTED


def test_null_plan_calls(lib):
    L, mod = lib
    assert L.wsimg_plan_destroy(None) == mod.WSIMG_OK
    assert L.wsimg_image(None, 0, None, None, None, 1e9, None, None) == mod.WSIMG_E_INVALID
    assert L.wsimg_grid(None, 0, None, None, None, 1e9, None, None) == mod.WSIMG_E_INVALID
    assert L.wsimg_set_timing(None, 1) == mod.WSIMG_E_INVALID
    assert L.wsimg_plan_set_stream(None, None) == mod.WSIMG_E_INVALID
    info = mod.PlanInfo()
    assert L.wsimg_plan_get_info(None, ctypes.byref(info)) == mod.WSIMG_E_INVALID


def test_binding_raises_without_library(tmp_path):
    from paper_2601_19714_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(ImportError):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._lib = saved
