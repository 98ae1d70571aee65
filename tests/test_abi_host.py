"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function include/offt.h declares, reject
bad arguments with the documented codes before touching a device, and report
OFFT_ERR_NO_DEVICE where no GPU is visible.
"""
import ctypes
import os
import re

import pytest

import paper_1501_07350_amd as offt
from paper_1501_07350_amd import _lib
from conftest import gpu_available

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "offt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(offt_[a-z_]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), f"libofft.so does not export {n}"
    # the binding describes exactly the declared set
    assert set(_lib.SIGNATURES) == set(names)


def test_error_strings_and_defaults():
    lib = _lib.load()
    for code in range(-7, 1):
        s = _lib.error_string(code)
        assert s and s != "unknown error"
    assert _lib.error_string(-99) == "unknown error"
    o = _lib.default_opts()
    assert o.tune == _lib.TUNE_NONE and o.reps == 2 and o.normalize_inverse == 0
    assert not o.forced_plan and not o.cache_path and not o.weights_path
    assert lib.offt_destroy(None) == 0


@pytest.mark.parametrize("dims,dtype,batch,code", [
    ((0, 4, 4), 0, 1, _lib.ERR_INVALID_ARG),
    ((4, -1, 4), 0, 1, _lib.ERR_INVALID_ARG),
    ((4, 4, 4), 2, 1, _lib.ERR_INVALID_ARG),
    ((4, 4, 4), 0, 0, _lib.ERR_INVALID_ARG),
    ((7, 4, 4), 0, 1, _lib.ERR_UNSUPPORTED_SIZE),
    ((4, 4, 14), 1, 1, _lib.ERR_UNSUPPORTED_SIZE),
    ((4, 2048, 4), 1, 1, _lib.ERR_UNSUPPORTED_SIZE),
    ((1024, 1024, 1024), 0, 1 << 40, _lib.ERR_INVALID_ARG),
])
def test_invalid_arguments_rejected_before_device(dims, dtype, batch, code):
    lib = _lib.load()
    h = lib.offt_plan(dims[0], dims[1], dims[2], dtype, batch)
    assert not h
    assert lib.offt_last_error() == code


def test_bad_options_rejected():
    lib = _lib.load()
    o = _lib.default_opts()
    o.tune = 9
    assert not lib.offt_plan_ex(8, 8, 8, 0, 1, ctypes.byref(o))
    assert lib.offt_last_error() == _lib.ERR_INVALID_ARG
    o = _lib.default_opts()
    o.tune = _lib.TUNE_FORCED   # forced without a plan string
    assert not lib.offt_plan_ex(8, 8, 8, 0, 1, ctypes.byref(o))
    assert lib.offt_last_error() == _lib.ERR_INVALID_ARG
    o.forced_plan = b"order=cba;a=3/8;b=8/8;c=8/8"   # radix 3 for length 8: no such kernel
    assert not lib.offt_plan_ex(8, 8, 8, 0, 1, ctypes.byref(o))
    assert lib.offt_last_error() == _lib.ERR_BAD_PLAN
    o.forced_plan = b"order=cca;a=8/8;b=8/8;c=8/8"   # repeated axis
    assert not lib.offt_plan_ex(8, 8, 8, 0, 1, ctypes.byref(o))
    assert lib.offt_last_error() == _lib.ERR_BAD_PLAN
    o.forced_plan = b"garbage"
    assert not lib.offt_plan_ex(8, 8, 8, 0, 1, ctypes.byref(o))
    assert lib.offt_last_error() == _lib.ERR_BAD_PLAN
    o = _lib.default_opts()
    o.reps = 0
    assert not lib.offt_plan_ex(8, 8, 8, 0, 1, ctypes.byref(o))
    assert lib.offt_last_error() == _lib.ERR_INVALID_ARG


def test_exec_rejects_null_handles():
    lib = _lib.load()
    assert lib.offt_exec_fwd(None, None, None, None) == _lib.ERR_INVALID_ARG
    assert lib.offt_exec_bwd(None, None, None, None) == _lib.ERR_INVALID_ARG
    assert lib.offt_plan_describe(None, None, 0) == _lib.ERR_INVALID_ARG
    assert lib.offt_workspace_bytes(None) == _lib.ERR_INVALID_ARG
    assert lib.offt_exec_many(None, None, None, -1, 1, None) < 0
    assert lib.offt_exec_pass(None, 0, -1, None, None, None) == _lib.ERR_INVALID_ARG
    assert lib.offt_exec_range(None, 0, 1, -1, None, None, None) == _lib.ERR_INVALID_ARG
    assert lib.offt_many_offset(None, 0) < 0


@pytest.mark.skipif(gpu_available(), reason="checks the no-device path")
def test_no_device_reported():
    lib = _lib.load()
    assert not lib.offt_plan(8, 8, 8, 0, 1)
    assert lib.offt_last_error() == _lib.ERR_NO_DEVICE
    buf = (ctypes.c_double * 16)()
    assert lib.offt_twiddles(8, 0, buf) == _lib.ERR_NO_DEVICE


def test_python_plan_raises_with_code():
    with pytest.raises(offt.OfftError) as ei:
        offt.Plan((7, 8, 8))
    assert ei.value.code == _lib.ERR_UNSUPPORTED_SIZE
    with pytest.raises(ValueError):
        offt.Plan((8,) * 6)                 # more axes than OFFT_MAX_DIMS
    with pytest.raises(offt.OfftError) as ei:
        offt.Plan((8, 8, 8, 7))             # 4-axis plans check the lengths too
    assert ei.value.code == _lib.ERR_UNSUPPORTED_SIZE
