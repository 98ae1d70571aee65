"""Host logic of grids with 4 and 5 axes: plan strings, the heuristic order,
rejection of unusable plans and arguments (no GPU)."""
import ctypes

import pytest
import torch

import paper_1501_07350_amd as offt
from paper_1501_07350_amd import _lib

C128, C64 = torch.complex128, torch.complex64


def fields(s):
    return dict(f.split("=", 1) for f in s.split(";"))


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape", [(64, 64, 64, 64), (32, 48, 30, 20, 16), (8, 1, 16, 1), (1, 1, 1, 1, 1)])
def test_heuristic_nd_plans(shape, dtype):
    s = offt.plan_string_nd(shape, dtype)
    f = fields(s)
    D = len(shape)
    assert f["order"] == "abcde"[:D][::-1]          # last axis first
    for i, n in enumerate(shape):
        assert (f["abcde"[i]] == "1") == (n == 1)
    assert offt.plan_string_nd(shape, dtype, s) == s


def test_nd_plan_strings_round_trip_and_fill_defaults():
    s = offt.plan_string_nd((8, 6, 10, 12), C128, "order=abcd;a=8/4;d=4x3/8")
    f = fields(s)
    assert f["order"] == "abcd" and f["a"] == "8/4" and f["d"] == "4x3/8"
    assert f["b"] != "1" and f["c"] != "1"


@pytest.mark.parametrize("plan", ["order=abc", "order=abcd;e=8/4", "order=abcd;d=4x3/8/p2", "order=aacd",
                                  "order=abcd;a=7/4", "order=abcd;rev=a", "order=abcd;b=3x2/3"])
def test_unusable_nd_plans_rejected(plan):
    with pytest.raises(offt.OfftError) as e:
        offt.plan_string_nd((8, 6, 10, 12), C128, plan)
    assert e.value.code == -6


def test_nd_arguments_rejected_before_the_device():
    lib = _lib.load()
    for ndim, dims in [(0, [4]), (6, [2] * 6), (4, [8, 7, 4, 4]), (4, [8, 0, 4, 4]), (5, [2048, 2, 2, 2, 2])]:
        arr = (ctypes.c_int64 * len(dims))(*dims)
        assert not lib.offt_plan_nd(ndim, arr, 0, 1, None)
        assert _lib.last_error() in (-1, -2)
    # reversed layout and 3-axis strings are rejected for 4-axis plans
    opts, keep = offt._make_opts(layout="cba")
    arr = (ctypes.c_int64 * 4)(8, 8, 8, 8)
    assert not lib.offt_plan_nd(4, arr, 0, 1, ctypes.byref(opts))
    assert _lib.last_error() == -1
    with pytest.raises(ValueError):
        offt.Plan((2,) * 6)
