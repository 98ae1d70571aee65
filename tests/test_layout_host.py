"""Host logic of the reversed (cba) output order: plan strings, the heuristic's
choice of transposing axis, and rejection of unusable plans (no GPU)."""
import numpy as np
import pytest
import torch

import paper_1501_07350_amd as offt

C128, C64 = torch.complex128, torch.complex64


def halves(s):
    fwd, bwd = s.split("|")
    return dict(f.split("=", 1) for f in fwd.split(";")), dict(f.split("=", 1) for f in bwd.split(";"))


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape,fwd_rev,bwd_rev", [
    ((512, 512, 512), "a", "a"),
    ((64, 48, 30), "a", "a"),
    ((1, 32, 40), "c", "a"),      # no axis a: the pass along c transposes
    ((30, 40, 1), "a", "c"),      # the backward plan's grid (1, 40, 30) has no axis a
    ((6, 1, 10), "a", "a"),
])
def test_heuristic_reversed_plans(shape, dtype, fwd_rev, bwd_rev):
    s = offt.plan_string(shape, dtype, "cba")
    f, b = halves(s)
    assert f["rev"] == fwd_rev and b["rev"] == bwd_rev
    assert f["order"] == "cba" and b["order"] == "cba"
    # the backward half names the axes of the cba input: its a is the grid's c
    assert f["a"] == "1" if shape[0] == 1 else f["a"] != "1"
    assert b["c"] == "1" if shape[0] == 1 else b["c"] != "1"
    assert offt.plan_string(shape, dtype, "cba", s) == s


@pytest.mark.parametrize("shape", [(1, 1, 60), (8, 1, 1), (1, 9, 1), (1, 1, 1)])
def test_one_axis_grids_need_no_transposing_pass(shape):
    s = offt.plan_string(shape, C128, "cba")
    assert "rev=" not in s and s.count("|") == 1


BASE = "order=cba;rev=a;a=16x16x2/4;b=16x16x2/4;c=16x16x2/4"


@pytest.mark.parametrize("plan", [
    BASE,                                              # no backward half
    BASE + "|order=cba;a=16x16x2/4;b=16x16x2/4;c=16x16x2/4",   # backward half without a transposing axis
    BASE + "|order=cba;rev=b;a=16x16x2/4;b=16x16x2/4;c=16x16x2/4",   # b cannot transpose
    "order=cba;rev=c;a=16x16x2/4/p2;b=16x16x2/4;c=16x16x2/4|" + BASE,   # parts on a contiguous cba axis
    "order=cba;rev=a;a=16x16x2/4/p4;b=16x16x2/4;c=16x16x2/4|" + BASE,   # no such kernel in 4 parts
])
def test_unusable_reversed_plans_rejected(plan):
    with pytest.raises(offt.OfftError) as e:
        offt.plan_string((512, 512, 512), C128, "cba", plan)
    assert e.value.code == -6


def test_transposing_pass_in_parts():
    # 2-part exchanges on the transposing axis: its strided side is strided,
    # and the first and last radix of 16x16x2 split into 2
    s = "order=cba;rev=a;a=16x16x2/4/p2;b=16x16x2/4;c=16x16x2/4|" + BASE
    assert offt.plan_string((512, 512, 512), C128, "cba", s) == s


def test_strided_reversed_axis_takes_parts():
    # after the transposing pass along c, axis b is strided on the cba grid
    # (stride Na) and accepts exchanges in parts; axis a is contiguous there
    s = "order=cba;rev=c;a=16x16x2/4;b=16x16x2/4/p2;c=16x16x2/4|" + BASE
    assert offt.plan_string((512, 512, 512), C128, "cba", s) == s


def test_natural_layout_rejects_reversed_strings():
    for plan in [BASE, BASE + "|" + BASE]:
        with pytest.raises(offt.OfftError):
            offt.plan_string((512, 512, 512), C128, "natural", plan)
    nat = offt.plan_string((512, 512, 512), C128, "natural")
    assert nat == offt.default_plan_string((512, 512, 512), C128)
    assert offt.plan_string((512, 512, 512), C128, "natural", nat) == nat


def test_one_axis_reversed_plan_rejects_a_transposing_axis():
    with pytest.raises(offt.OfftError):
        offt.plan_string((1, 1, 60), C128, "cba", "order=cba;rev=c;a=1;b=1;c=5x4x3/8|order=cba;a=5x4x3/8;b=1;c=1")


def test_bad_layout_names_rejected_before_the_device():
    with pytest.raises(ValueError):
        offt.plan_string((8, 8, 8), C128, "bca")
    with pytest.raises(ValueError):
        offt.Plan((8, 8, 8), layout="zyx")


def test_xcd_tile_order_in_plan_strings():
    """"/x" after an axis spec: the pass takes its tiles in XCD-contiguous order."""
    s = "order=bac;a=16x16x2/16/p2/x;b=32x16/32/p2;c=16x16x2/2/x"
    assert offt.plan_string((512, 512, 512), C128, "natural", s) == s
    r = "order=cba;rev=a;a=16x16x2/4/p2/x;b=16x16x2/4;c=16x16x2/4|" + BASE
    assert offt.plan_string((512, 512, 512), C128, "cba", r) == r
    assert offt.plan_string_nd((64, 64, 64, 64), C64, "order=dcba;a=16x4/32/x").startswith("order=dcba;a=16x4/32/x;")
    for bad in ["order=cba;c=16x16x2/2/y", "order=cba;c=16x16x2/2/x/p2", "order=cba;c=16x16x2/2/xx"]:
        with pytest.raises(offt.OfftError):
            offt.plan_string((512, 512, 512), C128, "natural", bad)


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape", [(512, 512, 512), (64, 48, 30), (1, 32, 40), (30, 40, 1), (6, 1, 9)])
def test_heuristic_tile_order_follows_the_stride(shape, dtype):
    """The heuristic plan takes the XCD-contiguous tile order ("/x") exactly on
    the axes whose lines are strided (a later axis longer than 1), except the
    lines strided by 2 MiB or more of a grid above 256 MiB, whose passes stream
    their data and keep the launch order."""
    f = dict(t.split("=", 1) for t in offt.default_plan_string(shape, dtype).split(";"))
    es = 16 if dtype == C128 else 8
    streams = np.prod(shape) * es > (256 << 20)
    for i, ax in enumerate("abc"):
        if shape[i] == 1:
            assert f[ax] == "1"
            continue
        strided = any(n > 1 for n in shape[i + 1:])
        long_stride = int(np.prod(shape[i + 1:])) * es >= (2 << 20)
        assert f[ax].endswith("/x") == (strided and not (streams and long_stride)), (ax, f[ax])


def test_access_mode_in_plan_strings():
    """"/s" and "/c" after an axis spec force streaming or cached grid-data
    accesses; without either the pass streams when the grids exceed 256 MiB."""
    s = "order=bca;a=16x16x2/16/p2/x/s;b=32x16/32/p2/c;c=16x16x2/2/s"
    assert offt.plan_string((512, 512, 512), C128, "natural", s) == s
    nd = offt.plan_string_nd((64, 64, 64, 64), C64, "order=dcba;a=16x4/32/c;d=8x8/4/x/s")
    assert ";a=16x4/32/c;" in nd and nd.endswith(";d=8x8/4/x/s")
    for bad in ["order=cba;c=16x16x2/2/s/x", "order=cba;c=16x16x2/2/q", "order=cba;c=16x16x2/2/s/c",
                "order=cba;c=16x16x2/2/ss"]:
        with pytest.raises(offt.OfftError):
            offt.plan_string((512, 512, 512), C128, "natural", bad)


def test_heuristic_tile_order_on_reversed_and_nd_plans():
    # the transposing pass keeps the launch order; on the cba grid after it,
    # axis b is strided (stride Na) and axis c is contiguous
    f, b = halves(offt.plan_string((512, 512, 512), C128, "cba"))
    assert f["rev"] == "a" and not f["a"].endswith("/x")
    assert f["b"].endswith("/x") and not f["c"].endswith("/x")
    nd = dict(t.split("=", 1) for t in offt.plan_string_nd((64, 64, 64, 64), C64).split(";"))
    assert [nd[ax].endswith("/x") for ax in "abcd"] == [True, True, True, False]


@pytest.mark.parametrize("L", [32, 64, 128, 160, 192, 256, 512])
def test_heuristic_contiguous_kernel_by_precision(L):
    """complex64 contiguous axes take a whole-line kernel of radix <= 8 at the
    default threads per line; complex128 ones keep the radix-16 kernels."""
    def c_spec(dtype):
        return dict(t.split("=", 1) for t in offt.default_plan_string((8, 8, L), dtype).split(";"))["c"]
    spec64 = c_spec(C64).split("/")
    seq = [int(r) for r in spec64[0].split("x")]
    assert max(seq) <= 8 and len(spec64) == 2          # radix <= 8, default threads per line, whole-line
    assert max(int(r) for r in c_spec(C128).split("/")[0].split("x")) == 16
