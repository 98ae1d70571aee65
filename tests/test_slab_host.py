"""Plan strings of the slab schedule (";slab=S"): parsed, written back in
canonical form, and rejected where the schedule does not fit (no GPU)."""
import pytest
import torch

import paper_1501_07350_amd as offt

C128, C64 = torch.complex128, torch.complex64
PLAN = "order=abc;a=16x16x2/16/p2;b=16x16x2/16/p2/x;c=8x8x8/2"


@pytest.mark.parametrize("slab,canonical", [("64", "64"), ("1", "1"), ("0064", "64"), ("4096", "4096")])
def test_slab_round_trip(slab, canonical):
    s = offt.plan_string((512, 512, 512), C128, "natural", f"{PLAN};slab={slab}")
    assert s == f"{PLAN};slab={canonical}"
    # the slab field may stand anywhere in the string
    t = offt.plan_string((512, 512, 512), C128, "natural", f"slab={slab};{PLAN}")
    assert t == s


def test_plan_without_slab_has_none():
    assert "slab" not in offt.plan_string((512, 512, 512), C128, "natural", PLAN)
    assert "slab" not in offt.default_plan_string((512, 512, 512), C128)


@pytest.mark.parametrize("shape,plan", [
    ((512, 512, 512), PLAN.replace("order=abc", "order=bac") + ";slab=64"),    # pass over a not first
    ((512, 512, 512), PLAN.replace("order=abc", "order=cba") + ";slab=64"),
    ((512, 512, 512), PLAN + ";slab=0"),
    ((512, 512, 512), PLAN + ";slab=-4"),
    ((512, 512, 512), PLAN + ";slab="),
    ((512, 512, 512), PLAN + ";slab=6x"),
    ((512, 512, 512), PLAN + ";slab=99999999999999"),
    ((1, 512, 512), "order=abc;a=1;b=16x16x2/16/p2/x;c=8x8x8/2;slab=4"),        # no pass over a
    ((512, 1, 1), "order=abc;a=16x16x2/16/p2;b=1;c=1;slab=4"),                 # nothing after it
])
def test_unusable_slab_plans_rejected(shape, plan):
    with pytest.raises(offt.OfftError) as e:
        offt.plan_string(shape, C128, "natural", plan)
    assert e.value.code == -6


def test_slab_not_in_reversed_layout():
    s = offt.plan_string((64, 48, 30), C64, "cba")
    fwd, bwd = s.split("|")
    with pytest.raises(offt.OfftError) as e:
        offt.plan_string((64, 48, 30), C64, "cba", f"{fwd};slab=4|{bwd}")
    assert e.value.code == -6


def test_slab_with_unit_axis_b_or_c():
    # one of b and c of length 1: the schedule covers the remaining pass
    base = offt.default_plan_string((64, 1, 30), C64)
    order = dict(f.split("=", 1) for f in base.split(";"))["order"]
    plan = base.replace(f"order={order}", "order=a" + order.replace("a", "")) + ";slab=8"
    assert offt.plan_string((64, 1, 30), C64, "natural", plan) == plan


def nd_with_first_axis_first(shape, dtype):
    base = offt.plan_string_nd(shape, dtype)
    order = dict(f.split("=", 1) for f in base.split(";"))["order"]
    return base.replace(f"order={order}", "order=a" + order.replace("a", ""))


@pytest.mark.parametrize("shape", [(16, 8, 6, 10), (6, 4, 5, 3, 8)])
def test_nd_slab_round_trip(shape):
    plan = nd_with_first_axis_first(shape, C64) + ";slab=3"
    assert offt.plan_string_nd(shape, C64, plan) == plan
    assert "slab" not in offt.plan_string_nd(shape, C64)


def test_nd_slab_needs_first_axis_first():
    shape = (16, 8, 6, 10)
    base = offt.plan_string_nd(shape, C64)          # heuristic order: last axis first
    assert not base.split(";")[0].endswith("=a") and "order=a" not in base
    with pytest.raises(offt.OfftError) as e:
        offt.plan_string_nd(shape, C64, base + ";slab=3")
    assert e.value.code == -6


@pytest.mark.parametrize("slab", ["0", "-1", "", "x"])
def test_nd_bad_slab_rejected(slab):
    shape = (16, 8, 6, 10)
    with pytest.raises(offt.OfftError) as e:
        offt.plan_string_nd(shape, C64, nd_with_first_axis_first(shape, C64) + f";slab={slab}")
    assert e.value.code == -6


PLAN_C = "order=cba;a=16x16x2/16/p2;b=16x16x2/16/p2/x;c=8x8x8/2"


@pytest.mark.parametrize("order", ["cba", "cab"])
@pytest.mark.parametrize("col", ["16", "64", "256"])
def test_column_block_round_trip(order, col):
    plan = PLAN_C.replace("order=cba", f"order={order}") + f";col={col}"
    assert offt.plan_string((512, 512, 512), C128, "natural", plan) == plan


@pytest.mark.parametrize("plan", [
    PLAN_C.replace("order=cba", "order=acb") + ";col=64",   # pass over c not first
    PLAN_C + ";col=48",                                     # not a power of two
    PLAN_C + ";col=512",                                    # the whole row
    PLAN_C + ";col=8",                                      # narrower than the 16-column tiles
    PLAN_C + ";col=0",
    PLAN_C + ";col=64;slab=4",                              # both schedules
])
def test_unusable_column_block_plans_rejected(plan):
    with pytest.raises(offt.OfftError) as e:
        offt.plan_string((512, 512, 512), C128, "natural", plan)
    assert e.value.code == -6


def test_column_block_not_on_a_ragged_row():
    # 48 columns split into blocks of 16 but not of 32; the strided tiles are
    # 16 columns wide
    plan = "order=cba;a=16x4/16/x;b=8x5/16/x;c=4x4x3/16"
    assert offt.plan_string((64, 40, 48), C64, "natural", plan + ";col=16") == plan + ";col=16"
    with pytest.raises(offt.OfftError):
        offt.plan_string((64, 40, 48), C64, "natural", plan + ";col=32")
    # tiles of 32 columns do not fit blocks of 16
    with pytest.raises(offt.OfftError):
        offt.plan_string((64, 40, 48), C64, "natural", plan.replace("/16/x", "/32/x") + ";col=16")


def test_every_plan_cache_entry_parses():
    """Every entry of the committed plan cache names compiled kernels and a
    schedule that fits its grid, and is written in canonical form (no
    device needed; tile sizes are checked against the device at plan time)."""
    import os
    path = os.path.join(os.path.dirname(offt.__file__), "data", "plan_cache_mi355x.txt")
    n = 0
    for line in open(path):
        head, plan, ms = line.rstrip("\n").split("\t")
        fields = dict(f.split("=", 1) for f in head.split())
        dims = tuple(int(v) for v in fields["dims"].split("x"))
        dtype = C128 if fields["dtype"] == "0" else C64
        assert float(ms) > 0
        if len(dims) == 3:
            layout = "cba" if fields.get("layout") == "cba" else "natural"
            assert offt.plan_string(dims, dtype, layout, plan) == plan, line
        else:
            assert offt.plan_string_nd(dims, dtype, plan) == plan, line
        n += 1
    assert n >= 10
