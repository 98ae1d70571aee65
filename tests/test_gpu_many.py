"""Uneven batches: one persistent launch (direct or replayed from a HIP graph)
over every (grid, axis pass, tile) work item -- with per-segment dependency
counters or level-synchronous with grid barriers -- and the level kernels,
against the CPU oracle and against the same plans run as separate launches.

The persistent executor runs the same tile code as the separate launches, so
with the same per-grid plans the results must agree bit for bit; every grid
must also meet the complex64 tolerance 2e-6 * log2(N_g) against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1501_07350_amd as offt
import synth

pytestmark = pytest.mark.gpu

C64, C128 = torch.complex64, torch.complex128


def packed_input(plan, dims, dtype, key0=synth.SEED):
    grids = synth.batch_grids(dims, dtype, key0=key0, device="cuda")
    return grids, plan.pack(grids)


def same_grids(plan, a, b):
    """Bitwise equality of every grid of two packed buffers (the alignment
    gaps between grids are never written)."""
    return all(torch.equal(u, v) for u, v in zip(plan.unpack(a), plan.unpack(b)))


def check_against_oracle(plan, grids, buf, dtype, sign=oracle.FORWARD, scale_inv=False, refs=None):
    worst = 0.0
    for g, (x, y) in enumerate(zip(grids, plan.unpack(buf))):
        ref = refs[g] if refs is not None else oracle.fft3(x.cpu().numpy().astype(np.complex128), sign)
        if scale_inv:
            ref = ref / x.numel()
        e = oracle.rel_l2(y.cpu().numpy(), ref)
        tol = oracle.tolerance(x.numel(), dtype == C64)
        assert e <= tol, (g, tuple(x.shape), e, tol)
        worst = max(worst, e / tol)
    return worst


def test_uneven_batch_64_grids_persistent_graph_vs_oracle_and_separate():
    dims = synth.uneven_batch_dims(64)
    plan = offt.ManyPlan(dims, dtype=C64)
    print(plan.describe().splitlines()[0], flush=True)
    grids, x = packed_input(plan, dims, C64)
    y_graph = plan.execute(x, use_graph=1)
    y_direct = plan.execute(x, use_graph=0)
    y_lgraph = plan.execute(x, use_graph=2)
    y_levels = plan.execute(x, use_graph=3)
    y_sgraph = plan.execute(x, use_graph=5)
    y_sync = plan.execute(x, use_graph=4)
    y_sep_same = plan.execute(x, use_graph=-2)
    y_sep_heur = plan.execute(x, use_graph=-1)
    torch.cuda.synchronize()
    assert plan.status() == 0
    assert same_grids(plan, y_graph, y_direct)
    assert same_grids(plan, y_graph, y_lgraph)
    assert same_grids(plan, y_graph, y_levels)
    assert same_grids(plan, y_graph, y_sgraph)
    assert same_grids(plan, y_graph, y_sync)
    assert same_grids(plan, y_graph, y_sep_same)
    assert same_grids(plan, y_graph, y_sep_heur)   # untuned plan: heuristic plans for both
    worst = check_against_oracle(plan, grids, y_graph, C64)
    print(f"64 grids: worst error / tolerance = {worst:.3e}", flush=True)


def test_uneven_batch_64_grids_tuned_every_launch_form_vs_oracle():
    """The benchmark's timed forms: exhaustively tuned per-grid plans, run as
    the grouped level graph, the level graph (the default), the
    level-synchronous graph, the queue-based persistent graph and separate
    launches; every one of the 64 grids against O3."""
    dims = synth.uneven_batch_dims(64)
    plan = offt.ManyPlan(dims, dtype=C64, tune="exhaustive")
    print(plan.describe().splitlines()[0], flush=True)
    grids, x = packed_input(plan, dims, C64)
    refs = [oracle.fft3(g.cpu().numpy().astype(np.complex128)) for g in grids]
    first = None
    assert "3 level groups" in plan.describe()     # 552 MB of grids in groups of at most 192 MiB
    for form in (offt.MANY_LEVELS_GROUPED_GRAPH, offt.MANY_LEVELS_GRAPH, offt.MANY_SYNC_GRAPH,
                 offt.MANY_PERSISTENT_GRAPH, offt.MANY_LEVELS, offt.MANY_SYNC, offt.MANY_PERSISTENT,
                 offt.MANY_SEPARATE_TUNED):
        print(f"form {form}", flush=True)
        y = plan.execute(x, use_graph=form)
        torch.cuda.synchronize()
        assert plan.status() == 0
        worst = check_against_oracle(plan, grids, y, C64, refs=refs)
        print(f"form {form}: worst error / tolerance over 64 grids = {worst:.3e}", flush=True)
        if first is None:
            first = y
        else:
            assert same_grids(plan, first, y), f"form {form} differs from the grouped level graph"


def test_graph_replays_match_eager_with_work_between():
    dims = synth.uneven_batch_dims(16, key=synth.KEY_DIMS + 7)
    plan = offt.ManyPlan(dims, dtype=C64)
    grids, x = packed_input(plan, dims, C64, key0=synth.SEED + 100)
    eager = plan.execute(x, use_graph=0)
    torch.cuda.synchronize()
    out = torch.empty_like(x)
    for rep in range(4):
        for mode in (1, 2, 5):   # persistent graph, level graph, level-synchronous graph
            # unrelated eager work and a sync between replays
            _ = (x * 2).sum()
            torch.cuda.synchronize()
            out.zero_()
            plan.execute(x, out=out, use_graph=mode)
            torch.cuda.synchronize()
            assert plan.status() == 0
            assert same_grids(plan, out, eager), f"replay {rep} of graph {mode} differs"
    # new buffers and direction: the graph's arguments are updated
    x2 = x.clone()
    z = plan.execute(x2, use_graph=1, direction=offt.BACKWARD)
    z2 = plan.execute(x2, use_graph=2, direction=offt.BACKWARD)
    z5 = plan.execute(x2, use_graph=5, direction=offt.BACKWARD)
    z_ref = plan.execute(x2, use_graph=-2, direction=offt.BACKWARD)
    torch.cuda.synchronize()
    assert plan.status() == 0
    assert same_grids(plan, z, z_ref)
    assert same_grids(plan, z2, z_ref)
    assert same_grids(plan, z5, z_ref)
    check_against_oracle(plan, grids, z, C64, sign=oracle.BACKWARD)


MIXED = [(2, 3, 5), (1, 1, 1), (9, 25, 27), (100, 4, 6), (48, 60, 64), (16, 1, 8), (5, 5, 5)]


@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_mixed_small_batch_separate_launches(dtype):
    # lengths outside the persistent executor's set (2, 3, 5, 9, 25, 27, 100)
    # and a 1x1x1 grid: separate launches, normalised round trip, in place
    plan = offt.ManyPlan(MIXED, dtype=dtype, normalize_inverse=True)
    assert "persistent executor unavailable" in plan.describe()
    grids, x = packed_input(plan, MIXED, dtype, key0=synth.SEED + 300)
    with pytest.raises(offt.OfftError) as ei:
        plan.execute(x, use_graph=1)
    assert ei.value.code == -2
    y = plan.execute(x, use_graph=-2)
    torch.cuda.synchronize()
    check_against_oracle(plan, grids, y, dtype)
    assert same_grids(plan, y, plan.execute(x, use_graph=-1))
    buf = y.clone()
    plan.execute(buf, out=buf, use_graph=-1, direction=offt.BACKWARD)
    torch.cuda.synchronize()
    for g, (a, b) in enumerate(zip(grids, plan.unpack(buf))):
        e = oracle.rel_l2(b.cpu().numpy(), a.cpu().numpy())
        assert e <= oracle.tolerance(a.numel(), dtype == C64), (g, e)


@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_mixed_small_batch_level_kernels(dtype):
    """Lengths outside the persistent executor's set run on the level kernels
    of the every-length executor: against the oracle, bit-identical to the
    same plans as separate launches, as the default form, and an in-place
    normalised round trip."""
    plan = offt.ManyPlan(MIXED, dtype=dtype, normalize_inverse=True)
    desc = plan.describe()
    print(desc.splitlines()[0], flush=True)
    assert "executor all" in desc and "level kernels unavailable" not in desc
    grids, x = packed_input(plan, MIXED, dtype, key0=synth.SEED + 310)
    y = plan.execute(x, use_graph=2)
    y_levels = plan.execute(x, use_graph=3)
    y_sep = plan.execute(x, use_graph=-2)
    y_default = plan.forward(x)
    torch.cuda.synchronize()
    check_against_oracle(plan, grids, y, dtype)
    assert same_grids(plan, y, y_levels)
    assert same_grids(plan, y, y_sep)
    assert same_grids(plan, y, y_default)
    buf = y.clone()
    plan.execute(buf, out=buf, use_graph=2, direction=offt.BACKWARD)
    torch.cuda.synchronize()
    for g, (a, b) in enumerate(zip(grids, plan.unpack(buf))):
        e = oracle.rel_l2(b.cpu().numpy(), a.cpu().numpy())
        assert e <= oracle.tolerance(a.numel(), dtype == C64), (g, e)


def every_length_dims():
    """Grids whose axes take every 2/3/5-smooth length from 2 to 160, three
    lengths per grid, short and long lengths mixed."""
    def smooth(n):
        for q in (2, 3, 5):
            while n % q == 0:
                n //= q
        return n == 1

    lengths = [n for n in range(2, 161) if smooth(n)]
    half = (len(lengths) + 1) // 2
    short, long_ = lengths[:half], lengths[half:][::-1]
    axes = [v for pair in zip(short, long_ + [1]) for v in pair]
    axes += [1] * (-len(axes) % 3)
    return [tuple(axes[i:i + 3]) for i in range(0, len(axes), 3)]


@pytest.mark.parametrize("tune", ["none", "exhaustive"])
def test_every_length_up_to_160_level_kernels(tune):
    """Every length the every-length executor compiles, in heuristic and in
    tuned plans, through the level kernels: against the oracle and bit for
    bit against the same plans as separate launches."""
    dims = every_length_dims()
    plan = offt.ManyPlan(dims, dtype=C64, tune=tune)
    print(plan.describe().splitlines()[0], flush=True)
    assert "executor all" in plan.describe()
    grids, x = packed_input(plan, dims, C64, key0=synth.SEED + 320)
    y = plan.forward(x)
    y_sep = plan.execute(x, use_graph=-2)
    torch.cuda.synchronize()
    assert same_grids(plan, y, y_sep)
    check_against_oracle(plan, grids, y, C64)


@pytest.mark.skip(reason="the work-queue persistent kernel of the executor for every length <= 160 stopped "
                         "responding on the GPU for this batch; its cause is not found (the tile code and loop "
                         "pass the CPU emulation in tests/test_emu.py), so that executor's persistent forms are "
                         "not built")
def test_mixed_small_batch_persistent_all_lengths():
    plan = offt.ManyPlan(MIXED, dtype=C64, normalize_inverse=True)
    grids, x = packed_input(plan, MIXED, C64, key0=synth.SEED + 300)
    y = plan.execute(x, use_graph=1)
    torch.cuda.synchronize()
    assert plan.status() == 0
    check_against_oracle(plan, grids, y, C64)


def test_batch_lengths_with_unit_axes_persistent():
    # lengths of the executor's set plus axes of length 1 (grids of 1 or 2 passes)
    dims = [(48, 1, 60), (1, 160, 1), (64, 80, 96), (150, 120, 1)]
    plan = offt.ManyPlan(dims, dtype=C64, normalize_inverse=True)
    assert "executor batch" in plan.describe()
    grids, x = packed_input(plan, dims, C64, key0=synth.SEED + 400)
    y = plan.execute(x, use_graph=1)
    torch.cuda.synchronize()
    assert plan.status() == 0
    check_against_oracle(plan, grids, y, C64)
    assert same_grids(plan, y, plan.execute(x, use_graph=-2))
    ys = plan.execute(x, use_graph=4)
    torch.cuda.synchronize()
    assert plan.status() == 0
    assert same_grids(plan, y, ys)
    buf = y.clone()
    plan.execute(buf, out=buf, use_graph=1, direction=offt.BACKWARD)
    torch.cuda.synchronize()
    assert plan.status() == 0
    for g, (a, b) in enumerate(zip(grids, plan.unpack(buf))):
        e = oracle.rel_l2(b.cpu().numpy(), a.cpu().numpy())
        assert e <= oracle.tolerance(a.numel(), True), (g, e)


def test_long_axis_has_no_persistent_executor():
    dims = [(256, 4, 4), (8, 8, 8)]
    plan = offt.ManyPlan(dims, dtype=C64)
    assert "level kernels unavailable" in plan.describe()
    grids, x = packed_input(plan, dims, C64)
    for form in (1, 2):
        with pytest.raises(offt.OfftError) as ei:
            plan.execute(x, use_graph=form)
        assert ei.value.code == -2
    y = plan.execute(x, use_graph=-1)
    torch.cuda.synchronize()
    check_against_oracle(plan, grids, y, C64)


def test_tuned_batch_plans_are_valid():
    dims = synth.uneven_batch_dims(6, key=synth.KEY_DIMS + 11)
    plan = offt.ManyPlan(dims, dtype=C64, tune="exhaustive")
    grids, x = packed_input(plan, dims, C64, key0=synth.SEED + 500)
    y = plan.execute(x, use_graph=1)
    y2 = plan.execute(x, use_graph=-2)
    y5 = plan.execute(x, use_graph=5)
    torch.cuda.synchronize()
    assert plan.status() == 0
    assert same_grids(plan, y, y2)
    assert same_grids(plan, y, y5)
    check_against_oracle(plan, grids, y, C64)
    for line in plan.describe().splitlines()[1:]:
        assert line.startswith("order=")


def test_default_launch_form():
    """offt_exec_many_fwd / _bwd: the level kernels from a graph where an
    executor covers the batch (bit-identical to use_graph=2 and to the
    grouped graph, 6), the tuned separate launches where it does not;
    backward round trip with 1/N."""
    dims = synth.uneven_batch_dims(8, key=synth.KEY_DIMS + 23)
    plan = offt.ManyPlan(dims, dtype=C64, normalize_inverse=True)
    grids, x = packed_input(plan, dims, C64, key0=synth.SEED + 700)
    y = plan.forward(x)
    y2 = plan.execute(x, use_graph=2)
    y6 = plan.execute(x, use_graph=6)
    z = plan.backward(y)
    torch.cuda.synchronize()
    assert same_grids(plan, y, y2) and same_grids(plan, y, y6)
    check_against_oracle(plan, grids, y, C64)
    for g, (a, b) in enumerate(zip(grids, plan.unpack(z))):
        assert oracle.rel_l2(b.cpu().numpy(), a.cpu().numpy()) <= oracle.tolerance(a.numel(), True), g
    dims = [(256, 4, 4), (8, 8, 8)]
    lplan = offt.ManyPlan(dims, dtype=C64)
    grids, x = packed_input(lplan, dims, C64)
    y = lplan.forward(x)
    y2 = lplan.execute(x, use_graph=-2)
    torch.cuda.synchronize()
    assert same_grids(lplan, y, y2)
    check_against_oracle(lplan, grids, y, C64)


def test_grouped_level_graph_many_groups():
    """24 complex128 grids of 128-160 points per axis (about 1.1 GiB, 42-53
    MiB each, so groups of a few grids under 192 MiB): the grouped graph
    equals the level graph bit for bit, every grid matches the oracle, and a
    call in place in the backward direction updates the graph."""
    lens = (128, 144, 150, 160)
    dims = [(lens[g % 4], lens[(g + 1) % 4], lens[(g + 3) % 4]) for g in range(24)]
    plan = offt.ManyPlan(dims, dtype=C128, normalize_inverse=True)
    ng = int(plan.describe().split(" level groups")[0].rsplit(" ", 1)[1])
    print(plan.describe().splitlines()[0], flush=True)
    assert ng >= 3
    grids, x = packed_input(plan, dims, C128, key0=synth.SEED + 800)
    y6 = plan.execute(x, use_graph=6)
    y2 = plan.execute(x, use_graph=2)
    torch.cuda.synchronize()
    assert same_grids(plan, y6, y2)
    check_against_oracle(plan, grids, y6, C128)
    buf = y6.clone()
    plan.execute(buf, out=buf, use_graph=6, direction=offt.BACKWARD)
    torch.cuda.synchronize()
    for g, (a, b) in enumerate(zip(grids, plan.unpack(buf))):
        e = oracle.rel_l2(b.cpu().numpy(), a.cpu().numpy())
        assert e <= oracle.tolerance(a.numel(), False), (g, e)
