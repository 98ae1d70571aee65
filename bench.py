#!/usr/bin/env python
"""Benchmark of the 3-D complex-to-complex FFT on one MI355X.

Workload (default): one forward 3-D transform of a 512x512x512 grid, complex128
(the headline value) and, measured in the same run, complex64; uniform [-1, 1)
synthetic entries from the seeded generator, resident in HBM before timing.
Plans are tuned at plan time (exhaustive tuning, excluded from the timed
region like the paper's initialization phase); the heuristic plan's times are
reported beside them.

A "step" is one forward transform: all axis passes with their fused
rearrangements.  W warm-up steps, then K timed steps; each pass is bracketed
by HIP events recorded on the stream the passes are launched on.

Prints ONE JSON line.  value = GFLOP/s by the 5 N log2 N convention for the
complex128 transform; the complex64 figures are in "f32".  roofline: the
slowest (dominant) pass kernel, algorithmic bytes 2 N s per launch divided by
its mean duration, against 8 TB/s HBM.  cpu_baseline: the CPU oracle's
recursive FFT timed on the host cores on one 512^3 complex128 transform.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3-D C2C FFT GFLOP/s (5N·log2N/t) + HBM GB/s at 512³, FP32 vs FP64"
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")
# Plan cache of the exhaustive tuner ("user-select after tuning once"): the
# timed plans are the ones the tuner chose on MI355X when the profiles were
# taken; a shape or device without an entry is tuned and appended.
PLAN_CACHE = os.path.join(ROOT, "paper_1501_07350_amd", "data", "plan_cache_mi355x.txt")

KERNEL_SOURCES = ["paper_1501_07350_amd/csrc/fft_device.hpp", "paper_1501_07350_amd/csrc/planner.cpp",
                  "paper_1501_07350_amd/csrc/gen_kernels.py"]


def _cache(tune: str):
    return PLAN_CACHE if (PLAN_CACHE and tune in ("exhaustive", "learned")) else None


# timed runs per candidate when a plan is tuned here (a cache miss): the
# minimum of 5 after a warm-up separates near-equal kernels more reliably than
# the library's default of 2
TUNE_REPS = 5


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pass_keys(plan: str):
    """Per-pass keys "axis=spec" of a plan string such as
    order=bca;a=16x16x2/16;b=16x16x2/16;c=16x16x2/2 (pass i transforms the
    i-th axis of the order that is longer than 1; an axis of length 1, spec
    "1", has no pass)."""
    fields = dict(f.split("=", 1) for f in plan.split("|")[0].strip().split(";"))
    return [f"{ax}={fields[ax]}" for ax in fields["order"] if fields[ax] != "1"]


def plan_schedule(plan: str):
    """("slab", planes per slab), ("col", columns per block) or (None, 0)
    for a plan string's block schedule (";slab=S" or ";col=W")."""
    for f in plan.split("|")[0].strip().split(";"):
        for key in ("slab", "col"):
            if f.startswith(key + "="):
                return key, int(f[len(key) + 1:])
    return None, 0


def plan_slab(plan: str) -> int:
    """Planes per slab or columns per block of a plan string's block
    schedule, or 0."""
    return plan_schedule(plan)[1]


def pass_groups(plan: str):
    """Pass indices timed together: each pass on its own, except that the
    passes of a slab or column-block schedule (every pass after the first)
    form one group, since they run interleaved block by block."""
    npass = len(pass_keys(plan))
    if plan_slab(plan) and npass > 1:
        return [[0], list(range(1, npass))]
    return [[i] for i in range(npass)]


def pass_label(plan: str, i: int) -> str:
    """Key "axis=spec" of pass i, with ";slab=S" for a pass of a slab schedule
    (its access modes and cache behaviour differ from the whole-grid pass)."""
    kind, size = plan_schedule(plan)
    keys = pass_keys(plan)
    return keys[i] + (f";{kind}={size}" if kind and i > 0 else "")


def group_key(plan: str, g) -> str:
    keys = pass_keys(plan)
    kind, size = plan_schedule(plan)
    key = "+".join(keys[i] for i in g)
    return key + (f";{kind}={size}" if len(g) > 1 else "")


def pass_launches(plan: str, planes: int, ncols: int | None = None):
    """Pass index of every kernel launch of one transform, in launch order
    (`planes` = Na x batch, `ncols` = Nc, by default `planes`: a slab or
    column-block schedule launches each of its passes once per block, block
    after block)."""
    npass = len(pass_keys(plan))
    kind, size = plan_schedule(plan)
    if not kind or npass < 2:
        return list(range(npass))
    nblocks = -(-planes // size) if kind == "slab" else (ncols or planes) // size
    return [0] + [i for _ in range(nblocks) for i in range(1, npass)]


def load_traffic(tag: str, key: str):
    """Measured HBM bytes per launch of one pass (from rocprofv3 PMC runs),
    only if they were taken on the current kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_source_hash():
        return None
    return d.get("workloads", {}).get(tag, {}).get("pass_bytes", {}).get(key)


def time_transform(n: int, dtype, steps: int, warmup: int, check: bool, tune: str = "exhaustive",
                   forced: str | None = None):
    import numpy as np
    import torch

    import paper_1501_07350_amd as offt
    import synth

    shape = (n, n, n)
    x = synth.complex_grid(shape, dtype, device="cuda")
    y = torch.empty_like(x)
    t0 = time.perf_counter()
    plan = offt.Plan(shape, dtype=dtype, tune=tune, forced_plan=forced, cache_path=_cache(tune), reps=TUNE_REPS)
    plan_s = time.perf_counter() - t0
    npass = plan.npasses()
    desc = plan.describe()
    # each pass timed on its own, a slab schedule's passes as one group
    # (launched as the transform launches them: interleaved slab by slab)
    groups = pass_groups(desc)
    ng = len(groups)
    stream = torch.cuda.current_stream()
    h = int(stream.cuda_stream)
    xp, yp = x.data_ptr(), y.data_ptr()

    def step():
        for g in groups:
            plan.exec_range(g[0], len(g), offt.FORWARD, xp, yp, h)

    for _ in range(warmup):
        step()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(ng + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        for j, g in enumerate(groups):
            ev[k][j].record(stream)
            plan.exec_range(g[0], len(g), offt.FORWARD, xp, yp, h)
        ev[k][ng].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pass_ms = [sum(ev[k][j].elapsed_time(ev[k][j + 1]) for k in range(steps)) / steps for j in range(ng)]
    total_ms = ev[0][0].elapsed_time(ev[steps - 1][ng])
    ms = total_ms / steps
    N = x.numel()
    s = x.element_size()
    # the transform just timed, checked before the copies below overwrite y
    checked = {}
    if check:
        import oracle
        xh = x.cpu().numpy().astype(np.complex128)
        yh = y.cpu().numpy()
        got, ref = [], []
        for ka, kb in ((0, 0), (3, 5), (n - 1, 7)):
            got.append(yh[ka, kb].astype(np.complex128))
            ref.append(oracle.dft3_line(xh, ka, kb))
        checked["check_rel_l2_sampled_lines"] = oracle.rel_l2(np.concatenate(got), np.concatenate(ref))
        checked["check_tolerance"] = oracle.tolerance(N, dtype == torch.complex64)
    # the copy of each pass's own memory accesses (offt_copy_pass): the same
    # tiles, threads, tile order and access mode, no arithmetic
    copy_ms = []
    for i in range(npass):
        for _ in range(warmup):
            plan.copy_pass(i, xp, yp, h)
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(steps):
            plan.copy_pass(i, xp, yp, h)
        c1.record(stream)
        torch.cuda.synchronize()
        copy_ms.append(c0.elapsed_time(c1) / steps)
    res = {
        "ms": ms,
        "gflops": 5.0 * N * math.log2(N) / (ms * 1e6),
        "eff_gbs": 6.0 * N * s / (ms * 1e6),
        "wall_ms_per_step": 1e3 * wall / steps,
        "plan": desc,
        "plan_seconds": plan_s,
        "pass_ms": pass_ms,
        "groups": groups,
        "pass_bytes": 2 * N * s,
        "copy_ms": copy_ms,
    }
    res.update(checked)
    plan.close()
    del x, y
    torch.cuda.empty_cache()
    return res


def time_reversed(n: int, dtype, steps: int, warmup: int, check: bool, tune: str = "exhaustive"):
    """Forward and backward transforms whose spectral side is in reversed
    (cba) order, beside the natural plan of the same tuning, in ms per
    transform (events around `steps` back-to-back executions)."""
    import numpy as np
    import torch

    import paper_1501_07350_amd as offt
    import synth

    shape = (n, n, n)
    x = synth.complex_grid(shape, dtype, device="cuda")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    h = int(stream.cuda_stream)

    def timed(plan, direction, src, dst):
        for _ in range(warmup):
            plan.exec_ptr(direction, src.data_ptr(), dst.data_ptr(), h)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.exec_ptr(direction, src.data_ptr(), dst.data_ptr(), h)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    res = {}
    for name, lay in (("natural", "natural"), ("reversed", "cba")):
        plan = offt.Plan(shape, dtype=dtype, tune=tune, layout=lay, cache_path=_cache(tune), reps=TUNE_REPS)
        fwd = timed(plan, offt.FORWARD, x, y)
        bwd = timed(plan, offt.BACKWARD, y, x)
        res[name] = {"fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4), "plan": plan.describe()}
        if name == "reversed" and check:
            import oracle
            x.copy_(synth.complex_grid(shape, dtype, device="cuda"))
            plan.forward(x, out=y.view(shape[::-1]))
            torch.cuda.synchronize()
            xh = x.cpu().numpy().astype(np.complex128)
            yh = y.view(shape[::-1]).cpu().numpy()
            got, ref = [], []
            for ka, kb in ((0, 0), (3, 5), (n - 1, 7)):
                got.append(yh[:, kb, ka].astype(np.complex128))     # Y[c, b, a] = X[a, b, c]
                ref.append(oracle.dft3_line(xh, ka, kb))
            res[name]["check_rel_l2_sampled_lines"] = oracle.rel_l2(np.concatenate(got), np.concatenate(ref))
            res[name]["check_tolerance"] = oracle.tolerance(x.numel(), dtype == torch.complex64)
        plan.close()
    res["reversed_over_natural_fwd"] = round(res["reversed"]["fwd_ms"] / res["natural"]["fwd_ms"], 3)
    del x, y
    torch.cuda.empty_cache()
    return res


def time_nd(shape, dtype, steps: int, warmup: int, check: bool, tune: str = "exhaustive"):
    """A grid of 4 or 5 axes: the tuned plan (kernels per axis, then every
    pass order) and the heuristic plan, ms per forward transform."""
    import numpy as np
    import torch

    import paper_1501_07350_amd as offt
    import synth

    x = synth.complex_grid(shape, dtype, device="cuda")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    h = int(stream.cuda_stream)
    N = x.numel()
    s = x.element_size()
    res = {"shape": list(shape), "dtype": "f64" if dtype == torch.complex128 else "f32"}
    for name, t in (("tuned", tune), ("heuristic", "none")):
        t0 = time.perf_counter()
        plan = offt.Plan(shape, dtype=dtype, tune=t, cache_path=_cache(t), reps=TUNE_REPS)
        plan_s = time.perf_counter() - t0
        for _ in range(warmup):
            plan.exec_ptr(offt.FORWARD, x.data_ptr(), y.data_ptr(), h)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.exec_ptr(offt.FORWARD, x.data_ptr(), y.data_ptr(), h)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        npass = plan.npasses()
        res[name] = {"ms": round(ms, 4), "gflops": round(5.0 * N * math.log2(N) / (ms * 1e6), 1),
                     "eff_gbs": round(2.0 * npass * N * s / (ms * 1e6), 1), "plan": plan.describe(),
                     "plan_seconds": round(plan_s, 3)}
        plan.close()
    if check:
        import oracle
        from oracle import ndim
        xh = x.cpu().numpy()
        yh = y.cpu().numpy()
        pts = [tuple(0 for _ in shape), tuple(min(i + 1, n - 1) for i, n in enumerate(shape)),
               tuple(n - 1 for n in shape)]
        got = np.array([yh[k] for k in pts], dtype=np.complex128)
        ref = np.array([ndim.dftn_point(xh, k) for k in pts])
        res["check_rel_l2_sampled_points"] = oracle.rel_l2(got, ref)
        res["check_tolerance"] = oracle.tolerance(N, dtype == torch.complex64)
    del x, y
    torch.cuda.empty_cache()
    return res


def reversed_runs(n: int, steps: int, warmup: int, check: bool):
    """The reversed (cba) output order at n^3, complex128 and complex64."""
    import torch

    return {"workload": f"{n}^3 forward with the output in cba order, and backward from it",
            "f64": time_reversed(n, torch.complex128, steps, warmup, check),
            "f32": time_reversed(n, torch.complex64, steps, warmup, check)}


def nd_runs(steps: int, warmup: int, check: bool):
    """The grids of 4 and 5 axes: 128^4 complex64 and complex128, 48^5 complex64."""
    import torch

    return [time_nd((128, 128, 128, 128), torch.complex64, steps, warmup, check),
            time_nd((128, 128, 128, 128), torch.complex128, steps, warmup, False),
            time_nd((48, 48, 48, 48, 48), torch.complex64, steps, warmup, check)]


def time_batch(steps: int, warmup: int, check: bool, count: int = 64):
    """Uneven batch of `count` complex64 grids (axes drawn from
    {48,...,160}): every launch form of the batch executor (the level kernels
    replayed from a HIP graph, the default, also grouped by
    Infinity-Cache-sized groups of grids; the level-synchronous and the
    work-queue persistent kernels) vs every grid's passes launched separately
    on the same stream."""
    import numpy as np
    import torch

    import paper_1501_07350_amd as offt
    import synth

    dims = synth.uneven_batch_dims(count)
    dtype = torch.complex64
    heur = offt.ManyPlan(dims, dtype=dtype, tune="none")
    t0 = time.perf_counter()
    tuned = offt.ManyPlan(dims, dtype=dtype, tune="exhaustive")
    tune_s = time.perf_counter() - t0
    grids = synth.batch_grids(dims, dtype, device="cuda")
    x = heur.pack(grids)
    y = torch.empty_like(x)
    h = int(torch.cuda.current_stream().cuda_stream)
    xp, yp = x.data_ptr(), y.data_ptr()
    variants = {
        "separate_heuristic": (heur, offt.MANY_SEPARATE_HEURISTIC),
        "separate_tuned": (tuned, offt.MANY_SEPARATE_TUNED),
        "persistent_tuned": (tuned, offt.MANY_PERSISTENT),
        "graph_tuned": (tuned, offt.MANY_PERSISTENT_GRAPH),
        "graph_heuristic": (heur, offt.MANY_PERSISTENT_GRAPH),
        "levels_tuned": (tuned, offt.MANY_LEVELS),
        "levels_graph_tuned": (tuned, offt.MANY_LEVELS_GRAPH),
        "levels_grouped_graph_tuned": (tuned, offt.MANY_LEVELS_GROUPED_GRAPH),
        "sync_tuned": (tuned, offt.MANY_SYNC),
        "sync_graph_tuned": (tuned, offt.MANY_SYNC_GRAPH),
    }
    ms = {}
    for name, (pl, mode) in variants.items():
        for _ in range(warmup):
            pl.exec_ptr(xp, yp, offt.FORWARD, mode, h)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            pl.exec_ptr(xp, yp, offt.FORWARD, mode, h)
        e1.record()
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1) / steps
        if mode >= 0 and pl.status() != 0:
            raise RuntimeError(f"persistent executor reported a dependency timeout ({name})")
    flop = sum(5.0 * a * b * c * math.log2(a * b * c) for a, b, c in dims)
    nbytes = sum(6.0 * a * b * c * 8 for a, b, c in dims)
    out = {
        "workload": f"{count} complex64 grids, axes uniform over {list(synth.BATCH_AXIS_LENGTHS)}",
        "elements": int(sum(a * b * c for a, b, c in dims)),
        "tune_seconds": round(tune_s, 3),
        "executor": tuned.describe().splitlines()[0],
        "ms": {k: round(v, 4) for k, v in ms.items()},
        "gflops": {k: round(flop / (v * 1e6), 1) for k, v in ms.items()},
        "eff_gbs": {k: round(nbytes / (v * 1e6), 1) for k, v in ms.items()},
        # the library's default form (offt_exec_many_fwd) and the fastest
        # single-kernel form; every form's time is in "ms"
        "default_form": "levels_graph_tuned",
        "speedup_levels_grouped_graph_tuned_vs_separate_heuristic": round(
            ms["separate_heuristic"] / ms["levels_grouped_graph_tuned"], 3),
        "speedup_levels_graph_tuned_vs_separate_heuristic": round(
            ms["separate_heuristic"] / ms["levels_graph_tuned"], 3),
        "speedup_sync_graph_tuned_vs_separate_heuristic": round(ms["separate_heuristic"] / ms["sync_graph_tuned"], 3),
    }
    if check:
        import oracle
        tuned.exec_ptr(xp, yp, offt.FORWARD, offt.MANY_LEVELS_GRAPH, h)
        torch.cuda.synchronize()
        worst = 0.0
        for g, yg in enumerate(tuned.unpack(y)):
            ref = oracle.fft3(grids[g].cpu().numpy().astype(np.complex128))
            e = oracle.rel_l2(yg.cpu().numpy(), ref)
            worst = max(worst, e / oracle.tolerance(grids[g].numel(), True))
        out["check_worst_error_over_tolerance_all_grids"] = worst
    heur.close()
    tuned.close()
    return out


def time_batch_any_lengths(steps: int, warmup: int, check: bool, count: int = 64):
    """Uneven batch of `count` complex64 grids with axes drawn from every
    2/3/5-smooth length 2..160 (the every-length executor, level kernels
    only) with the heuristic plans: level kernels, directly and from a HIP
    graph, vs every grid's passes launched separately."""
    import numpy as np
    import torch

    import paper_1501_07350_amd as offt
    import synth

    lengths = synth.smooth_lengths(2, 160)
    dims = synth.uneven_batch_dims(count, key=synth.KEY_DIMS + 101, lengths=lengths)
    dtype = torch.complex64
    plan = offt.ManyPlan(dims, dtype=dtype, tune="none")
    grids = synth.batch_grids(dims, dtype, key0=synth.SEED + 900, device="cuda")
    x = plan.pack(grids)
    y = torch.empty_like(x)
    h = int(torch.cuda.current_stream().cuda_stream)
    xp, yp = x.data_ptr(), y.data_ptr()
    variants = {"separate_heuristic": offt.MANY_SEPARATE_HEURISTIC,
                "levels_heuristic": offt.MANY_LEVELS,
                "levels_graph_heuristic": offt.MANY_LEVELS_GRAPH,
                "levels_grouped_graph_heuristic": offt.MANY_LEVELS_GROUPED_GRAPH}
    ms = {}
    for name, mode in variants.items():
        for _ in range(warmup):
            plan.exec_ptr(xp, yp, offt.FORWARD, mode, h)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            plan.exec_ptr(xp, yp, offt.FORWARD, mode, h)
        e1.record()
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1) / steps
    flop = sum(5.0 * a * b * c * math.log2(a * b * c) for a, b, c in dims if a * b * c > 1)
    nbytes = sum(6.0 * a * b * c * 8 for a, b, c in dims)
    out = {
        "workload": f"{count} complex64 grids, axes uniform over the 2/3/5-smooth lengths 2..160",
        "elements": int(sum(a * b * c for a, b, c in dims)),
        "executor": plan.describe().splitlines()[0],
        "ms": {k: round(v, 4) for k, v in ms.items()},
        "gflops": {k: round(flop / (v * 1e6), 1) for k, v in ms.items()},
        "eff_gbs": {k: round(nbytes / (v * 1e6), 1) for k, v in ms.items()},
        "speedup_levels_graph_vs_separate": round(ms["separate_heuristic"] / ms["levels_graph_heuristic"], 3),
    }
    if check:
        import oracle
        plan.exec_ptr(xp, yp, offt.FORWARD, offt.MANY_LEVELS_GRAPH, h)
        torch.cuda.synchronize()
        worst = 0.0
        for g, yg in enumerate(plan.unpack(y)):
            ref = oracle.fft3(grids[g].cpu().numpy().astype(np.complex128))
            e = oracle.rel_l2(yg.cpu().numpy(), ref)
            worst = max(worst, e / oracle.tolerance(grids[g].numel(), True))
        out["check_worst_error_over_tolerance_all_grids"] = worst
    plan.close()
    return out


def time_dist(n: int, dtype, steps: int, warmup: int, check: bool, nprocs=(2, 4, 8)):
    """The paper's distributed flow over Np virtual processes on this GPU
    (per-process line transforms, abc -> cab and cab -> cba transposes with
    pack, communicate, unpack; output in cba order): time of one forward
    transform with each communication method, the method the plan-time
    auto-tuning picks, and the elements each transpose moves between
    processes.  Block methods use groups of Np/2 processes."""
    import numpy as np
    import torch

    import paper_1501_07350_amd as offt
    import synth

    shape = (n, n, n)
    x = synth.complex_grid(shape, dtype, device="cuda")
    y = torch.empty(shape[::-1], dtype=dtype, device="cuda")
    h = int(torch.cuda.current_stream().cuda_stream)
    N = x.numel()
    out = {"workload": f"{n}x{n}x{n} {'complex128' if dtype == torch.complex128 else 'complex64'}, forward, "
                       f"output in cba order", "nprocs": {}}
    for np_ in nprocs:
        plan = offt.DistPlan(shape, np_, dtype=dtype, method="auto", block_size=max(1, np_ // 2), reps=3)
        ms = {}
        for m in offt.COMM_METHODS:
            def run():
                plan.exec_ptr(offt.FORWARD, x.data_ptr(), y.data_ptr(), h, method=m)

            for _ in range(warmup):
                run()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(steps):
                run()
            e1.record()
            torch.cuda.synchronize()
            ms[m] = round(e0.elapsed_time(e1) / steps, 4)
        moved = [int(sum(c for p, row in enumerate(plan.counts(st)) for q, c in enumerate(row) if p != q))
                 for st in (0, 1)]
        rec = {"decomposition": plan.describe().split(",")[1].strip(), "ms": ms,
               "auto_choice": plan.method, "auto_tuning_ms": {k: round(v, 4) for k, v in plan.method_times().items()},
               "elements_moved": {"abc->cab": moved[0], "cab->cba": moved[1]},
               "gflops_best": round(5.0 * N * math.log2(N) / (min(ms.values()) * 1e6), 1)}
        if check:
            import oracle
            plan.forward(x, out=y)
            torch.cuda.synchronize()
            xh = x.cpu().numpy().astype(np.complex128)
            yh = y.cpu().numpy()
            got, ref = [], []
            for ka, kb in ((0, 0), (3, 5), (n - 1, 7)):
                got.append(yh[:, kb, ka].astype(np.complex128))
                ref.append(oracle.dft3_line(xh, ka, kb))
            rec["check_rel_l2_sampled_lines"] = oracle.rel_l2(np.concatenate(got), np.concatenate(ref))
        out["nprocs"][str(np_)] = rec
        print(f"dist Np={np_}: {rec}", file=sys.stderr, flush=True)
        plan.close()
    del x, y
    torch.cuda.empty_cache()
    return out


def time_small(steps: int, warmup: int, check: bool, n: int = 32):
    """One n^3 complex128 grid, forward then inverse with 1/N,
    latency per round trip with the pass kernels launched directly and
    replayed from a HIP graph (use_graph)."""
    import numpy as np
    import torch

    import paper_1501_07350_amd as offt
    import synth

    shape = (n, n, n)
    x = synth.complex_grid(shape, torch.complex128, device="cuda")
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    h = int(torch.cuda.current_stream().cuda_stream)
    res = {"workload": f"{n}x{n}x{n} complex128, forward then inverse with 1/N", "us_per_round_trip": {}}
    for name, use_graph in (("direct", False), ("graph", True)):
        plan = offt.Plan(shape, dtype=torch.complex128, normalize_inverse=True, use_graph=use_graph)
        for _ in range(warmup):
            plan.exec_ptr(offt.FORWARD, x.data_ptr(), y.data_ptr(), h)
            plan.exec_ptr(offt.BACKWARD, y.data_ptr(), z.data_ptr(), h)
        reps = max(steps, 100)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            plan.exec_ptr(offt.FORWARD, x.data_ptr(), y.data_ptr(), h)
            plan.exec_ptr(offt.BACKWARD, y.data_ptr(), z.data_ptr(), h)
        e1.record()
        torch.cuda.synchronize()
        res["us_per_round_trip"][name] = round(1e3 * e0.elapsed_time(e1) / reps, 2)
        res["plan"] = plan.describe()
        plan.close()
    if check:
        import oracle
        xh = x.cpu().numpy()
        res["rel_l2_forward_vs_per_axis_dft"] = oracle.rel_l2(y.cpu().numpy(), oracle.dft3_axes(xh))
        res["rel_l2_round_trip"] = oracle.rel_l2(z.cpu().numpy(), xh)
        res["tolerance"] = oracle.tolerance(x.numel(), False)
    return res


def roofline(res, tag):
    """The dominant kernel: the slowest pass that runs as one launch over the
    whole grid (the passes of a slab schedule run as one launch per slab)."""
    groups = res["groups"]
    j = max((j for j in range(len(groups)) if len(groups[j]) == 1), key=lambda j: res["pass_ms"][j])
    i = groups[j][0]
    dur_ms = res["pass_ms"][j]
    achieved = res["pass_bytes"] / (dur_ms * 1e6)
    key = pass_keys(res["plan"])[i]
    copy_gbs = res["pass_bytes"] / (res["copy_ms"][i] * 1e6)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": load_traffic(tag, key), "kernel_pass": i,
            "kernel": key, "kernel_ms": round(dur_ms, 4), "algorithmic_bytes_per_launch": res["pass_bytes"],
            "copy_ceiling_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}


def copy_ceilings(res):
    """Per pass (per group of a slab schedule): the copy of the pass's own
    access pattern over the whole grid (GB/s of the algorithmic bytes) and
    the pass's rate as a fraction of it."""
    out = []
    for g, pm in zip(res["groups"], res["pass_ms"]):
        cm = sum(res["copy_ms"][i] for i in g)
        nbytes = res["pass_bytes"] * len(g)
        out.append({"pass": group_key(res["plan"], g), "copy_ms": round(cm, 4),
                    "copy_gbs": round(nbytes / (cm * 1e6), 1), "pass_gbs": round(nbytes / (pm * 1e6), 1),
                    "frac_of_copy": round(cm / pm, 4)})
    return out


def cpu_baseline(n: int):
    import numpy as np
    import torch

    import oracle
    import synth

    x = synth.complex_grid((n, n, n), torch.complex128).numpy()
    cores = oracle.max_threads()
    # repeat whole transforms until about 10 s of CPU work (at most 16)
    times = []
    while sum(times) < 10.0 and len(times) < 16:
        t0 = time.perf_counter()
        y = oracle.fft3(x)
        times.append(time.perf_counter() - t0)
        del y
    dt = sum(times) / len(times)
    N = x.size
    del x
    return {"value": round(5.0 * N * math.log2(N) / (dt * 1e9), 3), "unit": "GFLOP/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{len(times)} forward {n}^3 complex128 transforms of the same synthetic grid (the "
                      f"whole workload per execution), recursive radix-2/3/5 FFT along c, b, a in "
                      f"binary64, mean {dt:.2f} s each"}


def other_workloads_report(steps: int, warmup: int):
    """Every workload of the measurement plan besides the 512^3 headline:
    the 32^3 complex128 round trip, 256^3 complex128 (forward error vs the
    full oracle and round-trip error), 1024^3 complex64, and the CPU oracle
    timed on this host (O1 brute force, O2 per-axis DFT, O3 recursive FFT;
    all cores and one thread)."""
    import numpy as np
    import torch

    import oracle
    import paper_1501_07350_amd as offt
    import synth

    cpu = "unknown"
    try:
        cpu = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    rep = {"cpu_model": cpu, "cores": oracle.max_threads()}
    rep["round_trip_32cubed_c128"] = time_small(steps, warmup, True)

    def round_trip(n, dtype, check_full):
        shape = (n, n, n)
        x = synth.complex_grid(shape, dtype, device="cuda")
        plan = offt.Plan(shape, dtype=dtype, normalize_inverse=True, tune="exhaustive")
        y = plan.forward(x)
        z = plan.backward(y)
        torch.cuda.synchronize()
        d = {"plan": plan.describe(),
             "rel_l2_round_trip": float(((z - x).abs().double().pow(2).sum() / x.abs().double().pow(2).sum()).sqrt()),
             "tolerance": oracle.tolerance(x.numel(), dtype == torch.complex64)}
        if check_full:
            d["rel_l2_forward_vs_O3"] = oracle.rel_l2(y.cpu().numpy(), oracle.fft3(x.cpu().numpy()))
        plan.close()
        del x, y, z
        torch.cuda.empty_cache()
        return d

    r2 = time_transform(256, torch.complex128, steps, warmup, False, "exhaustive")
    rep["grid_256cubed_c128"] = {"workload": "256x256x256 complex128", "ms": round(r2["ms"], 4),
                      "gflops": round(r2["gflops"], 1), "eff_gbs": round(r2["eff_gbs"], 1),
                      "pass_ms": [round(v, 4) for v in r2["pass_ms"]], **round_trip(256, torch.complex128, True)}
    r3 = time_transform(1024, torch.complex64, steps, warmup, True, "exhaustive")
    rep["grid_1024cubed_c64"] = {"workload": "1024x1024x1024 complex64", "ms": round(r3["ms"], 4),
                           "gflops": round(r3["gflops"], 1), "eff_gbs": round(r3["eff_gbs"], 1),
                           "frac_of_peak_effective": round(r3["eff_gbs"] / PEAK_HBM_GBS, 4),
                           "pass_ms": [round(v, 4) for v in r3["pass_ms"]], "plan": r3["plan"],
                           "rel_l2_sampled_lines_vs_definition": r3["check_rel_l2_sampled_lines"],
                           **{k: v for k, v in round_trip(1024, torch.complex64, False).items() if k != "plan"}}

    def cpu_time(fn, n, threads, reps):
        x = synth.complex_grid((n, n, n), torch.complex128).numpy()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn(x, nthreads=threads)
            ts.append(time.perf_counter() - t0)
        N = x.size
        dt = sum(ts) / len(ts)
        return {"seconds": round(dt, 4), "gflops": round(5.0 * N * math.log2(N) / (dt * 1e9), 3),
                "threads": threads or oracle.max_threads(), "runs": reps}

    table = {}
    for name, fn, n, threads, reps in (("O1_brute_32", oracle.dft3_brute, 32, 0, 1),
                                       ("O2_axes_32", oracle.dft3_axes, 32, 0, 3),
                                       ("O2_axes_256", oracle.dft3_axes, 256, 0, 1),
                                       ("O3_fft_32", oracle.fft3, 32, 0, 10),
                                       ("O3_fft_256", oracle.fft3, 256, 0, 3),
                                       ("O3_fft_512", oracle.fft3, 512, 0, 3),
                                       ("O2_axes_32_1thread", oracle.dft3_axes, 32, 1, 3),
                                       ("O3_fft_32_1thread", oracle.fft3, 32, 1, 10),
                                       ("O3_fft_256_1thread", oracle.fft3, 256, 1, 1)):
        table[name] = cpu_time(fn, n, threads, reps)
        print(f"cpu {name}: {table[name]}", file=sys.stderr, flush=True)
    rep["cpu_oracle"] = table
    return rep


# ---------------------------------------------------------------- profiling ----
# rocprofv3 runs of this script (their commands head each summary under profiles/) are reduced to
# short text summaries and to profiles/pmc_traffic.json with the modes below.

CALIB_BYTES = 1 << 31   # bytes read (and written) by one calibration copy


def calibrate_copy(reps: int = 3):
    """Plain device-to-device copies of a known size (torch's copy kernel):
    HBM counters of a kernel that moves exactly CALIB_BYTES in and out."""
    import torch

    a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _find(d, suffix):
    for root, _, files in os.walk(d):
        for fn in files:
            if fn.endswith(suffix):
                return os.path.join(root, fn)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def _profiled_runs(log: str, n: int):
    """The transforms a profiled bench.py run timed, in launch order, from the
    JSON line it printed: [(tag, dtype label, plan)].  The run must use forced
    (or heuristic) plans so that no tuning dispatches sit among them."""
    line = [l for l in open(log) if l.startswith("{")][-1]
    d = json.loads(line)
    runs = [(f"{n}_f64", "complex128", d["plan"]), (f"{n}_f32", "complex64", d["f32"]["plan"])]
    h = d.get("heuristic_plan", {})
    if h.get("f64", {}).get("plan"):
        runs += [(f"{n}_f64", "complex128", h["f64"]["plan"]), (f"{n}_f32", "complex64", h["f32"]["plan"])]
    return runs


def _pass_dispatches(names, runs, steps, warmup, planes):
    """Split the fft_pass_kernel dispatches (in dispatch order) into
    runs x steps x passes (a pass of a slab schedule has one dispatch per
    slab); yields (run index, pass index, step, position)."""
    k = 0
    for r, (_, _, plan) in enumerate(runs):
        seq = pass_launches(plan, planes)
        for st in range(steps + warmup):
            for i in seq:
                yield r, i, st, k
                k += 1
    if k != len(names):
        raise RuntimeError(f"expected {k} pass dispatches, the trace holds {len(names)}")


def _per_step(items):
    """{(run, pass): {step: summed value}} -> {(run, pass): mean over steps}
    (a pass of a slab schedule sums its slabs' dispatches)."""
    return {key: sum(v.values()) / len(v) for key, v in items.items()}


def summarize_stats(d: str, log: str, command: str, n: int, steps: int, warmup: int) -> str:
    rows = _read_csv(_find(d, "kernel_stats.csv"))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}",
             f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total%':>7}  kernel"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"{int(r['Calls']):>6} {float(r['AverageNs'])/1e3:>10.2f} {float(r['MinNs'])/1e3:>10.2f} "
                     f"{float(r['MaxNs'])/1e3:>10.2f} {float(r['Percentage']):>7.2f}  {r['Name'][:150]}")
    runs = _profiled_runs(log, n)
    trace = _read_csv(_find(d, "kernel_trace.csv"))
    trace.sort(key=lambda r: int(r["Dispatch_Id"]))
    disp = [r for r in trace if "fft_pass_kernel" in r["Kernel_Name"]]
    dur, kname = {}, {}
    for r, i, st, k in _pass_dispatches(disp, runs, steps, warmup, n):
        if st >= warmup:
            x = disp[k]
            kname[(r, i)] = x["Kernel_Name"]
            steps_d = dur.setdefault((r, i), {})
            steps_d[st] = steps_d.get(st, 0.0) + (int(x["End_Timestamp"]) - int(x["Start_Timestamp"])) / 1e3
    dur = _per_step(dur)
    # the copy of each pass's accesses (offt_copy_pass), run after each
    # transform: per run, per pass, warmup + steps dispatches
    copies = [r for r in trace if "copy_pattern_kernel" in r["Kernel_Name"]]
    cdur = {}
    k = 0
    for r, (_, _, plan) in enumerate(runs):
        for i in range(len(pass_keys(plan))):
            for st in range(warmup + steps):
                if k < len(copies) and st >= warmup:
                    x = copies[k]
                    cdur.setdefault((r, i), []).append((int(x["End_Timestamp"]) - int(x["Start_Timestamp"])) / 1e3)
                k += 1
    if k != len(copies):
        raise RuntimeError(f"expected {k} copy dispatches, the trace holds {len(copies)}")
    es = {"complex128": 16, "complex64": 8}
    lines.append("")
    lines.append("# per-pass mean duration over the timed steps (from the dispatch trace; a pass of a slab")
    lines.append("# schedule summed over its slabs' dispatches), and the copy kernel of the same pass over the")
    lines.append("# whole grid (its tiles, threads, tile order and access mode, no arithmetic)")
    for r, (tag, label, plan) in enumerate(runs):
        lines.append(f"{n}^3 {label}, plan {plan}")
        nbytes = 2 * n ** 3 * es[label]
        for i in range(len(pass_keys(plan))):
            key = pass_label(plan, i)
            pm, name = dur[(r, i)], kname[(r, i)]
            cm = sum(cdur[(r, i)]) / len(cdur[(r, i)])
            lines.append(f"  pass {i} {key:<18} mean {pm:9.2f} us ({nbytes / (pm * 1e3):7.1f} GB/s), copy {cm:9.2f} us "
                         f"({nbytes / (cm * 1e3):7.1f} GB/s), of copy {cm / pm:6.3f}  {name[:100]}")
    return "\n".join(lines) + "\n"


def summarize_kernels(d: str, command: str, title: str, top: int = 20) -> str:
    """The kernel-statistics table of one rocprofv3 --stats run (the largest
    total time first)."""
    rows = _read_csv(_find(d, "kernel_stats.csv"))
    lines = [f"# rocprofv3 kernel statistics: {title}", f"# command: {command}",
             f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total%':>7}  kernel"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        lines.append(f"{int(r['Calls']):>6} {float(r['AverageNs'])/1e3:>10.2f} {float(r['MinNs'])/1e3:>10.2f} "
                     f"{float(r['MaxNs'])/1e3:>10.2f} {float(r['Percentage']):>7.2f}  {r['Name'][:150]}")
    return "\n".join(lines) + "\n"


def summarize_batch(d: str, command: str, steps: int, warmup: int) -> str:
    """Kernel-trace figures of the uneven-batch executors from one
    `--batch-only` run: per executor form, dispatches and mean duration; per
    execution, the summed kernel time, and for the forms replayed from a
    graph (the last `steps` executions) the span from the first kernel's
    start to the last one's end."""
    trace = _read_csv(_find(d, "kernel_trace.csv"))
    trace.sort(key=lambda r: int(r["Dispatch_Id"]))
    runs = steps + warmup

    def rows_of(key):
        return [r for r in trace if key in r["Kernel_Name"]]

    def dur(r):
        return (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3

    lines = ["# rocprofv3 kernel trace of the uneven-batch executors (64 complex64 grids, one forward each)",
             f"# command: {command}",
             f"# {steps} timed + {warmup} warm-up executions per form, in the order the bench runs them: the",
             "# persistent kernel (tuned, tuned in a graph, heuristic in a graph), the level kernels (direct, in a",
             "# graph, grouped in a graph), the level-synchronous kernel (direct, in a graph); the every-length",
             "# executor's level kernels run the second batch (64 grids, axes over every 2/3/5-smooth length",
             "# 2..160, heuristic plans: direct, in a graph, grouped in a graph)",
             f"{'form':<46} {'dispatches':>10} {'mean_us':>9} {'per_exec':>8} {'busy_us_per_exec':>17}"]

    def report(label, rows, execs, graph):
        if not rows:
            lines.append(f"{label:<46} {'none traced':>10}")
            return
        durs = [dur(r) for r in rows]
        per = len(rows) / execs
        lines.append(f"{label:<46} {len(rows):>10} {sum(durs) / len(rows):>9.2f} {per:>8.2f} "
                     f"{sum(durs) / execs:>17.2f}")
        if graph and per == int(per):
            k = int(per)
            tail = rows[len(rows) - steps * k:]
            spans = []
            for e in range(steps):
                grp = tail[e * k:(e + 1) * k]
                spans.append((max(int(r["End_Timestamp"]) for r in grp)
                              - min(int(r["Start_Timestamp"]) for r in grp)) / 1e3)
            busy = sum(dur(r) for r in tail) / steps
            lines.append(f"  graph replays: {k} kernels per execution, span first start to last end "
                         f"{sum(spans) / len(spans):.2f} us (min {min(spans):.2f}), summed kernel time {busy:.2f} us")

    report("persistent work-queue kernel", rows_of("many_kernel_batch_"), 3 * runs, False)
    for label, key in (("", "many_level_kernel_batch_"), ("every-length executor, ", "many_level_kernel_all_")):
        rows = rows_of(key)
        # direct and graph forms: 3 level kernels per execution; the grouped
        # graph: 3 per group, the rest
        n3 = 3 * runs
        report(f"{label}level kernels, direct", rows[:n3], runs, False)
        report(f"{label}level kernels, graph", rows[n3:2 * n3], runs, True)
        report(f"{label}level kernels, grouped graph", rows[2 * n3:], runs, True)
    report("level-synchronous persistent kernel", rows_of("many_sync_kernel_batch_"), 2 * runs, False)
    return "\n".join(lines) + "\n"


def summarize_reversed(d: str, log: str, command: str, n: int, steps: int, warmup: int) -> str:
    """Per-pass durations of the reversed (cba) output order from one
    rocprofv3 --kernel-trace run of `--reversed-only` (plans from the plan
    cache): for complex128 then complex64, the natural plan forward and
    backward, then the reversed plan forward and backward, `warmup + steps`
    transforms each, one dispatch per axis in the pass order.  The
    transposing pass is marked (T)."""
    res = None
    for line in open(log):
        if line.startswith("{"):
            res = json.loads(line)["reversed_output"]
    if res is None:
        raise RuntimeError(f"no result line in {log}")
    trace = _read_csv(_find(d, "kernel_trace.csv"))
    trace.sort(key=lambda r: int(r["Dispatch_Id"]))
    disp = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace
            if "fft_pass_kernel" in r["Kernel_Name"] or "fft_tpass_kernel" in r["Kernel_Name"]]
    lines = ["# rocprofv3 kernel trace of the reversed (cba) output order beside the natural one: mean duration",
             "# per pass dispatch over the timed transforms; GB/s = algorithmic 2*N*s bytes per pass / duration",
             f"# command: {command}"]
    N = n ** 3
    k = 0
    for dt in ("f64", "f32"):
        s_b = 16 if dt == "f64" else 8
        for name in ("natural", "reversed"):
            halves = res[dt][name]["plan"].split("|")
            for direction, half in (("fwd", halves[0]), ("bwd", halves[-1])):
                fields = dict(f.split("=", 1) for f in half.split(";"))
                ev = res[dt][name][f"{direction}_ms"]
                lines.append(f"{n}^3 {dt} {name} {direction} plan {half}: {ev * 1e3:.1f} us per transform (HIP events)")
                # a natural plan with a block schedule launches its later
                # passes once per block: per pass and transform, summed
                keys = pass_keys(half)
                per = [[0.0] * steps for _ in keys]
                for st in range(warmup + steps):
                    for i in pass_launches(half, n):
                        if k >= len(disp):
                            raise RuntimeError(f"the trace holds {len(disp)} pass dispatches, fewer than expected")
                        if st >= warmup:
                            per[i][st - warmup] += disp[k]
                        k += 1
                total = 0.0
                for i, key in enumerate(keys):
                    m = sum(per[i]) / len(per[i])
                    total += m
                    ax = key.split("=", 1)[0]
                    tag = " (T)" if fields.get("rev") == ax else ""
                    lines.append(f"  pass {i} {pass_label(half, i) + tag:<22} {m:9.2f} us  "
                                 f"{2.0 * N * s_b / (m * 1e3):7.1f} GB/s")
                lines.append(f"  summed pass time {total:.1f} us")
    if k != len(disp):
        raise RuntimeError(f"expected {k} pass dispatches, the trace holds {len(disp)}")
    return "\n".join(lines) + "\n"


def summarize_nd(d: str, log: str, command: str, steps: int, warmup: int) -> str:
    """Per-pass durations of the 4- and 5-axis transforms from one rocprofv3
    --kernel-trace run of `--nd-only` (plans from the plan cache, so every
    pass dispatch belongs to a timed or warm-up transform): for each grid,
    the tuned plan and then the heuristic plan, `warmup + steps` transforms
    of one dispatch per axis in the plan's pass order."""
    res = None
    for line in open(log):
        if line.startswith("{"):
            res = json.loads(line)["nd"]
    if res is None:
        raise RuntimeError(f"no result line in {log}")
    trace = _read_csv(_find(d, "kernel_trace.csv"))
    trace.sort(key=lambda r: int(r["Dispatch_Id"]))
    disp = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace
            if "fft_pass_kernel" in r["Kernel_Name"]]
    lines = ["# rocprofv3 kernel trace of the 4- and 5-axis transforms: mean duration per pass over the timed",
             "# transforms (a pass of a slab schedule summed over its slabs' dispatches); GB/s = algorithmic",
             "# 2*N*s bytes per pass / duration",
             f"# command: {command}"]
    k = 0
    for r in res:
        N = math.prod(r["shape"])
        s = 16 if r["dtype"] == "f64" else 8
        for name in ("tuned", "heuristic"):
            plan = r[name]["plan"]
            lines.append(f"{'x'.join(map(str, r['shape']))} {r['dtype']} {name} plan {plan}: "
                         f"{r[name]['ms'] * 1e3:.1f} us per transform (HIP events)")
            # a slab schedule launches its later passes once per slab: per pass
            # and transform, the slabs' dispatches are summed
            npass = len(pass_keys(plan))
            per = [[0.0] * steps for _ in range(npass)]
            seq = pass_launches(plan, r["shape"][0])
            for st in range(warmup + steps):
                for i in seq:
                    if k >= len(disp):
                        raise RuntimeError(f"the trace holds {len(disp)} pass dispatches, fewer than expected")
                    if st >= warmup:
                        per[i][st - warmup] += disp[k]
                    k += 1
            total = 0.0
            for i in range(npass):
                m = sum(per[i]) / len(per[i])
                total += m
                label = pass_label(plan, i)
                lines.append(f"  pass {i} {label:<16} {m:9.2f} us  {2.0 * N * s / (m * 1e3):7.1f} GB/s")
            lines.append(f"  summed pass time {total:.1f} us")
    if k != len(disp):
        raise RuntimeError(f"expected {k} pass dispatches, the trace holds {len(disp)}")
    return "\n".join(lines) + "\n"


def _pmc_per_dispatch(d: str, counter: str):
    """[(kernel_name, value_KiB)] in dispatch order for one counter."""
    rows = _read_csv(_find(d, "counter_collection.csv"))
    per = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        did = int(r["Dispatch_Id"])
        name, val = r["Kernel_Name"], float(r["Counter_Value"])
        prev = per.get(did)
        per[did] = (name, val + (prev[1] if prev else 0.0))
    return [per[k] for k in sorted(per)]


SQ_COUNTERS = ["SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
               "SQ_LDS_BANK_CONFLICT", "SQ_WAVES", "SQ_WAVE_CYCLES", "GRBM_GUI_ACTIVE"]
CU_NUM = 256
MAX_WAVES_PER_CU = 32
XCD_NUM = 8   # GRBM_GUI_ACTIVE arrives summed over the XCDs; rocprofv3's expressions take its max


def summarize_sq(d: str, log: str, command: str, n: int, steps: int, warmup: int) -> str:
    """Per-pass VALU / LDS figures from one rocprofv3 --pmc run of the SQ and
    GRBM counters above (with --kernel-trace for the durations), averaged
    over the timed steps.  Busy and conflict percentages use rocprofv3's own
    derived-metric expressions for this device (VALUBusy, LDSBankConflict,
    OccupancyPercent), with the LDS analogue of VALUBusy."""
    runs = _profiled_runs(log, n)
    vals = {c: _pmc_per_dispatch(d, c) for c in SQ_COUNTERS}
    names = [nm for nm, _ in vals["SQ_WAVES"]]
    idx = [i for i, nm in enumerate(names) if "fft_pass_kernel" in nm]
    trace = _read_csv(_find(d, "kernel_trace.csv"))
    trace.sort(key=lambda r: int(r["Dispatch_Id"]))
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace
            if "fft_pass_kernel" in r["Kernel_Name"]]
    if len(durs) != len(idx):
        raise RuntimeError(f"{len(idx)} counter dispatches but {len(durs)} traced pass dispatches")
    acc = {}
    for r, i, st, k in _pass_dispatches(idx, runs, steps, warmup, n):
        if st < warmup:
            continue
        a = acc.setdefault((r, i), {c: 0.0 for c in SQ_COUNTERS + ["us"]})
        for c in SQ_COUNTERS:
            a[c] += vals[c][idx[k]][1]
        a["us"] += durs[k]
        a.setdefault("steps", set()).add(st)
    lines = ["# rocprofv3 SQ / GRBM counters per axis pass (per pass and step, averaged over the timed steps;",
             "# a pass of a slab schedule summed over its slabs' dispatches)",
             f"# command: {command}",
             "# valu% = 100*SQ_ACTIVE_INST_VALU/CU_NUM/GRBM_GUI_ACTIVE (rocprofv3 VALUBusy); lds% the same with",
             "# SQ_ACTIVE_INST_LDS; conflict% = 100*SQ_LDS_BANK_CONFLICT/GRBM_GUI_ACTIVE/CU_NUM (LDSBankConflict);",
             "# occ% = 400*SQ_WAVE_CYCLES/GRBM_GUI_ACTIVE/CU_NUM/32 (OccupancyPercent); per-element counts are",
             "# wave instructions x 64 lanes / grid points; GRBM_GUI_ACTIVE (summed over the 8 XCDs in the CSV)",
             "# is divided by 8 for the max the expressions take; clock = that / dispatch duration",
             f"{'grid':<12} {'pass':<18} {'us':>8} {'GHz':>5} {'valu%':>6} {'lds%':>6} {'confl%':>7} {'occ%':>6} "
             f"{'valu/pt':>8} {'lds/pt':>7} {'vmem/pt':>8} {'waves':>8}"]
    for r, (tag, label, plan) in enumerate(runs):
        N = n ** 3
        for i in range(len(pass_keys(plan))):
            key = pass_label(plan, i)
            a = acc[(r, i)]
            m = {c: a[c] / len(a["steps"]) for c in SQ_COUNTERS + ["us"]}
            g = m["GRBM_GUI_ACTIVE"] / XCD_NUM
            lines.append(
                f"{n}^3 c{label[7:]:<5} {key:<18} {m['us']:8.1f} {g / m['us'] / 1e3:5.2f} "
                f"{100 * m['SQ_ACTIVE_INST_VALU'] / CU_NUM / g:6.1f} {100 * m['SQ_ACTIVE_INST_LDS'] / CU_NUM / g:6.1f} "
                f"{100 * m['SQ_LDS_BANK_CONFLICT'] / CU_NUM / g:7.2f} "
                f"{400 * m['SQ_WAVE_CYCLES'] / g / CU_NUM / MAX_WAVES_PER_CU:6.1f} "
                f"{m['SQ_INSTS_VALU'] * 64 / N:8.1f} {m['SQ_INSTS_LDS'] * 64 / N:7.2f} "
                f"{m['SQ_INSTS_VMEM'] * 64 / N:8.2f} {m['SQ_WAVES']:8.0f}")
    return "\n".join(lines) + "\n"


def summarize_pmc(fetch_dir: str, write_dir: str, log: str, n: int, steps: int, warmup: int, command: str):
    """Per-pass HBM bytes of the transforms, scaled by the copy calibration:
    factor = CALIB_BYTES / (counter bytes of one calibration copy).  Passes are
    keyed by "axis=spec" of their plan, per precision."""
    runs = _profiled_runs(log, n)
    out = {"kernel_hash": kernel_source_hash(), "command": command, "workloads": {}}
    # passes measured in earlier sessions on the same kernel sources stay in the
    # table (the tuner's choice among near-equal kernels varies by session)
    try:
        with open(TRAFFIC_FILE) as f:
            old = json.load(f)
        if old.get("kernel_hash") == out["kernel_hash"]:
            out["workloads"] = old.get("workloads", {})
            out["command"] = command + "; merged with the earlier sessions' passes on the same kernel sources"
    except (OSError, ValueError):
        pass
    text = [f"# HBM traffic per pass from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (a pass of a slab schedule",
            "# summed over its slabs' dispatches)",
            f"# command: {command}"]
    acc = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        disp = _pmc_per_dispatch(d, counter)
        passes = [x for x in disp if "fft_pass_kernel" in x[0]]
        copies = [x for x in disp if "copyBuffer" in x[0]]
        calib_kib = copies[-1][1]
        factor = CALIB_BYTES / (calib_kib * 1024.0)
        text.append(f"{counter}: calibration copy of {CALIB_BYTES} B in and out counted {calib_kib:.0f} KiB "
                    f"-> factor {factor:.4f}")
        vals = {}
        for r, i, st, k in _pass_dispatches(passes, runs, steps, warmup, n):
            if st >= warmup:
                per = vals.setdefault((r, i), {})
                per[st] = per.get(st, 0.0) + passes[k][1]
        for (r, i), kib in sorted(_per_step(vals).items()):
            tag, label, plan = runs[r]
            key = pass_label(plan, i)
            acc.setdefault((tag, key), {})[counter] = kib * 1024.0 * factor
            text.append(f"{tag} {key:<18} {counter}: {kib:.0f} KiB/pass -> {kib*1024*factor/1e9:.4f} GB scaled")
    for (tag, key), c in sorted(acc.items()):
        s = 16 if tag.endswith("f64") else 8
        alg = 2 * n ** 3 * s
        w = out["workloads"].setdefault(tag, {"algorithmic_bytes": alg, "pass_bytes": {}, "raw_bytes": {}})
        w["pass_bytes"][key] = round(c["FETCH_SIZE"] + c["WRITE_SIZE"])
        w["raw_bytes"][key] = {k: round(v) for k, v in c.items()}
    text.append("# every pass of the table (this session's and, on the same kernel sources, earlier ones)")
    for tag, w in sorted(out["workloads"].items()):
        alg = w["algorithmic_bytes"]
        for key, b in sorted(w["pass_bytes"].items()):
            text.append(f"{tag} {key:<18} measured {b/1e9:.4f} GB, algorithmic {alg/1e9:.4f} GB, "
                        f"amplification {b/alg:.3f}")
    return out, "\n".join(text) + "\n"


def main():
    global PLAN_CACHE
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled-line parity check")
    ap.add_argument("--calibrate", action="store_true", help="also run the copy-kernel calibration")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch (64 grids) timing")
    ap.add_argument("--tune", default="exhaustive", choices=["exhaustive", "none", "learned", "forced"],
                    help="plan selection of the timed transforms")
    ap.add_argument("--plan64", help="plan string for --tune forced (complex128)")
    ap.add_argument("--plan32", help="plan string for --tune forced (complex64)")
    ap.add_argument("--no-heuristic", action="store_true", help="skip the heuristic-plan comparison runs")
    ap.add_argument("--summarize-stats", nargs=2, metavar=("DIR", "LOG"),
                    help="reduce a rocprofv3 --stats output dir (LOG: the profiled run's stdout)")
    ap.add_argument("--summarize-sq", nargs=2, metavar=("DIR", "LOG"),
                    help="reduce a rocprofv3 --pmc run of the SQ/GRBM counters (VALU, LDS) to a per-pass table")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "LOG"),
                    help="reduce two rocprofv3 --pmc output dirs to profiles/pmc_traffic.json")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the uneven batch of 64 grids (to profile its executors)")
    ap.add_argument("--reversed-only", action="store_true",
                    help="time only the reversed (cba) output order at --n (to profile its passes)")
    ap.add_argument("--summarize-reversed", nargs=2, metavar=("DIR", "LOG"),
                    help="reduce a rocprofv3 --kernel-trace run of --reversed-only")
    ap.add_argument("--dist-only", action="store_true",
                    help="time only the distributed flow over virtual processes at --n")
    ap.add_argument("--nd-only", action="store_true",
                    help="time only the 4- and 5-axis grids (to profile their passes)")
    ap.add_argument("--summarize-nd", nargs=2, metavar=("DIR", "LOG"),
                    help="reduce a rocprofv3 --kernel-trace run of --nd-only")
    ap.add_argument("--summarize-kernels", metavar="DIR",
                    help="reduce a rocprofv3 --stats run to its kernel table (with --title)")
    ap.add_argument("--title", default="", help="title of a --summarize-kernels table")
    ap.add_argument("--summarize-batch", metavar="DIR",
                    help="reduce a rocprofv3 --kernel-trace run of --batch-only")
    ap.add_argument("--other-workloads", action="store_true",
                    help="report the 32^3 round trip, 256^3 complex128, 1024^3 complex64 and the CPU oracle table "
                         "instead")
    ap.add_argument("--plan-cache", default=PLAN_CACHE,
                    help="plan cache of the tuned plans ('none': tune afresh without a cache)")
    ap.add_argument("--command", default="", help="profiling command recorded in the summary")
    ap.add_argument("--out", help="summary text file")
    args = ap.parse_args()
    PLAN_CACHE = None if args.plan_cache == "none" else os.path.abspath(args.plan_cache)
    if args.summarize_stats:
        txt = summarize_stats(args.summarize_stats[0], args.summarize_stats[1], args.command, args.n,
                              args.steps, args.warmup)
        open(args.out, "w").write(txt) if args.out else print(txt)
        return
    if args.summarize_sq:
        txt = summarize_sq(args.summarize_sq[0], args.summarize_sq[1], args.command, args.n, args.steps,
                           args.warmup)
        open(args.out, "w").write(txt) if args.out else print(txt)
        return
    if args.summarize_reversed:
        txt = summarize_reversed(args.summarize_reversed[0], args.summarize_reversed[1], args.command, args.n,
                                 args.steps, args.warmup)
        open(args.out, "w").write(txt) if args.out else print(txt)
        return
    if args.summarize_nd:
        txt = summarize_nd(args.summarize_nd[0], args.summarize_nd[1], args.command, args.steps, args.warmup)
        open(args.out, "w").write(txt) if args.out else print(txt)
        return
    if args.summarize_kernels:
        txt = summarize_kernels(args.summarize_kernels, args.command, args.title)
        open(args.out, "w").write(txt) if args.out else print(txt)
        return
    if args.summarize_batch:
        txt = summarize_batch(args.summarize_batch, args.command, args.steps, args.warmup)
        open(args.out, "w").write(txt) if args.out else print(txt)
        return
    if args.summarize_pmc:
        d, txt = summarize_pmc(*args.summarize_pmc, args.n, args.steps, args.warmup, args.command)
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(d, f, indent=1)
        open(args.out, "w").write(txt) if args.out else print(txt)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the 3-D FFT is measured on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.other_workloads:
        print(json.dumps(other_workloads_report(args.steps, args.warmup)), flush=True)
        return
    if args.reversed_only:
        print(json.dumps({"reversed_output": reversed_runs(args.n, args.steps, args.warmup, not args.no_check)}),
              flush=True)
        return
    if args.dist_only:
        print(json.dumps({"dist": time_dist(args.n, torch.complex128, args.steps, args.warmup, not args.no_check)}),
              flush=True)
        return
    if args.nd_only:
        print(json.dumps({"nd": nd_runs(args.steps, args.warmup, not args.no_check)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch": time_batch(args.steps, args.warmup, not args.no_check),
                          "batch_any_lengths": time_batch_any_lengths(args.steps, args.warmup,
                                                                      not args.no_check)}), flush=True)
        return
    n = args.n
    # plans tuned at init (excluded from the timing, as the paper excludes its
    # initialization phase with auto-tuning); the heuristic plan beside them
    r64 = time_transform(n, torch.complex128, args.steps, args.warmup, not args.no_check, args.tune, args.plan64)
    r32 = time_transform(n, torch.complex64, args.steps, args.warmup, not args.no_check, args.tune, args.plan32)
    if args.no_heuristic:
        h64 = h32 = {"ms": float("nan"), "gflops": float("nan"), "plan": None}
    else:
        h64 = time_transform(n, torch.complex128, args.steps, args.warmup, False, tune="none")
        h32 = time_transform(n, torch.complex64, args.steps, args.warmup, False, tune="none")
    out = {
        "metric": METRIC,
        "value": round(r64["gflops"], 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3-D C2C FFT {n}x{n}x{n} complex128, forward, out of place "
                               f"(complex64 in 'f32')", "n": n, "global_batch": 1, "parallelism": "none"},
        "hbm_gbs_effective": round(r64["eff_gbs"], 1),
        "frac_of_peak_effective": round(r64["eff_gbs"] / PEAK_HBM_GBS, 4),
        "plan": r64["plan"],
        "plan_cache": os.path.relpath(PLAN_CACHE, ROOT) if PLAN_CACHE else None,
        "plan_tuning_seconds": round(r64["plan_seconds"], 3),
        "pass_ms": [round(v, 4) for v in r64["pass_ms"]],
        "copy_ceiling": copy_ceilings(r64),
        "heuristic_plan": {"f64": {"ms_per_step": round(h64["ms"], 4), "gflops": round(h64["gflops"], 1),
                                   "plan": h64["plan"]},
                           "f32": {"ms_per_step": round(h32["ms"], 4), "gflops": round(h32["gflops"], 1),
                                   "plan": h32["plan"]}},
        "f32": {"dtype": "f32", "value": round(r32["gflops"], 1), "unit": "GFLOP/s",
                "ms_per_step": round(r32["ms"], 4), "hbm_gbs_effective": round(r32["eff_gbs"], 1),
                "frac_of_peak_effective": round(r32["eff_gbs"] / PEAK_HBM_GBS, 4), "plan": r32["plan"],
                "plan_tuning_seconds": round(r32["plan_seconds"], 3),
                "pass_ms": [round(v, 4) for v in r32["pass_ms"]],
                "copy_ceiling": copy_ceilings(r32),
                "roofline": roofline(r32, f"{n}_f32")},
        "roofline": roofline(r64, f"{n}_f64"),
    }
    for key, r in (("check", r64), ("check_f32", r32)):
        if "check_rel_l2_sampled_lines" in r:
            out[key] = {"rel_l2_sampled_lines": r["check_rel_l2_sampled_lines"],
                        "tolerance": r["check_tolerance"],
                        "ok": bool(r["check_rel_l2_sampled_lines"] <= r["check_tolerance"])}
    if not args.no_batch:
        out["small"] = time_small(args.steps, args.warmup, not args.no_check)
        out["batch"] = time_batch(args.steps, args.warmup, not args.no_check)
        out["batch_any_lengths"] = time_batch_any_lengths(args.steps, args.warmup, not args.no_check)
        out["reversed_output"] = reversed_runs(n, args.steps, args.warmup, not args.no_check)
        out["nd"] = nd_runs(args.steps, args.warmup, not args.no_check)
        out["dist"] = time_dist(n, torch.complex128, args.steps, args.warmup, not args.no_check)
    if args.calibrate:
        calibrate_copy()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(out), flush=True)
    bad = [k for k in ("check", "check_f32") if k in out and not out[k]["ok"]]
    if bad:
        print(f"bench: the timed transform failed its check against the definition: {bad}", file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
