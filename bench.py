#!/usr/bin/env python
"""Benchmark of the 3-D complex-to-complex FFT on one MI355X.

Workload (default): one forward 3-D transform of a 512x512x512 grid, complex128
(the headline value) and, measured in the same run, complex64; uniform [-1, 1)
synthetic entries from the seeded generator, resident in HBM before timing.

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
KERNEL_SOURCES = ["paper_1501_07350_amd/csrc/fft_device.hpp", "paper_1501_07350_amd/csrc/planner.cpp",
                  "paper_1501_07350_amd/csrc/gen_kernels.py"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(tag: str):
    """Measured HBM bytes per launch of each pass (from rocprofv3 PMC runs),
    only if they were taken on the current kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_source_hash():
        return None
    return d.get("workloads", {}).get(tag)


def time_transform(n: int, dtype, steps: int, warmup: int, check: bool):
    import numpy as np
    import torch

    import paper_1501_07350_amd as offt
    import synth

    shape = (n, n, n)
    x = synth.complex_grid(shape, dtype, device="cuda")
    y = torch.empty_like(x)
    plan = offt.Plan(shape, dtype=dtype)
    npass = plan.npasses()
    stream = torch.cuda.current_stream()
    h = int(stream.cuda_stream)
    xp, yp = x.data_ptr(), y.data_ptr()

    def step():
        for i in range(npass):
            plan.exec_pass(i, offt.FORWARD, xp, yp, h)

    for _ in range(warmup):
        step()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(npass + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        for i in range(npass):
            ev[k][i].record(stream)
            plan.exec_pass(i, offt.FORWARD, xp, yp, h)
        ev[k][npass].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pass_ms = [sum(ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(steps)) / steps for i in range(npass)]
    total_ms = ev[0][0].elapsed_time(ev[steps - 1][npass])
    ms = total_ms / steps
    N = x.numel()
    s = x.element_size()
    res = {
        "ms": ms,
        "gflops": 5.0 * N * math.log2(N) / (ms * 1e6),
        "eff_gbs": 6.0 * N * s / (ms * 1e6),
        "wall_ms_per_step": 1e3 * wall / steps,
        "plan": plan.describe(),
        "pass_ms": pass_ms,
        "pass_bytes": 2 * N * s,
    }
    if check:
        import oracle
        xh = x.cpu().numpy().astype(np.complex128)
        yh = y.cpu().numpy()
        got, ref = [], []
        for ka, kb in ((0, 0), (3, 5), (n - 1, 7)):
            got.append(yh[ka, kb].astype(np.complex128))
            ref.append(oracle.dft3_line(xh, ka, kb))
        res["check_rel_l2_sampled_lines"] = oracle.rel_l2(np.concatenate(got), np.concatenate(ref))
        res["check_tolerance"] = oracle.tolerance(N, dtype == torch.complex64)
    plan.close()
    del x, y
    torch.cuda.empty_cache()
    return res


def roofline(res, tag):
    i = max(range(len(res["pass_ms"])), key=lambda j: res["pass_ms"][j])
    dur_ms = res["pass_ms"][i]
    achieved = res["pass_bytes"] / (dur_ms * 1e6)
    tr = load_traffic(tag)
    traffic = None
    if tr and len(tr.get("pass_bytes", [])) == len(res["pass_ms"]):
        traffic = tr["pass_bytes"][i]
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel_pass": i,
            "kernel_ms": round(dur_ms, 4), "algorithmic_bytes_per_launch": res["pass_bytes"]}


def cpu_baseline(n: int):
    import numpy as np
    import torch

    import oracle
    import synth

    x = synth.complex_grid((n, n, n), torch.complex128).numpy()
    cores = oracle.max_threads()
    t0 = time.perf_counter()
    y = oracle.fft3(x)
    dt = time.perf_counter() - t0
    N = x.size
    del x, y
    return {"value": round(5.0 * N * math.log2(N) / (dt * 1e9), 3), "unit": "GFLOP/s", "cores": cores,
            "kind": "oracle",
            "sample": f"one forward {n}^3 complex128 transform (the whole workload, one execution), "
                      f"recursive radix-2/3/5 FFT along c, b, a in binary64; {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled-line parity check")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the 3-D FFT is measured on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    n = args.n
    r64 = time_transform(n, torch.complex128, args.steps, args.warmup, not args.no_check)
    r32 = time_transform(n, torch.complex64, args.steps, args.warmup, not args.no_check)
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
        "pass_ms": [round(v, 4) for v in r64["pass_ms"]],
        "f32": {"dtype": "f32", "value": round(r32["gflops"], 1), "unit": "GFLOP/s",
                "ms_per_step": round(r32["ms"], 4), "hbm_gbs_effective": round(r32["eff_gbs"], 1),
                "frac_of_peak_effective": round(r32["eff_gbs"] / PEAK_HBM_GBS, 4), "plan": r32["plan"],
                "pass_ms": [round(v, 4) for v in r32["pass_ms"]],
                "roofline": roofline(r32, f"{n}_f32")},
        "roofline": roofline(r64, f"{n}_f64"),
    }
    for key, r in (("check", r64), ("check_f32", r32)):
        if "check_rel_l2_sampled_lines" in r:
            out[key] = {"rel_l2_sampled_lines": r["check_rel_l2_sampled_lines"],
                        "tolerance": r["check_tolerance"]}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
