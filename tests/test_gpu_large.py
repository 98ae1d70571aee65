"""Parity at the full workload sizes, against the full recursive oracle (O3)
element by element: 256^3 and 512^3 complex128, 512^3 and 1024^3 complex64.

Each size runs the heuristic plan and the tuned plan the benchmark times
(the plan-cache entry of that size and precision), in the benchmark's launch
configuration: the passes launched one by one with offt_exec_range (the
passes of a slab schedule as one range), out of place, on torch's current
stream, and compared bit for bit with the whole-transform call.  The error is the
relative L2 norm over the whole grid (tolerance 1e-12 for binary64,
2e-6 * log2(N) for binary32); the worst element error relative to the largest
reference magnitude is printed beside it.  The normalised round trip is
checked as well.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1501_07350_amd as offt
import synth

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PLAN_CACHE = os.path.join(ROOT, "paper_1501_07350_amd", "data", "plan_cache_mi355x.txt")


def cached_plan(n, dtype):
    """Natural-layout plan-cache entry of an n^3 grid, batch 1."""
    code = 0 if dtype == C128 else 1
    key = f"dtype={code} dims={n}x{n}x{n} batch=1 "
    with open(PLAN_CACHE) as f:
        for line in f:
            head, plan, _ = line.rstrip("\n").split("\t")
            if head.startswith(key) and "layout=" not in head:
                return plan
    return None


_REF = {}


def reference(n, dtype):
    """(device input, host input widened to binary64, O3 forward transform)
    of the seeded n^3 grid, computed once per module."""
    k = (n, dtype)
    if k not in _REF:
        _REF.clear()
        x = synth.complex_grid((n, n, n), dtype, device="cuda")
        xh = x.cpu().numpy().astype(np.complex128)
        _REF[k] = (x, xh, oracle.fft3(xh))
    return _REF[k]


def run_passes(plan, direction, x, y):
    """The benchmark's launch configuration, x -> y: each pass on its own,
    the passes of a slab schedule as one range (interleaved slab by slab)."""
    h = int(torch.cuda.current_stream().cuda_stream)
    for g in plan.pass_groups():
        plan.exec_range(g[0], len(g), direction, x.data_ptr(), y.data_ptr(), h)


def max_rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check_full(n, dtype, forced=None):
    x, xh, ref = reference(n, dtype)
    tune = "forced" if forced else "none"
    plan = offt.Plan((n, n, n), dtype=dtype, tune=tune, forced_plan=forced, normalize_inverse=True)
    print(f"case {n}^3 {dtype} plan {plan.describe()}", flush=True)
    y = torch.empty_like(x)
    run_passes(plan, offt.FORWARD, x, y)
    torch.cuda.synchronize()
    # the whole-transform call gives the same bits
    assert torch.equal(plan.forward(x), y)
    torch.cuda.synchronize()
    yh = y.cpu().numpy().astype(np.complex128)
    tol = oracle.tolerance(x.numel(), dtype == C64)
    e_full = oracle.rel_l2(yh, ref)
    e_max = max_rel(yh, ref)
    del yh
    z = torch.empty_like(x)
    run_passes(plan, offt.BACKWARD, y, z)
    torch.cuda.synchronize()
    e_rt = oracle.rel_l2(z.cpu().numpy(), xh)
    print(f"{n}^3 {dtype}: forward rel_l2 {e_full:.3e} (max element {e_max:.2e}), round trip {e_rt:.3e}, "
          f"tol {tol:.1e}", flush=True)
    plan.close()
    del y, z
    torch.cuda.empty_cache()
    assert e_full <= tol and e_rt <= tol


def test_256_complex128_heuristic():
    check_full(256, C128)


def test_256_complex128_tuned_cached_plan():
    plan = cached_plan(256, C128)
    assert plan, "plan cache has no 256^3 complex128 entry"
    check_full(256, C128, plan)


def test_512_complex128_heuristic():
    check_full(512, C128)


def test_512_complex128_tuned_cached_plan():
    plan = cached_plan(512, C128)
    assert plan, "plan cache has no 512^3 complex128 entry"
    check_full(512, C128, plan)


def test_512_complex64_heuristic():
    check_full(512, C64)


def test_512_complex64_tuned_cached_plan():
    plan = cached_plan(512, C64)
    assert plan, "plan cache has no 512^3 complex64 entry"
    check_full(512, C64, plan)


@pytest.mark.timeout(900)
def test_1024_complex64_heuristic():
    check_full(1024, C64)


@pytest.mark.timeout(900)
def test_1024_complex64_tuned_cached_plan():
    plan = cached_plan(1024, C64)
    assert plan, "plan cache has no 1024^3 complex64 entry"
    check_full(1024, C64, plan)
    _REF.clear()
