"""GPU parity of grids with 1, 2, 4 and 5 axes against the D-dimensional
oracle (through the C ABI).

4- and 5-axis plans run one pass per axis on the same kernels as the 3-D
path; 1- and 2-axis shapes are the 3-D plan of the padded shape.  Compared
element by element with oracle.ndim on the same seeded inputs, forward and
backward, in and out of place, every pass order of a 4-axis grid, the tuner's
order search, pass-by-pass launches and graph replay; larger grids against
the full oracle and on sampled points of the definition.  Tolerances as for
3-D grids (relative L2: 1e-12 complex128, 2e-6 log2 N complex64).
"""
import itertools

import numpy as np
import pytest
import torch

import oracle
import paper_1501_07350_amd as offt
import synth
from oracle import ndim

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64


def tol(n, dtype):
    return oracle.tolerance(n, dtype == C64)


def host(x):
    return x.detach().cpu().numpy().astype(np.complex128)


def gen(shape, dtype, key=synth.SEED):
    return synth.complex_grid(shape, dtype, key=key, device="cuda")


SHAPES = [(8, 6, 10, 12), (16, 16, 16, 16), (4, 5, 6, 8, 9), (2, 2, 2, 2, 2), (1, 16, 1, 30), (30, 1, 1, 1, 25),
          (3, 5, 4, 27, 2), (60,), (48, 40), (1, 1, 1, 1)]


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("batch", [1, 2])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_nd_forward_backward_vs_oracle(shape, batch, dtype):
    print(f"case {shape} batch {batch} {dtype}", flush=True)
    full = (batch,) + shape if batch > 1 else shape
    D = len(shape)
    x = gen(full, dtype)
    plan = offt.Plan(shape, dtype=dtype, batch=batch, normalize_inverse=True)
    y = plan.forward(x)
    torch.cuda.synchronize()
    xh = host(x)
    ref = ndim.fftn_batch(xh, D) if batch > 1 else ndim.fftn(xh)
    t = tol(int(np.prod(shape)), dtype)
    assert oracle.rel_l2(host(y), ref) <= t
    w = gen(full, dtype, key=synth.SEED + 9)
    z = plan.backward(w)
    torch.cuda.synchronize()
    wh = host(w)
    refb = (ndim.fftn_batch(wh, D, oracle.BACKWARD) if batch > 1 else ndim.fftn(wh, oracle.BACKWARD)) / np.prod(shape)
    assert oracle.rel_l2(host(z), refb) <= t
    # in place round trip
    buf = x.clone()
    plan.forward(buf, out=buf)
    plan.backward(buf, out=buf)
    torch.cuda.synchronize()
    assert oracle.rel_l2(host(buf), xh) <= t


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_every_pass_order_of_a_4_axis_grid(dtype):
    shape = (12, 10, 8, 18)
    x = gen(shape, dtype)
    ref = ndim.fftn(host(x))
    t = tol(x.numel(), dtype)
    for order in itertools.permutations("abcd"):
        plan = offt.Plan(shape, dtype=dtype, tune="forced", forced_plan="order=" + "".join(order))
        assert plan.describe().startswith("order=" + "".join(order))
        y = plan.forward(x)
        torch.cuda.synchronize()
        assert oracle.rel_l2(host(y), ref) <= t, order


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_sampled_pass_orders_of_a_5_axis_grid(dtype):
    shape = (6, 8, 5, 9, 10)
    x = gen(shape, dtype)
    ref = ndim.fftn(host(x))
    t = tol(x.numel(), dtype)
    perms = list(itertools.permutations("abcde"))
    for order in perms[::11]:
        plan = offt.Plan(shape, dtype=dtype, tune="forced", forced_plan="order=" + "".join(order))
        y = plan.forward(x)
        torch.cuda.synchronize()
        assert oracle.rel_l2(host(y), ref) <= t, order


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_tuned_order_search_and_cache(dtype, tmp_path):
    cache = str(tmp_path / "plans.txt")
    for shape in [(16, 24, 20, 30), (6, 8, 10, 12, 9)]:
        x = gen(shape, dtype)
        plan = offt.Plan(shape, dtype=dtype, tune="exhaustive", cache_path=cache)
        desc = plan.describe()
        print(f"tuned {shape} {dtype}: {desc}", flush=True)
        y = plan.forward(x)
        torch.cuda.synchronize()
        assert oracle.rel_l2(host(y), ndim.fftn(host(x))) <= tol(x.numel(), dtype)
        assert offt.Plan(shape, dtype=dtype, tune="exhaustive", cache_path=cache).describe() == desc
        assert offt.Plan(shape, dtype=dtype, tune="learned").describe().startswith("order=")


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_pass_by_pass_and_graph_replay(dtype):
    shape = (10, 12, 16, 6, 8)
    x = gen(shape, dtype)
    plan = offt.Plan(shape, dtype=dtype)
    y = plan.forward(x)
    y2 = torch.empty_like(y)
    for i in range(plan.npasses()):
        plan.exec_pass(i, offt.FORWARD, x.data_ptr(), y2.data_ptr())
    g = offt.Plan(shape, dtype=dtype, use_graph=True)
    for _ in range(3):
        y3 = g.forward(x)
        z3 = g.backward(y3)
        torch.cuda.synchronize()
        assert torch.equal(y3, y)
        assert torch.equal(z3, plan.backward(y))
    torch.cuda.synchronize()
    assert plan.npasses() == 5 and torch.equal(y, y2)


@pytest.mark.parametrize("shape,dtype", [((64, 64, 64, 64), C128), ((64, 64, 64, 64), C64), ((32, 32, 32, 32, 32), C64)],
                         ids=["64^4-c128", "64^4-c64", "32^5-c64"])
def test_larger_grids_full_oracle(shape, dtype):
    print(f"case {shape} {dtype}", flush=True)
    x = gen(shape, dtype)
    plan = offt.Plan(shape, dtype=dtype, normalize_inverse=True)
    y = plan.forward(x)
    torch.cuda.synchronize()
    xh = host(x)
    t = tol(x.numel(), dtype)
    e = oracle.rel_l2(host(y), ndim.fftn(xh))
    z = plan.backward(y)
    torch.cuda.synchronize()
    e_rt = oracle.rel_l2(host(z), xh)
    print(f"{shape} {dtype}: full {e:.2e} roundtrip {e_rt:.2e} plan {plan.describe()}", flush=True)
    assert e <= t and e_rt <= t


def test_128_4_complex64_sampled_points():
    """128^4 complex64 (2 GiB), the 4-axis workload the benchmark times:
    sampled points from the definition and the normalised round trip."""
    shape = (128, 128, 128, 128)
    print(f"case {shape} c64", flush=True)
    x = gen(shape, C64)
    plan = offt.Plan(shape, dtype=C64, normalize_inverse=True)
    y = plan.forward(x)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    yh = y.cpu().numpy()
    pts = [(0, 0, 0, 0), (1, 2, 3, 4), (127, 5, 64, 9), (33, 100, 7, 126)]
    got = np.array([yh[k] for k in pts], dtype=np.complex128)
    ref = np.array([ndim.dftn_point(xh, k) for k in pts])
    e_pts = oracle.rel_l2(got, ref)
    del yh
    z = plan.backward(y)
    torch.cuda.synchronize()
    e_rt = oracle.rel_l2(z.cpu().numpy(), xh)
    t = tol(x.numel(), C64)
    print(f"128^4 c64: points {e_pts:.2e} roundtrip {e_rt:.2e} plan {plan.describe()}", flush=True)
    assert e_pts <= t and e_rt <= t


def cached_nd_plan(shape, dtype):
    """Plan-cache entry of a grid (the tuned plan the benchmark times)."""
    import os
    path = os.path.join(os.path.dirname(offt.__file__), "data", "plan_cache_mi355x.txt")
    key = f"dtype={0 if dtype == C128 else 1} dims={'x'.join(map(str, shape))} batch=1 "
    for line in open(path):
        head, plan, _ = line.rstrip("\n").split("\t")
        if head.startswith(key) and "layout=" not in head:
            return plan
    return None


@pytest.mark.parametrize("shape,dtype", [((128, 128, 128, 128), C64), ((128, 128, 128, 128), C128),
                                         ((48, 48, 48, 48, 48), C64)], ids=["128^4-c64", "128^4-c128", "48^5-c64"])
def test_cached_tuned_plans_full_oracle(shape, dtype):
    """The tuned plans the benchmark times (plan cache, slab schedules
    included), through the whole-transform call, against the full oracle at
    every point; the normalised round trip."""
    plan_s = cached_nd_plan(shape, dtype)
    assert plan_s is not None
    print(f"case {shape} {dtype} {plan_s}", flush=True)
    x = gen(shape, dtype)
    plan = offt.Plan(shape, dtype=dtype, tune="forced", forced_plan=plan_s, normalize_inverse=True)
    assert plan.describe() == plan_s
    y = plan.forward(x)
    torch.cuda.synchronize()
    xh = host(x)
    t = tol(x.numel(), dtype)
    e = oracle.rel_l2(host(y), ndim.fftn(xh))
    z = plan.backward(y)
    torch.cuda.synchronize()
    e_rt = oracle.rel_l2(host(z), xh)
    print(f"{shape} {dtype}: full {e:.2e} roundtrip {e_rt:.2e}", flush=True)
    plan.close()
    assert e <= t and e_rt <= t


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_longest_axes_in_4_and_5_axis_grids(dtype):
    """Axes of 1024 points (exchanges in parts on the strided ones) inside 4-
    and 5-axis grids, against the full oracle."""
    for shape in [(1024, 3, 1024, 2), (2, 1024, 1, 3, 512)]:
        x = gen(shape, dtype)
        plan = offt.Plan(shape, dtype=dtype, normalize_inverse=True)
        y = plan.forward(x)
        z = plan.backward(y)
        torch.cuda.synchronize()
        xh = host(x)
        t = tol(x.numel(), dtype)
        assert oracle.rel_l2(host(y), ndim.fftn(xh)) <= t, (shape, plan.describe())
        assert oracle.rel_l2(host(z), xh) <= t
