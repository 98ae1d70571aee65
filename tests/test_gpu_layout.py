"""GPU parity of the reversed (cba) output order against the oracle (through
the C ABI).

The forward transform delivers Y[c, b, a] = X[a, b, c] (the cba order the
paper's transform finishes in) and the backward transform takes such input
back to natural order; both are compared element by element with
oracle.layout on the same seeded inputs.  Every transposing axis and pass
order is forced, in place and out of place, and the pass-by-pass launches,
the graph replay and the tuner are checked against the direct transform.
Tolerances as for the natural order (relative L2: 1e-12 complex128,
2e-6 log2 N complex64).
"""
import itertools
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1501_07350_amd as offt
import synth
from oracle import layout

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PLAN_CACHE = os.path.join(ROOT, "paper_1501_07350_amd", "data", "plan_cache_mi355x.txt")


def tol(n, dtype):
    return oracle.tolerance(n, dtype == C64)


def host(x):
    return x.detach().cpu().numpy().astype(np.complex128)


def gen(shape, dtype, key=synth.SEED):
    return synth.complex_grid(shape, dtype, key=key, device="cuda")


SHAPES = [(32, 32, 32), (12, 20, 30), (1, 32, 40), (30, 40, 1), (6, 1, 10), (5, 9, 1), (1, 1, 60), (64, 8, 48)]


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("batch", [1, 3])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_reversed_forward_and_backward_vs_oracle(shape, batch, dtype):
    print(f"case {shape} batch {batch} {dtype}", flush=True)
    full = (batch,) + shape if batch > 1 else shape
    x = gen(full, dtype)
    plan = offt.Plan(shape, dtype=dtype, batch=batch, layout="cba", normalize_inverse=True)
    y = plan.forward(x)
    torch.cuda.synchronize()
    assert tuple(y.shape[-3:]) == shape[::-1]
    xh = host(x)
    assert oracle.rel_l2(host(y), layout.fft3_reversed(xh)) <= tol(x.numel(), dtype)
    # backward of independent cba input, then the round trip
    w = gen(full[:-3] + shape[::-1], dtype, key=synth.SEED + 5)
    z = plan.backward(w)
    torch.cuda.synchronize()
    assert tuple(z.shape[-3:]) == shape
    ref = layout.fft3_from_reversed(host(w)) / np.prod(shape)
    assert oracle.rel_l2(host(z), ref) <= tol(x.numel(), dtype)
    back = plan.backward(y)
    torch.cuda.synchronize()
    assert oracle.rel_l2(host(back), xh) <= tol(x.numel(), dtype)


def forced_plans(shape, dtype):
    """Every (pass order, transposing axis) of the forward half, each with the
    heuristic backward half, with kernels left to the heuristic."""
    bwd = offt.plan_string(shape, dtype, "cba").split("|")[1]
    out = []
    for order in itertools.permutations("abc"):
        for rev in "ac":
            if shape["abc".index(rev)] > 1:
                out.append(f"order={''.join(order)};rev={rev}|{bwd}")
    return out


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("inplace", [False, True], ids=["oop", "inplace"])
@pytest.mark.parametrize("shape", [(48, 20, 36), (16, 1, 64), (60, 24, 1)], ids=lambda s: "x".join(map(str, s)))
def test_every_order_and_transposing_axis(shape, inplace, dtype):
    """The transposing pass first, in the middle and last, along a and along c,
    out of place and in place (where the plan's workspace carries the data);
    the backward direction with the transposing pass on each end as well."""
    x = gen(shape, dtype)
    xh = host(x)
    ref = layout.fft3_reversed(xh)
    t = tol(x.numel(), dtype)
    for fp in forced_plans(shape, dtype):
        # the backward half's orders too: swap roles by giving the same forms
        # to the reversed grid
        rs = shape[::-1]
        for bp in forced_plans(rs, dtype)[:3]:
            plan_str = fp.split("|")[0] + "|" + bp.split("|")[0]
            print(f"case {shape} {dtype} inplace={inplace} {plan_str}", flush=True)
            plan = offt.Plan(shape, dtype=dtype, layout="cba", tune="forced", forced_plan=plan_str)
            if inplace:
                buf = x.clone()
                plan.forward(buf, out=buf.view(rs))
                y = buf.view(rs)
            else:
                y = plan.forward(x)
            torch.cuda.synchronize()
            assert oracle.rel_l2(host(y), ref) <= t, plan_str
            if inplace:
                plan.backward(y, out=y.view(shape))
                z = y.view(shape)
            else:
                z = plan.backward(y)
            torch.cuda.synchronize()
            assert oracle.rel_l2(host(z) / np.prod(shape), xh) <= t, plan_str


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_pass_by_pass_equals_exec(dtype):
    """offt_exec_pass routes through the workspace exactly as exec does: the
    passes launched one by one give the same bits."""
    shape = (24, 30, 40)
    x = gen(shape, dtype)
    for plan_str in ["order=cba;rev=a", "order=cab;rev=c", "order=acb;rev=a"]:
        bwd = offt.plan_string(shape, dtype, "cba").split("|")[1]
        plan = offt.Plan(shape, dtype=dtype, layout="cba", tune="forced", forced_plan=plan_str + "|" + bwd)
        y = plan.forward(x)
        y2 = torch.empty_like(y)
        for i in range(plan.npasses()):
            plan.exec_pass(i, offt.FORWARD, x.data_ptr(), y2.data_ptr())
        z = plan.backward(y)
        z2 = torch.empty_like(z)
        for i in range(plan.npasses()):
            plan.exec_pass(i, offt.BACKWARD, y.data_ptr(), z2.data_ptr())
        torch.cuda.synchronize()
        assert torch.equal(y, y2) and torch.equal(z, z2), plan_str


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_graph_replay_of_reversed_plans(dtype):
    shape = (40, 36, 48)
    x = gen(shape, dtype)
    direct = offt.Plan(shape, dtype=dtype, layout="cba")
    graph = offt.Plan(shape, dtype=dtype, layout="cba", use_graph=True)
    y0 = direct.forward(x)
    z0 = direct.backward(y0)
    for _ in range(3):
        y = graph.forward(x)
        z = graph.backward(y)
        torch.cuda.synchronize()
        assert torch.equal(y, y0) and torch.equal(z, z0)


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_tuned_reversed_plan_and_cache(dtype, tmp_path):
    shape = (64, 96, 80)
    cache = str(tmp_path / "plans.txt")
    x = gen(shape, dtype)
    plan = offt.Plan(shape, dtype=dtype, layout="cba", tune="exhaustive", cache_path=cache)
    desc = plan.describe()
    print(f"tuned {shape} {dtype}: {desc}", flush=True)
    fwd, bwd = desc.split("|")
    assert "rev=" in fwd and "rev=" in bwd
    y = plan.forward(x)
    torch.cuda.synchronize()
    assert oracle.rel_l2(host(y), layout.fft3_reversed(host(x))) <= tol(x.numel(), dtype)
    again = offt.Plan(shape, dtype=dtype, layout="cba", tune="exhaustive", cache_path=cache)
    assert again.describe() == desc
    # the natural layout of the same shape does not pick up the reversed entry
    nat = offt.Plan(shape, dtype=dtype, tune="exhaustive", cache_path=cache)
    assert "|" not in nat.describe()


def test_workspace_and_one_axis_grids():
    shape = (64, 48, 30)
    nat = offt.Plan(shape, dtype=C128)
    rev = offt.Plan(shape, dtype=C128, layout="cba")
    assert rev.workspace_bytes() - nat.workspace_bytes() >= 64 * 48 * 30 * 16
    one = offt.Plan((1, 1, 60), dtype=C128, layout="cba")
    assert one.workspace_bytes() == offt.Plan((1, 1, 60), dtype=C128).workspace_bytes()
    x = gen((1, 1, 60), C128)
    assert torch.equal(one.forward(x).reshape(-1), offt.Plan((1, 1, 60), dtype=C128).forward(x).reshape(-1))


@pytest.mark.parametrize("n,dtype", [(512, C128), (512, C64)], ids=["512-c128", "512-c64"])
def test_full_size_sampled_lines(n, dtype):
    """512^3 with the heuristic reversed plan, out of place (the benchmark's
    tuned reversed plans are checked against the whole O3 transform in
    test_512_cached_reversed_plan_full_oracle): sampled lines from the
    definition, Parseval and the normalised round trip."""
    shape = (n, n, n)
    print(f"case {shape} {dtype} cba", flush=True)
    x = synth.complex_grid(shape, dtype, device="cuda")
    plan = offt.Plan(shape, dtype=dtype, layout="cba", normalize_inverse=True)
    y = plan.forward(x)
    torch.cuda.synchronize()
    t = tol(x.numel(), dtype)
    xh = host(x)
    yh = host(y)
    got, ref = [], []
    for ka, kb in [(0, 0), (1, 0), (0, 1), (5, 7), (17, 3), (n - 1, n - 1), (n - 2, 11), (100, n - 3)]:
        ref.append(oracle.dft3_line(xh, ka, kb))       # X[ka, kb, :]
        got.append(yh[:, kb, ka])                       # Y[:, kb, ka]
    e_lines = oracle.rel_l2(np.concatenate(got), np.concatenate(ref))
    e_pars = abs(np.sum(np.abs(yh) ** 2) / (xh.size * np.sum(np.abs(xh) ** 2)) - 1.0)
    del yh
    z = plan.backward(y)
    torch.cuda.synchronize()
    e_rt = oracle.rel_l2(host(z), xh)
    print(f"{shape} {dtype} cba: lines {e_lines:.2e} parseval {e_pars:.2e} roundtrip {e_rt:.2e} "
          f"plan {plan.describe()}", flush=True)
    assert e_lines <= t and e_pars <= t and e_rt <= t


def cached_reversed_plan(n, dtype):
    """Reversed-order (cba) plan-cache entry of an n^3 grid, batch 1: the
    forward and backward plan strings joined by '|'."""
    code = 0 if dtype == C128 else 1
    key = f"dtype={code} dims={n}x{n}x{n} batch=1 "
    with open(PLAN_CACHE) as f:
        for line in f:
            head, plan, _ = line.rstrip("\n").split("\t")
            if head.startswith(key) and "layout=cba" in head:
                return plan
    return None


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_512_cached_reversed_plan_full_oracle(dtype):
    """512^3 with the tuned reversed-order plans of the plan cache (those the
    benchmark's reversed-output runs time): the whole forward output against
    the O3 transform delivered in cba order, element by element, and the
    backward transform of it against the whole input (normalised)."""
    n = 512
    shape = (n, n, n)
    plan_str = cached_reversed_plan(n, dtype)
    assert plan_str, "plan cache has no 512^3 reversed-order entry"
    print(f"case {shape} {dtype} cba cached plan {plan_str}", flush=True)
    x = synth.complex_grid(shape, dtype, device="cuda")
    plan = offt.Plan(shape, dtype=dtype, layout="cba", tune="forced", forced_plan=plan_str,
                     normalize_inverse=True)
    y = plan.forward(x)
    torch.cuda.synchronize()
    t = tol(x.numel(), dtype)
    xh = host(x)
    yh = host(y)
    ref = layout.fft3_reversed(xh)
    e_fwd = oracle.rel_l2(yh, ref)
    e_max = float(np.max(np.abs(yh - ref)) / np.max(np.abs(ref)))
    del yh, ref
    z = plan.backward(y)
    torch.cuda.synchronize()
    e_rt = oracle.rel_l2(host(z), xh)
    print(f"{shape} {dtype} cba cached: forward {e_fwd:.2e} (max element {e_max:.2e}) round trip {e_rt:.2e} "
          f"tol {t:.1e} plan {plan.describe()}", flush=True)
    plan.close()
    assert e_fwd <= t and e_rt <= t


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("inplace", [False, True], ids=["oop", "inplace"])
@pytest.mark.parametrize("shape,fwd", [
    ((256, 6, 10), "order=cba;rev=a;a=16x16/16/p2"),     # rows out in 2 parts, transposing pass last
    ((256, 6, 10), "order=acb;rev=a;a=16x16/8/p4"),      # 4 parts, transposing pass first
    ((6, 10, 256), "order=cba;rev=c;c=16x16/16/p2"),     # rows in in 2 parts, first
    ((5, 12, 512), "order=abc;rev=c;c=16x16x2/16/p2"),   # rows in, last; 512-point lines
    ((512, 3, 5), "order=bca;rev=a;a=32x16/16/p2"),      # radix-32 first stage, 15 lines: one ragged tile
])
def test_transposing_pass_in_parts(shape, fwd, inplace, dtype):
    """Transposing passes whose exchanges and row side run in 2 and 4 parts,
    forward and backward, ragged tiles, against the oracle."""
    print(f"case {shape} {dtype} {fwd} inplace={inplace}", flush=True)
    rs = shape[::-1]
    bwd = offt.plan_string(rs, dtype, "cba").split("|")[0]
    plan = offt.Plan(shape, dtype=dtype, layout="cba", tune="forced", forced_plan=fwd + "|" + bwd,
                     normalize_inverse=True)
    assert fwd.split(";")[2] in plan.describe()
    x = gen(shape, dtype)
    xh = host(x)
    t = tol(x.numel(), dtype)
    if inplace:
        buf = x.clone()
        plan.forward(buf, out=buf.view(rs))
        y = buf.view(rs)
    else:
        y = plan.forward(x)
    torch.cuda.synchronize()
    assert oracle.rel_l2(host(y), layout.fft3_reversed(xh)) <= t
    z = plan.backward(y)
    torch.cuda.synchronize()
    assert oracle.rel_l2(host(z), xh) <= t


def test_largest_grid_reversed_sampled_lines():
    """1024^3 complex64 (8 GiB, the longest axes) in the reversed order with
    the plan's 8 GiB workspace: sampled lines from the definition and the
    normalised round trip."""
    n = 1024
    shape = (n, n, n)
    print(f"case {shape} c64 cba", flush=True)
    x = synth.complex_grid(shape, C64, device="cuda")
    plan = offt.Plan(shape, dtype=C64, layout="cba", normalize_inverse=True)
    y = plan.forward(x)
    torch.cuda.synchronize()
    t = tol(x.numel(), C64)
    xh = x.cpu().numpy()
    got, ref = [], []
    for ka, kb in [(0, 0), (1, 0), (5, 7), (n - 1, n - 1), (100, n - 3)]:
        ref.append(oracle.dft3_line(xh, ka, kb))
        got.append(y[:, kb, ka].cpu().numpy().astype(np.complex128))
    e_lines = oracle.rel_l2(np.concatenate(got), np.concatenate(ref))
    z = plan.backward(y)
    torch.cuda.synchronize()
    del y
    e_rt = oracle.rel_l2(z.cpu().numpy(), xh)
    print(f"1024^3 c64 cba: lines {e_lines:.2e} roundtrip {e_rt:.2e} plan {plan.describe()}", flush=True)
    assert e_lines <= t and e_rt <= t
