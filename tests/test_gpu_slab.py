"""Slab schedules (plan string ";slab=S"): after the whole-grid pass over a,
the passes over b and c run S planes (Nb x Nc, counted over the batch) at a
time, both passes of one slab before the next.  Every element goes through
the same arithmetic as without the schedule, so the result must equal the
same plan without ";slab=" bit for bit, and match the oracle's 3-D DFT
(Sec. 2, Eq. 1) within the tolerance.  Ragged last slabs, slabs that span
two grids of a batch, a unit axis, the backward direction with 1/N, in-place
execution, graph replay, and pass-by-pass / range-wise launches are covered."""
import numpy as np
import pytest
import torch

import oracle
import paper_1501_07350_amd as offt
import synth
from oracle import ndim

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64

# (shape, batch, planes per slab)
CASES = [((24, 20, 18), 1, 5), ((24, 20, 18), 3, 7), ((16, 12, 10), 2, 1), ((16, 12, 10), 1, 16),
         ((16, 12, 10), 2, 40), ((12, 1, 30), 2, 5), ((12, 30, 1), 1, 4), ((40, 48, 36), 1, 9)]


def plans(shape, dtype, S):
    """The heuristic plan with the pass over a moved first, without and with
    the slab schedule."""
    base = offt.default_plan_string(shape, dtype)
    order = dict(f.split("=", 1) for f in base.split(";"))["order"]
    plain = base.replace(f"order={order}", "order=a" + order.replace("a", ""))
    return plain, f"{plain};slab={S}"


def oracle_forward(x, shape, batch):
    xh = x.cpu().numpy().astype(np.complex128).reshape((batch,) + tuple(shape))
    return np.stack([oracle.fft3(g) for g in xh])


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape,batch,S", CASES, ids=lambda v: str(v))
def test_slab_schedule_bit_identical_and_vs_oracle(shape, batch, S, dtype):
    plain, slab = plans(shape, dtype, S)
    print(f"case {shape} batch {batch} {dtype}: {slab}", flush=True)
    full = ((batch,) if batch > 1 else ()) + tuple(shape)
    x = synth.complex_grid(full, dtype, device="cuda")
    p0 = offt.Plan(shape, dtype=dtype, batch=batch, tune="forced", forced_plan=plain, normalize_inverse=True)
    p1 = offt.Plan(shape, dtype=dtype, batch=batch, tune="forced", forced_plan=slab, normalize_inverse=True)
    assert p0.slab() == 0 and p1.slab() == S
    y0 = p0.forward(x)
    y1 = p1.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    ref = oracle_forward(x, shape, batch)
    tol = oracle.tolerance(int(np.prod(shape)), dtype == C64)
    assert oracle.rel_l2(y1.cpu().numpy().reshape(ref.shape), ref) <= tol
    # pass by pass (each over all its slabs) and range by range: the same bits
    h = int(torch.cuda.current_stream().cuda_stream)
    y2 = torch.empty_like(x)
    for i in range(p1.npasses()):
        p1.exec_pass(i, offt.FORWARD, x.data_ptr(), y2.data_ptr(), h)
    y3 = torch.empty_like(x)
    p1.exec_range(0, 1, offt.FORWARD, x.data_ptr(), y3.data_ptr(), h)
    if p1.npasses() > 1:
        p1.exec_range(1, p1.npasses() - 1, offt.FORWARD, x.data_ptr(), y3.data_ptr(), h)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2) and torch.equal(y1, y3)
    # backward with 1/N, in place, against the plain plan and the input
    z0 = y0.clone()
    p0.backward(z0, out=z0)
    z1 = y1.clone()
    p1.backward(z1, out=z1)
    torch.cuda.synchronize()
    assert torch.equal(z0, z1)
    assert oracle.rel_l2(z1.cpu().numpy(), x.cpu().numpy()) <= tol
    p0.close()
    p1.close()


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_slab_schedule_graph_replay(dtype):
    """The plan's HIP graph records the slab launches: every replay, with
    eager work between them, equals the eager result."""
    shape, batch, S = (24, 20, 18), 2, 7
    plain, slab = plans(shape, dtype, S)
    x = synth.complex_grid((batch,) + shape, dtype, device="cuda")
    eager = offt.Plan(shape, dtype=dtype, batch=batch, tune="forced", forced_plan=slab)
    graph = offt.Plan(shape, dtype=dtype, batch=batch, tune="forced", forced_plan=slab, use_graph=True)
    want = eager.forward(x)
    out = torch.empty_like(x)
    for r in range(4):
        graph.forward(x, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, want), r
        eager.forward(x * (r + 2))      # other work between replays
        torch.cuda.synchronize()


def test_range_rejects_bad_arguments():
    plan = offt.Plan((8, 8, 8), dtype=C64, tune="forced", forced_plan=plans((8, 8, 8), C64, 3)[1])
    x = synth.complex_grid((8, 8, 8), C64, device="cuda")
    for first, count in ((-1, 1), (0, 0), (0, 4), (3, 1), (2, 2)):
        with pytest.raises(offt.OfftError) as e:
            plan.exec_range(first, count, offt.FORWARD, x.data_ptr(), x.data_ptr())
        assert e.value.code == -1


def test_tuner_on_a_grid_above_512_mib():
    """The exhaustive tuner on a 640 MiB complex64 grid (where it also tries
    slab schedules): whatever it keeps matches the oracle on sampled lines,
    and its whole-transform call equals its ranges launched one by one."""
    shape = (320, 512, 512)
    x = synth.complex_grid(shape, C64, device="cuda")
    plan = offt.Plan(shape, dtype=C64, tune="exhaustive")
    print(f"tuned: {plan.describe()}", flush=True)
    y = plan.forward(x)
    y2 = torch.empty_like(x)
    h = int(torch.cuda.current_stream().cuda_stream)
    for g in plan.pass_groups():
        plan.exec_range(g[0], len(g), offt.FORWARD, x.data_ptr(), y2.data_ptr(), h)
    torch.cuda.synchronize()
    assert torch.equal(y, y2)
    xh = x.cpu().numpy().astype(np.complex128)
    yh = y.cpu().numpy()
    got, ref = [], []
    for ka, kb in ((0, 0), (7, 301), (319, 511)):
        got.append(yh[ka, kb].astype(np.complex128))
        ref.append(oracle.dft3_line(xh, ka, kb))
    e = oracle.rel_l2(np.concatenate(got), np.concatenate(ref))
    assert e <= oracle.tolerance(x.numel(), True), e
    plan.close()


# grids of 4 and 5 axes: (shape, batch, blocks of the trailing axes per slab)
ND_CASES = [((12, 8, 6, 10), 1, 5), ((6, 4, 5, 3, 8), 2, 4), ((10, 1, 6, 8), 1, 3), ((9, 6, 4, 10), 3, 2)]


def nd_plans(shape, dtype, S):
    base = offt.plan_string_nd(shape, dtype)
    order = dict(f.split("=", 1) for f in base.split(";"))["order"]
    plain = base.replace(f"order={order}", "order=a" + order.replace("a", ""))
    return plain, f"{plain};slab={S}"


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape,batch,S", ND_CASES, ids=lambda v: str(v))
def test_nd_slab_schedule_bit_identical_and_vs_oracle(shape, batch, S, dtype):
    plain, slab = nd_plans(shape, dtype, S)
    print(f"case {shape} batch {batch} {dtype}: {slab}", flush=True)
    full = ((batch,) if batch > 1 else ()) + tuple(shape)
    x = synth.complex_grid(full, dtype, device="cuda")
    p0 = offt.Plan(shape, dtype=dtype, batch=batch, tune="forced", forced_plan=plain, normalize_inverse=True)
    p1 = offt.Plan(shape, dtype=dtype, batch=batch, tune="forced", forced_plan=slab, normalize_inverse=True)
    assert p0.slab() == 0 and p1.slab() == S
    y0 = p0.forward(x)
    y1 = p1.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    xh = x.cpu().numpy().astype(np.complex128)
    ref = ndim.fftn_batch(xh, len(shape)) if batch > 1 else ndim.fftn(xh)
    tol = oracle.tolerance(int(np.prod(shape)), dtype == C64)
    assert oracle.rel_l2(y1.cpu().numpy(), ref) <= tol
    z1 = y1.clone()
    p1.backward(z1, out=z1)
    torch.cuda.synchronize()
    assert oracle.rel_l2(z1.cpu().numpy(), xh) <= tol
    p0.close()
    p1.close()


# column-block schedules: (shape, batch, columns per block)
COL_CASES = [((24, 20, 32), 1, 16), ((24, 20, 32), 2, 8), ((16, 12, 64), 1, 32), ((12, 1, 32), 2, 8),
             ((1, 12, 32), 1, 8), ((40, 48, 64), 1, 16)]


def col_plans(shape, dtype, w):
    """The heuristic plan with the pass over c first and the strided tiles
    at most w columns wide, without and with blocks of w columns."""
    base = offt.default_plan_string(shape, dtype)
    fields = [f.split("=", 1) for f in base.split(";")]
    out = []
    for k, v in fields:
        if k == "order":
            v = "c" + v.replace("c", "")
        elif k in ("a", "b") and v != "1":
            parts = v.split("/")
            parts[1] = str(min(int(parts[1]), w))
            v = "/".join(parts)
        out.append(f"{k}={v}")
    plain = ";".join(out)
    return plain, f"{plain};col={w}"


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape,batch,w", COL_CASES, ids=lambda v: str(v))
def test_column_block_schedule_bit_identical_and_vs_oracle(shape, batch, w, dtype):
    plain, blocked = col_plans(shape, dtype, w)
    print(f"case {shape} batch {batch} {dtype}: {blocked}", flush=True)
    full = ((batch,) if batch > 1 else ()) + tuple(shape)
    x = synth.complex_grid(full, dtype, device="cuda")
    p0 = offt.Plan(shape, dtype=dtype, batch=batch, tune="forced", forced_plan=plain, normalize_inverse=True)
    p1 = offt.Plan(shape, dtype=dtype, batch=batch, tune="forced", forced_plan=blocked, normalize_inverse=True)
    assert p0.col() == 0 and p1.col() == w
    y0 = p0.forward(x)
    y1 = p1.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    ref = oracle_forward(x, shape, batch)
    tol = oracle.tolerance(int(np.prod(shape)), dtype == C64)
    assert oracle.rel_l2(y1.cpu().numpy().reshape(ref.shape), ref) <= tol
    h = int(torch.cuda.current_stream().cuda_stream)
    y2 = torch.empty_like(x)
    for i in range(p1.npasses()):
        p1.exec_pass(i, offt.FORWARD, x.data_ptr(), y2.data_ptr(), h)
    y3 = torch.empty_like(x)
    for g in p1.pass_groups():
        p1.exec_range(g[0], len(g), offt.FORWARD, x.data_ptr(), y3.data_ptr(), h)
    z1 = y1.clone()
    p1.backward(z1, out=z1)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2) and torch.equal(y1, y3)
    assert oracle.rel_l2(z1.cpu().numpy(), x.cpu().numpy()) <= tol
    p0.close()
    p1.close()
