"""GPU parity of the HIP transform against the CPU oracle (through the C ABI).

Tolerances (relative L2 over the compared values): 1e-12 for complex128,
2e-6 * log2(N) for complex64 with N the grid's element count.  complex64
inputs are binary64 values rounded to binary32; the oracle consumes those
binary32 values widened exactly, so the error measured is the transform's.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1501_07350_amd as offt
import synth

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64


def tol(n, dtype):
    return oracle.tolerance(n, dtype == C64)


def gen(shape, dtype, key=synth.SEED, dev="cuda"):
    return synth.complex_grid(shape, dtype, key=key, device=dev)


def host(x):
    return x.detach().cpu().numpy().astype(np.complex128)


def run(shape, dtype, batch=1, inplace=False, forced=None, key=synth.SEED, normalize=False):
    full = (batch,) + tuple(shape) if batch > 1 else tuple(shape)
    x = gen(full, dtype, key)
    plan = offt.Plan(shape, dtype=dtype, batch=batch, tune="forced" if forced else "none",
                     forced_plan=forced, normalize_inverse=normalize)
    if inplace:
        y = x.clone()
        plan.forward(y, out=y)
    else:
        y = plan.forward(x)
    torch.cuda.synchronize()
    return plan, x, y


def ref3(xh, sign=oracle.FORWARD):
    if xh.ndim == 4:
        return np.stack([oracle.fft3(g, sign) for g in xh])
    return oracle.fft3(xh, sign)


# ------------------------------------------------------------ small workload ----
def test_32cubed_complex128_vs_brute_force():
    """32x32x32 complex128 forward vs the brute-force definition, then the
    inverse; round trip with 1/N."""
    plan, x, y = run((32, 32, 32), C128, normalize=True)
    xh = host(x)
    e_brute = oracle.rel_l2(host(y), oracle.dft3_brute(xh))
    e_axes = oracle.rel_l2(host(y), oracle.dft3_axes(xh))
    z = plan.backward(y)
    torch.cuda.synchronize()
    e_rt = oracle.rel_l2(host(z), xh)
    print(f"32^3 c128: brute {e_brute:.2e} axes {e_axes:.2e} roundtrip {e_rt:.2e}")
    assert e_brute <= 1e-12 and e_axes <= 1e-12 and e_rt <= 1e-12


TINY = [(1, 1, 1), (2, 3, 5), (5, 3, 2), (4, 4, 4), (8, 6, 10), (1, 9, 1), (3, 1, 16), (16, 1, 1),
        (1, 1, 2), (2, 1, 1), (6, 5, 4), (15, 12, 10), (9, 25, 27)]


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape", TINY, ids=lambda s: "x".join(map(str, s)))
def test_tiny_grids_vs_brute_force(shape, dtype):
    plan, x, y = run(shape, dtype)
    xh = host(x)
    ref = oracle.dft3_brute(xh)
    assert oracle.rel_l2(host(y), ref) <= tol(x.numel(), dtype)
    # backward, unnormalised
    z = plan.backward(x)
    torch.cuda.synchronize()
    assert oracle.rel_l2(host(z), oracle.dft3_brute(xh, oracle.BACKWARD)) <= tol(x.numel(), dtype)


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_batched_ragged_and_inplace(dtype):
    # batch of 5 grids, lines not a multiple of any tile width
    shape = (6, 10, 15)
    plan, x, y = run(shape, dtype, batch=5, key=synth.SEED + 9)
    ref = ref3(host(x))
    assert oracle.rel_l2(host(y), ref) <= tol(np.prod(shape), dtype)
    _, x2, y2 = run(shape, dtype, batch=5, inplace=True, key=synth.SEED + 9)
    assert torch.equal(y, y2), "in-place result differs from out-of-place"


# ------------------------------------------------------ every 1-D length ----
LENGTHS = [n for n in range(2, 1025) if synth.smooth_lengths(n, n)]


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_every_length_contiguous_lines(dtype):
    """Every 2/3/5-smooth length 2..1024 along the contiguous axis, 37 lines
    (ragged tile), against the 1-D oracle on each line."""
    bad = []
    for L in LENGTHS:
        plan, x, y = run((1, 1, L), dtype, batch=37, key=synth.SEED + L)
        xh = host(x).reshape(37, L)
        ref = oracle.fft1_lines(xh)
        e = oracle.rel_l2(host(y).reshape(37, L), ref)
        if e > tol(L, dtype):
            bad.append((L, e))
        plan.close()
    assert not bad, bad


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_every_length_strided_lines(dtype):
    """Every length along a strided axis: shape (L, 1, 20) puts L on axis a
    with stride 20 (not a multiple of the tile width: straddling tiles)."""
    bad = []
    for L in LENGTHS:
        plan, x, y = run((L, 1, 20), dtype, key=synth.SEED + 2 * L)
        xh = host(x)
        ref = np.moveaxis(oracle.fft1_lines(np.moveaxis(xh[:, 0, :], 0, 1)), 1, 0)
        # c axis (20) is transformed too: apply it to the reference
        ref = oracle.fft1_lines(ref)
        e = oracle.rel_l2(host(y)[:, 0, :], ref)
        if e > tol(20 * L, dtype):
            bad.append((L, e))
        plan.close()
    assert not bad, bad


def _gen_kernels():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(offt.__file__), "csrc", "gen_kernels.py")
    spec = importlib.util.spec_from_file_location("gen_kernels", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _all_forced_plans(shape, dtype):
    """Plan strings of every radix sequence per axis (default tile width)."""
    base = offt.Plan(shape, dtype=dtype).describe()
    fields = dict(kv.split("=") for kv in base.split(";"))
    plans = [base]
    gk = _gen_kernels()
    for ax, L in zip("abc", shape):
        if L <= 1:
            continue
        W0 = int(fields[ax].split("/")[1])
        for seq in gk.radix_seqs(L):
            # largest tile width <= the default one that fits this kernel
            W = W0
            while True:
                f2 = dict(fields)
                f2[ax] = "x".join(map(str, seq)) + f"/{W}"
                s = ";".join(f"{k}={v}" for k, v in f2.items())
                try:
                    offt.Plan(shape, dtype=dtype, tune="forced", forced_plan=s).close()
                    break
                except offt.OfftError as e:
                    assert e.code == -6 and W > 1, (s, e)
                    W //= 2
            if s not in plans:
                plans.append(s)
    return plans


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape", [(32, 32, 32), (48, 60, 80), (128, 16, 256), (1024, 2, 12), (6, 512, 10),
                                   (4, 6, 512)],
                         ids=lambda s: "x".join(map(str, s)))
def test_every_radix_sequence_and_order(shape, dtype):
    x = gen(shape, dtype, synth.SEED + 77)
    ref = oracle.fft3(host(x))
    plans = _all_forced_plans(shape, dtype)
    for order in ("abc", "acb", "bac", "bca", "cab"):
        plans.append(plans[0].replace("order=cba", "order=" + order))
    for ps in plans:
        p = offt.Plan(shape, dtype=dtype, tune="forced", forced_plan=ps)
        assert p.describe() == ps
        y = p.forward(x)
        torch.cuda.synchronize()
        e = oracle.rel_l2(host(y), ref)
        assert e <= tol(x.numel(), dtype), (ps, e)
        p.close()


def test_tile_widths_forced():
    shape = (64, 40, 96)
    for dtype in (C128, C64):
        x = gen(shape, dtype, synth.SEED + 5)
        ref = oracle.fft3(host(x))
        for W in (1, 2, 4, 8, 16):
            ps = f"order=cba;a=8x8/{W};b=8x5/{W};c=8x4x3/{W}"
            try:
                p = offt.Plan(shape, dtype=dtype, tune="forced", forced_plan=ps)
            except offt.OfftError:
                continue   # tile does not fit LDS / thread limit for this precision
            y = p.forward(x)
            torch.cuda.synchronize()
            assert oracle.rel_l2(host(y), ref) <= tol(x.numel(), dtype), (dtype, ps)
            p.close()


def _kernel_spec(L, seq, tpl, P, W):
    spec = "x".join(map(str, seq)) + f"/{W}"
    if tpl != L // max(seq):
        spec += f"/{tpl}"
    if P > 1:
        spec += f"/p{P}"
    return spec


# strided axes of power-of-two length >= 256 (the kernels with LDS exchanges
# in parts); lines per pass not a multiple of the tile width, so the last
# tile is ragged
@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape,axis", [((256, 12, 10), "a"), ((6, 512, 9), "b"), ((1024, 3, 5), "a")],
                         ids=["a256", "b512", "a1024"])
def test_strided_exchange_parts(shape, axis, dtype):
    """Every kernel whose LDS exchanges run in 2 or 4 parts, at every tile
    width that fits: within tolerance of the oracle, and bit-identical across
    tile widths (the width changes which threads and LDS slots carry a line,
    not the arithmetic).  Kernels of different part counts are separate
    compilations whose multiply-adds may be contracted differently, so they
    agree to rounding only."""
    gk = _gen_kernels()
    prec = "f64" if dtype == C128 else "f32"
    x = gen(shape, dtype, synth.SEED + 31)
    ref = oracle.fft3(host(x))
    base = offt.Plan(shape, dtype=dtype).describe()
    fields = dict(kv.split("=") for kv in base.split(";"))
    L = shape["abc".index(axis)]
    ents = [e for e in gk.entries(prec) if e[0] == L]
    tried = 0
    for (_, seq, tpl, P) in ents:
        if P == 1:
            continue
        whole = None
        for W in (64, 32, 16, 8, 4, 2, 1):
            f2 = dict(fields)
            f2[axis] = _kernel_spec(L, seq, tpl, P, W)
            ps = ";".join(f"{k}={v}" for k, v in f2.items())
            try:
                p = offt.Plan(shape, dtype=dtype, tune="forced", forced_plan=ps)
            except offt.OfftError:
                continue   # tile does not fit the thread or LDS limit
            assert p.describe() == ps
            y = p.forward(x)
            p.close()
            torch.cuda.synchronize()
            if whole is None:
                whole = y   # the widest tile of this kernel
            assert torch.equal(y, whole), ps
            e = oracle.rel_l2(host(y), ref)
            assert e <= tol(x.numel(), dtype), (ps, e)
            tried += 1
    assert tried > 0


def test_exchange_parts_rejected_for_contiguous_axes():
    """Kernels with exchanges in parts keep only part of each line in LDS:
    plan strings that put one on the contiguous axis are refused."""
    shape = (4, 4, 512)
    with pytest.raises(offt.OfftError):
        offt.Plan(shape, dtype=C128, tune="forced", forced_plan="order=cba;a=4/16;b=4/16;c=16x16x2/1/p2")


@pytest.mark.parametrize("shape,dtype", [((32, 32, 32), C128), ((48, 60, 80), C64)],
                         ids=["32cubed-c128", "48x60x80-c64"])
def test_tuner_candidates_choice_and_cache(shape, dtype, tmp_path):
    """Every candidate plan the tuners choose among meets the oracle; the
    exhaustive choice meets it; the plan cache replays the stored choice (the
    latest valid entry of the grid's key wins); offt_tune_table times every
    candidate."""
    from paper_1501_07350_amd import selector
    code = 0 if dtype == C128 else 1
    x = gen(shape, dtype, synth.SEED + 57)
    ref = oracle.fft3(host(x))
    plans, _ = selector.candidates(shape, 1, code)
    assert len(plans) == len(set(plans)) >= 6
    for ps in plans:
        p = offt.Plan(shape, dtype=dtype, tune="forced", forced_plan=ps)
        assert p.describe() == ps
        y = p.forward(x)
        torch.cuda.synchronize()
        assert oracle.rel_l2(host(y), ref) <= tol(x.numel(), dtype), ps
        p.close()
    cache = str(tmp_path / "plans.txt")
    tuned = offt.Plan(shape, dtype=dtype, tune="exhaustive", cache_path=cache)
    y = tuned.forward(x)
    torch.cuda.synchronize()
    assert oracle.rel_l2(host(y), ref) <= tol(x.numel(), dtype)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].split("\t")[1] == tuned.describe() and float(lines[0].split("\t")[2]) > 0
    again = offt.Plan(shape, dtype=dtype, tune="exhaustive", cache_path=cache)
    assert again.describe() == tuned.describe()
    # a later entry for the same key (another candidate) is the one replayed
    other = next(ps for ps in plans if ps != tuned.describe())
    with open(cache, "a") as f:
        f.write(lines[0].split("\t")[0] + "\t" + other + "\t1.0\n")
    assert offt.Plan(shape, dtype=dtype, tune="exhaustive", cache_path=cache).describe() == other
    # timings of the candidate list, as the selector's data collection takes them
    import ctypes
    from paper_1501_07350_amd import _lib
    buf = torch.zeros(x.numel() * 2, dtype=torch.float64 if dtype == C128 else torch.float32, device="cuda")
    times = np.zeros(len(plans), dtype=np.float32)
    n = _lib.check(_lib.load().offt_tune_table(shape[0], shape[1], shape[2], code, 1, 2,
                                               ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                                               ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream)),
                                               times.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), len(plans)))
    assert n == len(plans) and np.all(np.isfinite(times)) and np.all(times > 0)


# ------------------------------------------------------------- twiddles ----
def roots_extended(n):
    """exp(-2 pi i m / n) in x87 extended precision (independent of both the
    GPU generator and the oracle's binary64 table)."""
    pi = np.arctan(np.longdouble(1)) * 4
    m = np.arange(n, dtype=np.longdouble)
    ang = 2 * pi * m / np.longdouble(n)
    c, s = np.cos(ang), -np.sin(ang)
    # the quarter points are exact: 1, -i, -1, +i
    q = (4 * np.arange(n)) % n == 0
    k = (4 * np.arange(n))[q] // n
    c[q] = np.array([1, 0, -1, 0], dtype=np.longdouble)[k]
    s[q] = np.array([0, -1, 0, 1], dtype=np.longdouble)[k]
    return c, s


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 12, 60, 150, 512, 1000, 1024])
def test_twiddles_fp64_and_rounded_fp32(n):
    t64 = offt.twiddles(n, C128)
    cr, ci = roots_extended(n)
    # binary64 table within ~1 ulp of the extended-precision value
    err = np.maximum(np.abs(t64.real - cr), np.abs(t64.imag - ci)).astype(np.float64)
    assert np.max(err) <= 2.3e-16
    # and within the oracle table's own accuracy of the oracle
    assert np.max(np.abs(t64 - oracle.root_table(n))) <= 2e-15   # oracle: cos(2 pi m/n) in binary64
    # exact quarter points
    assert t64[0] == 1
    if n % 4 == 0:
        assert t64[n // 4] == -1j and t64[n // 2] == -1 and t64[3 * n // 4] == 1j
    # binary32: the binary64 value rounded to nearest; within one binary32 ulp
    # of RN(extended value), and equal to it almost everywhere
    t32 = offt.twiddles(n, C64)
    rr, ri = cr.astype(np.float32), ci.astype(np.float32)
    ulp_r = np.spacing(np.abs(rr)).astype(np.float64)
    ulp_i = np.spacing(np.abs(ri)).astype(np.float64)
    assert np.all(np.abs(t32.real.astype(np.float64) - rr) <= ulp_r)
    assert np.all(np.abs(t32.imag.astype(np.float64) - ri) <= ulp_i)
    assert np.mean((t32.real == rr) & (t32.imag == ri)) >= 0.99
    # and exactly RN of the device's own binary64 table
    assert np.array_equal(t32, t64.astype(np.complex64))


# ------------------------------------------------------- determinism etc ----
def test_bitwise_deterministic_and_stream_ordered():
    shape = (64, 64, 64)
    x = gen(shape, C64)
    plan = offt.Plan(shape, dtype=C64)
    y1 = plan.forward(x)
    y2 = plan.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        y3 = plan.forward(x)
    s.synchronize()
    assert torch.equal(y1, y3)


@pytest.mark.parametrize("shape,dtype", [((32, 32, 32), C128), ((48, 60, 80), C64), ((6, 512, 10), C64),
                                         ((1, 1, 1), C128)], ids=["32cubed-c128", "48x60x80-c64", "6x512x10-c64",
                                                                  "1x1x1"])
def test_graph_replay_matches_direct_launches(shape, dtype):
    """use_graph: the captured pass kernels give the direct launches' results
    bit for bit on every replay (eager work and a synchronisation between
    replays), after a change of buffers and direction, and in place."""
    x = gen(shape, dtype, synth.SEED + 41)
    direct = offt.Plan(shape, dtype=dtype, normalize_inverse=True)
    graph = offt.Plan(shape, dtype=dtype, normalize_inverse=True, use_graph=True)
    assert graph.describe() == direct.describe()
    ref_f = direct.forward(x)
    ref_b = direct.backward(ref_f)
    torch.cuda.synchronize()
    assert oracle.rel_l2(host(ref_f), oracle.fft3(host(x))) <= tol(x.numel(), dtype)
    out = torch.empty_like(x)
    for rep in range(3):
        _ = (x * 2).sum()
        torch.cuda.synchronize()
        out.zero_()
        graph.forward(x, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_f), f"replay {rep}"
    y = graph.backward(ref_f.clone())          # other buffers, other direction: graph updated
    torch.cuda.synchronize()
    assert torch.equal(y, ref_b)
    z = x.clone()
    graph.forward(z, out=z)                    # in place
    torch.cuda.synchronize()
    assert torch.equal(z, ref_f)
    graph.forward(x, out=out)                  # back to the first buffers
    torch.cuda.synchronize()
    assert torch.equal(out, ref_f)
    direct.close()
    graph.close()


def test_normalized_inverse_and_linearity():
    shape = (20, 24, 30)
    for dtype in (C128, C64):
        a = gen(shape, dtype, synth.SEED + 1)
        b = gen(shape, dtype, synth.SEED + 2)
        plan = offt.Plan(shape, dtype=dtype, normalize_inverse=True)
        z = plan.backward(plan.forward(a))
        torch.cuda.synchronize()
        assert oracle.rel_l2(host(z), host(a)) <= tol(a.numel(), dtype)
        fa, fb, fab = plan.forward(a), plan.forward(b), plan.forward(a + b)
        torch.cuda.synchronize()
        assert oracle.rel_l2(host(fab), host(fa) + host(fb)) <= tol(a.numel(), dtype)


@pytest.mark.parametrize("use_graph", [False, True], ids=["direct", "graph"])
def test_backward_normalize_per_call(use_graph):
    """backward(normalize=...) chooses the 1/N scaling per call: it equals the
    plan-level choice bit for bit, in either direction of the override, with
    direct launches and with graph replay."""
    shape = (12, 20, 30)
    for dtype in (C128, C64):
        x = gen(shape, dtype, synth.SEED + 3)
        plain = offt.Plan(shape, dtype=dtype, use_graph=use_graph)
        scaled = offt.Plan(shape, dtype=dtype, normalize_inverse=True, use_graph=use_graph)
        y = plain.forward(x)
        z_plain = plain.backward(y)
        z_scaled = scaled.backward(y)
        z1 = plain.backward(y, normalize=True)
        z0 = scaled.backward(y, normalize=False)
        zd = scaled.backward(y, normalize=None)
        torch.cuda.synchronize()
        assert torch.equal(z1, z_scaled) and torch.equal(zd, z_scaled) and torch.equal(z0, z_plain)
        assert oracle.rel_l2(host(z1), host(x)) <= tol(x.numel(), dtype)
        ref = oracle.fft3(host(y).astype(np.complex128), oracle.BACKWARD)
        assert oracle.rel_l2(host(z0), ref) <= tol(x.numel(), dtype)
        plain.close()
        scaled.close()


def _with_mode(plan, mode):
    """The plan string with every axis forced to access mode "/s" or "/c"."""
    def fix(spec):
        return spec if spec == "1" else spec + mode
    halves = []
    for half in plan.split("|"):
        parts = []
        for t in half.split(";"):
            k, v = t.split("=", 1)
            parts.append(f"{k}={fix(v)}" if k in "abcde" and len(k) == 1 else t)
        halves.append(";".join(parts))
    return "|".join(halves)


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape,layout", [((64, 48, 80), "natural"), ((30, 512, 12), "natural"),
                                          ((40, 24, 60), "cba"), ((6, 8, 10, 12), "natural")])
def test_streaming_and_cached_accesses_are_bit_identical(shape, layout, dtype):
    """Streaming ("/s") and cached ("/c") grid-data accesses only change how
    the loads and stores use the caches: the same plan gives the same bits
    either way, in every pass kind (contiguous, strided, transposing,
    4-axis), and matches the oracle."""
    x = gen(shape, dtype, synth.SEED + 11)
    heur = offt.Plan(shape, dtype=dtype, layout=layout)
    base = heur.describe()
    heur.close()
    outs = {}
    for mode in ("/s", "/c"):
        plan = offt.Plan(shape, dtype=dtype, layout=layout, tune="forced", forced_plan=_with_mode(base, mode))
        assert plan.describe() == _with_mode(base, mode)
        outs[mode] = plan.forward(x)
        torch.cuda.synchronize()
        plan.close()
    assert torch.equal(outs["/s"], outs["/c"])
    xh = host(x).astype(np.complex128)
    if len(shape) == 4:
        from oracle import ndim
        ref = ndim.fftn(xh)
    elif layout == "cba":
        from oracle import layout as lay
        ref = lay.fft3_reversed(xh)
    else:
        ref = oracle.fft3(xh)
    assert oracle.rel_l2(host(outs["/s"]), ref) <= tol(x.numel(), dtype)


def test_tensor_checks():
    plan = offt.Plan((8, 8, 8), dtype=C64)
    with pytest.raises(ValueError):
        plan.forward(torch.zeros((8, 8, 8), dtype=C128, device="cuda"))
    with pytest.raises(ValueError):
        plan.forward(torch.zeros((8, 8, 16), dtype=C64, device="cuda")[:, :, :8])
    with pytest.raises(ValueError):
        plan.forward(torch.zeros((8, 8, 8), dtype=C64))


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shape,axes", [((64, 48, 80), "abc"), ((30, 9, 512), "c"), ((512, 6, 10), "a"),
                                        ((5 * 9, 3, 64), "abc")])
def test_xcd_tile_order_is_bit_identical(shape, axes, dtype):
    """The XCD-contiguous tile order ("/x") only changes which workgroup runs
    which tile: tile counts divisible by 8 and not, contiguous and strided
    passes, exchanges in parts, and the transposing pass give the same bits."""
    x = gen(shape, dtype)
    base = offt.default_plan_string(shape, dtype).replace("/x", "")     # launch order everywhere
    fields = base.split(";")
    marked = ";".join(f + "/x" if f[0] in axes and f[1] == "=" and f[2:] != "1" else f for f in fields)
    assert marked != base
    p0 = offt.Plan(shape, dtype=dtype, tune="forced", forced_plan=base)
    p1 = offt.Plan(shape, dtype=dtype, tune="forced", forced_plan=marked)
    assert p1.describe() == marked
    y0, y1 = p0.forward(x), p1.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    assert oracle.rel_l2(host(y1), ref3(host(x))) <= tol(x.numel(), dtype)
    # the transposing pass of the reversed order
    rs = shape[::-1]
    fwd = offt.plan_string(shape, dtype, "cba").split("|")[0].replace("/x", "")
    bwd = offt.plan_string(rs, dtype, "cba").split("|")[0]
    if "rev=" in fwd:
        tax = fwd.split("rev=")[1][0]
        fx = ";".join(f + "/x" if f.startswith(tax + "=") else f for f in fwd.split(";"))
        r0 = offt.Plan(shape, dtype=dtype, layout="cba", tune="forced", forced_plan=fwd + "|" + bwd)
        r1 = offt.Plan(shape, dtype=dtype, layout="cba", tune="forced", forced_plan=fx + "|" + bwd)
        z0, z1 = r0.forward(x), r1.forward(x)
        torch.cuda.synchronize()
        assert torch.equal(z0, z1)
