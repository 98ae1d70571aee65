"""CPU emulation of the library's device code (no GPU).

tests/emu/hip_emu.h supplies just enough of HIP for fft_device.hpp and
many_device.hpp to compile as host C++; one workgroup runs as CPU threads
sharing a barrier that reports threads reaching different numbers of
__syncthreads() instead of hanging.  Built with AddressSanitizer and
UBSan, so an out-of-bounds LDS or global access in the tile code fails the
test.  The persistent batch loop runs as a single workgroup, which takes the
work items in order, so every dependency is met by construction; the check is
on the tile code, the barrier structure and the bookkeeping.
"""
import fcntl
import hashlib
import importlib.util
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

import oracle
import paper_1501_07350_amd as offt
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
CSRC = os.path.join(os.path.dirname(HERE), "paper_1501_07350_amd", "csrc")
BUILD = os.path.join(EMU, "_build")


def _load(name):
    spec = importlib.util.spec_from_file_location(name + "_emu", os.path.join(CSRC, name + ".py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def gen_kernels():
    return _load("gen_kernels")


def many_cases(prec, which):
    """Kernel cases of one of the library's batch executors (csrc/gen_many.py)."""
    return _load("gen_many").many_cases(prec, which)


# cases the emulated stand-alone passes add to the executor's: the radix-32
# butterfly, as a single stage and before a radix-2 stage
EXTRA_PASS_CASES = [(32, [32], 1), (64, [32, 2], 2)]


def plain_cases(gk, prec):
    return many_cases(prec, "all") + EXTRA_PASS_CASES


@pytest.fixture(scope="module")
def emu_binary():
    # the driver is built once per content (generated cases, driver, device
    # headers, command) into BUILD/<hash>; parallel test processes wait on a
    # lock for the one that builds it
    gk = gen_kernels()
    os.makedirs(BUILD, exist_ok=True)
    lines = ["template <typename V> struct EmuDispatch;"]
    for vt, prec in (("double2", "f64"), ("float2", "f32")):
        lines.append(f"template <> struct EmuDispatch<{vt}> {{")
        lines.append(f"  void operator()(int kid, const PassArgs& a, {vt}* lds, int64_t l0) const {{")
        lines.append("    switch (kid) {")
        for i, (L, seq, tpl) in enumerate(many_cases(prec, "all")):
            lines.append(f"      case {i}: pass_tile_coherent<{vt}, {L}, {tpl}, {', '.join(map(str, seq))}>(a, lds, l0); break;")
        lines.append("      default: break;\n    }\n  }\n};")
    lines.append("template <typename V> struct EmuDispatchPlain;")
    for vt, prec in (("double2", "f64"), ("float2", "f32")):
        lines.append(f"template <> struct EmuDispatchPlain<{vt}> {{")
        lines.append(f"  void operator()(int kid, int P, const PassArgs& a, {vt}* lds, int64_t l0) const {{")
        lines.append("    switch (kid) {")
        for i, (L, seq, tpl) in enumerate(plain_cases(gk, prec)):
            rad = ", ".join(map(str, seq))
            body = " else ".join([f"if (a.mode >= 2 && P == {P}) pass_tile_transpose<{vt}, {L}, {tpl}, {P}, {rad}>(a, lds, l0);"
                                  for P in (1, 2, 4) if gk.splits(L, seq, P) and gk.transposes(seq, P)] +
                                 [f"if (a.mode < 2 && P == {P}) pass_tile_parts<{vt}, {L}, {tpl}, {P}, {rad}>(a, lds, l0);"
                                  for P in (1, 2, 4) if gk.splits(L, seq, P)])
            lines.append(f"      case {i}: {body} break;")
        lines.append("      default: break;\n    }\n  }\n};")
    # the level kernels' and the level-synchronous form's dispatch over the
    # batch executor's cases, and the level kernels' over the every-length
    # executor's (plain stores)
    for struct, which in (("EmuLevelDispatch", "batch"), ("EmuLevelDispatchAll", "all")):
        lines.insert(0, f"template <typename V> struct {struct};")
        for vt, prec in (("double2", "f64"), ("float2", "f32")):
            lines.append(f"template <> struct {struct}<{vt}> {{")
            lines.append(f"  void operator()(int kid, const PassArgs& a, {vt}* lds, int64_t l0) const {{")
            lines.append("    switch (kid) {")
            for i, (L, seq, tpl) in enumerate(many_cases(prec, which)):
                lines.append(f"      case {i}: pass_tile<{vt}, {L}, {tpl}, {', '.join(map(str, seq))}>(a, lds, l0); break;")
            lines.append("      default: break;\n    }\n  }\n};")
    cases_text = "namespace offt {\n" + "\n".join(lines) + "\n}\n"
    flags = ["-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    h = hashlib.sha256(cases_text.encode() + " ".join(flags).encode())
    for d in (EMU, CSRC):
        for name in sorted(os.listdir(d)):
            if name.endswith((".h", ".hpp", ".cpp")):
                with open(os.path.join(d, name), "rb") as f:
                    h.update(name.encode() + f.read())
    build = os.path.join(BUILD, h.hexdigest()[:16])
    exe = os.path.join(build, "emu_driver")
    with open(os.path.join(BUILD, "lock"), "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        try:
            if not os.path.exists(exe):
                # drivers of older sources are not needed any more
                for old in os.listdir(BUILD):
                    if old != "lock" and os.path.isdir(os.path.join(BUILD, old)):
                        shutil.rmtree(os.path.join(BUILD, old), ignore_errors=True)
                os.makedirs(build, exist_ok=True)
                with open(os.path.join(build, "emu_cases.inc"), "w") as f:
                    f.write(cases_text)
                cmd = ["g++"] + flags + ["-I", EMU, "-I", build, "-I", CSRC, os.path.join(EMU, "emu_driver.cpp"),
                                         "-o", exe + ".tmp"]
                subprocess.run(cmd, check=True)
                os.replace(exe + ".tmp", exe)
        finally:
            fcntl.flock(lk, fcntl.LOCK_UN)
    yield exe


ORDER_NAMES = ["abc", "cab", "cba"]
# the flow's four transposes: forward abc -> cab -> cba, backward cba -> cab -> abc
TRANSPOSES = [(0, 1), (1, 2), (2, 1), (1, 0)]
# (shape, Np): 1-D and 2-D decompositions, unit axes, Np not dividing the lengths
ROUTE_CASES = [((8, 8, 8), 3), ((4, 6, 8), 5), ((4, 6, 8), 8), ((2, 12, 3), 6), ((1, 4, 6), 3), ((5, 1, 12), 4),
               ((6, 10, 9), 4), ((3, 5, 7), 1)]


@pytest.mark.parametrize("per_chunk", [0, 1], ids=["unpack_all", "unpack_per_chunk"])
@pytest.mark.parametrize("tr", TRANSPOSES, ids=lambda t: f"{ORDER_NAMES[t[0]]}-{ORDER_NAMES[t[1]]}")
@pytest.mark.parametrize("case", ROUTE_CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}-np{c[1]}")
def test_emulated_distributed_exchange(emu_binary, case, tr, per_chunk):
    """One exchange of the distributed flow with the library's own tables and
    pack / copy / unpack code, under AddressSanitizer on exactly sized
    arrays: every element lands where the reference oracle/dist.py puts it,
    and the chunk sizes equal the reference's counts."""
    from oracle import dist
    shape, np_ = case
    src_o, dst_o = ORDER_NAMES[tr[0]], ORDER_NAMES[tr[1]]
    r = subprocess.run([emu_binary, "route", *map(str, shape), str(np_), str(tr[0]), str(tr[1]), str(per_chunk)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[:500], r.stderr[-3000:])
    lines = r.stdout.splitlines()
    assert lines[0] == "OK"
    counts = np.array([[int(v) for v in ln.split()] for ln in lines[1:1 + np_]])
    out = np.array([int(v) for v in lines[1 + np_:]])
    n = int(np.prod(shape))
    code = np.arange(n, dtype=np.float64).astype(np.complex128)    # O_in index of every element
    local = [code[s:e] for s, e in dist.blocks(shape, src_o, np_)]
    want, m = dist.exchange(local, shape, src_o, dst_o, np_)
    assert np.array_equal(out, dist.gather(want).real.astype(np.int64))
    assert np.array_equal(counts, m)


def lds_idx(j):
    return j + (j >> 4)


def pitch(L):
    return (lds_idx(L - 1) + 1) | 1


def tile_lds_elems(W, L):
    return W * pitch(L) + L


def plan_passes(dims, dtype):
    """Passes of the heuristic plan, parsed from the library's plan string."""
    s = offt.default_plan_string(dims, dtype)
    fields = dict(kv.split("=") for kv in s.split(";"))
    out = []
    for ch in fields["order"]:
        ax = "abc".index(ch)
        L = dims[ax]
        if L <= 1:
            continue
        rad_s, *rest = fields[ch].split("/")
        rest = [t for t in rest if t != "x" and not t.startswith("p")]   # tile order, parts
        seq = [int(r) for r in rad_s.split("x")]
        W = int(rest[0])
        tpl = int(rest[1]) if len(rest) > 1 else L // max(seq)
        M2 = int(np.prod(dims[ax + 1:])) if ax < 2 else 1
        M1 = int(np.prod(dims[:ax])) if ax > 0 else 1
        out.append(dict(L=L, seq=seq, W=W, tpl=tpl, M1=M1, M2=M2, mode=1 if M2 > 1 else 0))
    return out


def grid_args(dims_list, dtype, which="all"):
    """Driver arguments of a batch: each grid's offset in the packed buffer
    (256-byte aligned, as the library packs) and its heuristic passes with
    their kernel cases; the driver builds the segment table with the
    library's own code (many_tables.hpp).  Returns (args, offsets, total,
    passes per grid)."""
    prec = "f64" if dtype == torch.complex128 else "f32"
    es = 16 if prec == "f64" else 8
    cases = many_cases(prec, which)
    align = 256 // es
    offs, off = [], 0
    for d in dims_list:
        offs.append(off)
        off += int(np.prod(d))
        off = (off + align - 1) // align * align
    total = off
    args = [str(len(dims_list))]
    npass = []
    for g, d in enumerate(dims_list):
        ps = plan_passes(d, dtype)
        npass.append(len(ps))
        args += [str(offs[g]), str(len(ps))]
        for p in ps:
            kid = cases.index((p["L"], p["seq"], p["tpl"]))
            args += [str(p["L"]), str(kid), str(p["mode"]), str(p["M1"] * p["M2"]), str(p["M2"]), str(p["tpl"])]
    args.append(str(total))
    return args, offs, total, npass


def run_many(exe, dims_list, dtype, nwg=1, sync=False, levels=False, which=None, group_bytes=None):
    """Run the batch loop of one form on the emulator: the work-queue loop
    over the every-length executor's cases, the level-synchronous loop or
    the level kernels over the batch executor's (the level kernels also over
    the every-length executor's, which="all")."""
    which = which or ("batch" if (sync or levels) else "all")
    args, offs, total, _ = grid_args(dims_list, dtype, which)
    code = "0" if dtype == torch.complex128 else "1"
    mode = ("levels_all" if which == "all" else "levels") if levels else "sync" if sync else "many"
    env = dict(os.environ, EMU_GROUP_BYTES=str(group_bytes)) if group_bytes else None
    r = subprocess.run([exe, mode, code, str(nwg)] + args, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[:500], r.stderr[-3000:])
    lines = r.stdout.splitlines()
    if group_bytes:
        assert lines[0].startswith("GROUPS"), lines[0]
        groups = int(lines[0].split()[1])
        lines = lines[1:]
    assert lines[0].startswith("OK"), lines[0]
    vals = np.array([[float(a) for a in ln.split()] for ln in lines[1:]])
    out = vals[:, 0] + 1j * vals[:, 1]
    assert out.size == total
    # the driver's input: in[i] = sin(0.37 i + 0.1) + i cos(0.91 i), rounded to the precision
    i = np.arange(total)
    xin = np.sin(0.37 * i + 0.1) + 1j * np.cos(0.91 * i)
    if dtype == torch.complex64:
        xin = xin.astype(np.complex64).astype(np.complex128)
    for g, d in enumerate(dims_list):
        n = int(np.prod(d))
        if n == 1:
            continue   # a one-point grid has no pass (the library copies it)
        x = xin[offs[g]:offs[g] + n].reshape(d)
        y = out[offs[g]:offs[g] + n].reshape(d)
        e = oracle.rel_l2(y, oracle.fft3(x))
        assert e <= oracle.tolerance(n, dtype == torch.complex64), (d, e)
    return groups if group_bytes else None


MIXED = [(2, 3, 5), (1, 1, 1), (9, 25, 27), (100, 4, 6), (48, 60, 64), (16, 1, 8), (5, 5, 5)]


@pytest.mark.parametrize("which", ["all", "batch"])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
def test_library_tables_invariants(emu_binary, dtype, which):
    """The segment table the library builds (many_tables.hpp, printed by the
    driver without running anything) for the mixed batch that once stopped
    and for the batch executor's lengths: every dependency is the same grid's
    segment one level lower, which is not a last pass and publishes one count
    per work item; first passes wait for nothing; every tile fits the
    launch's LDS and the workgroup's threads; items and tiles are numbered
    contiguously level by level."""
    dims = MIXED if which == "all" else [tuple(v if v in (1, 48, 60, 64) else 64 for v in d) for d in SYNC_DIMS]
    args, offs, total, npass = grid_args(dims, dtype, which)
    code = "0" if dtype == torch.complex128 else "1"
    r = subprocess.run([emu_binary, "tables", code, "1"] + args, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = r.stdout.splitlines()
    head = lines[0].split()
    assert head[0] == "TABLES"
    nseg, items, tiles, lds, threads, per_item = (int(head[i]) for i in (1, 3, 5, 8, 10, 12))
    segs = [list(map(int, ln.split())) for ln in lines[1:1 + nseg]]
    levels = [list(map(int, ln.split()[2:])) for ln in lines[1 + nseg:]]
    prec = "f64" if dtype == torch.complex128 else "f32"
    cases = many_cases(prec, which)
    es = 16 if prec == "f64" else 8
    assert nseg == sum(npass)
    item_next, tile_next = 0, 0
    for (i, lvl, off, nlines, M2, kid, logW, mode, ntiles, nitems, first, last, dep, item_base, tile_base) in segs:
        g = offs.index(off)
        L, seq, tpl = cases[kid]
        W = 1 << logW
        assert W * tpl <= threads
        assert tile_lds_elems(W, L) * es <= lds
        assert ntiles == (nlines + W - 1) // W and nitems == (ntiles + per_item - 1) // per_item
        assert first == (lvl == 0) and last == (lvl == npass[g] - 1)
        if lvl == 0:
            assert dep == -1
        else:
            d = segs[dep]
            assert d[2] == off and d[1] == lvl - 1 and d[11] == 0   # same grid, one level lower, not a last pass
        assert item_base == item_next and tile_base == tile_next   # contiguous, level-major order
        item_next += nitems
        tile_next += ntiles
    assert item_next == items and tile_next == tiles
    # level boundaries: the first item and tile of each level
    for lvl in range(3):
        first_seg = next((s for s in segs if s[1] == lvl), None)
        if first_seg is not None:
            assert levels[lvl] == [first_seg[13], first_seg[14]]
    assert levels[3] == [items, tiles]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
def test_emulated_persistent_loop_mixed_batch(emu_binary, dtype):
    run_many(emu_binary, MIXED, dtype)


@pytest.mark.parametrize("nwg", [2, 3])
def test_emulated_concurrent_workgroups_mixed_batch(emu_binary, nwg):
    """Several workgroups (one process each) race on the queue and the
    dependency counters in shared memory."""
    run_many(emu_binary, MIXED, torch.complex64, nwg=nwg)


def test_emulated_unmet_dependency_ends_within_one_spin_limit(emu_binary):
    """A dependency that is never met (the second pass of the largest grid
    made to wait on a grid's last pass, which publishes nothing): the first
    wait gives up after its spin limit and raises the error flag, and every
    later item then skips its wait and its tile, so the loop ends after about
    one spin limit instead of one per waiting item."""
    import time
    args, _, _, npass = grid_args(MIXED, torch.complex64, "all")
    # segment order of the library's table: level-major, grid order within a level
    order = [(lvl, g) for lvl in range(3) for g in range(len(MIXED)) if lvl < npass[g]]
    big = MIXED.index((48, 60, 64))
    waiting = order.index((1, big))
    last = next(i for i, (lvl, g) in enumerate(order) if lvl == npass[g] - 1 and g != big)
    t0 = time.perf_counter()
    r = subprocess.run([emu_binary, "many", "1", "1"] + args, capture_output=True, text=True, timeout=600)
    t_normal = time.perf_counter() - t0
    assert r.returncode == 0, r.stdout[:300]
    spin = 20000   # polls of at least 20 us each in the emulation: >= 0.4 s per full wait
    t0 = time.perf_counter()
    r = subprocess.run([emu_binary, "many", "1", "1"] + args + [str(waiting), str(last)], capture_output=True,
                       text=True, timeout=600, env={**os.environ, "EMU_SPIN_LIMIT": str(spin)})
    t_unmet = time.perf_counter() - t0
    assert r.returncode == 1 and "err=1" in r.stdout, (r.stdout[:300], r.stderr[-2000:])
    nitems = int(r.stdout.split("waiting_items=")[1].split()[0])
    assert nitems >= 8
    # one full wait beyond the normal run; one wait per waiting item would add
    # at least nitems * 0.4 s
    assert t_unmet < t_normal + 0.5 * nitems * spin * 20e-6, (t_normal, t_unmet, nitems)


def test_emulated_persistent_loop_batch_lengths(emu_binary):
    dims = synth.uneven_batch_dims(4, key=synth.KEY_DIMS + 99)
    dims = [tuple(min(v, 64) for v in d) for d in dims]   # small enough for CPU threads
    run_many(emu_binary, dims, torch.complex64)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
def test_emulated_every_case_once(emu_binary, dtype):
    """Every kernel case of the executor on a small strided and contiguous pass."""
    prec = "f64" if dtype == torch.complex128 else "f32"
    lengths = sorted({L for L, _, _ in many_cases(prec, "all")})
    dims = [d for L in lengths for d in ((L, 1, 3), (1, 2, L))]
    run_many(emu_binary, dims, dtype)


def run_pass(exe, dtype, L, seq, tpl, M1, M2, logW, logP):
    """One stand-alone axis pass through the emulated tile code, checked line
    by line against the oracle's naive DFT."""
    gk = gen_kernels()
    prec = "f64" if dtype == torch.complex128 else "f32"
    kid = plain_cases(gk, prec).index((L, seq, tpl))
    code = "0" if dtype == torch.complex128 else "1"
    args = [exe, "pass", code] + [str(v) for v in (kid, L, M1, M2, logW, logP, tpl)]
    r = subprocess.run(args, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[:500], r.stderr[-3000:])
    lines = r.stdout.splitlines()
    assert lines[0].startswith("OK"), lines[0]
    vals = np.array([[float(a) for a in ln.split()] for ln in lines[1:]])
    out = (vals[:, 0] + 1j * vals[:, 1]).reshape(M1, L, M2)
    i = np.arange(M1 * L * M2)
    x = np.sin(0.37 * i + 0.1) + 1j * np.cos(0.91 * i)
    if dtype == torch.complex64:
        x = x.astype(np.complex64).astype(np.complex128)
    x = x.reshape(M1, L, M2)
    lines_in = x.transpose(0, 2, 1).reshape(M1 * M2, L)        # every line along the pass axis
    want = oracle.fft1_lines(lines_in, method=0)               # naive DFT of each line
    got = out.transpose(0, 2, 1).reshape(M1 * M2, L)
    worst = max(oracle.rel_l2(got[i], want[i]) for i in range(M1 * M2))
    assert worst <= oracle.tolerance(L, dtype == torch.complex64), worst


def run_pass_block(exe, dtype, L, seq, tpl, M1, M2, logW, logP, logw, ld, off):
    """A strided pass restricted to one column block (2^logw columns from
    `off` in every row of `ld` columns): the block's lines match the naive
    DFT, every other element is left untouched (zero)."""
    gk = gen_kernels()
    prec = "f64" if dtype == torch.complex128 else "f32"
    kid = plain_cases(gk, prec).index((L, seq, tpl))
    code = "0" if dtype == torch.complex128 else "1"
    args = [exe, "pass", code] + [str(v) for v in (kid, L, M1, M2, logW, logP, tpl)]
    env = dict(os.environ, EMU_BLK=f"{logw} {ld} {off}")
    r = subprocess.run(args, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[:500], r.stderr[-3000:])
    lines = r.stdout.splitlines()
    assert lines[0].startswith("OK"), lines[0]
    vals = np.array([[float(a) for a in ln.split()] for ln in lines[1:]])
    out = (vals[:, 0] + 1j * vals[:, 1]).reshape(M1, L, M2)
    i = np.arange(M1 * L * M2)
    x = np.sin(0.37 * i + 0.1) + 1j * np.cos(0.91 * i)
    if dtype == torch.complex64:
        x = x.astype(np.complex64).astype(np.complex128)
    x = x.reshape(M1, L, M2)
    m2 = np.arange(M2)
    inside = ((m2 % ld) >= off) & ((m2 % ld) < off + (1 << logw))
    lines_in = x[:, :, inside].transpose(0, 2, 1).reshape(-1, L)
    want = oracle.fft1_lines(lines_in, method=0)
    got = out[:, :, inside].transpose(0, 2, 1).reshape(-1, L)
    worst = max(oracle.rel_l2(got[k], want[k]) for k in range(got.shape[0]))
    assert worst <= oracle.tolerance(L, dtype == torch.complex64), worst
    assert not np.any(out[:, :, ~inside]), "elements outside the block were written"


def run_tpass(exe, dtype, L, seq, tpl, M1, X, Y, logW, mode, logP=0):
    """One transposing pass through the emulated tile code: line l = m1*M2 + m2
    (M2 = X*Y) is strided in the [M1][L][M2] view and the contiguous row
    m1*M2 + (m2 mod X)*Y + m2 div X of the other buffer; mode 3 reads the
    strided side, mode 2 the rows.  Checked line by line against the
    oracle's naive DFT."""
    gk = gen_kernels()
    prec = "f64" if dtype == torch.complex128 else "f32"
    kid = plain_cases(gk, prec).index((L, seq, tpl))
    code = "0" if dtype == torch.complex128 else "1"
    M2 = X * Y
    args = [exe, "pass", code] + [str(v) for v in (kid, L, M1, M2, logW, logP, tpl, mode, X, Y)]
    r = subprocess.run(args, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[:500], r.stderr[-3000:])
    lines = r.stdout.splitlines()
    assert lines[0].startswith("OK"), lines[0]
    vals = np.array([[float(a) for a in ln.split()] for ln in lines[1:]])
    out = vals[:, 0] + 1j * vals[:, 1]
    i = np.arange(M1 * L * M2)
    x = np.sin(0.37 * i + 0.1) + 1j * np.cos(0.91 * i)
    if dtype == torch.complex64:
        x = x.astype(np.complex64).astype(np.complex128)
    m1, m2 = np.divmod(np.arange(M1 * M2), M2)
    row = m1 * M2 + (m2 % X) * Y + m2 // X
    assert sorted(row) == list(range(M1 * M2))      # the row map is a permutation
    strided_in = x.reshape(M1, L, M2).transpose(0, 2, 1).reshape(M1 * M2, L)
    if mode == 3:
        want = oracle.fft1_lines(strided_in, method=0)
        got = out.reshape(M1 * M2, L)[row]
    else:
        want = oracle.fft1_lines(x.reshape(M1 * M2, L)[row], method=0)
        got = out.reshape(M1, L, M2).transpose(0, 2, 1).reshape(M1 * M2, L)
    worst = max(oracle.rel_l2(got[k], want[k]) for k in range(M1 * M2))
    assert worst <= oracle.tolerance(L, dtype == torch.complex64), worst


# (L, radix sequence, threads per line, M1, X, Y, logW): transposing passes
# with a ragged last tile (M1*X*Y not a multiple of W), several batches (M1),
# X or Y of 1, multi-stage and single-stage sequences
TPASS_CASES = [
    (64, [8, 8], 8, 2, 5, 4, 4),
    (60, [5, 4, 3], 12, 3, 7, 2, 3),
    (128, [16, 8], 8, 1, 12, 3, 5),
    (48, [16, 3], 3, 2, 1, 9, 4),
    (32, [32], 1, 3, 6, 1, 2),
    (160, [16, 5, 2], 10, 1, 4, 5, 3),
]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("case", TPASS_CASES, ids=lambda c: f"L{c[0]}-{'x'.join(map(str, c[1]))}-M1_{c[3]}-X{c[4]}-Y{c[5]}-W{1 << c[6]}")
def test_emulated_transposing_pass(emu_binary, dtype, mode, case):
    L, seq, tpl, M1, X, Y, logW = case
    run_tpass(emu_binary, dtype, L, seq, tpl, M1, X, Y, logW, mode)


# transposing tiles whose exchanges and row side run in 2 and 4 parts:
# (L, radix sequence, threads per line, M1, X, Y, logW, logP), ragged tails,
# butterflies per thread of one and of several
TPASS_PART_CASES = [
    (64, [8, 8], 8, 2, 5, 4, 4, 1),
    (64, [8, 8], 8, 1, 6, 3, 3, 2),
    (128, [16, 8], 8, 1, 12, 3, 5, 1),
    (128, [8, 4, 4], 16, 3, 4, 5, 3, 1),
    (128, [8, 4, 4], 16, 1, 7, 3, 4, 2),
]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("case", TPASS_PART_CASES,
                         ids=lambda c: f"L{c[0]}-{'x'.join(map(str, c[1]))}-X{c[4]}-Y{c[5]}-W{1 << c[6]}-P{1 << c[7]}")
def test_emulated_transposing_pass_in_parts(emu_binary, dtype, mode, case):
    L, seq, tpl, M1, X, Y, logW, logP = case
    gk = gen_kernels()
    assert gk.splits(L, seq, 1 << logP) and gk.transposes(seq, 1 << logP)
    run_tpass(emu_binary, dtype, L, seq, tpl, M1, X, Y, logW, mode, logP)


# (L, radix sequence, threads per line, M1, M2, logW, logP): strided passes
# whose LDS exchanges run in 2 and 4 parts, with a ragged last tile (M1*M2
# not a multiple of W); the 2-stage and 3-stage sequences cover butterflies
# per thread of 1 and several, where the part of a butterfly is decided per
# thread and per register slot.
PART_CASES = [
    (64, [8, 8], 8, 2, 24, 4, 1),
    (64, [8, 8], 8, 2, 24, 4, 2),
    (128, [16, 8], 8, 1, 40, 5, 1),
    (128, [16, 8], 8, 1, 72, 5, 2),
    (128, [8, 4, 4], 16, 3, 20, 4, 1),
    (128, [8, 4, 4], 16, 3, 20, 3, 2),
]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
@pytest.mark.parametrize("case", PART_CASES, ids=lambda c: f"L{c[0]}-{'x'.join(map(str, c[1]))}-M2_{c[4]}-W{1 << c[5]}-P{1 << c[6]}")
def test_emulated_strided_pass_exchange_parts(emu_binary, dtype, case):
    L, seq, tpl, M1, M2, logW, logP = case
    assert gen_kernels().splits(L, seq, 1 << logP)
    run_pass(emu_binary, dtype, L, seq, tpl, M1, M2, logW, logP)


# the radix-32 butterfly: contiguous lines (M2 = 1) and strided lines with a
# ragged last tile, single stage and followed by a radix-2 stage
RADIX32_CASES = [
    (32, [32], 1, 7, 1, 2, 0),
    (32, [32], 1, 2, 12, 3, 0),
    (64, [32, 2], 2, 5, 1, 3, 0),
    (64, [32, 2], 2, 1, 40, 5, 0),
    (64, [32, 2], 2, 1, 40, 5, 1),
]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
@pytest.mark.parametrize("case", RADIX32_CASES, ids=lambda c: f"L{c[0]}-{'x'.join(map(str, c[1]))}-M1_{c[3]}-M2_{c[4]}-P{1 << c[6]}")
def test_emulated_radix32_pass(emu_binary, dtype, case):
    L, seq, tpl, M1, M2, logW, logP = case
    assert gen_kernels().splits(L, seq, 1 << logP)
    run_pass(emu_binary, dtype, L, seq, tpl, M1, M2, logW, logP)


# grids of the batch executor's lengths, with unit axes (one- and two-pass grids)
SYNC_DIMS = [(48, 1, 60), (1, 64, 1), (16 * 3, 60, 64), (80, 96, 1), (1, 1, 1), (120, 1, 128)]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
@pytest.mark.parametrize("nwg", [1, 3, 9])
def test_emulated_level_synchronous_body(emu_binary, dtype, nwg):
    """The level-synchronous persistent body: nwg workgroups (one process
    each) take the level's tiles round-robin, grid barriers between levels in
    shared memory; every workgroup arrives at both barriers, no wait times
    out, and every grid matches the oracle."""
    dims = [tuple(min(v, 64) if v > 1 else 1 for v in d) for d in SYNC_DIMS]
    dims = [tuple(v if v in (1, 48, 60, 64) else 64 for v in d) for d in dims]
    run_many(emu_binary, dims, dtype, nwg=nwg, sync=True)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
def test_emulated_level_kernels(emu_binary, dtype):
    """The level kernels' body: one workgroup per tile, each finding its
    segment in the library's tile table, level after level; every grid
    matches the oracle."""
    dims = [tuple(min(v, 64) if v > 1 else 1 for v in d) for d in SYNC_DIMS]
    dims = [tuple(v if v in (1, 48, 60, 64) else 64 for v in d) for d in dims]
    run_many(emu_binary, dims, dtype, levels=True)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
def test_emulated_level_kernels_every_length_executor(emu_binary, dtype):
    """The level kernels of the every-length executor over the mixed batch of
    small lengths (2, 3, 5, 9, 25, 27, 100, 16, 8, 48, 60, 64, and a 1x1x1
    grid): exactly the launch's LDS, the library's tables; every grid
    matches the oracle."""
    run_many(emu_binary, MIXED, dtype, levels=True, which="all")


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
@pytest.mark.parametrize("case", [
    # (L, seq, tpl, M1, M2, logW, logP, logw, ld, off): a pass along a over 6 rows
    # of 32 columns, blocks of 8 and 16; a pass along b (M2 = ld); a 2-part exchange
    (16, [16], 1, 1, 6 * 32, 3, 0, 3, 32, 16),
    (16, [16], 1, 1, 6 * 32, 2, 0, 4, 32, 0),
    (12, [4, 3], 3, 3, 32, 3, 0, 4, 32, 16),
    (64, [8, 8], 8, 2, 3 * 16, 2, 1, 3, 16, 8),
], ids=lambda v: str(v))
def test_emulated_column_block_pass(emu_binary, dtype, case):
    """The column-block addressing of strided passes (the column-block
    schedule): only the block's lines are transformed, each exactly."""
    L, seq, tpl, M1, M2, logW, logP, logw, ld, off = case
    assert (1 << logW) <= (1 << logw) and M2 % ld == 0 and off + (1 << logw) <= ld
    run_pass_block(emu_binary, dtype, L, seq, tpl, M1, M2, logW, logP, logw, ld, off)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
@pytest.mark.parametrize("group_bytes", [1, 300_000, 10 ** 12])
def test_emulated_grouped_level_schedule(emu_binary, dtype, group_bytes):
    """The grouped level schedule with the library's own group builder: the
    level kernels' body over each (group, level) range of the tile map, one
    group after the other -- one grid per group, a few grids per group, one
    group -- every grid matches the oracle."""
    dims = MIXED
    groups = run_many(emu_binary, dims, dtype, levels=True, which="all", group_bytes=group_bytes)
    ngrids = sum(1 for d in dims if int(np.prod(d)) > 1)
    if group_bytes == 1:
        assert groups >= ngrids
    if group_bytes == 10 ** 12:
        assert groups == 1
