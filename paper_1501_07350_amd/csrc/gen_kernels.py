"""Generate the explicit instantiations of the pass kernels and their registry.

For every 2/3/5-smooth length L <= 1024 and both precisions, one kernel per
radix sequence is compiled.  Radix sequences: the power-of-two part of L is
split into as few stages as possible with radix <= 16 (balanced), a
variant with radix <= 8 (balanced) and a greedy one (radix-16 stages plus one
remainder stage), and for 512 and 1024 also two radix-32-sized stages; each
factor 5 and 3 is its own stage.  Stages
run largest radix first.  Threads per line = L / (largest radix), so the
largest-radix stage does one butterfly per thread.

Output: <outdir>/kernels_<prec>_<part>.hip, each holding a slice of the
instantiations and a table; <outdir>/registry_parts.inc lists the tables.
"""
from __future__ import annotations

import os
import sys

MAX_L = 1024
PARTS = 8  # translation units per precision (compiled in parallel)


def smooth(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def exponents(n):
    e = []
    for p in (2, 3, 5):
        k = 0
        while n % p == 0:
            n //= p
            k += 1
        e.append(k)
    return e


def split_pow2(p, maxbits):
    """Split 2^p into the fewest stages of at most 2^maxbits, balanced."""
    if p == 0:
        return []
    ns = -(-p // maxbits)
    base, extra = divmod(p, ns)
    bits = [base + (1 if i < extra else 0) for i in range(ns)]
    return [1 << b for b in bits]


def radix_seqs(L):
    """Radix sequences of L: the power-of-two part split balanced with radix
    <= 16, balanced with radix <= 8, greedily into radix-16 stages, and (for
    2^9 and 2^10, where it saves a stage and so an LDS exchange) balanced
    with radix <= 32; each 3 and 5 is its own stage."""
    if L == 1:
        return []
    p, q, r = exponents(L)
    seqs = []
    greedy = [16] * (p // 4) + ([1 << (p % 4)] if p % 4 else [])
    splits2 = [split_pow2(p, 4), split_pow2(p, 3), greedy]
    if p >= 9:
        splits2.append(split_pow2(p, 5))
    for twos in splits2:
        seq = sorted(twos + [5] * r + [3] * q, reverse=True)
        if seq not in seqs:
            seqs.append(seq)
    return seqs


def max_threads(prec, L=None, seq=None, tpl=None):
    """Launch bound of a stand-alone pass kernel: 512 threads for binary64;
    1024 for binary32, except the variants with half the threads per line
    (two largest-radix butterflies per thread), which get 512 so that their
    registers fit without spilling (a strided tile of 32 columns still fits:
    that is what they are for).  A few binary32 kernels of L = 1024 at the
    1024 bound, and binary64 ones of radix 32 x 32, still spill 8-76 bytes
    per lane; the tuner weighs them like any other candidate."""
    if prec != "f32":
        return 512
    if seq is not None and tpl < L // max(seq):
        return 512
    return 1024


def lengths():
    return [n for n in range(2, MAX_L + 1) if smooth(n)]


def splits(L, seq, P):
    """Whether every LDS exchange of the radix sequence can run in P parts:
    P divides the next radix and the span times radix of the stage before
    divides L/P (fft_device.hpp, exchange_splits)."""
    if P == 1:
        return True
    if len(seq) < 2 or L % P:
        return False
    ns = 1
    for r, r2 in zip(seq, seq[1:]):
        if r2 % P or (L // P) % (ns * r):
            return False
        ns *= r
    return True


# Launch bound of the transposing kernels in both precisions: their row table
# and row-side copy add registers, and at 1024 threads (128 registers) the
# binary32 ones would spill.
TRANSPOSE_MAX_THREADS = 512


def transposes(seq, P):
    """Whether a kernel also comes as a transposing pass: with P parts its row
    side moves part by part, which needs P to divide the first radix (rows
    in) and the last radix (rows out)."""
    return P == 1 or (seq[0] % P == 0 and seq[-1] % P == 0)


# Lengths whose strided tiles also get kernels with LDS exchanges in 2 and 4
# parts: a wide tile of these fills the LDS, and only part of each line then
# needs to be resident at a time.
PARTS_MIN_L = 256


def entries(prec="f64", parts=True):
    """(L, radix sequence, threads per line, parts).  The default thread count
    is L / (largest radix); binary32 kernels of L >= 384 also come with half
    as many threads per line (two largest-radix butterflies per thread), which
    lets a strided tile span 32 columns (256-byte rows) under the thread
    limit.  Kernels of L >= PARTS_MIN_L whose exchanges split also come with
    2 and 4 parts (strided lines only)."""
    out = []
    for L in lengths():
        for seq in radix_seqs(L):
            tpl = L // max(seq)
            tpls = [tpl] + ([tpl // 2] if prec == "f32" and L >= 384 and tpl % 2 == 0 else [])
            for t in tpls:
                out.append((L, seq, t, 1))
            if parts and L >= PARTS_MIN_L:
                for P in (2, 4):
                    if splits(L, seq, P):
                        for t in tpls:
                            out.append((L, seq, t, P))
    return out


def emit(outdir):
    os.makedirs(outdir, exist_ok=True)
    tables = []
    for prec, vt, dcode in (("f64", "double2", 0), ("f32", "float2", 1)):
        ents = entries(prec)
        for part in range(PARTS):
            mine = ents[part::PARTS]
            name = f"kernels_{prec}_{part}"
            lines = [
                "// generated by gen_kernels.py -- do not edit",
                '#include "offt_internal.h"',
                '#include "fft_kernel.hpp"',
                "namespace offt {",
                "namespace {",
                "template <int MAXT, int L, int TPL, int P, int... Rs>",
                "hipError_t launch_one(const PassArgs& a, int64_t nblocks, int threads, size_t lds, hipStream_t s) {",
                f"    auto* k = &fft_pass_kernel<{vt}, MAXT, L, TPL, P, Rs...>;",
                "    static size_t lds_set = 65536;",
                "    if (lds > lds_set) {",
                "        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);",
                "        if (e != hipSuccess) return e;",
                "        lds_set = lds;",
                "    }",
                "    hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(threads), lds, s, a);",
                "    return hipGetLastError();",
                "}",
                "template <int L, int TPL, int P, int... Rs>",
                "hipError_t launch_t_one(const PassArgs& a, int64_t nblocks, int threads, size_t lds, hipStream_t s) {",
                f"    auto* k = &fft_tpass_kernel<{vt}, {TRANSPOSE_MAX_THREADS}, L, TPL, P, Rs...>;",
                "    static size_t lds_set = 65536;",
                "    if (lds > lds_set) {",
                "        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);",
                "        if (e != hipSuccess) return e;",
                "        lds_set = lds;",
                "    }",
                "    hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(threads), lds, s, a);",
                "    return hipGetLastError();",
                "}",
                "}  // namespace",
                f"extern KernelEntry g_{name}[];",
                f"extern const int g_{name}_n;",
                f"KernelEntry g_{name}[] = {{",
            ]
            for L, seq, tpl, P in mine:
                rad = ", ".join(str(x) for x in seq)
                padded = ", ".join(str(x) for x in (seq + [0] * (8 - len(seq))))
                # whole-line kernels, and kernels in parts whose first and last
                # radix split into the parts, also come as transposing passes
                lt = f"&launch_t_one<{L}, {tpl}, {P}, {rad}>" if transposes(seq, P) else "nullptr"
                mt = max_threads(prec, L, seq, tpl)
                lines.append(f"    {{{dcode}, {L}, {len(seq)}, {{{padded}}}, {tpl}, {mt}, {P}, "
                             f"&launch_one<{mt}, {L}, {tpl}, {P}, {rad}>, {lt}}},")
            lines.append("};")
            lines.append(f"const int g_{name}_n = {len(mine)};")
            lines.append("}  // namespace offt")
            path = os.path.join(outdir, name + ".hip")
            text = "\n".join(lines) + "\n"
            if not os.path.exists(path) or open(path).read() != text:
                with open(path, "w") as f:
                    f.write(text)
            tables.append(name)
    inc = []
    for t in tables:
        inc.append(f"extern KernelEntry g_{t}[]; extern const int g_{t}_n;")
    inc.append("#define OFFT_REGISTRY_TABLES \\")
    inc.append(" \\\n".join(f"    {{g_{t}, g_{t}_n}}," for t in tables))
    text = "\n".join(inc) + "\n"
    path = os.path.join(outdir, "registry_parts.inc")
    if not os.path.exists(path) or open(path).read() != text:
        with open(path, "w") as f:
            f.write(text)
    return [os.path.join(outdir, t + ".hip") for t in tables]


if __name__ == "__main__":
    outdir = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__), "_gen")
    files = emit(outdir)
    print(len(entries("f64")), "+", len(entries("f32")), "kernels in", len(files), "files")
