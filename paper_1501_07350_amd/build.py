"""Build the HIP library libofft.so for gfx950 in-tree.

Steps: generate the pass-kernel instantiations (csrc/gen_kernels.py) and the
batch executors (csrc/gen_many.py), compile
every source under csrc/ and csrc/_gen/ with hipcc in parallel, link into
paper_1501_07350_amd/libofft.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "_gen")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libofft.so")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed fp32 ops disabled on purpose (see DESIGN notes on code generation)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fused within one source expression only, so that the
    # rounding of a tile's arithmetic does not depend on the kernel it is
    # inlined into (stand-alone passes and the batch executors give the same
    # bits)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def sources():
    sys.path.insert(0, CSRC)
    try:
        import gen_kernels  # noqa: E402
        import gen_many  # noqa: E402
    finally:
        sys.path.pop(0)
    gen = gen_kernels.emit(GEN) + gen_many.emit_many(GEN)
    own = sorted(
        os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp"))
    )
    return own + gen


def _compile(src: str, verbose: bool) -> str:
    base = os.path.splitext(os.path.basename(src))[0]
    sub = "gen_" if os.path.dirname(src) == GEN else ""
    obj = os.path.join(OBJ, sub + base + ".o")
    cmd = [HIPCC, "-x", "hip", "-c", src, "-o", obj] + FLAGS
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
    if r.stderr.strip() and verbose:
        print(r.stderr[-2000:], flush=True)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    t0 = time.time()
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources in {time.time() - t0:.1f}s", flush=True)
    return LIB


def clean():
    shutil.rmtree(OBJ, ignore_errors=True)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
