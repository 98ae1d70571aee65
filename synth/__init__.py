"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no FFT arithmetic.  It produces the numbers the transforms
are fed with, so that the CPU oracle and the HIP library can be driven with
bit-identical inputs.

Generator: SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used counter-style so any
element can be produced independently of the others:

    state_j = key + (j + 1) * GAMMA              (mod 2^64)
    z = state_j
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    r_j = z ^ (z >> 31)

Uniform value in [-1, 1):  v_j = (r_j >> 11) * 2^-52 - 1, exact in binary64.
Grid element i (row-major, last axis fastest): re = v_{2i}, im = v_{2i+1}.
complex64 inputs are the binary64 values rounded to nearest-even binary32.

The implementation uses torch int64 arithmetic (two's-complement wrap-around)
so the same code runs on the CPU and on a GPU device; logical right shifts
are emulated with an arithmetic shift followed by a mask.
"""
from __future__ import annotations

import torch

SEED = 1501                     # base seed S of the synthetic workloads
KEY_DIMS = SEED + 1_000_000     # key for axis-length draws of batched grids
KEY_MLP = SEED + 2_000_000      # key for axis-length draws of selector grids

_M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
_MUL1 = 0xBF58476D1CE4E5B9
_MUL2 = 0x94D049BB133111EB


def _s64(u: int) -> int:
    """Reinterpret an unsigned 64-bit integer as signed (torch int64)."""
    u &= _M64
    return u - (1 << 64) if u >= (1 << 63) else u


def _srl(z: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _s64(_MUL1)
    z = (z ^ _srl(z, 27)) * _s64(_MUL2)
    return z ^ _srl(z, 31)


def splitmix64_int(key: int, start: int, count: int, device="cpu") -> torch.Tensor:
    """r_j for j in [start, start+count) as int64 bit patterns."""
    j = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    state = j * _s64(GAMMA) + _s64(key)
    return _mix(state)


def splitmix64_py(key: int, j: int) -> int:
    """Pure-Python r_j (unsigned), for spot checks and small integer draws."""
    z = (key + (j + 1) * GAMMA) & _M64
    z = ((z ^ (z >> 30)) * _MUL1) & _M64
    z = ((z ^ (z >> 27)) * _MUL2) & _M64
    return z ^ (z >> 31)


def uniform_pm1(key: int, start: int, count: int, device="cpu") -> torch.Tensor:
    """v_j in [-1, 1) as float64 for j in [start, start+count)."""
    r = splitmix64_int(key, start, count, device)
    return _srl(r, 11).to(torch.float64) * (2.0 ** -52) - 1.0


_CHUNK = 1 << 24  # values per generation chunk (bounds temporaries)


def complex_grid(shape, dtype=torch.complex128, key: int = SEED, device="cpu") -> torch.Tensor:
    """Contiguous complex tensor of `shape` filled with the seeded values.

    Element with flat index i gets re = v_{2i}, im = v_{2i+1}.  For
    torch.complex64 the binary64 values are rounded to nearest binary32.
    """
    if dtype not in (torch.complex128, torch.complex64):
        raise ValueError("dtype must be complex64 or complex128")
    n = 1
    for s in shape:
        n *= int(s)
    out = torch.empty(tuple(int(s) for s in shape), dtype=dtype, device=device)
    flat = torch.view_as_real(out.view(-1))  # (n, 2) real view
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    flat2 = flat.reshape(-1)
    total = 2 * n
    pos = 0
    while pos < total:
        cnt = min(_CHUNK, total - pos)
        flat2[pos:pos + cnt] = uniform_pm1(key, pos, cnt, device).to(rdt)
        pos += cnt
    return out


def batch_grids(dims_list, dtype=torch.complex64, key0: int = SEED, device="cpu"):
    """One seeded grid per entry of dims_list; grid g uses key key0 + g."""
    return [complex_grid(d, dtype, key0 + g, device) for g, d in enumerate(dims_list)]


def draw_index(key: int, j: int, n: int) -> int:
    """Integer in [0, n) from draw j of stream `key` (r_j mod n)."""
    return splitmix64_py(key, j) % n


BATCH_AXIS_LENGTHS = (48, 60, 64, 80, 96, 120, 128, 150, 160)


def uneven_batch_dims(count: int = 64, key: int = KEY_DIMS, lengths=BATCH_AXIS_LENGTHS):
    """Axis lengths for the uneven-batch workload: each of the 3*count axes is
    drawn independently and uniformly from `lengths` (BATCH_AXIS_LENGTHS by
    default)."""
    L = tuple(lengths)
    return [tuple(L[draw_index(key, 3 * g + k, len(L))] for k in range(3)) for g in range(count)]


def smooth_lengths(lo: int = 16, hi: int = 1024):
    """All 2/3/5-smooth integers in [lo, hi]."""
    out = []
    for n in range(lo, hi + 1):
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def selector_grids(count: int, key: int = KEY_MLP, skip: int = 0, max_elems: int = 1 << 28):
    """Random grids for plan-selector training/evaluation.

    Each accepted draw is (Na, Nb, Nc, batch, dtype_code) with axes uniform
    over the 2/3/5-smooth lengths in [16, 1024], batch uniform over
    {1, 2, 4, 8}, dtype code uniform over {0 (complex128), 1 (complex64)}, and
    batch*Na*Nb*Nc <= max_elems (draws violating it are rejected).  The first
    `skip` accepted draws are skipped, so train and held-out sets are disjoint
    slices of one stream.
    """
    L = smooth_lengths()
    out = []
    j = 0
    accepted = 0
    while len(out) < count:
        na = L[draw_index(key, j, len(L))]
        nb = L[draw_index(key, j + 1, len(L))]
        nc = L[draw_index(key, j + 2, len(L))]
        bt = (1, 2, 4, 8)[draw_index(key, j + 3, 4)]
        dt = draw_index(key, j + 4, 2)
        j += 5
        if bt * na * nb * nc > max_elems:
            continue
        if accepted >= skip:
            out.append((na, nb, nc, bt, dt))
        accepted += 1
    return out
