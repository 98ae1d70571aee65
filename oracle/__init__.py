"""CPU oracle for the 3-D complex-to-complex DFT -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The GPU library neither imports nor links it, and it shares no
code with the GPU library (only the seeded input generator in `synth` serves
both sides).

The arithmetic lives in offt_oracle.c (binary64, plain loops, OpenMP over
lines); this module marshals numpy arrays to it and adds the error metrics.

Transform definition (Duy & Ozaki, Sec. 2 Eq. 1 for the layout, Sec. 3.1.1
and Sec. 2's transpose order abc -> cab -> cba for the per-axis composition):
    X[ka,kb,kc] = sum_{a,b,c} x[a,b,c] W_Na^(a ka) W_Nb^(b kb) W_Nc^(c kc)
with W_n = exp(-2 pi i / n) forward and exp(+2 pi i / n) backward, both
unnormalised; the scaled inverse multiplies by 1/(Na Nb Nc).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "_build", "liboffs_oracle.so")
_lib = None

FORWARD = -1
BACKWARD = +1


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    sigs = {
        "oracle_root_table": [i64, ci, dp],
        "oracle_dft3_brute": [dp, dp, i64, i64, i64, ci, ci],
        "oracle_dft3_axes": [dp, dp, i64, i64, i64, ci, ci],
        "oracle_fft3": [dp, dp, i64, i64, i64, ci, ci],
        "oracle_fft1_lines": [dp, dp, i64, i64, ci, ci, ci],
        "oracle_dft3_line": [dp, dp, i64, i64, i64, i64, i64, ci, ci],
        "oracle_dft3_point": [dp, dp, i64, i64, i64, i64, i64, i64, ci],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ci
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ci
    _lib = lib
    return lib


def _as_c128(x) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(x), dtype=np.complex128)
    return x


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments")


def max_threads() -> int:
    return _load().oracle_max_threads()


def root_table(n: int, sign: int = FORWARD) -> np.ndarray:
    """W_n^m for m < n (binary64), exact at the quarter points."""
    out = np.empty(n, dtype=np.complex128)
    _check(_load().oracle_root_table(n, sign, _ptr(out)), "root_table")
    return out


def _grid_call(fname: str, x, sign: int, nthreads: int) -> np.ndarray:
    x = _as_c128(x)
    if x.ndim != 3:
        raise ValueError("expected a 3-D grid (Na, Nb, Nc)")
    y = np.empty_like(x)
    Na, Nb, Nc = x.shape
    _check(getattr(_load(), fname)(_ptr(x), _ptr(y), Na, Nb, Nc, sign, nthreads), fname)
    return y


def dft3_brute(x, sign: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """(O1) the plain triple sum, O(N^2)."""
    return _grid_call("oracle_dft3_brute", x, sign, nthreads)


def dft3_axes(x, sign: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """(O2) naive DFT along c, then b, then a."""
    return _grid_call("oracle_dft3_axes", x, sign, nthreads)


def fft3(x, sign: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """(O3) recursive mixed-radix 2/3/5 FFT along c, then b, then a."""
    return _grid_call("oracle_fft3", x, sign, nthreads)


def fft3_batch(x, sign: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """O3 applied to each grid of a (batch, Na, Nb, Nc) array."""
    x = _as_c128(x)
    return np.stack([fft3(x[g], sign, nthreads) for g in range(x.shape[0])])


def fft1_lines(x, sign: int = FORWARD, method: int = 1, nthreads: int = 0) -> np.ndarray:
    """1-D transform of every row of a (count, n) array; method 0 = naive DFT,
    1 = recursive FFT."""
    x = _as_c128(x)
    if x.ndim != 2:
        raise ValueError("expected (count, n)")
    y = np.empty_like(x)
    count, n = x.shape
    _check(_load().oracle_fft1_lines(_ptr(x), _ptr(y), n, count, sign, nthreads, method), "fft1_lines")
    return y


def dft3_line(x, ka: int, kb: int, sign: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """X[ka, kb, 0..Nc) straight from the definition (sum over a, b grouped per c)."""
    x = _as_c128(x)
    Na, Nb, Nc = x.shape
    y = np.empty(Nc, dtype=np.complex128)
    _check(_load().oracle_dft3_line(_ptr(x), _ptr(y), Na, Nb, Nc, ka, kb, sign, nthreads), "dft3_line")
    return y


def dft3_point(x, ka: int, kb: int, kc: int, sign: int = FORWARD) -> complex:
    """One output X[ka, kb, kc] from the plain triple sum."""
    x = _as_c128(x)
    Na, Nb, Nc = x.shape
    y = np.empty(1, dtype=np.complex128)
    _check(_load().oracle_dft3_point(_ptr(x), _ptr(y), Na, Nb, Nc, ka, kb, kc, sign), "dft3_point")
    return complex(y[0])


def rel_l2(y, ref) -> float:
    """||y - ref||_2 / ||ref||_2 in binary64 (numpy pairwise sums)."""
    y = np.asarray(y, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    num = np.sqrt(np.sum(np.abs(y - ref) ** 2))
    den = np.sqrt(np.sum(np.abs(ref) ** 2))
    return float(num / den) if den > 0 else float(num)


def rel_max(y, ref) -> float:
    """max|y - ref| / max|ref|."""
    y = np.asarray(y, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    den = np.max(np.abs(ref)) if ref.size else 0.0
    num = np.max(np.abs(y - ref)) if ref.size else 0.0
    return float(num / den) if den > 0 else float(num)


def tolerance(n_elems: int, complex64: bool) -> float:
    """Relative-L2 acceptance bound: 1e-12 for binary64, 2e-6 * log2(N) for
    binary32 (N = elements of the grid; at least 1 for tiny grids)."""
    if not complex64:
        return 1e-12
    return 2e-6 * max(1.0, float(np.log2(max(n_elems, 2))))
