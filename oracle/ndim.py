"""CPU oracle for D-dimensional complex transforms (D <= 5) -- TEST
INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the GPU library shares no code with it.

The paper's decomposition method covers multi-dimensional transforms, with
axes named a, b, c, ... for the first, second, third dimension (Sec. 1); its
future work extends the package beyond three dimensions (Sec. 5).  For a grid
of n_0 x ... x n_{D-1} points (row-major, the last axis fastest):

    X[k_0, ..., k_{D-1}] = sum over every j of x[j_0, ..., j_{D-1}]
                           * prod_i W_{n_i}^(j_i k_i)

with W_n = exp(-2 pi i / n) forward and exp(+2 pi i / n) backward, both
unnormalised.  The sum over each coordinate can be taken separately, so the
transform is the 1-D transform of every line along each axis in turn; the
order of the axes does not change the result.  `fftn` takes the axes from
the last to the first with the oracle's recursive FFT of each line (O3).
"""
from __future__ import annotations

import numpy as np

from . import BACKWARD, FORWARD, _as_c128, fft1_lines

__all__ = ["fftn", "fftn_batch", "dftn_point"]


def _along_axis(x: np.ndarray, axis: int, sign: int, nthreads: int) -> np.ndarray:
    """1-D transform of every line of `x` along `axis`."""
    moved = np.moveaxis(x, axis, -1)
    shape = moved.shape
    rows = np.ascontiguousarray(moved).reshape(-1, shape[-1])
    out = fft1_lines(rows, sign, method=1, nthreads=nthreads).reshape(shape)
    return np.ascontiguousarray(np.moveaxis(out, -1, axis))


def fftn(x, sign: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """The D-dimensional transform of one grid (1 <= D <= 5), axis by axis
    from the last to the first."""
    x = _as_c128(x)
    if not 1 <= x.ndim <= 5:
        raise ValueError("expected a grid of 1 to 5 dimensions")
    y = x.copy()
    for axis in reversed(range(x.ndim)):
        if x.shape[axis] > 1:
            y = _along_axis(y, axis, sign, nthreads)
    return y


def fftn_batch(x, ndim: int, sign: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """fftn of each grid of an array whose last `ndim` axes are the grid."""
    x = _as_c128(x)
    lead = x.shape[:-ndim]
    flat = x.reshape((-1,) + x.shape[-ndim:])
    return np.stack([fftn(g, sign, nthreads) for g in flat]).reshape(lead + x.shape[-ndim:])


def dftn_point(x, k, sign: int = FORWARD) -> complex:
    """One output X[k] straight from the D-fold sum of the definition, summed
    over one coordinate at a time, the first coordinate first: O(N) work per
    point, for sampled checks of large grids."""
    x = np.asarray(x)
    if len(k) != x.ndim:
        raise ValueError("index has the wrong number of coordinates")
    y = x
    for n, ki in zip(x.shape, k):
        j = np.arange(n)
        # exact exponent reduction: (j k) mod n before the division by n
        phase = np.exp(sign * 2j * np.pi * ((j * ki) % n) / n)
        y = np.tensordot(phase, y.astype(np.complex128, copy=False), axes=(0, 0))
    return complex(y)
