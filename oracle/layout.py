"""Reversed (cba) axis order of a transform's output -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the GPU library shares no code with it.

In the paper the 3-D transform finishes in the cba decomposition: after the
transpose order abc -> cab -> cba (Sec. 2) the data points are held in
ascending order of the c-, b- and a-coordinates, so the a-coordinate varies
fastest, and the output index set upon finishing differs from the one upon
starting (Sec. 3.1.1).  For one grid of Na x Nb x Nc points that order is the
array Y of shape (Nc, Nb, Na) with

    Y[c, b, a] = X[a, b, c]

where X is the transform in the natural (abc) order of the input.  The
backward transform of such a Y takes it back to natural order first.
"""
from __future__ import annotations

import numpy as np

from . import BACKWARD, FORWARD, fft3

__all__ = ["reverse_axes", "fft3_reversed", "fft3_from_reversed"]


def reverse_axes(x) -> np.ndarray:
    """Y[..., c, b, a] = x[..., a, b, c] for an array whose last three axes are
    (Na, Nb, Nc); leading axes (a batch) are kept.  Written as the flat-index
    map of the two orders: element (a, b, c) sits at (a*Nb + b)*Nc + c in the
    input and at (c*Nb + b)*Na + a in the output."""
    x = np.asarray(x)
    if x.ndim < 3:
        raise ValueError("expected (..., Na, Nb, Nc)")
    lead = x.shape[:-3]
    Na, Nb, Nc = x.shape[-3:]
    c, b, a = np.meshgrid(np.arange(Nc), np.arange(Nb), np.arange(Na), indexing="ij")
    src = ((a * Nb + b) * Nc + c).ravel()          # output position k reads input src[k]
    flat = x.reshape(lead + (Na * Nb * Nc,))
    return np.ascontiguousarray(flat[..., src].reshape(lead + (Nc, Nb, Na)))


def _per_grid(fn, x):
    x = np.asarray(x, dtype=np.complex128)
    if x.ndim == 3:
        return fn(x)
    if x.ndim == 4:
        return np.stack([fn(x[g]) for g in range(x.shape[0])])
    raise ValueError("expected (Na, Nb, Nc) or (batch, Na, Nb, Nc)")


def fft3_reversed(x, sign: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """Transform of each grid (O3) delivered in cba order: shape (Nc, Nb, Na),
    or (batch, Nc, Nb, Na) for a batch."""
    return _per_grid(lambda g: reverse_axes(fft3(g, sign, nthreads)), x)


def fft3_from_reversed(y, sign: int = BACKWARD, nthreads: int = 0) -> np.ndarray:
    """Transform of grids given in cba order (shape (Nc, Nb, Na), or with a
    leading batch axis), delivered in natural order (Na, Nb, Nc)."""
    return _per_grid(lambda g: fft3(reverse_axes(g), sign, nthreads), y)
