"""Brute-force reference of the paper's data distribution and transpose
volumes -- TEST INFRASTRUCTURE (only the tests call it).

Duy & Ozaki, Sec. 2: the grid is numbered row-wise (Eq. 1) and the linear
index range [0, N) is split into Np contiguous blocks; process `myid` owns
[f(myid), f(myid+1)) with f from Eq. 2: whole N2 x N3 planes when
Np <= N1, whole N3-lines when N1 < Np <= N1 N2.  The transform then moves
the data from the abc order to cab and on to cba (Fig. 1b), each order
decomposed the same way over its own leading dimensions.  The volume of a
transpose is the number of elements whose owner changes.

Everything here enumerates every element; it is meant for small grids.
"""
from __future__ import annotations

import numpy as np


def block_start(n1: int, n2: int, n3: int, np_: int, myid: int) -> int:
    """f(N1, N2, N3, Np, myid) of Eq. 2."""
    if not 1 <= np_ <= n1 * n2:
        raise ValueError("Eq. 2 covers 1 <= Np <= N1 N2")
    if np_ <= n1:
        return (n1 * myid // np_) * n2 * n3
    return (n1 * n2 * myid // np_) * n3


def owners(n1: int, n2: int, n3: int, np_: int) -> np.ndarray:
    """Owner process of every linear index of an (n1, n2, n3) row-major grid."""
    own = np.empty(n1 * n2 * n3, dtype=np.int64)
    for p in range(np_):
        own[block_start(n1, n2, n3, np_, p):block_start(n1, n2, n3, np_, p + 1)] = p
    return own


def transpose_counts(n1: int, n2: int, n3: int, np_: int, step: int) -> np.ndarray:
    """M[p, q] = elements that process p holds before the transpose and q
    after it.  step 0: abc -> cab, step 1: cab -> cba."""
    a, b, c = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    cab = owners(n3, n1, n2, np_)[c * n1 * n2 + a * n2 + b]
    if step == 0:
        src, dst = owners(n1, n2, n3, np_)[a * n2 * n3 + b * n3 + c], cab
    else:
        src, dst = cab, owners(n3, n2, n1, np_)[c * n2 * n1 + b * n1 + a]
    m = np.zeros((np_, np_), dtype=np.int64)
    np.add.at(m, (src.ravel(), dst.ravel()), 1)
    return m


def transpose_volume(n1: int, n2: int, n3: int, np_: int, step: int) -> int:
    """Elements that leave their process in the transpose."""
    m = transpose_counts(n1, n2, n3, np_, step)
    return int(m.sum() - np.trace(m))
