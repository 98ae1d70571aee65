"""Reference of the paper's distributed transform run by Np processes --
TEST INFRASTRUCTURE (only the tests and the benchmark's checks call it).

Duy & Ozaki, Sec. 2 and Sec. 3.1.1: the grid A(a, b, c) is numbered row-wise
(Eq. 1) and process `myid` owns the contiguous block [f(myid), f(myid+1)) of
the linear index, f of Eq. 2 taken over the leading dimensions of the order
the data is currently held in.  The forward calculation flow is

  1. the 1-D transform along c of every local line of the abc block,
  2. the transpose abc -> cab: every element moves to the process that owns
     its cab linear index (pack, communicate, unpack),
  3. the 1-D transform along b of every local line of the cab block,
  4. the transpose cab -> cba,
  5. the 1-D transform along a of every local line of the cba block,

and the data finishes in the cba decomposition (Fig. 1b).  The backward flow
runs the same steps in reverse order (a, cba -> cab, b, cab -> abc, c) with
the conjugate roots of unity.

Because each block is a contiguous range of its order's linear index and the
blocks follow the process order, the concatenation of all local arrays in
process order is the whole grid in that order.  The functions below keep the
processes' arrays separate and build every exchanged element's destination
explicitly from the owner map, as the processes would.
"""
from __future__ import annotations

import numpy as np

from . import BACKWARD, FORWARD, fft1_lines
from .decomp import block_start

# axis orders, slowest first: positions of the a, b and c axes
ORDERS = {"abc": (0, 1, 2), "cab": (2, 0, 1), "cba": (2, 1, 0)}


def order_dims(shape, order):
    """(N1, N2, N3) of a grid of `shape` = (Na, Nb, Nc) held in `order`."""
    return tuple(shape[ax] for ax in ORDERS[order])


def blocks(shape, order, np_):
    """[start, end) of every process's block of the linear index in `order`
    (Eq. 2 over that order's leading dimensions)."""
    n1, n2, n3 = order_dims(shape, order)
    s = [block_start(n1, n2, n3, np_, p) for p in range(np_ + 1)]
    return [(s[p], s[p + 1]) for p in range(np_)]


def linear_index(coords, shape, order):
    """Linear index in `order` of points with coordinates coords = (a, b, c)."""
    n1, n2, n3 = order_dims(shape, order)
    i1, i2, i3 = (coords[ax] for ax in ORDERS[order])
    return (i1 * n2 + i2) * n3 + i3


def coordinates(lin, shape, order):
    """(a, b, c) of the points with linear index `lin` in `order`."""
    n1, n2, n3 = order_dims(shape, order)
    i3 = lin % n3
    i2 = (lin // n3) % n2
    i1 = lin // (n2 * n3)
    out = [None, None, None]
    for ax, v in zip(ORDERS[order], (i1, i2, i3)):
        out[ax] = v
    return tuple(out)


def scatter(x, shape, np_):
    """The processes' abc blocks of a grid x (Na, Nb, Nc): list of 1-D arrays."""
    flat = np.asarray(x, dtype=np.complex128).reshape(-1)
    return [flat[s:e].copy() for s, e in blocks(shape, "abc", np_)]


def local_lines(local, shape, order, sign):
    """Step 1, 3 or 5: the 1-D transform of every local line along the fastest
    axis of `order` (each block holds whole lines)."""
    n3 = order_dims(shape, order)[2]
    return [fft1_lines(b.reshape(-1, n3), sign).reshape(-1) if b.size else b.copy() for b in local]


def exchange(local, shape, src_order, dst_order, np_):
    """Step 2 or 4: every element of every process goes to the process that
    owns its linear index in dst_order.  Returns (the new local arrays,
    counts[p][q] = elements process p sends to process q)."""
    src_blocks = blocks(shape, src_order, np_)
    dst_blocks = blocks(shape, dst_order, np_)
    out = [np.empty(e - s, dtype=np.complex128) for s, e in dst_blocks]
    counts = np.zeros((np_, np_), dtype=np.int64)
    for p, (s, e) in enumerate(src_blocks):
        lin_src = np.arange(s, e)
        lin_dst = linear_index(coordinates(lin_src, shape, src_order), shape, dst_order)
        for q, (ds, de) in enumerate(dst_blocks):
            sel = (lin_dst >= ds) & (lin_dst < de)
            counts[p, q] = int(sel.sum())
            out[q][lin_dst[sel] - ds] = local[p][lin_src[sel] - s]
    return out, counts


def forward_steps(x, np_):
    """The five steps of the forward flow for a grid x (Na, Nb, Nc).  Returns
    (states, counts): states[k] is the list of local arrays after step k + 1
    (orders abc, cab, cab, cba, cba) and counts the two exchange matrices."""
    shape = np.asarray(x).shape
    st = local_lines(scatter(x, shape, np_), shape, "abc", FORWARD)
    states = [st]
    st, m0 = exchange(st, shape, "abc", "cab", np_)
    states.append(st)
    st = local_lines(st, shape, "cab", FORWARD)
    states.append(st)
    st, m1 = exchange(st, shape, "cab", "cba", np_)
    states.append(st)
    st = local_lines(st, shape, "cba", FORWARD)
    states.append(st)
    return states, (m0, m1)


def backward_steps(y_local, shape, np_):
    """The five steps of the backward flow from the processes' cba blocks
    (unnormalised).  states[k] after step k + 1: orders cba, cab, cab, abc,
    abc."""
    st = local_lines(y_local, shape, "cba", BACKWARD)
    states = [st]
    st, m0 = exchange(st, shape, "cba", "cab", np_)
    states.append(st)
    st = local_lines(st, shape, "cab", BACKWARD)
    states.append(st)
    st, m1 = exchange(st, shape, "cab", "abc", np_)
    states.append(st)
    st = local_lines(st, shape, "abc", BACKWARD)
    states.append(st)
    return states, (m0, m1)


def gather(local):
    """Concatenation of the local arrays in process order: the grid in the
    order the blocks are held in."""
    return np.concatenate(local) if local else np.empty(0, dtype=np.complex128)


def max_processes(shape):
    """Largest Np that Eq. 2 covers for every order of the flow."""
    return min(order_dims(shape, o)[0] * order_dims(shape, o)[1] for o in ORDERS)
