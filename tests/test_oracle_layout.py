"""Pins for the oracle of the reversed (cba) output order (no GPU).

The reversed order is fixed by the definition Y[c, b, a] = X[a, b, c] (the
cba decomposition the paper's transform finishes in, Sec. 2 and Sec. 3.1.1).
The pins check it against things other than the oracle itself: coded
integer grids whose every value names its own (a, b, c), the plain triple
sum of the DFT written out here at every output point of tiny non-cubic
grids, the special case of one non-unit axis (both orders are the same
memory), the involution, and the round trip.  A mutation check shows that
plausible mistakes in the index map (another axis permutation, a transposed
pair) fail a pin.
"""
import itertools

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import layout

SHAPES = [(2, 3, 5), (3, 1, 4), (1, 4, 6), (4, 6, 1), (5, 2, 3), (6, 1, 1), (2, 2, 2)]


def coded(shape):
    """x[a, b, c] = 10000 a + 100 b + c (every value names its position)."""
    Na, Nb, Nc = shape
    a, b, c = np.meshgrid(np.arange(Na), np.arange(Nb), np.arange(Nc), indexing="ij")
    return (10000 * a + 100 * b + c).astype(np.int64)


def pin_coded(rev, shape):
    y = rev(coded(shape))
    Na, Nb, Nc = shape
    if y.shape != (Nc, Nb, Na):
        return False
    return all(y[c, b, a] == 10000 * a + 100 * b + c
               for a, b, c in itertools.product(range(Na), range(Nb), range(Nc)))


def dft_sum(x, ka, kb, kc, sign=-1):
    """The plain triple sum of the definition at one output point."""
    Na, Nb, Nc = x.shape
    s = 0j
    for a, b, c in itertools.product(range(Na), range(Nb), range(Nc)):
        s += x[a, b, c] * np.exp(sign * 2j * np.pi * (a * ka / Na + b * kb / Nb + c * kc / Nc))
    return s


@pytest.mark.parametrize("shape", SHAPES)
def test_reverse_axes_moves_every_point(shape):
    assert pin_coded(layout.reverse_axes, shape)


@pytest.mark.parametrize("shape", SHAPES)
def test_reversed_forward_is_the_definition_at_every_point(shape):
    x = synth.complex_grid(shape, torch.complex128, key=synth.SEED + 71).numpy()
    y = layout.fft3_reversed(x)
    Na, Nb, Nc = shape
    assert y.shape == (Nc, Nb, Na)
    worst = 0.0
    for a, b, c in itertools.product(range(Na), range(Nb), range(Nc)):
        ref = dft_sum(x, a, b, c)
        worst = max(worst, abs(y[c, b, a] - ref) / max(1.0, abs(ref)))
    assert worst < 1e-13


@pytest.mark.parametrize("shape", [(7, 1, 1), (1, 9, 1), (1, 1, 12)])
def test_one_axis_grids_keep_their_memory_order(shape):
    x = synth.complex_grid(shape, torch.complex128, key=synth.SEED + 72).numpy()
    assert np.array_equal(layout.reverse_axes(x).ravel(), x.ravel())


def test_reverse_is_an_involution_and_keeps_a_batch():
    x = synth.complex_grid((3, 4, 5, 6), torch.complex128, key=synth.SEED + 73).numpy()
    y = layout.reverse_axes(x)
    assert y.shape == (3, 6, 5, 4)
    for g in range(3):
        assert np.array_equal(y[g], layout.reverse_axes(x[g]))
    assert np.array_equal(layout.reverse_axes(y), x)


@pytest.mark.parametrize("shape", [(4, 6, 10), (3, 5, 2), (8, 1, 9)])
def test_round_trip_through_the_reversed_order(shape):
    x = synth.complex_grid((2,) + shape, torch.complex128, key=synth.SEED + 74).numpy()
    y = layout.fft3_reversed(x)
    back = layout.fft3_from_reversed(y) / np.prod(shape)
    assert oracle.rel_l2(back, x) < 1e-14


def test_backward_from_reversed_is_the_definition():
    """Backward transform of a cba-ordered grid: the conjugate-sign triple sum
    over the natural-order points."""
    shape = (3, 2, 4)
    y = synth.complex_grid((4, 2, 3), torch.complex128, key=synth.SEED + 75).numpy()   # cba order
    got = layout.fft3_from_reversed(y)
    x_nat = np.empty(shape, np.complex128)
    for a, b, c in itertools.product(range(3), range(2), range(4)):
        x_nat[a, b, c] = y[c, b, a]
    for ka, kb, kc in itertools.product(range(3), range(2), range(4)):
        assert abs(got[ka, kb, kc] - dft_sum(x_nat, ka, kb, kc, sign=+1)) < 1e-12


def test_mutations_of_the_index_map_fail_a_pin():
    """Other axis orders one could write by mistake: each fails the coded pin
    on a grid with three different lengths."""
    def perm(order):
        return lambda x: np.ascontiguousarray(np.transpose(np.asarray(x), order))
    shape = (2, 3, 5)
    assert pin_coded(perm((2, 1, 0)), shape)                 # the right one, written another way
    for order in [(0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (1, 0, 2)]:
        assert not pin_coded(perm(order), shape), order
