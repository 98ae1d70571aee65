"""Pins for the D-dimensional oracle (no GPU).

Checked against things other than itself: the D-fold sum of the definition
written out here at every point of tiny 4-D and 5-D grids, an independent
library (numpy.fft.fftn), grids with unit axes that reduce to the pinned 3-D
oracle, separable inputs whose transform is the outer product of 1-D
transforms (closed form), Parseval and the round trip.  A mutation check
shows that a dropped axis, a wrong sign or exchanged axis lengths fail a
pin.
"""
import itertools

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import ndim

TINY = [(2, 3, 2, 5), (3, 1, 4, 2), (2, 2, 2, 2, 2), (3, 2, 1, 2, 3), (5, 4), (6,)]


def grid(shape, seed=0):
    return synth.complex_grid(shape, torch.complex128, key=synth.SEED + 300 + seed).numpy()


def dft_sum(x, k, sign=-1):
    """The plain D-fold sum at one output point."""
    s = 0j
    for j in itertools.product(*(range(n) for n in x.shape)):
        ph = sum(ji * ki / n for ji, ki, n in zip(j, k, x.shape))
        s += x[j] * np.exp(sign * 2j * np.pi * ph)
    return s


@pytest.mark.parametrize("shape", TINY, ids=lambda s: "x".join(map(str, s)))
def test_fftn_is_the_definition_at_every_point(shape):
    x = grid(shape)
    y = ndim.fftn(x)
    worst = 0.0
    for k in itertools.product(*(range(n) for n in shape)):
        ref = dft_sum(x, k)
        worst = max(worst, abs(y[k] - ref) / max(1.0, abs(ref)))
    assert worst < 1e-13


@pytest.mark.parametrize("shape", [(8, 6, 10, 12), (4, 5, 6, 8, 9), (16, 16, 16, 16), (30, 1, 25, 1)])
def test_fftn_matches_numpy(shape):
    x = grid(shape, 1)
    for sign, ref in ((oracle.FORWARD, np.fft.fftn(x)), (oracle.BACKWARD, np.fft.ifftn(x) * x.size)):
        assert oracle.rel_l2(ndim.fftn(x, sign), ref) < 1e-14


def test_unit_axes_reduce_to_the_3d_oracle():
    x = grid((6, 1, 10, 12), 2)
    assert oracle.rel_l2(ndim.fftn(x)[:, 0], oracle.fft3(x[:, 0])) < 1e-15
    x5 = grid((1, 9, 1, 8, 10), 3)
    assert oracle.rel_l2(ndim.fftn(x5)[0, :, 0], oracle.fft3(x5[0, :, 0])) < 1e-15


def test_separable_input_gives_the_outer_product():
    """x = u0 (x) u1 (x) u2 (x) u3  =>  X = F u0 (x) F u1 (x) F u2 (x) F u3, each
    F the textbook n-point DFT matrix applied directly."""
    lens = (4, 6, 5, 3)
    us = [synth.complex_grid((n,), torch.complex128, key=synth.SEED + 310 + i).numpy() for i, n in enumerate(lens)]
    x = us[0]
    for u in us[1:]:
        x = np.multiply.outer(x, u)
    ref = None
    for n, u in zip(lens, us):
        F = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
        fu = F @ u
        ref = fu if ref is None else np.multiply.outer(ref, fu)
    assert oracle.rel_l2(ndim.fftn(x), ref) < 1e-14


def test_parseval_round_trip_and_batch():
    x = grid((3, 6, 5, 4, 8), 4)
    y = ndim.fftn(x)
    assert abs(np.sum(abs(y) ** 2) / (x.size * np.sum(abs(x) ** 2)) - 1) < 1e-14
    assert oracle.rel_l2(ndim.fftn(y, oracle.BACKWARD) / x.size, x) < 1e-15
    b = np.stack([x, 2 * x])
    yb = ndim.fftn_batch(b, 5)
    assert oracle.rel_l2(yb[0], y) == 0.0 and oracle.rel_l2(yb[1], 2 * y) < 1e-16


def test_sampled_points_match_the_transform():
    x = grid((8, 6, 10, 12), 5)
    y = ndim.fftn(x)
    for k in [(0, 0, 0, 0), (1, 2, 3, 4), (7, 5, 9, 11), (3, 0, 5, 6)]:
        assert abs(ndim.dftn_point(x, k) - y[k]) <= 1e-12 * np.max(abs(y))


def test_mutations_fail_a_pin():
    """A dropped axis, the wrong sign and exchanged axis lengths each disagree
    with the D-fold sum."""
    shape = (2, 3, 2, 5)
    x = grid(shape, 6)
    ref = np.array([dft_sum(x, k) for k in itertools.product(*(range(n) for n in shape))]).reshape(shape)

    def drop_axis(v):
        y = v.copy()
        for axis in (3, 2, 1):                      # axis 0 forgotten
            y = np.fft.fft(y, axis=axis)
        return y

    def wrong_sign(v):
        return ndim.fftn(v, oracle.BACKWARD)

    def mixed_axes(v):
        # the grid read with two axis lengths exchanged (a layout mistake)
        return ndim.fftn(v.reshape(2, 5, 2, 3)).reshape(shape)

    assert oracle.rel_l2(ndim.fftn(x), ref) < 1e-13
    assert oracle.rel_l2(drop_axis(x), ref) > 0.1
    assert oracle.rel_l2(wrong_sign(x), ref) > 0.1
    assert oracle.rel_l2(mixed_axes(x), ref) > 0.1
