"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: an independent
library run (numpy.fft), the brute-force definition on tiny grids, textbook
closed forms (impulses, constants, single modes, small DFT matrices in
radicals), and invariants (Parseval, round trip, linearity, shift theorem,
Hermitian symmetry).  A mutation test then shows that plausible mistakes
(wrong sign, transposed operand, dropped term, wrong twiddle index, missing
axis) each fail at least one pin.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TINY = [(1, 1, 1), (2, 3, 5), (4, 4, 4), (5, 3, 2), (8, 6, 10), (1, 9, 1), (3, 1, 16), (16, 16, 16)]
TIGHT = 1e-13


def rand_grid(shape, seed=0):
    x = synth.complex_grid(shape, torch.complex128, key=synth.SEED + seed)
    return x.numpy()


# ---------------------------------------------------------------- pins ----
def pin_numpy(fn, shape, seed=0):
    x = rand_grid(shape, seed)
    return oracle.rel_l2(fn(x, oracle.FORWARD), np.fft.fftn(x)) <= TIGHT


def pin_impulse(fn, shape, pos):
    Na, Nb, Nc = shape
    x = np.zeros(shape, np.complex128)
    x[pos] = 1.0
    ka, kb, kc = np.meshgrid(np.arange(Na), np.arange(Nb), np.arange(Nc), indexing="ij")
    a0, b0, c0 = pos
    expect = np.exp(-2j * np.pi * (a0 * ka / Na + b0 * kb / Nb + c0 * kc / Nc))
    return oracle.rel_l2(fn(x, oracle.FORWARD), expect) <= TIGHT


def pin_single_mode(fn, shape, mode):
    Na, Nb, Nc = shape
    a, b, c = np.meshgrid(np.arange(Na), np.arange(Nb), np.arange(Nc), indexing="ij")
    p, q, r = mode
    x = np.exp(2j * np.pi * (p * a / Na + q * b / Nb + r * c / Nc))
    expect = np.zeros(shape, np.complex128)
    expect[mode] = Na * Nb * Nc
    return oracle.rel_l2(fn(x, oracle.FORWARD), expect) <= TIGHT


def pin_parseval(fn, shape):
    x = rand_grid(shape, 3)
    y = fn(x, oracle.FORWARD)
    lhs = np.sum(np.abs(y) ** 2)
    rhs = x.size * np.sum(np.abs(x) ** 2)
    return abs(lhs - rhs) / rhs <= TIGHT


def pin_roundtrip(fn, shape):
    x = rand_grid(shape, 4)
    z = fn(fn(x, oracle.FORWARD), oracle.BACKWARD) / x.size
    return oracle.rel_l2(z, x) <= TIGHT


def all_pins(fn):
    res = {
        "numpy_8x6x10": pin_numpy(fn, (8, 6, 10)),
        "numpy_5x12x9": pin_numpy(fn, (5, 12, 9), 1),
        "impulse_a": pin_impulse(fn, (6, 4, 5), (1, 0, 0)),
        "impulse_abc": pin_impulse(fn, (6, 4, 5), (2, 3, 1)),
        "mode": pin_single_mode(fn, (6, 4, 5), (1, 2, 3)),
        "parseval": pin_parseval(fn, (6, 4, 5)),
        "roundtrip": pin_roundtrip(fn, (6, 4, 5)),
    }
    return res


# ------------------------------------------------------- the oracle parts ----
@pytest.mark.parametrize("method", ["brute", "axes", "fft"])
def test_all_pins_hold(method):
    fn = {"brute": oracle.dft3_brute, "axes": oracle.dft3_axes, "fft": oracle.fft3}[method]
    res = all_pins(fn)
    assert all(res.values()), res


@pytest.mark.parametrize("shape", TINY)
def test_three_parts_agree_with_brute_force(shape):
    x = rand_grid(shape, 7)
    for sign in (oracle.FORWARD, oracle.BACKWARD):
        ref = oracle.dft3_brute(x, sign)
        assert oracle.rel_l2(oracle.dft3_axes(x, sign), ref) <= TIGHT
        assert oracle.rel_l2(oracle.fft3(x, sign), ref) <= TIGHT


@pytest.mark.parametrize("shape", [(32, 32, 32), (27, 25, 16), (64, 48, 60), (1, 1, 1000)])
def test_fft3_vs_numpy_library_run(shape):
    x = rand_grid(shape, 11)
    assert oracle.rel_l2(oracle.fft3(x), np.fft.fftn(x)) <= TIGHT
    assert oracle.rel_l2(oracle.fft3(x, oracle.BACKWARD), np.fft.ifftn(x) * x.size) <= TIGHT


def test_brute_force_32cubed_vs_numpy():
    # 32^3 complex128, the small workload: brute force is the definition itself.
    x = synth.complex_grid((32, 32, 32), torch.complex128).numpy()
    y = oracle.dft3_brute(x)
    assert oracle.rel_l2(y, np.fft.fftn(x)) <= 1e-13


def test_impulse_at_origin_is_exactly_ones():
    for fn in (oracle.dft3_brute, oracle.dft3_axes, oracle.fft3):
        x = np.zeros((4, 6, 10), np.complex128)
        x[0, 0, 0] = 1.0
        assert np.array_equal(fn(x), np.ones_like(x))


def test_constant_gives_scaled_delta():
    x = np.ones((6, 10, 8), np.complex128)
    y = oracle.fft3(x)
    expect = np.zeros_like(x)
    expect[0, 0, 0] = x.size
    assert oracle.rel_l2(y, expect) <= TIGHT


def _radical_roots():
    env = {"sqrt": math.sqrt}
    roots = {}
    with open(os.path.join(GOLDEN, "dft_textbook.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            n, re_s, im_s = line.split()
            roots[int(n)] = complex(eval(re_s, env), eval(im_s, env))
    return roots


def test_small_dft_matrices_from_radicals():
    """Columns of the DFT matrix for the radix lengths match W_n^(jk) built by
    repeated multiplication of the radical closed form of W_n."""
    roots = _radical_roots()
    assert set(roots) >= {2, 3, 4, 5, 8, 16}
    for n, w in roots.items():
        powers = [complex(1, 0)]
        for _ in range(n - 1):
            powers.append(powers[-1] * w)
        expect = np.array([[powers[(j * k) % n] for k in range(n)] for j in range(n)])
        for method in (0, 1):
            got = oracle.fft1_lines(np.eye(n, dtype=np.complex128), oracle.FORWARD, method)
            assert np.max(np.abs(got - expect)) <= 1e-15 * n, (n, method)
        # the table itself
        assert np.max(np.abs(oracle.root_table(n) - np.array(powers))) <= 1e-15 * n


def test_root_table_exact_quarter_points():
    for n in (4, 8, 12, 16, 20, 60, 1024):
        t = oracle.root_table(n)
        assert t[0] == 1 and t[n // 2] == -1 and t[n // 4] == -1j and t[3 * n // 4] == 1j
        assert np.max(np.abs(np.abs(t) - 1)) <= 4.5e-16
    tb = oracle.root_table(12, oracle.BACKWARD)
    assert np.array_equal(tb, np.conj(oracle.root_table(12)))


def test_linearity_shift_and_hermitian():
    shape = (6, 8, 10)
    x1, x2 = rand_grid(shape, 21), rand_grid(shape, 22)
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    assert oracle.rel_l2(oracle.fft3(a * x1 + b * x2), a * oracle.fft3(x1) + b * oracle.fft3(x2)) <= TIGHT
    # circular shift by (s0, s1, s2) multiplies X by a phase ramp
    s = (1, 3, 7)
    ka, kb, kc = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    ramp = np.exp(-2j * np.pi * (s[0] * ka / shape[0] + s[1] * kb / shape[1] + s[2] * kc / shape[2]))
    shifted = np.roll(x1, s, axis=(0, 1, 2))
    assert oracle.rel_l2(oracle.fft3(shifted), ramp * oracle.fft3(x1)) <= TIGHT
    # real input -> X[-k] = conj(X[k])
    xr = x1.real.astype(np.complex128)
    y = oracle.fft3(xr)
    flip = np.roll(y[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))
    assert oracle.rel_l2(flip, np.conj(y)) <= TIGHT
    # backward = conj(forward(conj(x)))
    assert oracle.rel_l2(oracle.fft3(x1, oracle.BACKWARD), np.conj(oracle.fft3(np.conj(x1)))) <= TIGHT


def test_separability_per_axis_lines():
    """Each axis pass equals the 1-D oracle on every line of that axis."""
    x = rand_grid((6, 10, 12), 31)
    # c axis only: a 1x1xNc pass on each (a,b) row == fft1_lines on rows
    rows = x.reshape(-1, 12)
    y_rows = oracle.fft1_lines(rows).reshape(x.shape)
    assert oracle.rel_l2(y_rows, np.fft.fft(x, axis=2)) <= TIGHT
    full = oracle.fft3(x)
    step_b = oracle.fft1_lines(np.moveaxis(y_rows, 1, 2).reshape(-1, 10)).reshape(6, 12, 10)
    step_b = np.moveaxis(step_b, 2, 1)
    step_a = oracle.fft1_lines(np.moveaxis(step_b, 0, 2).reshape(-1, 6)).reshape(10, 12, 6)
    step_a = np.moveaxis(step_a, 2, 0)
    assert oracle.rel_l2(step_a, full) <= TIGHT


def test_sampled_line_and_point_match_full_transform():
    x = rand_grid((24, 20, 30), 41)
    full = oracle.fft3(x)
    for ka, kb in [(0, 0), (5, 19), (23, 7)]:
        assert oracle.rel_l2(oracle.dft3_line(x, ka, kb), full[ka, kb]) <= TIGHT
        assert oracle.rel_l2(oracle.dft3_line(x, ka, kb, oracle.BACKWARD),
                             oracle.fft3(x, oracle.BACKWARD)[ka, kb]) <= TIGHT
    for p in [(0, 0, 0), (3, 4, 29), (23, 19, 1)]:
        assert abs(oracle.dft3_point(x, *p) - full[p]) <= TIGHT * np.max(np.abs(full))


def test_fft3_roundoff_grows_like_log_n():
    """Textbook bound: rms round-off of Cooley-Tukey is O(eps log2 N); the
    fp64 tolerance 1e-12 is ~4500 eps, far above what the oracle produces."""
    for n in (16, 64, 128):
        x = rand_grid((n, n, n), 51)
        err = oracle.rel_l2(oracle.fft3(x), np.fft.fftn(x))
        assert err <= 2.0 * np.finfo(np.float64).eps * math.log2(n ** 3)


def test_bad_arguments_rejected():
    with pytest.raises(ValueError):
        oracle.fft3(np.zeros((7, 2, 2), np.complex128))  # prime 7 unsupported by O3
    with pytest.raises(ValueError):
        oracle.dft3_line(np.zeros((2, 2, 2), np.complex128), 2, 0)


# -------------------------------------------------------------- mutations ----
def _mutants():
    def wrong_sign(x, s):
        return oracle.fft3(x, -s)

    def transposed(x, s):
        # b and c swapped: transform the grid read as (Na, Nc, Nb)
        xt = np.ascontiguousarray(x.reshape(x.shape[0], x.shape[2], x.shape[1]))
        return oracle.fft3(xt, s).reshape(x.shape)

    def dropped_term(x, s):
        x2 = x.copy().reshape(-1)
        x2[-1] = 0
        return oracle.fft3(x2.reshape(x.shape), s)

    def missing_axis(x, s):
        return np.fft.fft(np.fft.fft(x, axis=2), axis=1) if s < 0 else np.fft.ifft(
            np.fft.ifft(x, axis=2), axis=1) * x.shape[1] * x.shape[2]

    def wrong_index(x, s):
        y = oracle.fft3(x, s)
        return np.roll(y, 1, axis=2)

    def conj_twiddle_on_one_axis(x, s):
        y = np.fft.fft(x, axis=2) if s < 0 else np.fft.ifft(x, axis=2) * x.shape[2]
        y = np.fft.ifft(y, axis=1) * x.shape[1] if s < 0 else np.fft.fft(y, axis=1)
        return np.fft.fft(y, axis=0) if s < 0 else np.fft.ifft(y, axis=0) * x.shape[0]

    return [wrong_sign, transposed, dropped_term, missing_axis, wrong_index, conj_twiddle_on_one_axis]


@pytest.mark.parametrize("mutant", _mutants(), ids=lambda f: f.__name__)
def test_pins_catch_planted_mistakes(mutant):
    res = all_pins(mutant)
    assert not all(res.values()), f"mutant {mutant.__name__} passed every pin: {res}"


# --------------------------------------------------------- the generator ----
def test_generator_matches_published_splitmix64():
    # Reference values of SplitMix64 from its published definition, computed
    # with Python integers: the torch int64 implementation must agree.
    r = synth.splitmix64_int(synth.SEED, 0, 16)
    for j in range(16):
        expect = synth.splitmix64_py(synth.SEED, j)
        got = int(r[j]) & ((1 << 64) - 1)
        assert got == expect
    # seed 0, first output of the sequential generator started at state 0
    assert synth.splitmix64_py(0, 0) == 0xE220A8397B1DCDAF


def test_generator_values_and_rounding():
    v = synth.uniform_pm1(synth.SEED, 0, 1 << 16)
    assert v.min() >= -1.0 and v.max() < 1.0
    assert abs(float(v.mean())) < 0.01
    g64 = synth.complex_grid((4, 5, 6), torch.complex128)
    g32 = synth.complex_grid((4, 5, 6), torch.complex64)
    assert torch.equal(g32, g64.to(torch.complex64))
    flat = torch.view_as_real(g64.reshape(-1)).reshape(-1)
    assert torch.equal(flat, synth.uniform_pm1(synth.SEED, 0, flat.numel()))
    # random access: a window equals the same slice of a longer draw
    assert torch.equal(synth.uniform_pm1(7, 1000, 10), synth.uniform_pm1(7, 0, 1010)[1000:])


def test_paper_tuning_arithmetic_fixture():
    vals = {}
    with open(os.path.join(GOLDEN, "paper_values.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()[:2]
                vals[k] = float(v)
    runs = vals["tune_candidates"] * vals["tune_reps"]
    assert runs == vals["tune_runs"]
    pct = 100.0 * runs / (runs + vals["exec_runs_example"])
    assert round(pct, 2) == vals["tune_overhead_percent"]
