"""Pins of the distributed-flow reference oracle/dist.py (CPU only).

The reference runs the paper's calculation flow over Np processes (Sec. 2,
Eq. 2 blocks; Sec. 3.1.1 steps; transpose order abc -> cab -> cba of
Fig. 1b).  It is pinned against things it does not share code with:
numpy.fft along single axes and over the whole grid, the brute-force owner
enumeration of oracle/decomp.py, coded grids whose values name their own
coordinates, the round trip, and mutations that must fail.
"""
import numpy as np
import pytest

from oracle import decomp, dist

SHAPES = [(4, 6, 8), (5, 3, 4), (8, 8, 8), (6, 10, 9), (2, 12, 3), (1, 4, 6)]


def cases():
    out = []
    for shape in SHAPES:
        lim = dist.max_processes(shape)
        for np_ in sorted({1, 2, 3, 4, 5, 8, shape[0] + 1, lim} & set(range(1, lim + 1))):
            out.append((shape, np_))
    return out


CASES = cases()


def grid(shape, seed=5):
    r = np.random.default_rng(seed)
    return r.uniform(-1, 1, shape) + 1j * r.uniform(-1, 1, shape)


def in_order(g, order):
    """A (Na, Nb, Nc) array held in `order`, flattened (numpy transpose)."""
    return np.ascontiguousarray(np.transpose(g, dist.ORDERS[order])).reshape(-1)


@pytest.mark.parametrize("shape,np_", CASES, ids=lambda v: str(v))
def test_every_state_of_the_forward_flow(shape, np_):
    x = grid(shape)
    states, (m0, m1) = dist.forward_steps(x, np_)
    c = np.fft.fft(x, axis=2)
    cb = np.fft.fft(c, axis=1)
    cba = np.fft.fft(cb, axis=0)
    want = [in_order(c, "abc"), in_order(c, "cab"), in_order(cb, "cab"), in_order(cb, "cba"),
            in_order(cba, "cba")]
    for k, (st, w) in enumerate(zip(states, want)):
        g = dist.gather(st)
        assert np.max(np.abs(g - w)) <= 1e-12 * max(1.0, np.max(np.abs(w))), k
    # the finishing cba distribution of the whole transform
    assert np.allclose(dist.gather(states[-1]), np.fft.fftn(x).transpose(2, 1, 0).reshape(-1), atol=1e-12)


@pytest.mark.parametrize("shape,np_", CASES, ids=lambda v: str(v))
def test_exchange_counts_match_the_owner_enumeration(shape, np_):
    na, nb, nc = shape
    _, (m0, m1) = dist.forward_steps(grid(shape), np_)
    assert np.array_equal(m0, decomp.transpose_counts(na, nb, nc, np_, 0))
    assert np.array_equal(m1, decomp.transpose_counts(na, nb, nc, np_, 1))
    # the backward flow runs the two exchanges in reverse: transposed matrices
    states, _ = dist.forward_steps(grid(shape), np_)
    _, (b0, b1) = dist.backward_steps(states[-1], shape, np_)
    assert np.array_equal(b0, m1.T) and np.array_equal(b1, m0.T)


@pytest.mark.parametrize("shape,np_", CASES, ids=lambda v: str(v))
def test_blocks_follow_eq2_and_hold_whole_lines(shape, np_):
    for order in dist.ORDERS:
        n1, n2, n3 = dist.order_dims(shape, order)
        b = dist.blocks(shape, order, np_)
        assert b[0][0] == 0 and b[-1][1] == n1 * n2 * n3
        assert all(b[p][1] == b[p + 1][0] for p in range(np_ - 1))
        unit = n2 * n3 if np_ <= n1 else n3
        assert all((e - s) % unit == 0 for s, e in b)


@pytest.mark.parametrize("shape,np_", [(s, n) for s, n in CASES if n > 1], ids=lambda v: str(v))
def test_exchange_moves_each_point_to_its_owner(shape, np_):
    """A coded grid (value = a + 100 b + 10^4 c) after each exchange: every
    process holds exactly the points its block of the new order names."""
    a, b, c = np.meshgrid(*(np.arange(n) for n in shape), indexing="ij")
    code = (a + 100 * b + 10000 * c).astype(np.complex128)
    local = dist.scatter(code, shape, np_)
    cab, _ = dist.exchange(local, shape, "abc", "cab", np_)
    for q, (s, e) in enumerate(dist.blocks(shape, "cab", np_)):
        ca, cb, cc = dist.coordinates(np.arange(s, e), shape, "cab")
        assert np.array_equal(cab[q].real, ca + 100 * cb + 10000 * cc)
    cba, _ = dist.exchange(cab, shape, "cab", "cba", np_)
    for q, (s, e) in enumerate(dist.blocks(shape, "cba", np_)):
        ca, cb, cc = dist.coordinates(np.arange(s, e), shape, "cba")
        assert np.array_equal(cba[q].real, ca + 100 * cb + 10000 * cc)
    back, _ = dist.exchange(cba, shape, "cba", "abc", np_)
    assert np.array_equal(dist.gather(back), code.reshape(-1))


@pytest.mark.parametrize("shape,np_", CASES, ids=lambda v: str(v))
def test_round_trip(shape, np_):
    x = grid(shape, 9)
    states, _ = dist.forward_steps(x, np_)
    back, _ = dist.backward_steps(states[-1], shape, np_)
    z = dist.gather(back[-1]) / x.size
    assert np.max(np.abs(z - x.reshape(-1))) <= 1e-13


def test_one_process_exchanges_nothing():
    x = grid((6, 10, 9))
    states, (m0, m1) = dist.forward_steps(x, 1)
    assert m0.shape == (1, 1) and m0[0, 0] == x.size and m1[0, 0] == x.size


def test_mutations_fail_a_pin():
    """Plausible mistakes in the flow are caught: blocks of the wrong order,
    the wrong axis transformed, and a conjugated step."""
    shape, np_ = (6, 10, 9), 4
    x = grid(shape)
    want = np.fft.fftn(x).transpose(2, 1, 0).reshape(-1)
    orig_blocks = dist.blocks

    def wrong_blocks(shp, order, n):
        return orig_blocks(shp, "abc", n)   # every order split as abc

    dist.blocks = wrong_blocks
    try:
        # the gathered grid does not see block boundaries; the counts do
        _, (m0, _) = dist.forward_steps(x, np_)
        assert not np.array_equal(m0, decomp.transpose_counts(*shape, np_, 0))
    finally:
        dist.blocks = orig_blocks
    # the wrong axis: transform along the slowest axis of each order
    st = dist.scatter(x, shape, np_)
    bad = [np.fft.fft(b.reshape(-1, shape[2]), axis=0).reshape(-1) for b in st]
    assert not np.allclose(dist.gather(bad), np.fft.fft(x, axis=2).reshape(-1))
    # a backward step in a forward flow
    states, _ = dist.forward_steps(np.conj(x), np_)
    assert not np.allclose(dist.gather(states[-1]), want)
