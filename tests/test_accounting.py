"""Byte and volume accounting (host only, no GPU).

Per decomposition: the library's block distribution (Duy & Ozaki, Sec. 2,
Eq. 2) and transpose element counts against a brute-force enumeration
(oracle/decomp.py), closed forms of the 1-D decomposition, the localisation
of Fig. 1b, and the 256^3 statements of Sec. 4.1.  Per plan: the predicted
bytes of a pass against the HBM traffic rocprofv3 measured for the committed
profiles ("theory and practice", Sec. 4.1)."""
import json
import os

import numpy as np
import pytest
import torch

import paper_1501_07350_amd as offt
from oracle import decomp as ref

HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC = os.path.join(os.path.dirname(HERE), "profiles", "pmc_traffic.json")

GRIDS = [(8, 6, 10), (5, 7, 3), (16, 4, 12), (12, 12, 12), (3, 9, 4)]


@pytest.mark.parametrize("dims", GRIDS, ids=lambda d: "x".join(map(str, d)))
def test_block_distribution_matches_eq2(dims):
    n1, n2, n3 = dims
    for np_ in range(1, n1 * n2 + 1):
        starts = [offt.decomp_start(n1, n2, n3, np_, p) for p in range(np_ + 1)]
        assert starts == [ref.block_start(n1, n2, n3, np_, p) for p in range(np_ + 1)]
        assert starts[0] == 0 and starts[-1] == n1 * n2 * n3 and starts == sorted(starts)
        unit = n2 * n3 if np_ <= n1 else n3          # whole planes (1-D) or whole lines (2-D)
        sizes = np.diff(starts)
        assert np.all(sizes % unit == 0)
        assert sizes.max() - sizes.min() <= unit       # block distribution: balanced to one unit


@pytest.mark.parametrize("dims", GRIDS, ids=lambda d: "x".join(map(str, d)))
@pytest.mark.parametrize("step", [0, 1], ids=["abc-cab", "cab-cba"])
def test_transpose_counts_match_brute_force(dims, step):
    n1, n2, n3 = dims
    limit = min(n1 * n2, n3 * n1) if step == 0 else min(n3 * n1, n3 * n2)
    for np_ in sorted({1, 2, 3, 4, 5, 7, n1, n1 + 1, n3, n3 + 1, limit} & set(range(1, limit + 1))):
        m = ref.transpose_counts(n1, n2, n3, np_, step)
        got = np.array([[offt.transpose_count(n1, n2, n3, np_, step, p, q) for q in range(np_)]
                        for p in range(np_)])
        assert np.array_equal(got, m), (np_, step)
        assert offt.transpose_volume(n1, n2, n3, np_, step) == ref.transpose_volume(n1, n2, n3, np_, step)


def test_one_d_decomposition_closed_forms():
    # Np dividing N1 and N3: every process keeps 1/Np of its slab and sends the
    # rest, so abc -> cab moves N (Np - 1) / Np elements; with Np <= N3 the
    # cab and cba orders share their c-slabs and cab -> cba is local (Fig. 1b)
    for (n1, n2, n3) in [(8, 6, 10), (16, 4, 12), (64, 64, 64), (256, 256, 256)]:
        N = n1 * n2 * n3
        for np_ in (1, 2, 4):
            if n1 % np_ or n3 % np_:
                continue
            assert offt.transpose_volume(n1, n2, n3, np_, 0) == N * (np_ - 1) // np_
            assert offt.transpose_volume(n1, n2, n3, np_, 1) == 0
        for np_ in range(1, min(n1, n3) + 1, max(1, min(n1, n3) // 7)):
            assert offt.transpose_volume(n1, n2, n3, np_, 1) == 0


def test_volume_at_256_cubed_switches_to_2d_beyond_256_processes():
    """Sec. 4.1: at 256^3 the decomposition is 1-D up to 256 processes and 2-D
    beyond, with a surge in volume from 256 to 512 processes.  Bytes as the
    paper scales them: elements x 16 B (double complex) x 2 (send + receive)."""
    n = 256
    vol = {}
    for np_ in (2, 4, 16, 64, 128, 256, 512, 1024, 4096):
        v0 = offt.transpose_volume(n, n, n, np_, 0)
        v1 = offt.transpose_volume(n, n, n, np_, 1)
        vol[np_] = (v0 + v1) * 16 * 2
        if np_ <= n:
            assert v1 == 0 and v0 == n ** 3 * (np_ - 1) // np_   # one transpose step only
        else:
            assert v1 > 0                                         # 2-D: cab -> cba no longer local
    assert vol[512] > 1.5 * vol[256]
    assert all(vol[a] <= vol[b] for a, b in zip(sorted(vol), sorted(vol)[1:]))


def test_invalid_decompositions_are_rejected():
    with pytest.raises(offt.OfftError):
        offt.decomp_start(4, 4, 4, 17, 0)        # Np > N1 N2: outside Eq. 2
    with pytest.raises(offt.OfftError):
        offt.transpose_volume(4, 4, 2, 9, 0)     # cab order: Np > N3 N1
    with pytest.raises(offt.OfftError):
        offt.transpose_count(4, 4, 4, 4, 2, 0, 0)
    with pytest.raises(offt.OfftError):
        offt.transpose_count(4, 4, 4, 4, 0, 0, 4)


def test_pass_bytes():
    assert offt.pass_bytes((512, 512, 512), torch.complex128) == 2 * 512 ** 3 * 16
    assert offt.pass_bytes((48, 60, 80), torch.complex64, batch=3) == 2 * 3 * 48 * 60 * 80 * 8
    with pytest.raises(offt.OfftError):
        offt.pass_bytes((7, 4, 4))


@pytest.mark.skipif(not os.path.exists(TRAFFIC), reason="no committed rocprofv3 traffic profile")
def test_predicted_pass_bytes_equal_measured_hbm_traffic():
    """Every pass the committed profile measured (FETCH_SIZE + WRITE_SIZE,
    scaled by a plain copy's counters) at 512^3 and 1024^3 moved the
    predicted bytes within 1% (the kernels with 2-part exchanges at 32
    complex64 columns up to 1.0%, the tuned plans within 0.3%; bound 1.5%)."""
    d = json.load(open(TRAFFIC))
    checked = 0
    for tag, w in d["workloads"].items():
        n = int(tag.split("_")[0])
        dtype = torch.complex128 if tag.endswith("f64") else torch.complex64
        predicted = offt.pass_bytes((n, n, n), dtype)
        assert w["algorithmic_bytes"] == predicted
        for key, measured in w["pass_bytes"].items():
            assert abs(measured / predicted - 1) <= 0.015, (tag, key, measured, predicted)
            checked += 1
    assert checked >= 4
    assert {"512_f64", "512_f32", "1024_f32"} <= set(d["workloads"])
