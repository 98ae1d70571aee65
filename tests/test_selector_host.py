"""Learned plan selector, host side (no GPU): candidates, features, weights
file handling, and -- on the committed MI355X timing dataset and weights --
what the trained network gains over the heuristic plan and what it saves
against exhaustive tuning, measured on held-out grids."""
import json
import os

import numpy as np
import pytest

import paper_1501_07350_amd as offt
from paper_1501_07350_amd import _lib, selector
import synth

D = selector.feature_dim()


def test_candidates_and_features():
    plans, feats = selector.candidates((64, 48, 60), 1, 1)
    assert feats.shape == (len(plans), D)
    assert plans[0] == offt.default_plan_string((64, 48, 60), __import__("torch").complex64)
    assert len(set(plans)) == len(plans)
    assert np.array_equal(selector.plan_features((64, 48, 60), 1, 1, plans), feats)
    # log2 of the axes, batch, precision flag, one-hot order
    f = feats[0]
    assert np.allclose(f[:3], np.log2([64, 48, 60])) and f[3] == 0 and f[4] == 1
    assert f[6:12].sum() == 1 and f[6] == 1    # order cba


def test_weights_io_and_errors(tmp_path):
    p = np.random.default_rng(0).standard_normal(_lib.load().offt_mlp_nparams(D, 64)).astype(np.float32) * 0.1
    w = tmp_path / "w.txt"
    selector.write_weights(str(w), np.zeros(D), np.ones(D), 1.0, 2.0, p)
    plans, feats = selector.candidates((32, 32, 32), 1, 0)
    s = selector.scores(str(w), feats)
    assert s.shape == (len(plans),) and np.all(np.isfinite(s))
    assert selector.choose(str(w), (32, 32, 32), 1, 0) == plans[int(np.argmin(s))]
    bad = tmp_path / "bad.txt"
    bad.write_text("offt-selector 1\ndims 45 64\n")
    with pytest.raises(_lib.OfftError) as ei:
        selector.scores(str(bad), feats)
    assert ei.value.code == _lib.ERR_IO
    with pytest.raises(_lib.OfftError):
        selector.scores(str(tmp_path / "none.txt"), feats)
    wrong = tmp_path / "wrong.txt"
    selector.write_weights(str(wrong), np.zeros(10), np.ones(10), 0, 1, np.zeros(_lib.load().offt_mlp_nparams(10, 64)))
    with pytest.raises(_lib.OfftError):
        selector.scores(str(wrong), feats[:, :10].copy())


def test_selector_grids_are_seeded_and_bounded():
    g = synth.selector_grids(300)
    assert g == synth.selector_grids(300)
    L = set(synth.smooth_lengths())
    for a, b, c, bt, dt in g:
        assert {a, b, c} <= L and bt in (1, 2, 4, 8) and dt in (0, 1) and a * b * c * bt <= 1 << 28
    assert synth.selector_grids(5, skip=295) == g[295:]


@pytest.mark.skipif(not (os.path.exists(selector.DATASET) and os.path.exists(selector.WEIGHTS)),
                    reason="the MI355X timing dataset and trained weights are not present")
def test_learned_selector_gain_on_heldout_grids():
    records = selector.read_dataset(selector.DATASET)
    train_r, held = selector.split(records)
    assert len(held) >= 100 and len(train_r) >= 1000
    ev = selector.evaluate(held, selector.WEIGHTS)
    print(json.dumps(ev, indent=1))
    # better than the heuristic plan the library uses without tuning ...
    assert ev["regret_learned"]["mean"] < ev["regret_heuristic"]["mean"]
    assert ev["speedup_learned_over_heuristic_geomean"] > 1.0
    # ... at a tiny fraction of exhaustive tuning's cost
    assert ev["selection_us_mean"] * 1e-3 < 0.05 * ev["exhaustive_tuning_ms_mean"]


def test_access_mode_candidates_and_feature():
    """The candidate list ends with the heuristic plan with one axis's access
    mode switched (cached for a grid above 256 MiB, where passes stream by
    default; streaming below), and the per-axis access-mode feature follows
    the mode the pass runs with."""
    per_axis = 15
    for dims, batch, dtype, suffix, default_mode in (((512, 512, 512), 1, 0, "/c", 1.0),
                                                     ((64, 48, 60), 1, 1, "/s", 0.0)):
        plans, feats = selector.candidates(dims, batch, dtype)
        switched = [i for i, p in enumerate(plans) if suffix in p]
        assert len(switched) == 3, plans
        assert switched == list(range(len(plans) - 3, len(plans)))
        mode = feats[:, 12 + per_axis - 1::per_axis]          # the mode feature of axes a, b, c
        assert np.all(mode[0] == default_mode)
        flipped = []
        for i in switched:
            f = np.flatnonzero(mode[i] != default_mode)
            assert len(f) == 1, (plans[i], mode[i])
            flipped.append(int(f[0]))
        assert sorted(flipped) == [0, 1, 2]
