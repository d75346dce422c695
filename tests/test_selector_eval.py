"""The selector's evaluation helpers on small synthetic label sets (CPU):
the V6 mask, the fixed policy's fallback, the autotune cost with a missing
variant, the label-noise measure and the label file's source-hash check."""
import json
import os

import numpy as np
import pytest

from paper_1101_0091_amd import selector as sel
from paper_1101_0091_amd.selector import labels as lab
from paper_1101_0091_amd.selector import train

NAN = float("nan")


def test_masked_argmin_ignores_v6_without_a_time():
    P = np.array([[3.0, 2.0, 2.0, 2.0, 1.0, 2.0, 0.0],
                  [3.0, 2.0, 2.0, 2.0, 1.0, 2.0, 0.0]])
    T = np.array([[9.0, 8, 8, 8, 5, 8, 4],
                  [9.0, 8, 8, 8, 5, 8, NAN]])
    assert sel.masked_argmin(P, T).tolist() == [6, 4]


def test_fixed_policy_falls_back_to_v4():
    T = np.array([[9.0, 8, 8, 8, 5, 8, 4],
                  [9.0, 8, 8, 8, 5, 8, NAN]])
    assert sel.fixed_times(T, 6).tolist() == [4.0, 5.0]
    assert sel.fixed_times(T, 0).tolist() == [9.0, 9.0]
    assert sel.best_times(T).tolist() == [4.0, 5.0]


def test_autotune_cost_skips_missing_variants():
    # every variant: warm-up + one timed launch (2 t), four more (6 t) when
    # within 1.5x of the best time seen before it
    t = [10.0, 4.0, 5.0, 20.0, 4.0, 7.0, NAN]
    cost = (6 * 10 + 6 * 4 + 6 * 5 + 2 * 20 + 6 * 4 + 2 * 7) / 4.0
    assert sel.autotune_cost(t) == pytest.approx(cost)


def test_evaluate_on_a_planted_set():
    """A network output equal to the true log times picks the best variant
    everywhere: hit rate 1 and geomean 1; the fixed policy pays where its
    variant is not the best."""
    rng = np.random.default_rng(0)
    n = 40
    T = rng.uniform(1, 2, size=(n, 7))
    T[: n // 2, 6] = NAN
    F = rng.uniform(0, 1, size=(n, 16))
    tr, te = np.arange(0, n, 2), np.arange(1, n, 2)
    P = np.log2(T[te])
    rep = sel.evaluate(F, T, tr, te, np.nan_to_num(P, nan=0.0))
    assert rep["mlp_hit_rate"] == 1.0
    assert rep["mlp_geomean_vs_best"] == pytest.approx(1.0)
    assert rep["fixed_geomean_vs_best"] >= 1.0
    assert rep["heldout_with_v6_copy"] == int(np.sum(~np.isnan(T[te, 6])))


def _write_labels(path, rows):
    with open(path, "w") as f:
        for r in rows:
            f.write(json.dumps(r) + "\n")


def test_label_noise(tmp_path):
    rows = []
    for i, (a, b) in enumerate(((1.0, 1.1), (2.0, 2.0))):
        rows.append({"id": i, "features": [0.0] * 16, "us": [a, 3.0, 3, 3, 3, 3, None],
                     "us_rep": [b, 3.0, 3, 3, 3, 3, None]})
    p = str(tmp_path / "l.jsonl")
    _write_labels(p, rows)
    nz = train.label_noise(p)
    # variant 0 is the best in both records: max/min 1.1 and 1.0
    assert nz["label_noise_best_geomean"] == pytest.approx(np.sqrt(1.1))
    assert nz["label_best_variant_flip_rate"] == 0.0
    T = train.targets(train.load_labels(p)[2])
    assert np.isnan(T[:, 6]).all() and np.allclose(np.nanmean(T, axis=1), 0.0)


def test_label_file_refuses_other_sources(tmp_path):
    p = str(tmp_path / "sub" / "l.jsonl")
    lab.check_meta(p)  # new file: writes the sidecar (and the folder)
    meta = sel.labels_meta(p)
    assert meta["kernel_source_hash"] == sel.source_hash()
    _write_labels(p, [{"id": 0}])
    lab.check_meta(p)  # same sources: accepted
    meta["kernel_source_hash"] = "0" * 16
    with open(sel.labels_meta_path(p), "w") as f:
        json.dump(meta, f)
    with pytest.raises(SystemExit):
        lab.check_meta(p)
    assert os.path.exists(sel.labels_meta_path(p))
