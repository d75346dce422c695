"""What the trained selector network gains over the method without it.

Uses the committed label run (every variant timed on the GPU for 512 seeded
matrices) and the committed weights (trained on the GPU with the library's
own kernels). The held-out choices are recomputed with the float64 oracle
network, so this test needs no GPU. Selector accuracy itself is not pinned by
the paper (it has no learned component): the exhaustive autotuner's timings
decide which choice was right."""
import json
import os

import numpy as np
import pytest

from oracle import mlp
from paper_1101_0091_amd.selector import (DEFAULT_LABELS, DEFAULT_WEIGHTS, evaluate, geomean,
                                          split_ids, unpack_weights)
from paper_1101_0091_amd.selector.train import load_labels

pytestmark = pytest.mark.skipif(not (os.path.exists(DEFAULT_LABELS) and
                                     os.path.exists(DEFAULT_WEIGHTS)),
                                reason="selector labels/weights not generated yet")


def _heldout_predictions():
    recs, F, T, ids = load_labels(DEFAULT_LABELS)
    theta, mu, sigma, lo, hi, margin = unpack_weights(DEFAULT_WEIGHTS)
    tr, te = split_ids(ids)
    X = ((F.astype(np.float32) - mu) / sigma).astype(np.float64)
    P = mlp.forward(theta.astype(np.float64), X[te])[0]
    return F, T, tr, te, P, (lo, hi, margin)


def test_split_is_384_128():
    recs, F, T, ids = load_labels(DEFAULT_LABELS)
    assert len(ids) == 512 and len(set(ids.tolist())) == 512
    tr, te = split_ids(ids)
    assert len(tr) == 384 and len(te) == 128 and not set(tr) & set(te)
    assert np.all(T > 0)


def test_network_beats_fixed_variant_and_rule():
    F, T, tr, te, P, _ = _heldout_predictions()
    rep = evaluate(F, T, tr, te, P)
    # the method without the network: the best single variant on the training set
    assert rep["mlp_geomean_vs_best"] < rep["fixed_geomean_vs_best"]
    assert rep["mlp_geomean_vs_best"] < rep["rule_geomean_vs_best"]
    assert rep["mlp_geomean_vs_best"] < 1.05
    assert rep["mlp_hit_rate"] > 0.7


def test_report_matches_oracle_recomputation():
    """The GPU-side evaluation written at training time agrees with the
    float64 oracle forward on the same weights."""
    F, T, tr, te, P, _ = _heldout_predictions()
    rep = json.load(open(os.path.join(os.path.dirname(DEFAULT_WEIGHTS), "report.json")))
    ours = evaluate(F, T, tr, te, P)
    assert rep["fixed_variant"] == ours["fixed_variant"]
    assert abs(rep["mlp_geomean_vs_best"] - ours["mlp_geomean_vs_best"]) < 5e-3


def test_selection_cost_vs_autotune():
    """Choosing by the network costs one tiny forward pass; the autotuner
    runs every variant several times (its cost in multiples of one product)."""
    F, T, tr, te, P, _ = _heldout_predictions()
    from paper_1101_0091_amd.selector import autotune_cost as cost_of
    autotune_cost = np.array([cost_of(t) for t in T[te]])
    assert np.all(autotune_cost >= 12.0)  # at least warm-up + timed launch of each of 6
    assert geomean(autotune_cost) > 20
