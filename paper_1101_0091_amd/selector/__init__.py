"""Kernel-variant selector: weights file format, train/held-out split and
the evaluation against the exhaustive autotuner.

The network itself (16 -> 64 -> 64 -> 6, ReLU) runs inside libspmv: its
forward/backward/Adam kernels train it (``train.py``) and plan creation runs
its forward kernel on the plan's row-statistics features.

Weights file (little endian): 8-byte magic ``SPMVSEL1``, then float32
params[5638], mu[16], sigma[16], lo[16], hi[16], margin[1].
"""
from __future__ import annotations

import os

import numpy as np

MAGIC = b"SPMVSEL1"
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights.bin")
DEFAULT_LABELS = os.path.join(HERE, "labels_family512.jsonl")
SPLIT_SEED = 5


def pack_weights(path, theta, mu, sigma, lo, hi, margin):
    with open(path, "wb") as f:
        f.write(MAGIC)
        for a in (theta, mu, sigma, lo, hi, np.array([margin])):
            f.write(np.asarray(a, dtype="<f4").tobytes())


def unpack_weights(path):
    raw = open(path, "rb").read()
    if raw[:8] != MAGIC:
        raise ValueError(f"{path}: not a selector weights file")
    a = np.frombuffer(raw[8:], dtype="<f4")
    if a.size != 5638 + 16 * 4 + 1:
        raise ValueError(f"{path}: wrong size")
    o = 0
    out = []
    for n in (5638, 16, 16, 16, 16, 1):
        out.append(a[o:o + n].copy())
        o += n
    theta, mu, sigma, lo, hi, margin = out
    return theta, mu, sigma, lo, hi, float(margin[0])


def split_ids(ids):
    """Seeded 384/128 split of the matrix collection (indices into ids)."""
    n = len(ids)
    perm = np.random.default_rng(SPLIT_SEED).permutation(n)
    ntr = int(round(0.75 * n))
    return np.sort(perm[:ntr]), np.sort(perm[ntr:])


def geomean(x):
    x = np.asarray(x, dtype=np.float64)
    return float(np.exp(np.mean(np.log(x))))


def threshold_rule(F, T, tr):
    """Best rule 'variant a if mean row length <= thr else variant b' on the
    training set (the hand-written heuristic the selector is compared with)."""
    best = None
    nnzr = F[:, 2]
    for thr in np.unique(np.quantile(nnzr[tr], np.linspace(0, 1, 41))):
        for a in range(6):
            for b in range(6):
                ch = np.where(nnzr[tr] <= thr, a, b)
                g = geomean(T[tr, ch] / T[tr].min(axis=1)) if len(tr) else 1.0
                if best is None or g < best[0]:
                    best = (g, float(thr), a, b)
    return best


def autotune_cost(times) -> float:
    """Cost of the library's autotune in multiples of the fastest variant's
    product, from per-variant times: every variant gets one warm-up and one
    timed launch, and four more when it is within 1.5x of the best time seen
    before it (the schedule of `autotune` in api.hip)."""
    best, cost = float("inf"), 0.0
    for t in times:
        cost += (6.0 if t <= 1.5 * best else 2.0) * t
        best = min(best, t)
    return cost / min(times)


def evaluate(F, T, tr, te, pred_te):
    """Held-out comparison: geomean(t_choice / t_best) for the network, the
    best single fixed variant (chosen on the training set) and the threshold
    rule; plus hit rate and how often the confidence check would fall back."""
    best_te = T[te].min(axis=1)
    fixed = int(np.argmin([geomean(T[tr, v] / T[tr].min(axis=1)) for v in range(6)]))
    _, thr, a, b = threshold_rule(F, T, tr)
    mlp_choice = np.argmin(pred_te, axis=1)
    rule_choice = np.where(F[te, 2] <= thr, a, b)
    srt = np.sort(pred_te, axis=1)
    gap = srt[:, 1] - srt[:, 0]
    rep = {
        "n_train": int(len(tr)), "n_heldout": int(len(te)),
        "mlp_geomean_vs_best": geomean(T[te, mlp_choice] / best_te),
        "fixed_variant": fixed,
        "fixed_geomean_vs_best": geomean(T[te, fixed] / best_te),
        "rule": {"thr_mean_row_len": thr, "below": a, "above": b},
        "rule_geomean_vs_best": geomean(T[te, rule_choice] / best_te),
        "mlp_hit_rate": float(np.mean(mlp_choice == np.argmin(T[te], axis=1))),
        "best_variant_histogram_heldout": np.bincount(np.argmin(T[te], axis=1), minlength=6).tolist(),
        "mlp_choice_histogram_heldout": np.bincount(mlp_choice, minlength=6).tolist(),
        "gap_median": float(np.median(gap)),
        "autotune_cost_over_best": float(np.mean([autotune_cost(t) for t in T[te]])),
    }
    return rep
