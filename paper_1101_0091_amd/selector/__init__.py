"""Kernel-variant selector: weights file format, train/held-out split, the
label set's kernel-source hash and the evaluation against the exhaustive
autotuner.

The network itself (16 -> 64 -> 64 -> 7, ReLU) runs inside libspmv: its
forward/backward/Adam kernels train it (``train.py``) and plan creation runs
its forward kernel on the plan's row-statistics features. Output v is the
predicted relative log2 time of variant Vv; V6 counts only for plans that
hold the chunked copy.

Weights file (little endian): 8-byte magic ``SPMVSEL2``, then float32
params[5703], mu[16], sigma[16], lo[16], hi[16], margin[1].
"""
from __future__ import annotations

import hashlib
import json
import os
import re

import numpy as np

MAGIC = b"SPMVSEL2"
N_OUT = 7
N_PARAMS = 5703
V4, V6 = 4, 6
HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "csrc")
DEFAULT_WEIGHTS = os.path.join(HERE, "weights.bin")
DEFAULT_LABELS = os.path.join(HERE, "labels_family512.jsonl")
SPLIT_SEED = 5
# the sources of the V0-V6 product kernels, the V4 forms, and the create-time
# analysis that computes the features and chooses the V4 form's tables
LABEL_SOURCES = ("spmv_kernels.hip", "sell.hip", "window.hip", "device.hpp", "common.hpp",
                 "analysis.hip")


def code_only(text: str) -> str:
    """Source text without comments and with whitespace collapsed: an edit to a
    comment does not change a kernel."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash(files=LABEL_SOURCES) -> str:
    """First 16 hex digits of the SHA-256 of the code of `files` (in csrc)."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f)) as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def labels_meta_path(labels_path: str) -> str:
    return os.path.splitext(labels_path)[0] + ".meta.json"


def labels_meta(labels_path: str) -> dict:
    with open(labels_meta_path(labels_path)) as f:
        return json.load(f)


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
    if a.size != N_PARAMS + 16 * 4 + 1:
        raise ValueError(f"{path}: wrong size")
    o = 0
    out = []
    for n in (N_PARAMS, 16, 16, 16, 16, 1):
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


def fixed_times(T, v):
    """Times of the fixed policy 'always Vv' (V6 where the plan holds the
    copy, else V4, the library's default variant)."""
    t = T[:, v].copy()
    miss = np.isnan(t)
    t[miss] = T[miss, V4]
    return t


def best_times(T):
    return np.nanmin(T, axis=1)


def masked_argmin(P, T):
    """Per row, the output with the smallest value among the variants that
    have a time (V6 is masked where the copy did not fit), as plan creation
    does."""
    P = np.where(np.isnan(T), np.inf, P)
    return np.argmin(P, axis=1)


def threshold_rule(F, T, tr):
    """Best rule 'variant a if mean row length <= thr else variant b' on the
    training set (the hand-written heuristic the selector is compared with)."""
    best = None
    nnzr = F[:, 2]
    bt = best_times(T[tr])
    ft = [fixed_times(T[tr], v) for v in range(N_OUT)]
    for thr in np.unique(np.quantile(nnzr[tr], np.linspace(0, 1, 41))):
        low = nnzr[tr] <= thr
        for a in range(N_OUT):
            for b in range(N_OUT):
                g = geomean(np.where(low, ft[a], ft[b]) / bt) if len(tr) else 1.0
                if best is None or g < best[0]:
                    best = (g, float(thr), a, b)
    return best


def autotune_cost(times) -> float:
    """Cost of the library's autotune in multiples of the fastest variant's
    product, from per-variant times (NaN: variant absent): every variant gets
    one warm-up and one timed launch, and four more when it is within 1.5x of
    the best time seen before it (the schedule of `autotune` in api.hip)."""
    best, cost = float("inf"), 0.0
    ts = [t for t in times if not np.isnan(t)]
    for t in ts:
        cost += (6.0 if t <= 1.5 * best else 2.0) * t
        best = min(best, t)
    return cost / min(ts)


def evaluate(F, T, tr, te, pred_te):
    """Held-out comparison: geomean(t_choice / t_best) for the network, the
    best single fixed variant (chosen on the training set) and the threshold
    rule; plus hit rate, the choice histograms and the predicted gaps."""
    best_te = best_times(T[te])
    fixed = int(np.argmin([geomean(fixed_times(T[tr], v) / best_times(T[tr]))
                           for v in range(N_OUT)]))
    _, thr, a, b = threshold_rule(F, T, tr)
    mlp_choice = masked_argmin(pred_te, T[te])
    rule_t = np.where(F[te, 2] <= thr, fixed_times(T[te], a), fixed_times(T[te], b))
    P = np.where(np.isnan(T[te]), np.inf, pred_te)
    srt = np.sort(P, axis=1)
    gap = srt[:, 1] - srt[:, 0]
    best_v = np.nanargmin(T[te], axis=1)
    rep = {
        "n_train": int(len(tr)), "n_heldout": int(len(te)),
        "mlp_geomean_vs_best": geomean(T[te][np.arange(len(te)), mlp_choice] / best_te),
        "fixed_variant": fixed,
        "fixed_geomean_vs_best": geomean(fixed_times(T[te], fixed) / best_te),
        "rule": {"thr_mean_row_len": thr, "below": a, "above": b},
        "rule_geomean_vs_best": geomean(rule_t / best_te),
        "mlp_hit_rate": float(np.mean(mlp_choice == best_v)),
        "best_variant_histogram_heldout": np.bincount(best_v, minlength=N_OUT).tolist(),
        "mlp_choice_histogram_heldout": np.bincount(mlp_choice, minlength=N_OUT).tolist(),
        "heldout_with_v6_copy": int(np.sum(~np.isnan(T[te, V6]))),
        "gap_median": float(np.median(gap)),
        "autotune_cost_over_best": float(np.mean([autotune_cost(t) for t in T[te]])),
    }
    return rep
