"""Train the kernel-variant selector on the GPU with libspmv's own network
kernels (spmv_mlp_forward / spmv_mlp_backward / spmv_mlp_adam), then write
the packed weights file and a held-out evaluation report.

Target per matrix and variant: relative log2 time, log2 t_v minus the mean
over the variants timed on that matrix (the network ranks variants; the
argmin of the usable outputs is the choice). V6 has no time where the chunked
copy did not fit; its target is then NaN, which the loss skips. Inputs: the
16 row-statistics features, standardised with the training-set mean and
standard deviation.

    python -m paper_1101_0091_amd.selector.train --labels FILE --out-dir DIR
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

from . import N_OUT, N_PARAMS, evaluate, geomean, labels_meta, pack_weights, split_ids

SHAPES = [(64, 16), (64,), (64, 64), (64,), (N_OUT, 64), (N_OUT,)]


def he_init(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = math.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-lim, lim, size=s))
        else:
            parts.append(np.zeros(s))
    theta = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
    assert theta.size == N_PARAMS
    return theta


def load_labels(path, key="us"):
    """Records sorted by id, features F, times T[:, 7] (NaN: not timed), ids."""
    recs = [json.loads(line) for line in open(path) if line.strip()]
    recs.sort(key=lambda r: r["id"])
    F = np.array([r["features"] for r in recs], dtype=np.float64)
    T = np.array([[np.nan if t is None else t for t in r[key]] for r in recs], dtype=np.float64)
    ids = np.array([r["id"] for r in recs])
    return recs, F, T, ids


def targets(T):
    lt = np.log2(T)
    return lt - np.nanmean(lt, axis=1, keepdims=True)


def label_noise(path):
    """Run-to-run spread of the labels: geomean over matrices and variants of
    max(t1, t2) / min(t1, t2) for the two timing passes, and the same for the
    best variant of the first pass alone."""
    _, _, T1, _ = load_labels(path, "us")
    _, _, T2, _ = load_labels(path, "us_rep")
    ok = ~np.isnan(T1) & ~np.isnan(T2)
    r = np.maximum(T1[ok], T2[ok]) / np.minimum(T1[ok], T2[ok])
    b = np.nanargmin(T1, axis=1)
    rb = np.array([max(T1[i, v], T2[i, v]) / min(T1[i, v], T2[i, v]) for i, v in enumerate(b)])
    # the fraction of matrices whose best variant differs between the passes
    flip = float(np.mean(np.nanargmin(T1, axis=1) != np.nanargmin(T2, axis=1)))
    return {"label_noise_geomean": geomean(r), "label_noise_best_geomean": geomean(rb),
            "label_best_variant_flip_rate": flip}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--labels", required=True)
    ap.add_argument("--out-dir", required=True)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--margin", type=float, default=0.05)
    args = ap.parse_args(argv)
    import torch

    import paper_1101_0091_amd as pkg

    recs, F, T, ids = load_labels(args.labels)
    tr, te = split_ids(ids)
    mu = F[tr].mean(axis=0)
    sd = F[tr].std(axis=0)
    sd[sd < 1e-6] = 1.0
    X = ((F - mu) / sd).astype(np.float32)
    Y = targets(T).astype(np.float32)
    dev = torch.device("cuda:0")
    Xtr = torch.from_numpy(X[tr]).to(dev)
    Ytr = torch.from_numpy(Y[tr]).to(dev)
    nb = int(Xtr.shape[0])
    th = torch.from_numpy(he_init(args.seed)).to(dev)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    g = torch.empty_like(th)
    P = torch.empty((nb, N_OUT), dtype=torch.float32, device=dev)
    Z1 = torch.empty((nb, 64), dtype=torch.float32, device=dev)
    Z2 = torch.empty((nb, 64), dtype=torch.float32, device=dev)
    scratch = torch.empty(nb * (N_OUT + 64 + 64), dtype=torch.float32, device=dev)
    have = ~torch.isnan(Ytr)
    hist = []
    for t in range(1, args.steps + 1):
        pkg.spmv_mlp_forward(th, Xtr, nb, P, Z1, Z2)
        if t == 1 or t % 500 == 0 or t == args.steps:
            loss = float(torch.where(have, (P - Ytr) ** 2, 0.0).sum()) / P.numel()
            hist.append((t, loss))
            print(f"[train] step {t} loss {loss:.5f}", flush=True)
        pkg.spmv_mlp_backward(th, Xtr, Z1, Z2, P, Ytr, nb, scratch, g)
        lr = args.lr * (0.1 ** (t / args.steps))
        pkg.spmv_mlp_adam(th, g, m, v, t, lr)
    theta = th.cpu().numpy()
    # feature range accepted without fallback: training range widened by 10% of its span
    lo = F[tr].min(axis=0)
    hi = F[tr].max(axis=0)
    pad = 0.1 * (hi - lo) + 1e-9
    os.makedirs(args.out_dir, exist_ok=True)
    wpath = os.path.join(args.out_dir, "weights.bin")
    pack_weights(wpath, theta, mu.astype(np.float32), sd.astype(np.float32),
                 (lo - pad).astype(np.float32), (hi + pad).astype(np.float32), args.margin)
    # held-out predictions with the GPU forward kernel
    Xte = torch.from_numpy(X[te]).to(dev)
    Pte = torch.empty((len(te), N_OUT), dtype=torch.float32, device=dev)
    Z1e = torch.empty((len(te), 64), dtype=torch.float32, device=dev)
    Z2e = torch.empty((len(te), 64), dtype=torch.float32, device=dev)
    pkg.spmv_mlp_forward(th, Xte, len(te), Pte, Z1e, Z2e)
    rep = evaluate(F, T, tr, te, Pte.cpu().numpy())
    rep.update(label_noise(args.labels))
    rep["kernel_source_hash"] = labels_meta(args.labels)["kernel_source_hash"]
    rep["loss_history"] = hist
    rep["steps"] = args.steps
    rep["lr"] = args.lr
    json.dump(rep, open(os.path.join(args.out_dir, "report.json"), "w"), indent=1)
    print(json.dumps({k: rep[k] for k in rep if k != "loss_history"}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
