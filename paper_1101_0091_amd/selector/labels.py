"""Label run for the kernel-variant selector: time every variant V0-V6 on the
seeded matrix collection (N log-uniform in [1e4, 2e7]; uniform, power-law
or banded rows) and append one JSON line per matrix. V4 runs in the form the
plan chooses by default; V6 only where the chunked copy fits its reserve
(else its time is null). Every variant is timed in two separate passes (the
median of 7 launches each), so the label noise can be measured.

The sidecar FILE.meta.json holds the hash of the kernel sources the labels
were taken with; a run refuses to append to labels of other sources.
Resumable: matrices already in the output file are skipped.

    python -m paper_1101_0091_amd.selector.labels --out FILE [--start 0 --stop 512]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import LABEL_SOURCES, labels_meta_path, source_hash

SEED = 5
NLO, NHI = 1e4, 2e7


def time_variants(M, Bd, C, variants, reps=7, warmup=2):
    import numpy as np
    import torch
    s = torch.cuda.current_stream()
    out = []
    for v in variants:
        M.variant = v
        for _ in range(warmup):
            M.apply(Bd, C)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(s)
            M.apply(Bd, C)
            b.record(s)
        torch.cuda.synchronize()
        out.append(float(np.median([a.elapsed_time(b) for a, b in ev])) * 1000.0)
    return out


def check_meta(path: str) -> None:
    """Write the sidecar for a new label file, or check an existing one."""
    meta = {"kernel_source_hash": source_hash(), "files": list(LABEL_SOURCES),
            "variants": "V0-V6", "seed": SEED, "n_range": [NLO, NHI]}
    mp = labels_meta_path(path)
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    if os.path.exists(path) and os.path.getsize(path) > 0:
        old = json.load(open(mp)) if os.path.exists(mp) else {}
        if old.get("kernel_source_hash") != meta["kernel_source_hash"]:
            raise SystemExit(f"{path} was labelled with other kernel sources "
                             f"({old.get('kernel_source_hash')} != {meta['kernel_source_hash']}); "
                             "start a new file")
    else:
        with open(mp, "w") as f:
            json.dump(meta, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--stop", type=int, default=512)
    args = ap.parse_args(argv)
    check_meta(args.out)
    import torch

    import crsgen
    import paper_1101_0091_amd as pkg
    done = set()
    if os.path.exists(args.out):
        for line in open(args.out):
            try:
                done.add(json.loads(line)["id"])
            except (ValueError, KeyError):
                pass
    dev = torch.device("cuda:0")
    for i in range(args.start, args.stop):
        if i in done:
            continue
        t0 = time.time()
        A, prm = crsgen.family_matrix(SEED, i, NLO, NHI)
        B = crsgen.uniform_vec(A.n_cols, SEED)
        tg = time.time() - t0
        M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(4) | pkg.SPMV_FLAG_SELL,
                                   device=dev)
        Bd = torch.from_numpy(B).to(dev)
        C = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
        has6 = M.sell_slots is not None
        vs = list(range(7 if has6 else 6))
        us = time_variants(M, Bd, C, vs)
        us_rep = time_variants(M, Bd, C, vs)
        if not has6:
            us.append(None)
            us_rep.append(None)
        rec = {"id": i, "n": A.n_rows, "nnz": A.nnz, "family": crsgen.FAMILY_NAMES[prm["family"]],
               "width": prm["width"], "features": [float(x) for x in M.features],
               "us": [None if t is None else round(t, 3) for t in us],
               "us_rep": [None if t is None else round(t, 3) for t in us_rep],
               "v4_form": pkg.V4_FORMS[M.v4_form], "sell_slots": M.sell_slots,
               "gen_s": round(tg, 2)}
        with open(args.out, "a") as f:
            f.write(json.dumps(rec) + "\n")
        best = min(range(len(vs)), key=lambda v: us[v])
        print(f"[labels] {i} n={A.n_rows} nnz={A.nnz} {rec['family']} best=V{best} "
              f"us={rec['us']} ({time.time() - t0:.1f}s)", flush=True)
        del M, Bd, C, A
        torch.cuda.empty_cache()


if __name__ == "__main__":
    sys.exit(main())
