"""Label run for the kernel-variant selector: time every variant on the
seeded matrix collection (N log-uniform in [1e4, 2e7]; uniform, power-law
or banded rows) and append one JSON line per matrix. Resumable: matrices
already in the output file are skipped.

    python -m paper_1101_0091_amd.selector.labels --out FILE [--start 0 --stop 512]
    python -m paper_1101_0091_amd.selector.labels --out FILE --retime-v6

--retime-v6 re-times only V6 for the records of FILE that have a chunked
copy and rewrites FILE (the V0-V5 times are kept).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

SEED = 5
NLO, NHI = 1e4, 2e7


def time_variants(M, Bd, C, reps=7, warmup=2, variants=None):
    import numpy as np
    import torch

    import paper_1101_0091_amd as pkg
    s = torch.cuda.current_stream()
    out = []
    for v in (range(pkg.SPMV_NUM_SELECTOR_OUTPUTS) if variants is None else variants):
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--stop", type=int, default=512)
    ap.add_argument("--retime-v6", action="store_true")
    args = ap.parse_args(argv)
    if args.retime_v6:
        return retime_v6(args.out)
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
        us = time_variants(M, Bd, C)
        # V6 (chunked copy) is outside the selector's outputs; its time is kept
        # for reference where the copy fits its reserve
        us6 = (time_variants(M, Bd, C, variants=(pkg.SPMV_V6_SELL64,))[0]
               if M.sell_slots is not None else None)
        rec = {"id": i, "n": A.n_rows, "nnz": A.nnz, "family": crsgen.FAMILY_NAMES[prm["family"]],
               "width": prm["width"], "features": [float(x) for x in M.features],
               "us": [round(t, 3) for t in us], "gen_s": round(tg, 2),
               "us_v6": None if us6 is None else round(us6, 3),
               "sell_slots": M.sell_slots}
        with open(args.out, "a") as f:
            f.write(json.dumps(rec) + "\n")
        print(f"[labels] {i} n={A.n_rows} nnz={A.nnz} {rec['family']} best=V{us.index(min(us))} "
              f"us={rec['us']} ({time.time() - t0:.1f}s)", flush=True)
        del M, Bd, C, A
        torch.cuda.empty_cache()


def retime_v6(path):
    import torch

    import crsgen
    import paper_1101_0091_amd as pkg
    recs = [json.loads(line) for line in open(path)]
    dev = torch.device("cuda:0")
    for r in recs:
        if r.get("sell_slots") is None:
            continue
        t0 = time.time()
        A, _ = crsgen.family_matrix(SEED, r["id"], NLO, NHI)
        B = crsgen.uniform_vec(A.n_cols, SEED)
        M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(6) | pkg.SPMV_FLAG_SELL,
                                   device=dev)
        Bd = torch.from_numpy(B).to(dev)
        C = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
        r["us_v6"] = round(time_variants(M, Bd, C, variants=(pkg.SPMV_V6_SELL64,))[0], 3)
        print(f"[labels] {r['id']} V6 {r['us_v6']} us, best of V0-V5 {min(r['us'])} us "
              f"({time.time() - t0:.1f}s)", flush=True)
        del M, Bd, C, A
        torch.cuda.empty_cache()
    with open(path, "w") as f:
        for r in recs:
            f.write(json.dumps(r) + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
