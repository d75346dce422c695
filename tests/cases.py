"""Seeded parity cases (host CRS + B), shared by the GPU tests.

Sizes are chosen so the oracle finishes in well under a second per case yet
the matrices span many LDS row blocks and end in ragged tails; the edge cases
cover empty matrices, empty rows, rows longer than a row block, duplicate and
unsorted columns, and rectangular shapes.
"""
from __future__ import annotations

import numpy as np

import crsgen
from crsgen import CRS


def long_rows(seed=7) -> CRS:
    """Short rows, empty rows and a few rows far longer than one LDS block."""
    rng = np.random.default_rng(seed)
    n, ncol = 20_000, 30_000
    lens = rng.integers(0, 12, size=n)
    lens[rng.random(n) < 0.1] = 0
    for r in (0, 17, 5000, 5001, 19_999):
        lens[r] = int(rng.integers(2049, 12_000))
    lens[7000:7004] = 2048
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(ncol, size=l, replace=False)) for l in lens]
                        ).astype(np.int32)
    va = rng.standard_normal(ci.shape[0])
    return CRS(n, ncol, rp, ci, va)


def mostly_empty(seed=8) -> CRS:
    """50k rows, 0.5% non-empty: LDS blocks full of empty rows."""
    rng = np.random.default_rng(seed)
    n = 50_000
    lens = np.zeros(n, dtype=np.int64)
    nz = rng.choice(n, size=250, replace=False)
    lens[nz] = rng.integers(1, 200, size=250)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(n, size=l, replace=False)) for l in lens if l]
                        ).astype(np.int32)
    return CRS(n, n, rp, ci, rng.standard_normal(ci.shape[0]))


def powerlaw(n=60_000) -> CRS:
    for idx in range(100):
        if crsgen.family_params(5, idx, 1e4, 2e7)["family"] == 1:
            return crsgen.family_matrix(5, idx, 1e4, 2e7, n_override=n)[0]
    raise RuntimeError("no power-law matrix")


def banded(n=40_000) -> CRS:
    for idx in range(100):
        if crsgen.family_params(5, idx, 1e4, 2e7)["family"] == 2:
            return crsgen.family_matrix(5, idx, 1e4, 2e7, n_override=n)[0]
    raise RuntimeError("no banded matrix")


def hand() -> CRS:
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_example.json")))
    return CRS(g["n_rows"], g["n_cols"], np.array(g["row_ptr"], np.int32),
               np.array(g["col_idx"], np.int32), np.array(g["val"]))


def empty(n_rows, n_cols) -> CRS:
    return CRS(n_rows, n_cols, np.zeros(n_rows + 1, np.int32), np.zeros(0, np.int32),
               np.zeros(0))


CASES = {
    "hand": hand,
    "irregular_dup_unsorted": lambda: crsgen.random_crs(5000, 4000, seed=21, max_len=40,
                                                        empty_frac=0.2, allow_dup=True,
                                                        unsorted=True),
    "laplace2d_256": lambda: crsgen.laplace2d(256),
    "hamiltonian_200k": lambda: crsgen.hamiltonian(200_000, seed=2),
    "mesh3d_48_permuted": lambda: crsgen.mesh3d(48, seed=3)[0],
    "powerlaw_60k": powerlaw,
    "banded_40k": banded,
    "long_rows": long_rows,
    "mostly_empty": mostly_empty,
    "rect_wide": lambda: crsgen.random_crs(1000, 100_000, seed=31, max_len=300),
    "rect_tall": lambda: crsgen.random_crs(100_000, 10, seed=32, max_len=10),
    "nnz0": lambda: empty(1000, 700),
    "rows0": lambda: empty(0, 5),
    "one_row": lambda: crsgen.random_crs(1, 9000, seed=33, max_len=8000, empty_frac=0.0),
}


def rhs(A: CRS, seed=1) -> np.ndarray:
    return crsgen.uniform_vec(A.n_cols, seed)
