"""The host baseline (the paper's OpenMP node scheme, Sect. 2) sums every
row in the oracle's order, so its C equals the oracle's bit for bit on any
thread count; the triad reports a positive bandwidth."""
import numpy as np
import pytest

import crsgen
import oracle
import oracle.node as node
from cases import CASES, rhs


@pytest.mark.parametrize("name", ["hand", "irregular_dup_unsorted", "mesh3d_48_permuted",
                                  "long_rows", "mostly_empty", "nnz0", "one_row", "rect_tall"])
def test_node_product_equals_oracle(name):
    A = CASES[name]()
    B = rhs(A)
    Cref, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
    C, reps, secs = node.spmv_bench(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val, B,
                                    min_seconds=0.0, max_reps=2)
    assert 1 <= reps <= 2 and secs >= 0.0
    assert np.array_equal(C.view(np.int64), Cref.view(np.int64))


def test_node_threads_and_triad():
    assert node.threads() >= 1
    assert node.triad_gbs(1 << 20, 2) > 0.0
