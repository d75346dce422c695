"""The CPU oracle against the paper's definition and the mathematics
(exact rationals, dense products, closed-form eigenpairs, integer
exactness, permutation identity, edge cases), plus planted-mistake checks
that show the pins catch a dropped term, a wrong sign, a shifted index and a
transposed operand."""
import os
import subprocess

import pytest

import oracle
from oracle_pins import ALL_PINS

LIB = oracle.load()


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin(LIB)


MUTANTS = {
    # (original text, mutated text): first occurrence is inside oracle_spmv
    "dropped_last_term": ("j < row_ptr[i + 1]; ++j) {\n      double prod = val[j] * B[col_idx[j]];",
                          "j < row_ptr[i + 1] - 1; ++j) {\n      double prod = val[j] * B[col_idx[j]];"),
    "wrong_sign": ("acc = acc + prod;", "acc = acc - prod;"),
    "shifted_index": ("double prod = val[j] * B[col_idx[j]];",
                      "double prod = val[j] * B[col_idx[j] > 0 ? col_idx[j] - 1 : 0];"),
    "transposed_operand": ("double prod = val[j] * B[col_idx[j]];",
                           "double prod = val[j] * B[i < 0 ? 0 : i % (col_idx[j] + 1)];"),
    "abs_dropped_in_bound": ("mag = mag + fabs(prod);", "mag = mag + prod;"),
    "spmm_wrong_column": ("B[(int64_t)col_idx[j] * ldb + c]", "B[(int64_t)col_idx[j] * ldb]"),
    "check_misses_col_range": ("(int64_t)col_idx[j] >= n_cols", "(int64_t)col_idx[j] > n_cols"),
    "features_bin_edge": ("l <= 16 ? 2", "l <= 15 ? 2"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    old, new = MUTANTS[name]
    assert old in src, name
    mutant_src = tmp_path / "oracle_mutant.c"
    mutant_src.write_text(src.replace(old, new, 1))
    so = str(tmp_path / "liboracle_mutant.so")
    oracle.build(str(mutant_src), so)
    lib = oracle.load(so)
    caught = []
    for pin in ALL_PINS:
        try:
            pin(lib)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
