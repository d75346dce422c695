"""Seeded generators: shapes, structure and thread-count independence."""
import numpy as np
import pytest

import crsgen
import oracle


def test_philox_known_answers():
    # Known-answer vectors of Philox4x32-10 (Salmon et al., SC'11)
    assert crsgen.philox4x32_10([0, 0, 0, 0], [0, 0]) == (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)
    assert crsgen.philox4x32_10([0xffffffff] * 4, [0xffffffff] * 2) == (
        0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)
    assert crsgen.philox4x32_10([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344],
                                [0xa4093822, 0x299f31d0]) == (
        0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)


def _valid(A):
    assert oracle.check_crs(A.n_rows, A.n_cols, A.row_ptr, A.col_idx) == 0
    for i in range(0, A.n_rows, max(1, A.n_rows // 997)):
        c = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_laplace2d_config1():
    A = crsgen.laplace2d(256)
    assert A.n_rows == 65536 and A.nnz == 326656
    _valid(A)
    assert set(np.unique(A.val)) == {-1.0, 4.0}


def test_hamiltonian_symmetric():
    n = 50_000
    A = crsgen.hamiltonian(n, seed=2)
    _valid(A)
    d = crsgen.hamiltonian_offsets(n, 2)
    assert len(set(d.tolist())) == 7 and d.min() >= 1 and d.max() <= n // 2
    assert A.nnz == n + 2 * int(np.sum(n - d))
    # exact symmetry: the transpose has identical arrays
    import scipy.sparse as sp
    M = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(n, n))
    T = M.T.tocsr()
    T.sort_indices()
    assert np.array_equal(T.indptr, A.row_ptr) and np.array_equal(T.indices, A.col_idx)
    assert np.array_equal(T.data, A.val)


def test_hamiltonian_full_size_counts():
    d = crsgen.hamiltonian_offsets(6_000_000, 2)
    nnz = 6_000_000 + 2 * int(np.sum(6_000_000 - d))
    assert 84e6 <= nnz <= 90e6


def test_mesh3d_permutation_and_dominance():
    m = 24
    A, p = crsgen.mesh3d(m, seed=3, block=4096)
    _valid(A)
    n = m**3
    # p is a bijection inside every block of 4096
    for b in range(0, n, 4096):
        blk = p[b:b + 4096]
        assert np.array_equal(np.sort(blk), np.arange(b, min(b + 4096, n)))
    # diagonally dominant: a_ii = 1 + sum_{j != i} |a_ij|
    rows = np.repeat(np.arange(n), A.row_lengths())
    diag = A.col_idx == rows
    assert np.sum(diag) == n
    off = np.zeros(n)
    np.add.at(off, rows[~diag], np.abs(A.val[~diag]))
    assert np.allclose(A.val[diag], 1.0 + off, rtol=1e-15, atol=0)
    # stencil count 7N - 6m^2 plus extras on ~5% of rows
    extra = A.nnz - (7 * n - 6 * m * m)
    assert 0.02 * n * 15.5 < extra < 0.08 * n * 15.5


def test_thread_count_independence():
    ref = crsgen.mesh3d(16, seed=5)[0]
    f_ref = crsgen.family_matrix(5, 3, 1e4, 2e4)[0]
    t0 = crsgen.num_threads()
    try:
        crsgen.set_threads(1)
        one = crsgen.mesh3d(16, seed=5)[0]
        f_one = crsgen.family_matrix(5, 3, 1e4, 2e4)[0]
    finally:
        crsgen.set_threads(t0)
    for a, b in ((ref, one), (f_ref, f_one)):
        assert np.array_equal(a.row_ptr, b.row_ptr)
        assert np.array_equal(a.col_idx, b.col_idx)
        assert np.array_equal(a.val, b.val)


def test_powerlaw_mean():
    cdf = np.array([crsgen.powerlaw_cdf(l) for l in range(1, 5001)])
    pmf = np.diff(np.concatenate([[0.0], cdf]))
    mean = float(np.sum(pmf * np.arange(1, 5001)))
    assert mean == pytest.approx(4.05, abs=0.05)


@pytest.mark.parametrize("idx", range(9))
def test_family_matrices(idx):
    A, prm = crsgen.family_matrix(5, idx, 1e4, 3e4)
    _valid(A)
    L = A.row_lengths()
    if prm["family"] == 0:
        assert L.min() >= 1 and L.max() <= 30
    elif prm["family"] == 1:
        assert L.min() >= 1 and L.max() <= 5000
    else:
        assert 3 <= prm["width"] <= 64 and L.max() == prm["width"]


def test_family_small_n_dense_rows():
    # power-law rows longer than N are clipped to N (all columns)
    for idx in range(40):
        prm = crsgen.family_params(6, idx, 100, 5000)
        if prm["family"] == 1:
            A, _ = crsgen.family_matrix(6, idx, 100, 5000, n_override=120)
            _valid(A)
            assert A.row_lengths().max() <= 120
            break
