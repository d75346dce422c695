"""Reverse Cuthill-McKee ordering (host code in the library): a valid
permutation that narrows the band like scipy's implementation, recovers a
shuffled chain, and keeps the product (checked on the CPU with the oracle on
the permuted problem)."""
import numpy as np
import pytest

import crsgen
import oracle
import paper_1101_0091_amd as pkg


def bandwidth(rp, ci):
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return int(np.max(np.abs(ci.astype(np.int64) - rows))) if len(ci) else 0


def test_permutation_and_band_vs_scipy():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    for m, seed in ((16, 1), (24, 3)):
        A, _ = crsgen.mesh3d(m, seed=seed, block=512)
        perm = pkg.spmv_rcm_order(A.n_rows, A.row_ptr, A.col_idx)
        assert np.array_equal(np.sort(perm), np.arange(A.n_rows))
        rp, ci, va = pkg.spmv_permute_crs(A.n_rows, A.row_ptr, A.col_idx, A.val, perm)
        M = csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_rows))
        sp = reverse_cuthill_mckee(M + M.T, symmetric_mode=True)
        srp, sci, _ = pkg.spmv_permute_crs(A.n_rows, A.row_ptr, A.col_idx, A.val, sp)
        ours, ref, before = bandwidth(rp, ci), bandwidth(srp, sci), bandwidth(A.row_ptr, A.col_idx)
        assert ours < before
        assert ours <= 1.25 * ref, (ours, ref)


def test_shuffled_chain_recovers_band_one():
    n = 5000
    A = crsgen.laplace1d(n)
    rng = np.random.default_rng(0)
    shuffle = rng.permutation(n).astype(np.int32)
    rp, ci, va = pkg.spmv_permute_crs(n, A.row_ptr, A.col_idx, A.val, shuffle)
    assert bandwidth(rp, ci) > 100
    perm = pkg.spmv_rcm_order(n, rp, ci)
    rp2, ci2, _ = pkg.spmv_permute_crs(n, rp, ci, va, perm)
    assert bandwidth(rp2, ci2) == 1


def test_components_and_isolated_vertices():
    # two chains and three isolated vertices
    rows = [[1], [0, 2], [1], [], [5], [4], [], []]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.array([c for r in rows for c in r], dtype=np.int32)
    perm = pkg.spmv_rcm_order(8, rp, ci)
    assert np.array_equal(np.sort(perm), np.arange(8))


def test_permuted_product_identity():
    """(P A P^T)(P B) = P (A B) within the bound, through permute_crs."""
    A, _ = crsgen.mesh3d(20, seed=5, block=1024)
    perm = pkg.spmv_rcm_order(A.n_rows, A.row_ptr, A.col_idx)
    rp, ci, va = pkg.spmv_permute_crs(A.n_rows, A.row_ptr, A.col_idx, A.val, perm)
    B = crsgen.uniform_vec(A.n_rows, 5)
    C, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
    Cp, Sp = oracle.spmv(A.n_rows, rp, ci, va, B[perm])
    ok, worst = oracle.bound_ok(Cp, C[perm], rp, Sp)
    assert ok, worst


def test_symmetric_part_ignores_one_sided_extras():
    """With random one-sided extras the A + A^T graph is small-world and RCM
    cannot narrow it; ordering by the two-sided part recovers the stencil band."""
    A, _ = crsgen.mesh3d(24, seed=3, block=4096)
    full = pkg.spmv_rcm_order(A.n_rows, A.row_ptr, A.col_idx, symmetric_part=False)
    sym = pkg.spmv_rcm_order(A.n_rows, A.row_ptr, A.col_idx, symmetric_part=True)
    def median_dist(perm):
        rp, ci, _ = pkg.spmv_permute_crs(A.n_rows, A.row_ptr, A.col_idx, A.val, perm)
        rows = np.repeat(np.arange(A.n_rows), np.diff(rp))
        return float(np.median(np.abs(ci.astype(np.int64) - rows)))
    assert median_dist(sym) < median_dist(full)
    assert median_dist(sym) <= 2 * 24 * 24


def test_permute_matches_numpy_definition():
    A = crsgen.random_crs(300, 300, seed=4, max_len=9, allow_dup=False)
    perm = np.random.default_rng(1).permutation(300).astype(np.int32)
    rp, ci, va = pkg.spmv_permute_crs(300, A.row_ptr, A.col_idx, A.val, perm)
    D = A.to_dense()
    P = np.zeros((300, 300)); P[np.arange(300), perm] = 1.0
    E = crsgen.CRS(300, 300, rp, ci, va).to_dense()
    assert np.array_equal(E, P @ D @ P.T)


def test_rejects_bad_row_ptr():
    with pytest.raises(pkg.SpmvError) as e:
        pkg.spmv_rcm_order(3, np.array([0, 2, 1, 3]), np.array([0, 1, 2]))
    assert e.value.status == pkg.SPMV_ERR_BAD_CRS
