"""Locality reordering on the GPU path (the paper's Sect. 1.3.1 use of RCM):
the reverse Cuthill-McKee order and the symmetric permutation are host
library calls; the reordered product P A P^T (P B) runs through every
variant and V4 form and is checked row by row against the oracle of the
reordered matrix and against P (A B), the oracle of the original one."""
import numpy as np
import pytest

import crsgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1101_0091_amd as pkg  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("m", [48, 128])
def test_rcm_ordered_mesh_product(m):
    A = crsgen.mesh3d(m, seed=3)[0]
    B = crsgen.uniform_vec(A.n_cols, 3)
    perm = pkg.spmv_rcm_order(A.n_rows, A.row_ptr, A.col_idx, symmetric_part=True)
    assert np.array_equal(np.sort(perm), np.arange(A.n_rows))
    rp, ci, va = pkg.spmv_permute_crs(A.n_rows, A.row_ptr, A.col_idx, A.val, perm)
    PB = np.ascontiguousarray(B[perm])
    Cp, Sp = oracle.spmv(A.n_rows, rp, ci, va, PB)   # oracle of P A P^T (P B)
    C0, S0 = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)  # oracle of A B
    # the permutation only moves rows and reorders entries within a row: the
    # same terms, so the same magnitude sums, and P (A B) within the bound
    assert np.allclose(Sp, S0[perm], rtol=1e-12, atol=0)
    ok, worst = oracle.bound_ok(Cp, C0[perm], rp, Sp)
    assert ok, worst
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, rp, ci, va,
                      flags=pkg.SPMV_FLAG_VARIANT(4) | pkg.SPMV_FLAG_SELL, device=DEV)
    Bd = torch.from_numpy(PB).to(DEV)
    for v in range(pkg.SPMV_NUM_VARIANTS):
        if v == pkg.SPMV_V6_SELL64 and M.sell_slots is None:
            continue
        M.variant = v
        for f in ((0, 1, 2) if v == 4 else (None,)):
            if f is not None:
                M.v4_form = f
            C = M.apply(Bd).cpu().numpy()
            ok, worst = oracle.bound_ok(C, Cp, rp, Sp)
            assert ok, (v, f, worst)
            ok, worst = oracle.bound_ok(C, C0[perm], rp, Sp)
            assert ok, (v, f, "P(AB)", worst)
            if v == 4 and f == 2:  # the window form sums in CRS order: bit for bit
                assert np.array_equal(C.view(np.int64), Cp.view(np.int64))
