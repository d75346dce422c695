"""Local/remote split product (eq. (2) kernel structure) against the oracle:
pass 0 alone equals the product of the local entries; both passes equal the
whole product within the bound."""
import numpy as np
import pytest

import crsgen
import oracle
from cases import CASES, rhs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_1101_0091_amd as pkg  # noqa: E402

DEV = "cuda:0"


def _local_part(A, lo, hi):
    keep = (A.col_idx >= lo) & (A.col_idx < hi)
    rows = np.repeat(np.arange(A.n_rows), A.row_lengths())
    lens = np.bincount(rows[keep], minlength=A.n_rows)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    return crsgen.CRS(A.n_rows, A.n_cols, rp, A.col_idx[keep], A.val[keep])


@pytest.mark.parametrize("name,frac", [("hamiltonian_200k", (0.4, 0.6)),
                                       ("mesh3d_48_permuted", (0.25, 0.5)),
                                       ("long_rows", (0.0, 0.3)),
                                       ("powerlaw_60k", (0.0, 1.0)),
                                       ("irregular_dup_unsorted", (0.5, 0.5)),
                                       ("nnz0", (0.1, 0.9))])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_split_vs_oracle(name, frac, dt):
    A, B = CASES[name](), None
    B = rhs(A)
    lo, hi = int(frac[0] * A.n_cols), int(frac[1] * A.n_cols)
    if dt == "f32":
        A = crsgen.CRS(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.astype(np.float32))
        B = B.astype(np.float32)
    tdt = torch.float32 if dt == "f32" else torch.float64
    S = pkg.SplitMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val, lo, hi, val_dtype=tdt,
                        device=DEV)
    Al = _local_part(A, lo, hi)
    assert S.nnz_local == Al.nnz and S.nnz_local + S.nnz_remote == A.nnz
    Bd = torch.from_numpy(B).to(DEV)
    C = torch.full((A.n_rows,), float("nan"), dtype=torch.float64, device=DEV)
    S.apply(Bd, C, pass_=0)
    Cl, Sl = oracle.spmv(Al.n_rows, Al.row_ptr, Al.col_idx, Al.val, B)
    ok, worst = oracle.bound_ok(C.cpu().numpy(), Cl, Al.row_ptr, Sl)
    assert ok, worst
    S.apply(Bd, C, pass_=1)
    Cref, Sref = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
    ok, worst = oracle.bound_ok(C.cpu().numpy(), Cref, A.row_ptr, Sref)
    assert ok, worst
    C2 = S.apply(Bd)
    assert torch.equal(C2, C)  # both passes in one call: same bits


def test_split_rejects_bad_window_and_crs():
    A = crsgen.laplace2d(16)
    with pytest.raises(pkg.SpmvError):
        pkg.SplitMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val, 10, 5, device=DEV)
    bad = A.col_idx.copy()
    bad[3] = A.n_cols
    with pytest.raises(pkg.SpmvError) as e:
        pkg.SplitMatrix(A.n_rows, A.n_cols, A.row_ptr, bad, A.val, 0, 10, device=DEV)
    assert e.value.status == pkg.SPMV_ERR_BAD_CRS
