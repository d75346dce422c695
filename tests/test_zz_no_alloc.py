"""spmv_cg_solve_noalloc (the solver scratch held by the library in a static
device array) against spmv_cg_solve with a caller-supplied workspace: the
same kernels in the same order, so the same iteration count, residual and x
bit for bit -- on calls in a row, each pair's second with a smaller system,
through the four-launch iteration (V4 plans) and the two-launch one (V0
plans), in float64 and float32 storage; a system beyond the scratch is
refused and the largest one that fits runs."""
import numpy as np
import pytest

import crsgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_1101_0091_amd as pkg  # noqa: E402

DEV = "cuda:0"
N_MAX = 931_680


def _solve(M, b, tol, noalloc, check_every=10):
    n = b.shape[0]
    bd = torch.from_numpy(b).to(DEV)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    if noalloc:
        it, rr = pkg.spmv_cg_solve_noalloc(M.handle, bd, x, tol, 3000, check_every)
    else:
        ws_bytes = pkg.spmv_cg_workspace_size(n)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=DEV)
        it, rr = pkg.spmv_cg_solve(M.handle, bd, x, tol, 3000, check_every, False, ws, ws_bytes)
    torch.cuda.synchronize()
    return x.cpu().numpy(), it, rr


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_noalloc_cg_equals_workspace_cg(dt):
    tol = 1e-10 if dt == "f64" else 1e-5
    for m, v in ((256, 4), (96, 4), (200, 0), (64, 0)):  # each second call smaller
        A = crsgen.laplace2d(m)
        xs = crsgen.uniform_vec(A.n_rows, 8)
        b, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, xs)
        if dt == "f32":
            M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.astype(np.float32),
                              val_dtype=torch.float32, flags=pkg.SPMV_FLAG_VARIANT(v),
                              device=DEV)
        else:
            M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(v), device=DEV)
        x_na, it_na, rr_na = _solve(M, b, tol, noalloc=True)
        x_ws, it_ws, rr_ws = _solve(M, b, tol, noalloc=False)
        assert it_na == it_ws and rr_na == rr_ws, (m, dt)
        assert np.array_equal(x_na.view(np.int64), x_ws.view(np.int64)), (m, dt)
        assert rr_na <= tol
        Ax, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, x_na)
        assert np.linalg.norm(b - Ax) / np.linalg.norm(b) <= 10 * tol


def _diag(n):
    rp = np.arange(n + 1, dtype=np.int32)
    return pkg.CRSMatrix(n, n, rp, rp[:-1], np.full(n, 2.0), flags=pkg.SPMV_FLAG_VARIANT(0),
                         device=DEV)


def test_noalloc_cg_size_limit():
    big = _diag(N_MAX + 1)
    x = torch.zeros(N_MAX + 1, dtype=torch.float64, device=DEV)
    b = torch.ones(N_MAX + 1, dtype=torch.float64, device=DEV)
    with pytest.raises(pkg.SpmvError) as e:
        pkg.spmv_cg_solve_noalloc(big.handle, b, x, 1e-12, 10, 1)
    assert e.value.status == pkg.SPMV_ERR_UNSUPPORTED
    del big, x, b
    # the largest system that fits: 2 I x = b converges in one step to b / 2
    # (alpha = b.b / (2 b.b) = 1/2 exactly, so the residual is exactly zero)
    M = _diag(N_MAX)
    bh = crsgen.uniform_vec(N_MAX, 9)
    x_na, it_na, rr_na = _solve(M, bh, 1e-12, noalloc=True, check_every=1)
    x_ws, it_ws, rr_ws = _solve(M, bh, 1e-12, noalloc=False, check_every=1)
    assert it_na == it_ws == 1 and rr_na == rr_ws
    assert np.array_equal(x_na, x_ws) and np.array_equal(x_na, bh / 2)
