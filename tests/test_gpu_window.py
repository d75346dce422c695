"""V4 in its window form (B windows staged per 4096-row super-block, each
row's products added by one lane in CRS order): its results equal the
oracle's bit for bit, since it performs the oracle's operations (rounded
product, then sum, ascending j) in the oracle's order -- for every parity
case, both storage precisions, non-finite B, the full-size permuted mesh and
a B too large for 32-bit buffer offsets."""
import numpy as np
import pytest

import crsgen
import oracle
from cases import CASES, rhs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1101_0091_amd as pkg  # noqa: E402

DEV = "cuda:0"
WIN = pkg.SPMV_FLAG_VARIANT(4) | pkg.SPMV_FLAG_V4_WINDOWS


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _bits(x):
    return np.ascontiguousarray(x).view(np.int64)


def _inputs(A, B, dt):
    if dt == "f32":
        return A.val.astype(np.float32), B.astype(np.float32), torch.float32
    return A.val, B, torch.float64


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_window_form_bit_exact(name, dt):
    A = CASES[name]()
    val_h, B_h, tdt = _inputs(A, rhs(A), dt)
    Cref, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, val_h, B_h)
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val_h, val_dtype=tdt,
                      flags=WIN, device=DEV)
    assert M.v4_form == pkg.SPMV_V4_WINDOWS
    assert 0 <= M.win_covered <= A.nnz
    C = torch.full((A.n_rows,), float("nan"), dtype=torch.float64, device=DEV)
    M.apply(_gpu(B_h), C)
    assert np.array_equal(_bits(C.cpu().numpy()), _bits(Cref)), (name, dt)
    # switching the form of an existing plan gives the same bits
    M.v4_form = pkg.SPMV_V4_PLAIN
    M.v4_form = pkg.SPMV_V4_WINDOWS
    C2 = M.apply(_gpu(B_h))
    assert torch.equal(C, C2)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_window_form_nonfinite_B(dt):
    """NaN and infinities in B, inside and outside the windows: the same
    operations in the same order give NaN where the oracle does and the same
    finite values and infinities elsewhere."""
    A = crsgen.mesh3d(48, seed=3)[0]
    B = rhs(A)
    rng = np.random.default_rng(5)
    idx = rng.choice(A.n_cols, size=64, replace=False)
    B[idx[:24]] = np.nan
    B[idx[24:44]] = np.inf
    B[idx[44:]] = -np.inf
    val_h, B_h, tdt = _inputs(A, B, dt)
    Cref, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, val_h, B_h)
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val_h, val_dtype=tdt,
                      flags=WIN, device=DEV)
    C = M.apply(_gpu(B_h)).cpu().numpy()
    nan = np.isnan(Cref)
    assert nan.any() and np.isinf(Cref).any()
    assert np.array_equal(np.isnan(C), nan)
    assert np.array_equal(_bits(C[~nan]), _bits(Cref[~nan]))


def test_window_form_full_size_mesh():
    """The permuted 3D stencil with random extras at full size (N = 21.95M):
    the default plan takes the window form, and every row equals the oracle's
    bit for bit in float64 and float32 storage (the latter also against the
    staged V4 form within the bound)."""
    A = crsgen.mesh3d(280, seed=3)[0]
    B = crsgen.uniform_vec(A.n_cols, 3)
    Cref, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
    M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(4), device=DEV)
    assert M.v4_form == pkg.SPMV_V4_WINDOWS
    assert M.win_covered >= 0.7 * A.nnz
    C = M.apply(_gpu(B)).cpu().numpy()
    assert np.array_equal(_bits(C), _bits(Cref))
    del M
    v32, b32 = A.val.astype(np.float32), B.astype(np.float32)
    C32ref, S32 = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, v32, b32)
    M32 = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, v32, val_dtype=torch.float32,
                        flags=pkg.SPMV_FLAG_VARIANT(4), device=DEV)
    assert M32.v4_form == pkg.SPMV_V4_WINDOWS
    Bd = _gpu(b32)
    C32 = M32.apply(Bd).cpu().numpy()
    assert np.array_equal(_bits(C32), _bits(C32ref))
    # the staged form with float32 B windows, every row within the bound
    M32.v4_form = pkg.SPMV_V4_STAGED
    ok, worst = oracle.bound_ok(M32.apply(Bd).cpu().numpy(), C32ref, A.row_ptr, S32)
    assert ok, worst
    del M32
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_window_form_wide_B(dt):
    """n_cols past 2^32 bytes of B: the kernel reads B through 64-bit
    addresses instead of a buffer resource. The oracle runs on the columns the
    matrix touches (same products in the same order)."""
    n_cols = 540_000_000 if dt == "f64" else 1_080_000_000
    rng = np.random.default_rng(9)
    n = 20_000
    lens = rng.integers(0, 9, size=n)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    # half the columns near the diagonal block (windows), half anywhere
    near = (np.arange(rp[-1]) % 2 == 0)
    ci = np.where(near, rng.integers(0, 8192, size=rp[-1]),
                  rng.integers(0, n_cols, size=rp[-1])).astype(np.int32)
    va = rng.standard_normal(rp[-1])
    tdt = torch.float32 if dt == "f32" else torch.float64
    # B[j] = ((j * 40503) mod 65521 - 32760) / 2^16, built on the device
    # (exact in both precisions, so host and device values agree bit for bit)
    j = torch.arange(n_cols, dtype=torch.int64, device=DEV)
    Bd = (((j * 40503) % 65521 - 32760).to(torch.float64) * 2.0**-16).to(tdt)
    del j
    uniq, inv = np.unique(ci, return_inverse=True)
    jj = uniq.astype(np.int64)
    Bu = (((jj * 40503) % 65521 - 32760).astype(np.float64) * 2.0**-16).astype(
        np.float32 if dt == "f32" else np.float64)
    val_h = va.astype(np.float32) if dt == "f32" else va
    Cref, _ = oracle.spmv(n, rp, inv.astype(np.int32), val_h, Bu)
    M = pkg.CRSMatrix(n, n_cols, rp, ci, val_h, val_dtype=tdt, flags=WIN, device=DEV)
    C = M.apply(Bd).cpu().numpy()
    assert np.array_equal(_bits(C), _bits(Cref))
    del Bd, M
    torch.cuda.empty_cache()
