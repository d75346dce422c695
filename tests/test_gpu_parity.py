"""GPU parity: every kernel variant, both storage precisions, multi-RHS, the
uneven batch, graph replay and the analysis outputs against the CPU oracle,
through the C ABI. Acceptance: |C_gpu - C_oracle| <= 8 nnz_row 2^-53 S_i per
row; integer-valued inputs and FP32-stored integers bit-exact."""
import numpy as np
import pytest

import crsgen
import oracle
from cases import CASES, rhs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1101_0091_amd as pkg  # noqa: E402

DEV = "cuda:0"
NV = pkg.SPMV_NUM_VARIANTS


SELL = pkg.SPMV_FLAG_SELL


def variants(M):
    """Every variant the plan has (V6 only where its chunked copy was built)."""
    return [v for v in range(NV) if v != pkg.SPMV_V6_SELL64 or M.sell_slots is not None]


def sell_expected(A):
    """Slots of the V6 copy (64 x sum over 64-row chunks of the longest row)
    and whether they fit the reserve of 1.5 nnz + 4096 slots."""
    lens = np.diff(A.row_ptr.astype(np.int64))
    nch = (A.n_rows + 63) // 64
    padded = np.zeros(nch * 64, np.int64)
    padded[:A.n_rows] = lens
    slots = 64 * int(padded.reshape(nch, 64).max(axis=1).sum()) if nch else 0
    cap = (A.nnz + A.nnz // 2 + 4096 + 63) // 64 * 64
    return slots, slots <= cap


def _gpu(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.to(DEV) if dtype is None else t.to(DEV, dtype)


_cache = {}


def case(name):
    if name not in _cache:
        A = CASES[name]()
        _cache[name] = (A, rhs(A))
    return _cache[name]


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_all_variants_vs_oracle(name, dt):
    A, B = case(name)
    if dt == "f32":
        val_h, B_h = A.val.astype(np.float32), B.astype(np.float32)
        tdt = torch.float32
    else:
        val_h, B_h, tdt = A.val, B, torch.float64
    Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, val_h, B_h)
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val_h, val_dtype=tdt,
                      flags=pkg.SPMV_FLAG_VARIANT(4) | SELL, device=DEV)
    Bd = _gpu(B_h)
    for v in variants(M):
        M.variant = v
        C = torch.full((A.n_rows,), float("nan"), dtype=torch.float64, device=DEV)
        M.apply(Bd, C)
        ok, worst = oracle.bound_ok(C.cpu().numpy(), Cref, A.row_ptr, S)
        assert ok, f"{name} {dt} variant {v}: worst/bound {worst}"


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_v4_both_staging_forms(name, dt):
    """V4 with B staging forced on (exact spans, and windows around the rows
    for wider blocks, where gathers outside the window read B) and forced off."""
    A, B = case(name)
    if dt == "f32":
        val_h, B_h, tdt = A.val.astype(np.float32), B.astype(np.float32), torch.float32
    else:
        val_h, B_h, tdt = A.val, B, torch.float64
    Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, val_h, B_h)
    Bd = _gpu(B_h)
    outs = []
    for form in (pkg.SPMV_FLAG_V4_STAGE_ON, pkg.SPMV_FLAG_V4_STAGE_OFF):
        M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val_h, val_dtype=tdt,
                          flags=pkg.SPMV_FLAG_VARIANT(4) | form, device=DEV)
        C = torch.full((A.n_rows,), float("nan"), dtype=torch.float64, device=DEV)
        M.apply(Bd, C)
        ok, worst = oracle.bound_ok(C.cpu().numpy(), Cref, A.row_ptr, S)
        assert ok, (name, dt, form, worst)
        outs.append(C)
    # staging changes where B is read from, not the arithmetic: bitwise equal
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_integer_inputs_bit_exact(dt):
    A = crsgen.random_crs(30_000, 20_000, seed=41, max_len=3000, empty_frac=0.05,
                          integer=True)
    B = crsgen.int_vec(A.n_cols, 41, 0, -8, 8)
    Cref, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
    tdt = torch.float32 if dt == "f32" else torch.float64
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val, val_dtype=tdt,
                      flags=pkg.SPMV_FLAG_VARIANT(0) | SELL, device=DEV)
    Bd = _gpu(B, tdt)
    for v in variants(M):
        M.variant = v
        assert np.array_equal(M.apply(Bd).cpu().numpy(), Cref), v


def test_diagonal_bit_exact():
    n = 100_000
    rng = np.random.default_rng(5)
    d, B = rng.standard_normal(n), rng.standard_normal(n)
    M = pkg.CRSMatrix(n, n, np.arange(n + 1), np.arange(n), d, flags=SELL, device=DEV)
    assert M.sell_slots == (n + 63) // 64 * 64
    for v in variants(M):
        M.variant = v
        assert np.array_equal(M.apply(_gpu(B)).cpu().numpy(), d * B), v


@pytest.mark.parametrize("v", [0, 4, 5, 6])
def test_concurrent_applies_on_two_streams(v):
    """A plan is const under apply: two streams multiplying the same plan by
    different B into different C at the same time give bitwise the results
    of the sequential products (V4 in its B-staging form, V6 through its
    8-bit deltas, and multi-RHS from the copy)."""
    A, _ = case("hamiltonian_200k")
    flags = pkg.SPMV_FLAG_VARIANT(v) | SELL | (pkg.SPMV_FLAG_V4_STAGE_ON if v == 4 else 0)
    M = pkg.CRSMatrix.from_crs(A, flags=flags, device=DEV)
    if v == 6:
        assert M.sell_deltas[0] > 0
    B1, B2 = _gpu(crsgen.uniform_vec(A.n_cols, 11)), _gpu(crsgen.uniform_vec(A.n_cols, 12))
    Bk = _gpu(crsgen.uniform_vec(A.n_cols * 4, 13).reshape(A.n_cols, 4))
    ref1, ref2, refk = M.apply(B1), M.apply(B2), M.spmm(Bk)
    torch.cuda.synchronize()
    reps = 16
    C1 = torch.empty((reps, A.n_rows), dtype=torch.float64, device=DEV)
    C2 = torch.empty_like(C1)
    Ck = torch.empty((reps, A.n_rows, 4), dtype=torch.float64, device=DEV)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    for i in range(reps):
        M.apply(B1, C1[i], stream=s1)
        M.apply(B2, C2[i], stream=s2)
        M.spmm(Bk, Ck[i], stream=s1 if i % 2 else s2)
    torch.cuda.synchronize()
    for i in range(reps):
        assert torch.equal(C1[i], ref1) and torch.equal(C2[i], ref2), (v, i)
        assert torch.equal(Ck[i], refk), (v, i)
    Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B1.cpu().numpy())
    ok, worst = oracle.bound_ok(ref1.cpu().numpy(), Cref, A.row_ptr, S)
    assert ok, worst


def test_deterministic_repeats():
    """Run to run, 50 repeats of every product path give the same bits (the
    race detector): every variant on power-law rows, the three V4 forms on
    the permuted stencil, V6 and its lane-group multi-RHS kernel on the
    Hamiltonian-like matrix, and the batch's persistent kernels (whose tile
    order changes from launch to launch; each tile's sums do not)."""
    reps = 50
    A, B = case("powerlaw_60k")
    M = pkg.CRSMatrix.from_crs(A, device=DEV)
    Bd = _gpu(B)
    for v in variants(M):
        M.variant = v
        first = M.apply(Bd).clone()
        for _ in range(reps):
            assert torch.equal(M.apply(Bd), first), v
    Am, Bm = case("mesh3d_48_permuted")
    Mm = pkg.CRSMatrix.from_crs(Am, flags=pkg.SPMV_FLAG_VARIANT(4), device=DEV)
    Bmd = _gpu(Bm)
    for f in (pkg.SPMV_V4_PLAIN, pkg.SPMV_V4_STAGED, pkg.SPMV_V4_WINDOWS):
        Mm.v4_form = f
        first = Mm.apply(Bmd).clone()
        for _ in range(reps):
            assert torch.equal(Mm.apply(Bmd), first), f
    Ah, Bh = case("hamiltonian_200k")
    Mh = pkg.CRSMatrix.from_crs(Ah, flags=pkg.SPMV_FLAG_VARIANT(6) | SELL, device=DEV)
    first = Mh.apply(_gpu(Bh)).clone()
    for _ in range(reps):
        assert torch.equal(Mh.apply(_gpu(Bh)), first)
    Bk = _gpu(crsgen.uniform_vec(Ah.n_cols * 8, 4).reshape(Ah.n_cols, 8))
    first = Mh.spmm(Bk).clone()
    for _ in range(reps):
        assert torch.equal(Mh.spmm(Bk), first)
    mats = _batch_mats(300, 8)
    Bt = pkg.Batch(mats, device=DEV)
    B_all = _gpu(crsgen.uniform_vec(int(Bt.n_cols.sum()), 8))
    C_all = torch.zeros(int(Bt.n_rows.sum()), dtype=torch.float64, device=DEV)
    Bp, Cp, _, _ = Bt.pointers(B_all, C_all)
    for mode in (pkg.SPMV_BATCH_STATIC, pkg.SPMV_BATCH_DYNAMIC):
        Bt.set_mode(mode)
        Bt.apply(Bp, Cp)
        first = C_all.clone()
        for _ in range(reps):
            C_all.fill_(float("nan"))
            Bt.apply(Bp, Cp)
            assert torch.equal(C_all, first), mode


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 8, 10, 16, 32, 33, 64, 100])
def test_spmm_vs_oracle(k, dt):
    A = crsgen.laplace2d(256) if k <= 32 else crsgen.random_crs(3000, 2000, seed=k, max_len=50)
    Bh = crsgen.uniform_vec(A.n_cols * k, 4).reshape(A.n_cols, k)
    tdt = torch.float32 if dt == "f32" else torch.float64
    if dt == "f32":
        Bh = Bh.astype(np.float32)
        val = A.val.astype(np.float32)
    else:
        val = A.val
    Cref, S = oracle.spmm(A.n_rows, A.row_ptr, A.col_idx, val, Bh)
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val, val_dtype=tdt, device=DEV)
    C = M.spmm(_gpu(Bh)).cpu().numpy()
    ok, worst = oracle.bound_ok(C, Cref, A.row_ptr, S)
    assert ok, worst
    # padded leading dimensions: ldb = k + 3 takes the scalar path, ldb = k + 2
    # the column groups its parity allows (with a partial group where k is odd)
    for pad in (3, 2):
        Bp = torch.zeros((A.n_cols, k + pad), dtype=tdt, device=DEV)
        Bp[:, :k] = _gpu(Bh)
        Cp = torch.full((A.n_rows, k + 1), 7.0, dtype=torch.float64, device=DEV)
        pkg.spmm_apply(M.handle, k, Bp, k + pad, M.code, Cp, k + 1)
        Cp = Cp.cpu().numpy()
        ok, worst = oracle.bound_ok(Cp[:, :k], Cref, A.row_ptr, S)
        assert ok, (pad, worst)
        assert np.all(Cp[:, k] == 7.0)  # untouched padding column


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8, 9, 16, 17, 32, 64])
@pytest.mark.parametrize("name", ["hamiltonian_200k", "laplace2d_256"])
def test_spmm_from_v6_copy(name, k, dt):
    """A plan running V6 multiplies blocks of right-hand sides from its chunked
    copy when its rows average at least 8 entries (lane groups per row for
    k = 8, 16, 32 in float64 and 8 .. 64 in float32; else column blocks of
    up to 8, vector loads of B row segments, a scalar partial last block),
    else with the row-group kernel (the 5-point Laplacian); also with padded
    leading dimensions, odd (scalar paths) and aligned (lane groups)."""
    A, _ = case(name)
    Bh = crsgen.uniform_vec(A.n_cols * k, 5).reshape(A.n_cols, k)
    tdt = torch.float32 if dt == "f32" else torch.float64
    val = A.val.astype(np.float32) if dt == "f32" else A.val
    if dt == "f32":
        Bh = Bh.astype(np.float32)
    Cref, S = oracle.spmm(A.n_rows, A.row_ptr, A.col_idx, val, Bh)
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val, val_dtype=tdt,
                      flags=pkg.SPMV_FLAG_VARIANT(6) | SELL, device=DEV)
    C = M.spmm(_gpu(Bh)).cpu().numpy()
    ok, worst = oracle.bound_ok(C, Cref, A.row_ptr, S)
    assert ok, worst
    Bp = torch.zeros((A.n_cols, k + 3), dtype=tdt, device=DEV)
    Bp[:, :k] = _gpu(Bh)
    Cp = torch.full((A.n_rows, k + 1), 7.0, dtype=torch.float64, device=DEV)
    pkg.spmm_apply(M.handle, k, Bp, k + 3, M.code, Cp, k + 1)
    Cp = Cp.cpu().numpy()
    assert oracle.bound_ok(Cp[:, :k], Cref, A.row_ptr, S)[0]
    assert np.all(Cp[:, k] == 7.0)
    Ba = torch.zeros((A.n_cols, k + 4), dtype=tdt, device=DEV)
    Ba[:, :k] = _gpu(Bh)
    Ca = torch.full((A.n_rows, k + 2), 7.0, dtype=torch.float64, device=DEV)
    pkg.spmm_apply(M.handle, k, Ba, k + 4, M.code, Ca, k + 2)
    Ca = Ca.cpu().numpy()
    assert oracle.bound_ok(Ca[:, :k], Cref, A.row_ptr, S)[0]
    assert np.all(Ca[:, k:] == 7.0)


@pytest.mark.parametrize("flags", [pkg.SPMV_FLAG_VARIANT(6) | pkg.SPMV_FLAG_SELL,
                                   pkg.SPMV_FLAG_VARIANT(4) | pkg.SPMV_FLAG_V4_WINDOWS,
                                   pkg.SPMV_FLAG_VARIANT(2)])
def test_spmm_single_column_is_the_single_product(flags):
    """k = 1 with unit leading dimensions runs the plan's single product (rows
    averaging at least 8 entries here): the same bits as spmv_apply; a
    strided single column takes the multi-RHS kernels and stays within the
    bound."""
    A, B = case("hamiltonian_200k")
    Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
    M = pkg.CRSMatrix.from_crs(A, flags=flags, device=DEV)
    Bd = _gpu(B)
    C1 = M.apply(Bd)
    Cm = torch.full((A.n_rows, 1), float("nan"), dtype=torch.float64, device=DEV)
    pkg.spmm_apply(M.handle, 1, Bd.view(A.n_cols, 1), 1, M.code, Cm, 1)
    assert torch.equal(Cm[:, 0], C1)
    Bs = torch.zeros((A.n_cols, 2), dtype=torch.float64, device=DEV)
    Bs[:, 0] = Bd
    Cs = torch.full((A.n_rows, 2), 7.0, dtype=torch.float64, device=DEV)
    pkg.spmm_apply(M.handle, 1, Bs, 2, M.code, Cs, 2)
    Cs = Cs.cpu().numpy()
    assert oracle.bound_ok(Cs[:, 0], Cref, A.row_ptr, S)[0]
    assert np.all(Cs[:, 1] == 7.0)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("k", [2, 4, 6, 8, 16])
def test_spmm_from_v6_copy_misaligned_B(k, dt):
    """B starting 1 or 2 elements past an aligned address: the vector loads of
    B row segments need 16 bytes of alignment (8 for float32 pairs), and a B
    that lacks it takes the scalar path with the same products."""
    A, _ = case("hamiltonian_200k")
    tdt = torch.float32 if dt == "f32" else torch.float64
    val = A.val.astype(np.float32) if dt == "f32" else A.val
    Bh = crsgen.uniform_vec(A.n_cols * k, 6).reshape(A.n_cols, k)
    if dt == "f32":
        Bh = Bh.astype(np.float32)
    Cref, S = oracle.spmm(A.n_rows, A.row_ptr, A.col_idx, val, Bh)
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val, val_dtype=tdt,
                      flags=pkg.SPMV_FLAG_VARIANT(6) | SELL, device=DEV)
    aligned = M.spmm(_gpu(Bh))
    for off in (1, 2):
        flat = torch.zeros(A.n_cols * k + off, dtype=tdt, device=DEV)
        Bv = flat[off:].view(A.n_cols, k)
        Bv.copy_(_gpu(Bh))
        C = torch.empty((A.n_rows, k), dtype=torch.float64, device=DEV)
        pkg.spmm_apply(M.handle, k, Bv, k, M.code, C, k)
        ok, worst = oracle.bound_ok(C.cpu().numpy(), Cref, A.row_ptr, S)
        assert ok, (off, worst)
        # the same slots summed in the same order: bitwise equal to the aligned B
        assert torch.equal(C, aligned), off


def test_full_size_hamiltonian_and_mesh():
    """Workloads at full size (N = 6.0M and 21.95M), every row checked, with
    the plans the benchmark builds (V6 copy requested; it fits the
    Hamiltonian-like matrix and not the mesh, whose chunks are 3.7x padded)."""
    for name, A in (("hamiltonian_6M", crsgen.hamiltonian(6_000_000, seed=2)),
                    ("mesh3d_280", crsgen.mesh3d(280, seed=3)[0])):
        B = crsgen.uniform_vec(A.n_cols, 2 if name.startswith("ham") else 3)
        Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
        M = pkg.CRSMatrix.from_crs(A, flags=SELL, device=DEV)
        slots, fits = sell_expected(A)
        assert fits == name.startswith("ham")
        assert M.sell_slots == (slots if fits else None)
        Bd = _gpu(B)
        for v in (6, 4, 5, 1, 0) if fits else (4, 5, 1, 0):
            M.variant = v
            ok, worst = oracle.bound_ok(M.apply(Bd).cpu().numpy(), Cref, A.row_ptr, S)
            assert ok, (name, v, worst)
        # V4 with B staging forced on (row windows on these wide-span blocks)
        Ms = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(4) | pkg.SPMV_FLAG_V4_STAGE_ON,
                                    device=DEV)
        ok, worst = oracle.bound_ok(Ms.apply(Bd).cpu().numpy(), Cref, A.row_ptr, S)
        assert ok, (name, "v4 staged", worst)
        del Ms
        # FP32 storage against the widened-input oracle
        v32, b32 = A.val.astype(np.float32), B.astype(np.float32)
        C32ref, S32 = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, v32, b32)
        M32 = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, v32,
                            val_dtype=torch.float32, flags=SELL, device=DEV)
        for v in (6, 4) if fits else (4,):
            M32.variant = v
            ok, worst = oracle.bound_ok(M32.apply(_gpu(b32)).cpu().numpy(), C32ref, A.row_ptr,
                                        S32)
            assert ok, (name, "f32", v, worst)
        del M, M32
        torch.cuda.empty_cache()


def test_full_size_spmm_hamiltonian():
    """Multi-RHS on the full N = 6.0M Hamiltonian-like matrix with the plan the
    benchmark times (autotuned, V6 copy requested), from the chunked copy
    through its 8-bit deltas: k = 2 in column blocks, k = 8, 16 and 32 in
    lane groups (k = 32: 1.5 GB of B, XCD-contiguous chunk order); every
    entry checked against the oracle."""
    A = crsgen.hamiltonian(6_000_000, seed=2)
    M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_SELECT_AUTOTUNE | SELL, device=DEV)
    assert M.variant == pkg.SPMV_V6_SELL64
    for k in (2, 8, 16, 32):
        Bh = crsgen.uniform_vec(A.n_cols * k, 4).reshape(A.n_cols, k)
        Cref, S = oracle.spmm(A.n_rows, A.row_ptr, A.col_idx, A.val, Bh)
        C = M.spmm(_gpu(Bh)).cpu().numpy()
        ok, worst = oracle.bound_ok(C, Cref, A.row_ptr, S)
        assert ok, (k, worst)
        del Cref, S, C
    del M
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["laplace2d_256", "powerlaw_60k", "mostly_empty", "hand",
                                  "rect_wide", "nnz0", "rows0"])
def test_features_vs_oracle(name):
    A, _ = case(name)
    M = pkg.CRSMatrix.from_crs(A, device=DEV)
    f = M.features
    ref = oracle.row_features(A.n_rows, A.row_ptr, A.col_idx)
    assert np.allclose(f, ref, rtol=1e-12, atol=0), (f, ref)


BAD = {
    "row_ptr0": (3, 4, [1, 2, 2, 5], [0, 3, 1, 2, 3]),
    "decreasing": (3, 4, [0, 3, 2, 5], [0, 3, 1, 2, 3]),
    "last_ne_nnz": (3, 4, [0, 2, 2, 4], [0, 3, 1, 2, 3]),
    "col_high": (3, 4, [0, 2, 2, 5], [0, 4, 1, 2, 3]),
    "col_negative": (3, 4, [0, 2, 2, 5], [0, 3, -1, 2, 3]),
}


@pytest.mark.parametrize("name", list(BAD))
def test_bad_crs_rejected(name):
    n, nc, rp, ci = BAD[name]
    with pytest.raises(pkg.SpmvError) as e:
        pkg.CRSMatrix(n, nc, np.array(rp), np.array(ci), np.ones(len(ci)), device=DEV)
    assert e.value.status == pkg.SPMV_ERR_BAD_CRS
    # the device is still healthy afterwards
    A = crsgen.laplace2d(8)
    pkg.CRSMatrix.from_crs(A, device=DEV).apply(_gpu(rhs(A)))
    torch.cuda.synchronize()


@pytest.mark.parametrize("sell", [False, True])
def test_autotune_selects_fastest(sell):
    A, B = case("hamiltonian_200k")
    M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_SELECT_AUTOTUNE | (SELL if sell else 0),
                               device=DEV)
    t = pkg.spmv_get_autotune_times(M.handle)
    assert t.shape == (NV,) and np.all(t > 0) and M.variant == int(np.argmin(t))
    assert np.isfinite(t[pkg.SPMV_V6_SELL64]) == sell
    Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
    assert oracle.bound_ok(M.apply(_gpu(B)).cpu().numpy(), Cref, A.row_ptr, S)[0]


@pytest.mark.parametrize("name", list(CASES))
def test_sell_copy_size_and_availability(name):
    """The V6 copy has exactly 64 x (sum of chunk widths) slots and exists iff
    that fits the reserve; without it V6 cannot be selected."""
    A, B = case(name)
    slots, fits = sell_expected(A)
    M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(4) | SELL, device=DEV)
    assert M.sell_slots == (slots if fits else None)
    if fits:
        M6 = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(6) | SELL, device=DEV)
        assert M6.variant == 6
        Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
        assert oracle.bound_ok(M6.apply(_gpu(B)).cpu().numpy(), Cref, A.row_ptr, S)[0]
    else:
        with pytest.raises(pkg.SpmvError) as e:
            M.variant = 6
        assert e.value.status == pkg.SPMV_ERR_STATE and M.variant == 4
        with pytest.raises(pkg.SpmvError) as e:
            pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(6) | SELL, device=DEV)
        assert e.value.status == pkg.SPMV_ERR_UNSUPPORTED
    # a plan built without the flag never has the copy
    M0 = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(4), device=DEV)
    assert M0.sell_slots is None


def test_sell_padding_and_nonfinite_B():
    """Padded slots never read B: an infinite or NaN B entry reaches only the
    rows that reference it, as in the CRS definition."""
    rng = np.random.default_rng(11)
    n = 1000
    lens = rng.integers(0, 9, size=n)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(n - 1, size=l, replace=False)) + 1 for l in lens]
                        ).astype(np.int32)  # column 0 never referenced
    va = rng.standard_normal(ci.shape[0])
    A = crsgen.CRS(n, n, rp, ci, va)
    B = crsgen.uniform_vec(n, 3)
    B[0] = np.inf
    Cref, S = oracle.spmv(n, rp, ci, va, B)
    assert np.all(np.isfinite(Cref))
    M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(6) | SELL, device=DEV)
    assert M.sell_slots > A.nnz
    C = M.apply(_gpu(B)).cpu().numpy()
    assert np.all(np.isfinite(C)) and oracle.bound_ok(C, Cref, rp, S)[0]


# ------------------------------------------------------------------ batch

def _batch_mats(count, seed, nlo=100, nhi=5000):
    return [crsgen.family_matrix(seed, i, nlo, nhi)[0] for i in range(count)]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batch_vs_oracle_and_each(dt):
    mats = _batch_mats(200, 6)
    tdt = torch.float32 if dt == "f32" else torch.float64
    if dt == "f32":
        mats = [crsgen.CRS(m.n_rows, m.n_cols, m.row_ptr, m.col_idx, m.val.astype(np.float32))
                for m in mats]
    Bt = pkg.Batch(mats, val_dtype=tdt, device=DEV)
    ncols = int(Bt.n_cols.sum())
    Bh = crsgen.uniform_vec(ncols, 6)
    if dt == "f32":
        Bh = Bh.astype(np.float32)
    B_all = _gpu(Bh)
    C_all = torch.full((int(Bt.n_rows.sum()),), float("nan"), dtype=torch.float64, device=DEV)
    Bd, Cd, bh, ch = Bt.pointers(B_all, C_all)
    Bt.apply(Bd, Cd)
    C1 = C_all.clone()
    for m, A in enumerate(mats):
        b = Bh[Bt.col_off[m]:Bt.col_off[m + 1]]
        Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, b)
        got = C1[Bt.row_off[m]:Bt.row_off[m + 1]].cpu().numpy()
        ok, worst = oracle.bound_ok(got, Cref, A.row_ptr, S)
        assert ok, (m, worst)
    C_all.fill_(float("nan"))
    Bt.apply_each(bh, ch)
    assert torch.equal(C_all, C1)  # same tiles, same order: bitwise
    for mode in (pkg.SPMV_BATCH_STATIC, pkg.SPMV_BATCH_TILE_GRID, pkg.SPMV_BATCH_DYNAMIC):
        Bt.set_mode(mode)
        for _ in range(3):  # repeated launches: the dynamic counters reset themselves
            C_all.fill_(float("nan"))
            Bt.apply(Bd, Cd)
            assert torch.equal(C_all, C1), mode


@pytest.mark.parametrize("count", [1, 2, 3, 5, 9])
def test_batch_fewer_tiles_than_queues(count):
    """Batches of a few small matrices: a persistent grid smaller than the 8
    per-XCD ranges (static: as many ranges as workgroups; dynamic: every
    range still drained by stealing), each mode against the oracle and
    bitwise equal to the tile grid, repeated so the dynamic counters reset."""
    mats = [crsgen.family_matrix(4, i, 100, 400)[0] for i in range(count)]
    Bt = pkg.Batch(mats, device=DEV)
    Bh = crsgen.uniform_vec(int(Bt.n_cols.sum()), 4)
    B_all = _gpu(Bh)
    C_all = torch.full((int(Bt.n_rows.sum()),), float("nan"), dtype=torch.float64, device=DEV)
    Bd, Cd, _, _ = Bt.pointers(B_all, C_all)
    Bt.set_mode(pkg.SPMV_BATCH_TILE_GRID)
    Bt.apply(Bd, Cd)
    ref = C_all.clone()
    got = ref.cpu().numpy()
    for m, A in enumerate(mats):
        b = Bh[Bt.col_off[m]:Bt.col_off[m + 1]]
        Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, b)
        assert oracle.bound_ok(got[Bt.row_off[m]:Bt.row_off[m + 1]], Cref, A.row_ptr, S)[0], m
    for mode in (pkg.SPMV_BATCH_STATIC, pkg.SPMV_BATCH_DYNAMIC):
        Bt.set_mode(mode)
        for _ in range(3):
            C_all.fill_(float("nan"))
            Bt.apply(Bd, Cd)
            assert torch.equal(C_all, ref), (mode, Bt.ntiles)


def test_graph_replay_matches_eager():
    mats = _batch_mats(300, 7)
    Bt = pkg.Batch(mats, device=DEV)
    B_all = _gpu(crsgen.uniform_vec(int(Bt.n_cols.sum()), 7))
    C_all = torch.zeros(int(Bt.n_rows.sum()), dtype=torch.float64, device=DEV)
    Bd, Cd, bh, ch = Bt.pointers(B_all, C_all)
    Bt.apply(Bd, Cd)
    eager = C_all.clone()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        pkg.spmv_graph_begin(s)
        Bt.apply(Bd, Cd, stream=s)
        g1 = pkg.spmv_graph_end(s)
        pkg.spmv_graph_begin(s)
        Bt.apply_each(bh, ch, stream=s)
        g2 = pkg.spmv_graph_end(s)
    try:
        for g in (g1, g2, g1, g2, g1):
            C_all.fill_(-1.0)
            torch.cuda.synchronize()
            pkg.spmv_graph_launch(g, s)
            s.synchronize()
            assert torch.equal(C_all, eager)
            # eager work between replays
            Bt.apply(Bd, Cd)
            torch.cuda.synchronize()
    finally:
        pkg.spmv_graph_destroy(g1)
        pkg.spmv_graph_destroy(g2)


@pytest.mark.parametrize("name", ["mesh3d_48_permuted", "hamiltonian_200k"])
def test_single_matrix_graph_replay(name):
    A, B = case(name)
    M = pkg.CRSMatrix.from_crs(A, flags=SELL, device=DEV)
    Bd = _gpu(B)
    C = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    for v in variants(M):
        M.variant = v
        eager = M.apply(Bd).clone()
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        pkg.spmv_graph_begin(s)
        pkg.spmv_apply(M.handle, Bd, pkg.SPMV_F64, C, s)
        g = pkg.spmv_graph_end(s)
        for _ in range(3):
            C.fill_(0.0)
            torch.cuda.synchronize()
            pkg.spmv_graph_launch(g, s)
            s.synchronize()
            assert torch.equal(C, eager), v
            M.apply(Bd)
        pkg.spmv_graph_destroy(g)


@pytest.mark.parametrize("name", ["hamiltonian_200k", "mesh3d_48_permuted", "laplace2d_256"])
def test_fp32_storage_error_vs_fp64_oracle(name):
    """FP32-stored val and B against the FP64-input oracle. Rounding each
    input to float32 perturbs every product by at most 2^-23 + 2^-48 of its
    magnitude; the float64 sums add at most gamma_n on each side, so
    |C32 - C64| <= (2^-23 + 2^-48 + 2 gamma_n (1 + 2^-23)) S_i. Reports the
    observed worst ratio and the relative 2-norm error."""
    A, B = case(name)
    Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.astype(np.float32),
                      val_dtype=torch.float32, device=DEV)
    C = M.apply(_gpu(B.astype(np.float32))).cpu().numpy()
    n = np.diff(A.row_ptr).astype(np.float64)
    u = 2.0 ** -53
    gam = n * u / (1 - n * u)
    tol = (2.0 ** -23 + 2.0 ** -48 + 2 * gam * (1 + 2.0 ** -23)) * S
    d = np.abs(C - Cref)
    assert np.all(d <= tol)
    nz = S > 0
    print(f"{name}: max |dC|/S = {np.max(d[nz] / S[nz]):.3e}, "
          f"rel 2-norm = {np.linalg.norm(C - Cref) / np.linalg.norm(Cref):.3e}")


def test_spmm_fp32_storage_error_per_column():
    A = crsgen.laplace2d(256)
    k = 32
    Bh = crsgen.uniform_vec(A.n_cols * k, 4).reshape(A.n_cols, k)
    Cref, S = oracle.spmm(A.n_rows, A.row_ptr, A.col_idx, A.val, Bh)
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.astype(np.float32),
                      val_dtype=torch.float32, device=DEV)
    C = M.spmm(_gpu(Bh.astype(np.float32))).cpu().numpy()
    n = np.diff(A.row_ptr).astype(np.float64)[:, None]
    gam = n * 2.0 ** -53 / (1 - n * 2.0 ** -53)
    assert np.all(np.abs(C - Cref) <= (2.0 ** -23 + 2.0 ** -48 + 2 * gam * (1 + 2.0 ** -23)) * S)
    col_err = np.linalg.norm(C - Cref, axis=0) / np.linalg.norm(Cref, axis=0)
    assert np.all(col_err < 1e-6)


def _banded_ragged(n, half, seed, jitter):
    """Rows i with columns [i-half, i+half] clipped, a seeded number (0..jitter)
    of them dropped per row, so chunk widths are odd and even and rows inside
    a chunk differ in length."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        c = np.arange(max(0, i - half), min(n, i + half + 1))
        drop = rng.integers(0, jitter + 1)
        if drop:
            c = np.delete(c, rng.choice(len(c), size=min(drop, len(c)), replace=False))
        rows.append(np.full(len(c), i))
        cols.append(c)
    lens = np.array([len(c) for c in cols])
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate(cols).astype(np.int32)
    return crsgen.CRS(n, n, rp, ci, rng.standard_normal(ci.shape[0]))


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("k", [4, 8, 16, 32])
def test_spmm_lanes_ragged_last_chunk(k, dt):
    """The lane-group multi-RHS kernel on 10,007 rows (the last 64-row chunk
    holds 23 rows) with rows of different lengths: every entry against the
    oracle, bitwise equal to the column-block/row-group path that an odd
    leading dimension selects, and the 64 C rows past the matrix untouched."""
    A = _banded_ragged(10_007, 20, seed=11, jitter=3)
    n = A.n_rows
    tdt = torch.float32 if dt == "f32" else torch.float64
    val = A.val.astype(np.float32) if dt == "f32" else A.val
    Bh = crsgen.uniform_vec(A.n_cols * k, 7).reshape(A.n_cols, k)
    if dt == "f32":
        Bh = Bh.astype(np.float32)
    Cref, S = oracle.spmm(A.n_rows, A.row_ptr, A.col_idx, val, Bh)
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val, val_dtype=tdt,
                      flags=pkg.SPMV_FLAG_VARIANT(6) | SELL, device=DEV)
    assert M.sell_slots is not None
    Cbig = torch.full((n + 64, k), 7.0, dtype=torch.float64, device=DEV)
    pkg.spmm_apply(M.handle, k, _gpu(Bh), k, M.code, Cbig, k)
    C = Cbig[:n].cpu().numpy()
    ok, worst = oracle.bound_ok(C, Cref, A.row_ptr, S)
    assert ok, worst
    assert torch.all(Cbig[n:] == 7.0)
    # an odd leading dimension of B takes the scalar paths: same products, same order
    Bo = torch.zeros((A.n_cols, k + 1), dtype=tdt, device=DEV)
    Bo[:, :k] = _gpu(Bh)
    Co = torch.empty((n, k), dtype=torch.float64, device=DEV)
    pkg.spmm_apply(M.handle, k, Bo, k + 1, M.code, Co, k)
    assert torch.equal(Co, Cbig[:n])


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n,half,jitter", [(10_007, 20, 3), (4_099, 7, 1), (130, 1, 1),
                                           (65, 40, 0), (64, 0, 0)])
def test_sell_layout_rounds_and_ragged_tail(n, half, jitter, dt):
    """V6 over chunk widths that need several 8-pair rounds, odd last slots,
    rows of different lengths inside a chunk and a ragged last chunk."""
    A = _banded_ragged(n, half, seed=n, jitter=jitter)
    B = crsgen.uniform_vec(n, 9)
    if dt == "f32":
        val, Bh, tdt = A.val.astype(np.float32), B.astype(np.float32), torch.float32
    else:
        val, Bh, tdt = A.val, B, torch.float64
    Cref, S = oracle.spmv(n, A.row_ptr, A.col_idx, val, Bh)
    M = pkg.CRSMatrix(n, n, A.row_ptr, A.col_idx, val, val_dtype=tdt,
                      flags=pkg.SPMV_FLAG_VARIANT(6) | SELL, device=DEV)
    slots, fits = sell_expected(A)
    assert fits and M.sell_slots == slots
    C = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
    M.apply(_gpu(Bh), C)
    ok, worst = oracle.bound_ok(C.cpu().numpy(), Cref, A.row_ptr, S)
    assert ok, worst


def _span_matrix(spans, n_cols):
    """One 64-row chunk per entry of `spans`: row l of chunk k has a nonzero
    in column 1000 k + (l spans[k]) // 63, so slot 0 of chunk k covers exactly
    spans[k] + 1 columns, and even rows a second one in the next column (odd
    rows pad slot 1)."""
    rng = np.random.default_rng(len(spans))
    cols = []
    for k, sp in enumerate(spans):
        for l in range(64):
            c = 1000 * k + (l * sp) // 63
            cols.append([c, c + 1] if l % 2 == 0 else [c])
    lens = np.array([len(c) for c in cols])
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate(cols).astype(np.int32)
    return crsgen.CRS(len(cols), n_cols, rp, ci, rng.standard_normal(ci.shape[0]))


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_sell_column_deltas_at_their_limit(dt):
    """A chunk is read through 8-bit deltas exactly when each of its slots
    spans at most 0xFE columns, else through 16-bit deltas when each spans at
    most 0xFFFE (the all-ones delta marks padding); either way the product is
    bitwise the one read through the 4-byte columns, and within the bound of
    the oracle."""
    spans = [0, 1, 63, 0xFE, 0xFF, 0xFFFE, 0xFFFF, 0x10000, 1_000_000]
    A = _span_matrix(spans, 2_000_000)
    B = crsgen.uniform_vec(A.n_cols, 12)
    tdt = torch.float32 if dt == "f32" else torch.float64
    val = A.val.astype(np.float32) if dt == "f32" else A.val
    Bh = B.astype(np.float32) if dt == "f32" else B
    Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, val, Bh)
    outs = []
    for wide, expect in ((False, (4, 2)), (True, (0, 0))):
        fl = pkg.SPMV_FLAG_VARIANT(6) | SELL | (pkg.SPMV_FLAG_SELL_WIDE if wide else 0)
        M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val, val_dtype=tdt,
                          flags=fl, device=DEV)
        assert M.sell_deltas == expect + (len(spans),)
        C = M.apply(_gpu(Bh)).cpu().numpy()
        ok, worst = oracle.bound_ok(C, Cref, A.row_ptr, S)
        assert ok, (wide, worst)
        outs.append(C)
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("name", ["hand", "laplace2d_256", "hamiltonian_200k", "banded_40k",
                                  "nnz0", "rows0"])  # the cases whose copy fits its reserve
def test_sell_deltas_bitwise_equal_wide(name, dt):
    """Every case read through the deltas where they fit gives bitwise the
    product (and the multi-RHS product) of the copy read through its 4-byte
    columns."""
    A, B = case(name)
    tdt = torch.float32 if dt == "f32" else torch.float64
    val = A.val.astype(np.float32) if dt == "f32" else A.val
    Bd = _gpu(B.astype(np.float32) if dt == "f32" else B)
    tdB = torch.float32 if dt == "f32" else torch.float64
    Bk = {k: torch.from_numpy(crsgen.uniform_vec(A.n_cols * k, 40 + k)).to(DEV, tdB).reshape(
        A.n_cols, k) for k in (3, 8)}
    outs, narrow, mm = [], [], []
    for wide in (False, True):
        fl = pkg.SPMV_FLAG_VARIANT(4) | SELL | (pkg.SPMV_FLAG_SELL_WIDE if wide else 0)
        M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val, val_dtype=tdt,
                          flags=fl, device=DEV)
        M.variant = 6
        narrow.append(M.sell_deltas)
        outs.append(M.apply(Bd).cpu().numpy())
        # from the copy where rows average at least 8 entries (k <= 8)
        mm.append([M.spmm(Bk[k]).cpu().numpy() for k in (3, 8)])
    assert narrow[1][:2] == (0, 0)
    for x, y in zip(mm[0], mm[1]):
        assert np.array_equal(x, y)
    n8, n16, nch = narrow[0]
    if name in ("laplace2d_256", "banded_40k"):
        assert n8 + n16 == nch  # a band: every chunk on deltas
    if name == "hamiltonian_200k":  # 8-bit except near the ends of the long diagonals
        assert n8 >= 0.9 * nch
    assert np.array_equal(outs[0], outs[1])


def _two_col(n, ncols, far, seed):
    """n rows: even rows hold columns 0 and `far`, odd rows column 1, so the
    one tile of the matrix spans exactly `far` columns."""
    rng = np.random.default_rng(seed)
    cols = [[0, far] if i % 2 == 0 else [1] for i in range(n)]
    lens = np.array([len(c) for c in cols])
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate(cols).astype(np.int32)
    return crsgen.CRS(n, ncols, rp, ci, rng.standard_normal(ci.shape[0]))


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batch_column_delta_widths(dt):
    """Tile columns are read as 8-bit deltas up to a span of 0xFF, 16-bit up to
    0xFFFF and as the 4-byte columns beyond: every width against the oracle,
    and bitwise equal to the single-matrix staged row-block product (the same
    blocks, products and sums)."""
    mats = [_two_col(64, 300, 0xFF, 1), _two_col(64, 300, 0x100, 2),
            _two_col(64, 70_000, 0xFFFF, 3), _two_col(64, 70_000, 0x10000, 4),
            crsgen.random_crs(1000, 200_000, seed=5, max_len=40), _banded_ragged(3000, 9, 6, 2)]
    tdt = torch.float32 if dt == "f32" else torch.float64
    if dt == "f32":
        mats = [crsgen.CRS(m.n_rows, m.n_cols, m.row_ptr, m.col_idx, m.val.astype(np.float32))
                for m in mats]
    Bt = pkg.Batch(mats, val_dtype=tdt, device=DEV)
    Bh = crsgen.uniform_vec(int(Bt.n_cols.sum()), 7)
    if dt == "f32":
        Bh = Bh.astype(np.float32)
    B_all = _gpu(Bh)
    C_all = torch.full((int(Bt.n_rows.sum()),), float("nan"), dtype=torch.float64, device=DEV)
    Bd, Cd, bh, ch = Bt.pointers(B_all, C_all)
    Bt.apply(Bd, Cd)
    for m, A in enumerate(mats):
        b = Bh[Bt.col_off[m]:Bt.col_off[m + 1]]
        Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, b)
        got = C_all[Bt.row_off[m]:Bt.row_off[m + 1]]
        ok, worst = oracle.bound_ok(got.cpu().numpy(), Cref, A.row_ptr, S)
        assert ok, (m, worst)
        M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val, val_dtype=tdt,
                          flags=pkg.SPMV_FLAG_VARIANT(4) | pkg.SPMV_FLAG_V4_STAGE_ON, device=DEV)
        assert torch.equal(M.apply(_gpu(b)), got), m


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("shape", ["empty_chunks", "one_column", "ragged_last"])
def test_sell_deltas_degenerate_chunks(shape, dt):
    """Chunks of width 0 next to full ones, a single column (every span 0),
    and a last chunk of 1 row: V6 through its deltas against the oracle and
    bitwise against its 4-byte columns."""
    rng = np.random.default_rng(17)
    if shape == "empty_chunks":  # every other chunk empty, the rest 1..3 entries per row
        n, nc = 64 * 9, 500
        lens = np.array([0 if (i // 64) % 2 == 0 else 1 + i % 3 for i in range(n)])
    elif shape == "one_column":
        n, nc = 300, 1
        lens = (np.arange(n) % 2).astype(np.int64)
    else:  # 64 k + 1 rows: the last chunk holds one row
        n, nc = 64 * 5 + 1, 2000
        lens = rng.integers(1, 9, size=n)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(nc, size=l, replace=False)) for l in lens]
                        ).astype(np.int32)
    va = rng.standard_normal(ci.shape[0])
    B = crsgen.uniform_vec(nc, 19)
    tdt = torch.float32 if dt == "f32" else torch.float64
    if dt == "f32":
        va, B = va.astype(np.float32), B.astype(np.float32)
    Cref, S = oracle.spmv(n, rp, ci, va, B)
    outs = []
    for wide in (False, True):
        fl = pkg.SPMV_FLAG_VARIANT(6) | SELL | (pkg.SPMV_FLAG_SELL_WIDE if wide else 0)
        M = pkg.CRSMatrix(n, nc, rp, ci, va, val_dtype=tdt, flags=fl, device=DEV)
        C = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
        M.apply(_gpu(B), C)
        got = C.cpu().numpy()
        ok, worst = oracle.bound_ok(got, Cref, rp, S)
        assert ok, (wide, worst)
        outs.append(got)
        if not wide:
            n8, n16, nch = M.sell_deltas
            assert n8 + n16 == nch  # every span here is below 0xFF or 0xFFFF
    assert np.array_equal(outs[0], outs[1])


def test_batch_full_size_4096():
    """The batch the benchmark times (4096 matrices, seed 6, N log-uniform in
    [100, 5000]) in its launch mode (one tile-grid launch): every row of every
    matrix against the oracle; the persistent grids (static ranges, and claims
    from per-XCD queues, repeated so the counters' self-reset is used) and the
    graphs of the tile grid and of the dynamic kernel bitwise equal."""
    mats = _batch_mats(4096, 6)
    Bt = pkg.Batch(mats, device=DEV)
    Bh = crsgen.uniform_vec(int(Bt.n_cols.sum()), 6)
    B_all = _gpu(Bh)
    C_all = torch.full((int(Bt.n_rows.sum()),), float("nan"), dtype=torch.float64, device=DEV)
    Bd, Cd, bh, ch = Bt.pointers(B_all, C_all)
    Bt.set_mode(pkg.SPMV_BATCH_TILE_GRID)
    Bt.apply(Bd, Cd)
    got = C_all.cpu().numpy()
    for m, A in enumerate(mats):
        b = Bh[Bt.col_off[m]:Bt.col_off[m + 1]]
        Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, b)
        ok, worst = oracle.bound_ok(got[Bt.row_off[m]:Bt.row_off[m + 1]], Cref, A.row_ptr, S)
        assert ok, (m, worst)
    first = C_all.clone()
    for mode in (pkg.SPMV_BATCH_STATIC, pkg.SPMV_BATCH_DYNAMIC):
        Bt.set_mode(mode)
        for _ in range(3):
            C_all.fill_(float("nan"))
            Bt.apply(Bd, Cd)
            assert torch.equal(C_all, first), mode
    s = torch.cuda.Stream()
    for mode in (pkg.SPMV_BATCH_TILE_GRID, pkg.SPMV_BATCH_DYNAMIC):
        Bt.set_mode(mode)
        torch.cuda.synchronize()
        pkg.spmv_graph_begin(s)
        Bt.apply(Bd, Cd, stream=s)
        g = pkg.spmv_graph_end(s)
        try:
            for _ in range(3):
                C_all.fill_(float("nan"))
                torch.cuda.synchronize()
                pkg.spmv_graph_launch(g, s)
                s.synchronize()
                assert torch.equal(C_all, first), mode
        finally:
            pkg.spmv_graph_destroy(g)


@pytest.mark.parametrize("mode", ["default", "mlp"])
def test_selector_plan_masks_v6(mode):
    """The network's outputs are the same for a plan with and without the V6
    copy; the default mode takes V6 where the copy is held and the smallest
    predicted time over V0-V5 where it is not; both multiply correctly."""
    A, B = case("hamiltonian_200k")
    flags = pkg.SPMV_SELECT_DEFAULT if mode == "default" else pkg.SPMV_SELECT_MLP
    M0 = pkg.CRSMatrix.from_crs(A, flags=flags, device=DEV)
    M = pkg.CRSMatrix.from_crs(A, flags=flags | SELL, device=DEV)
    assert M.sell_slots is not None
    if pkg.spmv_selector_loaded():
        p0, p = pkg.spmv_get_predictions(M0.handle), pkg.spmv_get_predictions(M.handle)
        assert np.array_equal(p0, p)
        if mode == "default":
            assert M0.v4_form != pkg.SPMV_V4_WINDOWS
            assert M0.variant == int(np.argmin(p[:6]))
            assert M.variant == pkg.SPMV_V6_SELL64
    Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
    assert oracle.bound_ok(M.apply(_gpu(B)).cpu().numpy(), Cref, A.row_ptr, S)[0]
    assert oracle.bound_ok(M0.apply(_gpu(B)).cpu().numpy(), Cref, A.row_ptr, S)[0]


def test_default_mode_takes_the_window_form():
    """The default mode on the permuted 3D stencil with extras: the plan's
    windows hold most nonzeros, so it runs V4 in its window form whatever the
    network ranks first, and equals the oracle bit for bit."""
    A = crsgen.mesh3d(130, seed=3)[0]  # 2.2M rows: 537 super-blocks
    B = rhs(A)
    M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_SELECT_DEFAULT | SELL, device=DEV)
    assert M.v4_form == pkg.SPMV_V4_WINDOWS
    assert M.variant == 4  # V4_lds_block
    Cref, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
    C = M.apply(_gpu(B)).cpu().numpy()
    assert np.array_equal(C.view(np.int64), Cref.view(np.int64))


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("name", ["laplace2d_256", "hamiltonian_200k", "powerlaw_60k",
                                  "long_rows", "mostly_empty"])
def test_nonfinite_B_propagates(name, dt):
    """NaN and infinite B entries propagate by IEEE rules in every variant
    (and both V4 forms): C is NaN exactly where the oracle's is, infinite
    where it is infinite with the same sign, and within the bound elsewhere.
    Padded and masked slots never touch B."""
    A, B = case(name)
    B = B.copy()
    rng = np.random.default_rng(17)
    pick = rng.choice(A.n_cols, size=min(A.n_cols, 40), replace=False)
    B[pick[:20]] = np.nan
    B[pick[20:30]] = np.inf
    B[pick[30:]] = -np.inf
    if dt == "f32":
        val_h, B_h, tdt = A.val.astype(np.float32), B.astype(np.float32), torch.float32
    else:
        val_h, B_h, tdt = A.val, B, torch.float64
    Cref, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, val_h, B_h)
    fin = np.isfinite(Cref)
    Bd = _gpu(B_h)
    for form in (pkg.SPMV_FLAG_V4_STAGE_ON, pkg.SPMV_FLAG_V4_STAGE_OFF):
        M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val_h, val_dtype=tdt,
                          flags=pkg.SPMV_FLAG_VARIANT(4) | SELL | form, device=DEV)
        for v in variants(M):
            M.variant = v
            C = M.apply(Bd).cpu().numpy()
            assert np.array_equal(np.isnan(C), np.isnan(Cref)), (name, dt, v)
            assert np.array_equal(C[np.isinf(Cref)], Cref[np.isinf(Cref)]), (name, dt, v)
            rp = A.row_ptr
            ok, worst = oracle.bound_ok(np.where(fin, C, 0.0), np.where(fin, Cref, 0.0), rp,
                                        np.where(fin, S, 0.0))
            assert ok, (name, dt, v, worst)
    # the multi-RHS form on the same inputs, two columns
    Bk = np.stack([B_h, B_h[::-1].copy()], axis=1)
    Ck_ref, Sk = oracle.spmm(A.n_rows, A.row_ptr, A.col_idx, val_h, Bk)
    Ck = M.spmm(_gpu(Bk)).cpu().numpy()
    assert np.array_equal(np.isnan(Ck), np.isnan(Ck_ref))
