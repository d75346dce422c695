"""CG and Lanczos on top of the product, checked against closed forms of the
2D Laplacian: the exact solution of A x = A x*, and the extreme eigenvalues
4 +- 4 cos(pi/(m+1)). True residuals are recomputed with the CPU oracle."""
import math

import numpy as np
import pytest

import crsgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_1101_0091_amd as pkg  # noqa: E402

DEV = "cuda:0"


def _cg(M, b, tol, maxit=3000, graph=False, check_every=10):
    n = b.shape[0]
    ws_bytes = pkg.spmv_cg_workspace_size(n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=DEV)
    bd = torch.from_numpy(b).to(DEV)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    s = torch.cuda.Stream() if graph else None
    torch.cuda.synchronize()
    it, rr = pkg.spmv_cg_solve(M.handle, bd, x, tol, maxit, check_every, graph, ws, ws_bytes,
                               s)
    torch.cuda.synchronize()
    return x.cpu().numpy(), it, rr


@pytest.fixture(scope="module")
def lap128():
    A = crsgen.laplace2d(128)
    xs = crsgen.uniform_vec(A.n_rows, 8)
    b, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, xs)
    return A, xs, b


def test_cg_solves_laplacian(lap128):
    A, xs, b = lap128
    M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(4), device=DEV)
    x, it, rr = _cg(M, b, 1e-10)
    assert rr <= 1e-10 and 100 < it < 1000
    Ax, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, x)
    assert np.linalg.norm(b - Ax) / np.linalg.norm(b) <= 1e-9
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-6


def test_cg_graph_replay_and_variants_bitwise(lap128):
    A, xs, b = lap128
    M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(4), device=DEV)
    x1, it1, r1 = _cg(M, b, 1e-10)
    x2, it2, r2 = _cg(M, b, 1e-10, graph=True)
    x3, it3, r3 = _cg(M, b, 1e-10)
    assert it1 == it2 == it3 and r1 == r2 == r3
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3)
    # other variants round the products differently; the solutions agree to
    # the solver tolerance
    outs = []
    for v in (0, 4, 5):
        M.variant = v
        outs.append(_cg(M, b, 1e-8)[0])
    for o in outs[1:]:
        assert np.linalg.norm(o - outs[0]) <= 1e-6 * np.linalg.norm(outs[0])


def test_cg_fp32_storage_effect(lap128):
    """FP32 storage of the (exactly representable) Laplacian with a float32
    copy of the search direction: convergence stalls near float32 accuracy."""
    A, xs, b = lap128
    M32 = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.astype(np.float32),
                        val_dtype=torch.float32, device=DEV)
    x, it, rr = _cg(M32, b, 1e-5)
    Ax, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, x)
    true = np.linalg.norm(b - Ax) / np.linalg.norm(b)
    assert rr <= 1e-5 and true <= 1e-4
    print(f"fp32-storage CG: {it} iterations to 1e-5, true residual {true:.2e}")


def test_cg_rejects_bad_arguments(lap128):
    A, xs, b = lap128
    M = pkg.CRSMatrix.from_crs(A, device=DEV)
    with pytest.raises(pkg.SpmvError):
        pkg.spmv_cg_solve(M.handle, torch.zeros(A.n_rows, dtype=torch.float64, device=DEV),
                          torch.zeros(A.n_rows, dtype=torch.float64, device=DEV), 1e-8, 10, 1,
                          False, torch.empty(256, dtype=torch.uint8, device=DEV), 256)
    R = crsgen.random_crs(10, 12, seed=1)
    MR = pkg.CRSMatrix.from_crs(R, device=DEV)
    n = pkg.spmv_cg_workspace_size(10)
    with pytest.raises(pkg.SpmvError):
        pkg.spmv_cg_solve(MR.handle, torch.zeros(10, dtype=torch.float64, device=DEV),
                          torch.zeros(10, dtype=torch.float64, device=DEV), 1e-8, 10, 1, False,
                          torch.empty(n, dtype=torch.uint8, device=DEV), n)


@pytest.mark.parametrize("variant", [None, 0])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_lanczos_extreme_eigenvalues(dt, variant):
    """Default plan, and a V0 plan (two launches per step)."""
    from scipy.linalg import eigvalsh_tridiagonal
    m, k = 64, 300
    A = crsgen.laplace2d(m)
    tdt = torch.float32 if dt == "f32" else torch.float64
    val = A.val.astype(np.float32) if dt == "f32" else A.val
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val, val_dtype=tdt,
                      flags=0 if variant is None else pkg.SPMV_FLAG_VARIANT(variant), device=DEV)
    v0 = torch.from_numpy(crsgen.uniform_vec(A.n_rows, 7)).to(DEV)
    nb = pkg.spmv_lanczos_workspace_size(A.n_rows, k)
    ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
    al, be = pkg.spmv_lanczos(M.handle, v0, k, ws, nb)
    al2, be2 = pkg.spmv_lanczos(M.handle, v0, k, ws, nb)
    assert np.array_equal(al, al2) and np.array_equal(be, be2)
    th = eigvalsh_tridiagonal(al, be[:-1])
    c = math.cos(math.pi / (m + 1))
    tol = 1e-10 if dt == "f64" else 1e-5
    assert abs(th[-1] - (4 + 4 * c)) <= tol
    assert abs(th[0] - (4 - 4 * c)) <= tol


def _cpu_cg(A, b, iters):
    """Textbook CG in float64 with the oracle's product (no stopping test)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    for _ in range(iters):
        Ap, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, p)
        a = rr / (p @ Ap)
        x += a * p
        r -= a * Ap
        rr, rr_old = r @ r, rr
        p = r + (rr / rr_old) * p
    return x, math.sqrt(rr) / np.linalg.norm(b)


@pytest.mark.parametrize("variant", [4, 0, 1])
@pytest.mark.parametrize("graph", [False, True])
def test_cg_fixed_iterations_match_cpu_cg(lap128, graph, variant):
    """Each iteration's scalars come from the fused reductions (the last
    workgroup sums the partials); 25 iterations against a CPU CG pin every
    alpha and beta along the way -- in four launches per iteration (V4) and
    in two (V0, V1: search-direction update, product and p.Ap in one)."""
    A, xs, b = lap128
    M = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_FLAG_VARIANT(variant), device=DEV)
    xr, rr_ref = _cpu_cg(A, b, 25)
    first = None
    for rep in range(5):  # the counters must be back at zero for every later solve
        x, it, rr = _cg(M, b, 0.0, maxit=25, graph=graph, check_every=5)
        assert it == 25
        assert np.linalg.norm(x - xr) <= 1e-11 * np.linalg.norm(xr)
        assert abs(rr - rr_ref) <= 1e-9 * rr_ref
        if first is None:
            first = (x, rr)
        assert np.array_equal(x, first[0]) and rr == first[1]  # run to run: bitwise


@pytest.mark.parametrize("variant", [None, 0])
def test_lanczos_first_steps_match_cpu(variant):
    m, k = 48, 12
    A = crsgen.laplace2d(m)
    M = pkg.CRSMatrix.from_crs(A, flags=0 if variant is None else pkg.SPMV_FLAG_VARIANT(variant),
                               device=DEV)
    v0 = crsgen.uniform_vec(A.n_rows, 9)
    nb = pkg.spmv_lanczos_workspace_size(A.n_rows, k)
    ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
    al, be = pkg.spmv_lanczos(M.handle, torch.from_numpy(v0).to(DEV), k, ws, nb)
    v, vp, bprev = v0 / np.linalg.norm(v0), np.zeros_like(v0), 0.0
    for j in range(k):
        w, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, v)
        w = w - bprev * vp
        a = w @ v
        w = w - a * v
        bn = np.linalg.norm(w)
        assert abs(al[j] - a) <= 1e-12 * 8
        assert abs(be[j] - bn) <= 1e-12 * 8
        v, vp, bprev = w / bn, v, bn


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_cg_on_the_chunked_copy(lap128, dt):
    """CG whose product is V6 read through its column deltas: eager and
    graph-replayed iterations bitwise equal, and the solution converged."""
    A, xs, b = lap128
    tdt = torch.float32 if dt == "f32" else torch.float64
    val = A.val.astype(np.float32) if dt == "f32" else A.val
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, val, val_dtype=tdt,
                      flags=pkg.SPMV_FLAG_VARIANT(6) | pkg.SPMV_FLAG_SELL, device=DEV)
    n8, n16, nch = M.sell_deltas
    assert n8 + n16 == nch
    tol = 1e-5 if dt == "f32" else 1e-10
    x1, it1, r1 = _cg(M, b, tol)
    x2, it2, r2 = _cg(M, b, tol, graph=True)
    assert it1 == it2 and r1 == r2 and np.array_equal(x1, x2)
    Ax, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, x1)
    assert np.linalg.norm(b - Ax) / np.linalg.norm(b) <= (1e-4 if dt == "f32" else 1e-9)


def _diag_plan(d, variant, dt):
    n = d.shape[0]
    rp = np.arange(n + 1, dtype=np.int32)
    val = d.astype(np.float32) if dt == "f32" else d
    return pkg.CRSMatrix(n, n, rp, rp[:-1], val,
                         val_dtype=torch.float32 if dt == "f32" else torch.float64,
                         flags=pkg.SPMV_FLAG_VARIANT(variant), device=DEV)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n", [70_001, 300_007])
def test_two_launch_cg_equals_four_launch(n, dt):
    """On a diagonal matrix every variant's product is the same single
    rounded product, so CG through the one-launch step (V0 plan) and through
    the four launches (V4 plan) perform the same operations: x and the
    residual equal bit for bit after 40 iterations, eager and graph-replayed
    (300,007 rows take the reduction grid's stride loop twice)."""
    rng = np.random.default_rng(n)
    d = 1.0 + rng.integers(0, 4096, size=n) / 1024.0  # exact in float32 too
    b = rng.uniform(-1, 1, size=n)
    out = []
    for v in (0, 4):
        M = _diag_plan(d, v, dt)
        for graph in (False, True):
            x, it, rr = _cg(M, b, 0.0, maxit=40, graph=graph, check_every=8)
            assert it == 40
            out.append((x, rr))
    for x, rr in out[1:]:
        assert rr == out[0][1]
        assert np.array_equal(x.view(np.int64), out[0][0].view(np.int64))


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_two_launch_lanczos_equals_four_launch(dt):
    """The same argument for Lanczos: on a diagonal matrix the one-launch
    step (V0 plan) and the four-launch step (V4 plan) give the same alpha and
    beta bit for bit over 60 steps, in both storage precisions."""
    rng = np.random.default_rng(11)
    n = 90_001
    d = 1.0 + rng.integers(0, 4096, size=n) / 1024.0
    v0 = torch.from_numpy(rng.uniform(-1, 1, size=n)).to(DEV)
    k = 60
    nb = pkg.spmv_lanczos_workspace_size(n, k)
    ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
    out = []
    for v in (0, 4):
        M = _diag_plan(d, v, dt)
        out.append(pkg.spmv_lanczos(M.handle, v0, k, ws, nb))
    (a0, b0), (a4, b4) = out
    assert np.array_equal(np.asarray(a0).view(np.int64), np.asarray(a4).view(np.int64))
    assert np.array_equal(np.asarray(b0).view(np.int64), np.asarray(b4).view(np.int64))
