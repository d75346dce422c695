"""Pins of the CPU oracle against facts that do not come from the oracle.

Each pin takes an oracle library handle (``oracle.load(path)``) so the
mutation test can run the same pins against deliberately broken builds of the
oracle and show that every planted mistake is caught.
"""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np

import crsgen
import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U = Fraction(1, 2**53)


def _exact_rows(A: crsgen.CRS, B: np.ndarray):
    """Exact rational C_i and S_i = sum |a_ij b_j| (brute force)."""
    C, S = [], []
    for i in range(A.n_rows):
        c = Fraction(0)
        s = Fraction(0)
        for j in range(A.row_ptr[i], A.row_ptr[i + 1]):
            p = Fraction(float(A.val[j])) * Fraction(float(B[A.col_idx[j]]))
            c += p
            s += abs(p)
        C.append(c)
        S.append(s)
    return C, S


def pin_hand_example(lib):
    """The hand-worked 4x5 example (golden file)."""
    g = json.load(open(os.path.join(GOLDEN, "hand_example.json")))
    C, _ = oracle.spmv(g["n_rows"], np.array(g["row_ptr"]), np.array(g["col_idx"]),
                       np.array(g["val"]), np.array(g["B"]), lib=lib)
    assert np.array_equal(C, np.array(g["C"])), (C, g["C"])


def pin_fraction(lib, cases=40):
    """|oracle - exact| <= gamma_n * S (Higham's recursive-summation bound),
    and S itself within the same relative bound, on tiny irregular CRS."""
    for seed in range(cases):
        rng = np.random.default_rng(1000 + seed)
        nr = int(rng.integers(1, 13))
        nc = int(rng.integers(1, 13))
        A = crsgen.random_crs(nr, nc, seed=seed, max_len=6, empty_frac=0.2,
                              allow_dup=bool(seed % 3 == 0), unsorted=bool(seed % 2))
        B = rng.standard_normal(nc) * np.exp(rng.uniform(-20, 20, size=nc))
        C, S = oracle.spmv(nr, A.row_ptr, A.col_idx, A.val, B, lib=lib)
        Ce, Se = _exact_rows(A, B)
        for i in range(nr):
            n = int(A.row_ptr[i + 1] - A.row_ptr[i])
            gam = n * U / (1 - n * U) if n else Fraction(0)
            assert abs(Fraction(float(C[i])) - Ce[i]) <= gam * Se[i], (seed, i)
            assert abs(Fraction(float(S[i])) - Se[i]) <= gam * Se[i], (seed, i)


def pin_dense(lib):
    """Against numpy's dense product on small rectangular matrices."""
    for seed in range(6):
        nr, nc = 30 + 7 * seed, 50 - 3 * seed
        A = crsgen.random_crs(nr, nc, seed=50 + seed, max_len=12, empty_frac=0.15)
        B = np.random.default_rng(seed).uniform(-1, 1, nc)
        C, S = oracle.spmv(nr, A.row_ptr, A.col_idx, A.val, B, lib=lib)
        D = A.to_dense() @ B
        ok, worst = oracle.bound_ok(C, D, A.row_ptr, S, factor=8.0)
        assert ok, (seed, worst)


def pin_diagonal(lib):
    """Diagonal and identity: C = d * B with one rounding, bit-exact."""
    n = 1000
    rng = np.random.default_rng(7)
    d = rng.standard_normal(n)
    B = rng.standard_normal(n)
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    C, _ = oracle.spmv(n, rp, ci, d, B, lib=lib)
    assert np.array_equal(C, d * B)
    C, _ = oracle.spmv(n, rp, ci, np.ones(n), B, lib=lib)
    assert np.array_equal(C, B)


def pin_integer(lib):
    """Integer-valued A and B: every partial sum is exact, so C is the exact
    integer product (computed in int64) bit for bit."""
    A = crsgen.random_crs(3000, 2500, seed=11, max_len=200, empty_frac=0.05, integer=True)
    B = np.random.default_rng(12).integers(-8, 9, size=2500)
    C, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B.astype(np.float64), lib=lib)
    rows = np.repeat(np.arange(A.n_rows), A.row_lengths())
    exact = np.zeros(A.n_rows, dtype=np.int64)
    np.add.at(exact, rows, A.val.astype(np.int64) * B[A.col_idx])
    assert np.array_equal(C, exact.astype(np.float64))
    # row sums: B = 1
    C1, _ = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, np.ones(2500), lib=lib)
    rs = np.zeros(A.n_rows, dtype=np.int64)
    np.add.at(rs, rows, A.val.astype(np.int64))
    assert np.array_equal(C1, rs.astype(np.float64))


def _sin_exact_arg(idx, k, n1):
    """sin(pi * idx * k / n1) with the angle reduced exactly in integers, so the
    argument carries at most a few ulp of 2*pi (the vector is then accurate to
    about 16 u absolutely)."""
    r = (np.asarray(idx, dtype=np.int64) * k) % (2 * n1)
    return np.sin(math.pi * r / n1)


def _eig_check(A, v, lam, lib):
    C, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, v, lib=lib)
    u = 2.0**-53
    nrow = np.diff(A.row_ptr).astype(np.float64)
    absrow = np.zeros(A.n_rows)
    np.add.at(absrow, np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr)), np.abs(A.val))
    # rounding of the product (<= 8 n u S) plus the error of the computed
    # eigenvector entries (<= 16 u each) propagated through A and lambda
    tol = 8 * nrow * u * S + (abs(lam) + absrow + 1.0) * 16 * u
    assert np.all(np.abs(C - lam * v) <= tol)
    rq = float(v @ C) / float(v @ v)
    assert abs(rq - lam) <= 1e-13 * max(abs(lam), 1e-3)


def pin_laplace_eigen(lib):
    """Closed-form eigenpairs of tridiag(-1,2,-1) and the 2D 5-point stencil:
    lambda_k = 2 - 2 cos(k pi/(n+1)), v_k(j) = sin(j k pi/(n+1)), and the
    product form on the m x m grid."""
    n = 500
    A = crsgen.laplace1d(n)
    j = np.arange(1, n + 1)
    for k in (1, 2, 77, 250, 499, 500):
        th = k * math.pi / (n + 1)
        _eig_check(A, _sin_exact_arg(j, k, n + 1), 2.0 - 2.0 * math.cos(th), lib)
    m = 256
    A2 = crsgen.laplace2d(m)
    x = np.arange(1, m + 1)
    for (k, l) in ((1, 1), (3, 200), (128, 129), (256, 256), (17, 5)):
        tk, tl = k * math.pi / (m + 1), l * math.pi / (m + 1)
        # index = x + m*y: the x factor varies fastest
        v = np.outer(_sin_exact_arg(x, l, m + 1), _sin_exact_arg(x, k, m + 1)).ravel()
        _eig_check(A2, v, 4.0 - 2.0 * math.cos(tk) - 2.0 * math.cos(tl), lib)


def pin_permutation(lib):
    """(P A P^T)(P B) = P (A B) within the bound: ties the permuted stencil to
    the unpermuted one (same seed, same values)."""
    m = 20
    A, _ = crsgen.mesh3d(m, seed=9, block=None)
    Ap, p = crsgen.mesh3d(m, seed=9, block=512)
    B = crsgen.uniform_vec(A.n_rows, 9)
    C, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B, lib=lib)
    Cp, Sp = oracle.spmv(Ap.n_rows, Ap.row_ptr, Ap.col_idx, Ap.val, B[p], lib=lib)
    ok, worst = oracle.bound_ok(Cp, C[p], Ap.row_ptr, Sp)
    assert ok, worst


def pin_edges(lib):
    """Empty matrix, empty rows (+0.0 exactly), duplicates summed, unsorted
    columns (order only changes rounding), rectangular shapes."""
    C, S = oracle.spmv(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0),
                       np.zeros(3), lib=lib)
    assert C.shape == (0,)
    C, S = oracle.spmv(5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0),
                       np.ones(2), lib=lib)
    assert np.array_equal(C, np.zeros(5)) and not np.any(np.signbit(C))
    # duplicates: row 0 = 1.5*B[2] + 2.5*B[2]
    C, _ = oracle.spmv(1, np.array([0, 2]), np.array([2, 2]), np.array([1.5, 2.5]),
                       np.array([0.0, 0.0, 2.0]), lib=lib)
    assert C[0] == 8.0
    # products that cancel: -0 + +0 rows give +0
    C, _ = oracle.spmv(1, np.array([0, 2]), np.array([0, 1]), np.array([-1.0, 1.0]),
                       np.array([0.0, 0.0]), lib=lib)
    assert C[0] == 0.0


def pin_spmm(lib):
    """Multi-RHS: each column against exact rationals; and against dense."""
    A = crsgen.random_crs(9, 7, seed=3, max_len=5, empty_frac=0.2)
    rng = np.random.default_rng(4)
    B = rng.standard_normal((7, 5))
    C, S = oracle.spmm(A.n_rows, A.row_ptr, A.col_idx, A.val, B, lib=lib)
    for c in range(5):
        Ce, Se = _exact_rows(A, B[:, c])
        for i in range(A.n_rows):
            n = int(A.row_ptr[i + 1] - A.row_ptr[i])
            gam = n * U / (1 - n * U) if n else Fraction(0)
            assert abs(Fraction(float(C[i, c])) - Ce[i]) <= gam * Se[i]
    A2 = crsgen.random_crs(60, 40, seed=5, max_len=10)
    B2 = rng.uniform(-1, 1, (40, 8))
    C2, S2 = oracle.spmm(A2.n_rows, A2.row_ptr, A2.col_idx, A2.val, B2, lib=lib)
    ok, worst = oracle.bound_ok(C2, A2.to_dense() @ B2, A2.row_ptr, S2)
    assert ok, worst


def pin_check_crs(lib):
    """Each violation of the CRS definition is reported; valid input passes."""
    rp = np.array([0, 2, 2, 5], np.int32)
    ci = np.array([0, 3, 1, 2, 3], np.int32)
    assert oracle.check_crs(3, 4, rp, ci, lib=lib) == 0
    assert oracle.check_crs(3, 3, rp, ci, lib=lib) == -2          # col >= n_cols
    assert oracle.check_crs(3, 4, rp, np.array([0, 3, -1, 2, 3]), lib=lib) == -2
    assert oracle.check_crs(3, 4, np.array([1, 2, 2, 5]), ci, nnz=5, lib=lib) == -2
    assert oracle.check_crs(3, 4, np.array([0, 2, 1, 5]), ci, lib=lib) == -2
    assert oracle.check_crs(3, 4, np.array([0, 2, 2, 4]), ci, nnz=5, lib=lib) == -2
    assert oracle.check_crs(0, 0, np.array([0]), np.zeros(0), lib=lib) == 0


def pin_features(lib):
    """Features of the hand example and closed forms for the 2D Laplacian."""
    g = json.load(open(os.path.join(GOLDEN, "hand_example.json")))
    f = oracle.row_features(g["n_rows"], np.array(g["row_ptr"]), np.array(g["col_idx"]),
                            lib=lib)
    assert np.allclose(f, g["features"]["values"], rtol=1e-15, atol=0), f
    m = 64
    A = crsgen.laplace2d(m)
    f = oracle.row_features(A.n_rows, A.row_ptr, A.col_idx, lib=lib)
    N, nnz = m * m, 5 * m * m - 4 * m
    n3, n4, n5 = 4, 4 * (m - 2), (m - 2) ** 2
    mean = nnz / N
    var = (9 * n3 + 16 * n4 + 25 * n5) / N - mean**2
    # |col-row| in {0, 1, m}: log buckets 0, 1, floor(log2(m+1)); the 2(m-1)m
    # horizontal pairs give 1, the 2(m-1)m vertical pairs give log2(m+1)
    hor = 2 * (m - 1) * m
    ver = 2 * (m - 1) * m
    want = [math.log2(N), math.log2(nnz), mean, math.sqrt(var), math.log2(6), 3,
            0, (n3 + n4) / N, n5 / N, 0, 0, 0, 0,
            (hor * 1 + ver * int(math.floor(math.log2(m + 1)))) / nnz, 1.0, 5 / mean]
    assert np.allclose(f, want, rtol=1e-14, atol=1e-15), (f, want)
    # one row at each side of every bin edge: lengths 0,1,4,5,16,17,64,65,1024,1025
    lens = [0, 1, 4, 5, 16, 17, 64, 65, 1024, 1025]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.arange(l) for l in lens]).astype(np.int32)
    f = oracle.row_features(len(lens), rp, ci, lib=lib)
    assert np.array_equal(f[6:12], np.array([1, 2, 2, 2, 2, 1]) / 10.0), f[6:12]
    assert f[5] == 0 and f[4] == math.log2(1026)
    assert f[12] == (65 + 1024 + 1025) / sum(lens)


ALL_PINS = [pin_hand_example, pin_fraction, pin_dense, pin_diagonal, pin_integer,
            pin_laplace_eigen, pin_permutation, pin_edges, pin_spmm, pin_check_crs,
            pin_features]
