"""Seeded synthetic inputs: CRS matrices and dense vectors.

This package only builds inputs. It contains none of the sparse
matrix-vector arithmetic, and both the CPU oracle and the GPU library are fed
from it. The heavy generators are C (``crsgen.c``, OpenMP, Philox4x32-10
counter-based random numbers), so the arrays are identical for any thread
count. Small irregular test matrices come from ``numpy.random.default_rng``.

CRS layout (the paper's Sect. 1.2 "Compressed Row Storage"): ``row_ptr``
int32[n_rows+1] with 0-based offsets, ``col_idx`` int32[nnz], ``val``
float64[nnz]; this package always emits sorted, distinct columns per row.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libcrsgen.so")
_SRC = os.path.join(_HERE, "crsgen.c")


def build() -> str:
    """Compile ``libcrsgen.so`` in place (gcc, OpenMP)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64, u32, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
        sig = {
            "crsgen_philox4x32_10": [P, P, P],
            "crsgen_uniform_vec": [u32, u32, i64, P],
            "crsgen_int_vec": [u32, u32, i64, i32, i32, P],
            "crsgen_laplace2d": [i32, P, P, P],
            "crsgen_laplace1d": [i32, P, P, P],
            "crsgen_ham_offsets": [u32, i64, P],
            "crsgen_ham_rowlens": [i64, P, P],
            "crsgen_ham_fill": [u32, i64, P, P, P, P],
            "crsgen_block_perm": [u32, i64, i32, P],
            "crsgen_mesh_rowlens": [u32, i32, u32, i32, P, P],
            "crsgen_mesh_fill": [u32, i32, u32, i32, P, P, P, P, P],
            "crsgen_family_params": [u32, u32, f64, f64, P],
            "crsgen_family_rowlens": [u32, u32, i64, i32, i32, P],
            "crsgen_family_fill": [u32, u32, i64, i32, i32, P, P, P],
            "crsgen_powerlaw_cdf": [i32],
            "crsgen_num_threads": [],
            "crsgen_set_threads": [ctypes.c_int],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None
        L.crsgen_powerlaw_cdf.restype = f64
        L.crsgen_num_threads.restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


@dataclass
class CRS:
    """A CRS matrix held in host numpy arrays."""
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray  # int32[n_rows+1]
    col_idx: np.ndarray  # int32[nnz]
    val: np.ndarray      # float64[nnz] (or float32 after .astype)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n_rows, self.n_cols), dtype=np.float64)
        rows = np.repeat(np.arange(self.n_rows), self.row_lengths())
        np.add.at(d, (rows, self.col_idx), self.val.astype(np.float64))
        return d


def _row_ptr_from_lens(lens: np.ndarray) -> np.ndarray:
    rp = np.zeros(lens.shape[0] + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    if rp[-1] >= 2**31:
        raise ValueError(f"nnz={rp[-1]} does not fit int32 row_ptr")
    return rp.astype(np.int32)


# ---------------------------------------------------------------- primitives

def philox4x32_10(ctr, key) -> tuple:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _lib().crsgen_philox4x32_10(_p(c), _p(k), _p(out))
    return tuple(int(x) for x in out)


def set_threads(t: int) -> None:
    _lib().crsgen_set_threads(int(t))


def num_threads() -> int:
    return int(_lib().crsgen_num_threads())


def uniform_vec(n: int, seed: int, stream: int = 0) -> np.ndarray:
    """float64[n] uniform in [-1, 1)."""
    out = np.empty(int(n), dtype=np.float64)
    _lib().crsgen_uniform_vec(seed, stream, int(n), _p(out))
    return out


def int_vec(n: int, seed: int, stream: int, lo: int, hi: int) -> np.ndarray:
    """float64[n] holding integers uniform in [lo, hi]."""
    out = np.empty(int(n), dtype=np.float64)
    _lib().crsgen_int_vec(seed, stream, int(n), lo, hi, _p(out))
    return out


def powerlaw_cdf(l: int) -> float:
    return float(_lib().crsgen_powerlaw_cdf(int(l)))


# ---------------------------------------------------------------- matrices

def laplace2d(m: int) -> CRS:
    """2D 5-point Laplacian on an m x m grid, natural order, diag 4, off -1."""
    n = m * m
    nnz = 5 * n - 4 * m
    rp = np.empty(n + 1, dtype=np.int32)
    ci = np.empty(nnz, dtype=np.int32)
    va = np.empty(nnz, dtype=np.float64)
    _lib().crsgen_laplace2d(m, _p(rp), _p(ci), _p(va))
    return CRS(n, n, rp, ci, va)


def laplace1d(n: int) -> CRS:
    """1D tridiag(-1, 2, -1)."""
    nnz = 3 * n - 2 if n > 1 else n
    rp = np.empty(n + 1, dtype=np.int32)
    ci = np.empty(nnz, dtype=np.int32)
    va = np.empty(nnz, dtype=np.float64)
    _lib().crsgen_laplace1d(n, _p(rp), _p(ci), _p(va))
    return CRS(n, n, rp, ci, va)


def hamiltonian_offsets(n: int, seed: int) -> np.ndarray:
    d = np.zeros(7, dtype=np.int32)
    _lib().crsgen_ham_offsets(seed, int(n), _p(d))
    return d


def hamiltonian(n: int, seed: int) -> CRS:
    """Symmetric: N(0,1) diagonal plus 7 offset pairs +-d_k (log-uniform 1..N/2)."""
    d = hamiltonian_offsets(n, seed)
    lens = np.empty(n, dtype=np.int32)
    _lib().crsgen_ham_rowlens(int(n), _p(d), _p(lens))
    rp = _row_ptr_from_lens(lens)
    ci = np.empty(int(rp[-1]), dtype=np.int32)
    va = np.empty(int(rp[-1]), dtype=np.float64)
    _lib().crsgen_ham_fill(seed, int(n), _p(d), _p(rp), _p(ci), _p(va))
    return CRS(n, n, rp, ci, va)


def block_perm(n: int, seed: int, block: int = 4096) -> np.ndarray:
    """p[new] = old, a random permutation inside each block of `block` indices."""
    p = np.empty(n, dtype=np.int32)
    _lib().crsgen_block_perm(seed, int(n), block, _p(p))
    return p


def mesh3d(m: int, seed: int, extra_frac: float = 0.05, max_extra: int = 30,
           block: int | None = 4096) -> tuple[CRS, np.ndarray | None]:
    """3D 7-point stencil on m^3 + random extras, block-permuted.

    Returns (A', p) with A' = P A P^T, p[new] = old (None if unpermuted).
    """
    n = m * m * m
    ppm = int(round(extra_frac * 1e6))
    p = q = None
    if block:
        p = block_perm(n, seed, block)
        q = np.empty(n, dtype=np.int32)
        q[p] = np.arange(n, dtype=np.int32)
    lens = np.empty(n, dtype=np.int32)
    _lib().crsgen_mesh_rowlens(seed, m, ppm, max_extra, _p(p), _p(lens))
    rp = _row_ptr_from_lens(lens)
    ci = np.empty(int(rp[-1]), dtype=np.int32)
    va = np.empty(int(rp[-1]), dtype=np.float64)
    _lib().crsgen_mesh_fill(seed, m, ppm, max_extra, _p(p), _p(q), _p(rp), _p(ci), _p(va))
    return CRS(n, n, rp, ci, va), p


FAMILY_NAMES = ("uniform", "powerlaw", "banded")


def family_params(seed: int, idx: int, nlo: float, nhi: float) -> dict:
    out = np.zeros(3, dtype=np.int64)
    _lib().crsgen_family_params(seed, idx, float(nlo), float(nhi), _p(out))
    return {"n": int(out[0]), "family": int(out[1]), "width": int(out[2])}


def family_matrix(seed: int, idx: int, nlo: float, nhi: float,
                  n_override: int | None = None) -> tuple[CRS, dict]:
    """Matrix `idx` of a seeded collection (uniform / power-law / banded rows)."""
    prm = family_params(seed, idx, nlo, nhi)
    n = int(n_override) if n_override is not None else prm["n"]
    prm["n"] = n
    lens = np.empty(n, dtype=np.int32)
    _lib().crsgen_family_rowlens(seed, idx, n, prm["family"], prm["width"], _p(lens))
    rp = _row_ptr_from_lens(lens)
    ci = np.empty(int(rp[-1]), dtype=np.int32)
    va = np.empty(int(rp[-1]), dtype=np.float64)
    _lib().crsgen_family_fill(seed, idx, n, prm["family"], prm["width"], _p(rp), _p(ci), _p(va))
    return CRS(n, n, rp, ci, va), prm


def random_crs(n_rows: int, n_cols: int, seed: int, max_len: int = 8,
               empty_frac: float = 0.1, allow_dup: bool = False,
               unsorted: bool = False, integer: bool = False) -> CRS:
    """Small irregular CRS for tests: empty rows, optional duplicate or
    unsorted columns, optional small-integer values."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, size=n_rows)
    lens[rng.random(n_rows) < empty_frac] = 0
    if not allow_dup and n_cols > 0:
        lens = np.minimum(lens, n_cols)
    if n_cols == 0:
        lens[:] = 0
    rp = _row_ptr_from_lens(lens.astype(np.int64))
    cols = []
    for L in lens:
        if L == 0:
            continue
        if allow_dup:
            c = rng.integers(0, n_cols, size=L)
        else:
            c = rng.choice(n_cols, size=L, replace=False)
        c = np.sort(c) if not unsorted else c
        cols.append(c)
    ci = (np.concatenate(cols) if cols else np.zeros(0)).astype(np.int32)
    if integer:
        va = rng.integers(-8, 9, size=ci.shape[0]).astype(np.float64)
    else:
        va = rng.standard_normal(ci.shape[0])
    return CRS(n_rows, n_cols, rp, ci, va)


# ---------------------------------------------------------------- workloads

#: The five workloads. Config 2 and 3 are synthetic stand-ins for the paper's
#: Holstein-Hubbard (N=6.2e6, N_nzr~15) and sAMG (N=2.2e7, N_nzr~7) matrices.
CONFIG_SEEDS = {1: 1, 2: 2, 3: 3, 4: 4, "5a": 5, "5b": 6}


def config_matrix(cfg, scale: str = "full") -> CRS:
    """Matrix of workload `cfg` (1..4). scale='small' gives a shrunken copy
    of the same family for fast parity tests."""
    if cfg in (1, 4):
        return laplace2d(256 if scale == "full" else 64)
    if cfg == 2:
        return hamiltonian(6_000_000 if scale == "full" else 200_000, seed=CONFIG_SEEDS[2])
    if cfg == 3:
        A, _ = mesh3d(280 if scale == "full" else 48, seed=CONFIG_SEEDS[3])
        return A
    raise ValueError(cfg)


def config_rhs(cfg, n: int, k: int = 1) -> np.ndarray:
    """B for workload `cfg`: U[-1,1), shape (n,) or row-major (n, k)."""
    seed = CONFIG_SEEDS[cfg]
    if k == 1:
        return uniform_vec(n, seed, 0)
    return uniform_vec(n * k, seed, 0).reshape(n, k)


def loguniform_n(u: float, lo: float, hi: float) -> int:
    return int(math.floor(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo))) + 0.5))
