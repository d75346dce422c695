"""CPU oracle for the CRS spMVM hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``, never by the product package. It
shares no code with the GPU path; both are fed by the seeded generators in
``crsgen`` (inputs only).

* :func:`spmv`, :func:`spmm` -- the paper's CRS loop (Sect. 1.2) in plain
  single-threaded C, float64, no FMA contraction (``oracle.c``).
* :func:`check_crs` -- structural validity of a CRS triple.
* :func:`row_features` -- the selector's 16 row-statistics features.
* :mod:`oracle.mlp` -- float64 forward/backward/update of the selector MLP.
* :func:`bound_ok` -- the per-row acceptance bound
  ``|C_gpu - C_ref| <= 8 * nnz_row * 2^-53 * S_i``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

ORACLE_CFLAGS = ["-O1", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]

U = 2.0 ** -53  # unit roundoff of float64


def build(src: str = _SRC, out: str = _SO) -> str:
    """Compile the oracle with gcc (no FMA contraction)."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *ORACLE_CFLAGS, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def load(path: str = _SO):
    """Load an oracle shared object (the default one, or a test's variant)."""
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(path)
    P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.oracle_check_crs.argtypes = [i64, i64, i64, P, P]
    L.oracle_check_crs.restype = ctypes.c_int
    L.oracle_spmv.argtypes = [i64, P, P, P, P, P, P]
    L.oracle_spmv.restype = None
    L.oracle_spmm.argtypes = [i64, i32, P, P, P, P, i64, P, i64, P]
    L.oracle_spmm.restype = None
    L.oracle_row_features.argtypes = [i64, P, P, P]
    L.oracle_row_features.restype = None
    return L


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        _lib_handle = load()
    return _lib_handle


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def check_crs(n_rows, n_cols, row_ptr, col_idx, nnz=None, lib=None) -> int:
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    nnz = int(ci.shape[0]) if nnz is None else int(nnz)
    return int((lib or _lib()).oracle_check_crs(int(n_rows), int(n_cols), nnz, _p(rp), _p(ci)))


def spmv(n_rows, row_ptr, col_idx, val, B, lib=None):
    """Return (C, S): C = A*B in float64 and the per-row magnitude sums S.

    float32 inputs are widened to float64 exactly before the loop (the
    reference for FP32-stored values and B)."""
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    va = _c(val, np.float64)
    b = _c(B, np.float64)
    C = np.empty(int(n_rows), dtype=np.float64)
    S = np.empty(int(n_rows), dtype=np.float64)
    (lib or _lib()).oracle_spmv(int(n_rows), _p(rp), _p(ci), _p(va), _p(b), _p(C), _p(S))
    return C, S


def spmm(n_rows, row_ptr, col_idx, val, B, lib=None):
    """Row-major multi-RHS: B (n_cols, k) -> (C (n_rows, k), S (n_rows, k))."""
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    va = _c(val, np.float64)
    b = _c(B, np.float64)
    k = int(b.shape[1])
    C = np.empty((int(n_rows), k), dtype=np.float64)
    S = np.empty((int(n_rows), k), dtype=np.float64)
    (lib or _lib()).oracle_spmm(int(n_rows), k, _p(rp), _p(ci), _p(va), _p(b), k, _p(C), k,
                                _p(S))
    return C, S


def row_features(n_rows, row_ptr, col_idx, lib=None) -> np.ndarray:
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    f = np.zeros(16, dtype=np.float64)
    (lib or _lib()).oracle_row_features(int(n_rows), _p(rp), _p(ci), _p(f))
    return f


def row_nnz(row_ptr) -> np.ndarray:
    return np.diff(np.asarray(row_ptr, dtype=np.int64))


def bound(row_ptr, S, factor: float = 8.0) -> np.ndarray:
    """Per-row tolerance factor * nnz_row * 2^-53 * S_i (S may be (n,) or (n,k))."""
    n = row_nnz(row_ptr).astype(np.float64)
    if S.ndim == 2:
        n = n[:, None]
    return factor * n * U * S


def bound_ok(C_test, C_ref, row_ptr, S, factor: float = 8.0):
    """(ok, worst) where worst = max |diff| / bound over rows with bound > 0.

    Rows with no entries, and rows whose S_i is zero, must match exactly
    (+0 and -0 are equal)."""
    C_test = np.asarray(C_test, dtype=np.float64)
    C_ref = np.asarray(C_ref, dtype=np.float64)
    tol = bound(row_ptr, S, factor)
    diff = np.abs(C_test - C_ref)
    exact = tol == 0
    ok_exact = bool(np.all(diff[exact] == 0))
    nz = ~exact
    ratio = diff[nz] / tol[nz] if np.any(nz) else np.zeros(1)
    worst = float(ratio.max()) if ratio.size else 0.0
    return bool(ok_exact and np.all(ratio <= 1.0) and np.all(np.isfinite(C_test))), worst
