"""Host baseline (benchmark infrastructure, like the oracle): the paper's
node-level scheme for the CRS product (Sect. 2) -- OpenMP threads over the row
loop with a static schedule and first-touch placement -- plus a STREAM-style
triad, on all cores of the host. Built from ``node.c`` by :func:`build`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libnode.so")
_SRC = os.path.join(_HERE, "node.c")

# no FMA contraction (each row sums exactly as the oracle does); generic x86-64
# code, since the library built here may run on another host
NODE_CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-std=c11", "-D_POSIX_C_SOURCE=200809L", "-D_ISOC11_SOURCE"]


def build() -> str:
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", *NODE_CFLAGS, "-o", tmp, _SRC])
    os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(_SO)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.node_threads.argtypes = []
        L.node_threads.restype = ctypes.c_int
        L.node_spmv_bench.argtypes = [i64, i64, P, P, P, P, P, ctypes.c_double, i32, P, P]
        L.node_spmv_bench.restype = ctypes.c_int
        L.node_triad.argtypes = [i64, i32, P]
        L.node_triad.restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    return int(_lib().node_threads())


def spmv_bench(n_rows, n_cols, row_ptr, col_idx, val, B, min_seconds=5.0, max_reps=1000):
    """(C, reps, seconds): the threaded product timed over `reps` passes."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = np.ascontiguousarray(val, dtype=np.float64)
    b = np.ascontiguousarray(B, dtype=np.float64)
    C = np.empty(int(n_rows), dtype=np.float64)
    reps, secs = ctypes.c_int32(0), ctypes.c_double(0.0)
    st = _lib().node_spmv_bench(int(n_rows), int(n_cols), _p(rp), _p(ci), _p(va), _p(b), _p(C),
                                float(min_seconds), int(max_reps), ctypes.byref(reps),
                                ctypes.byref(secs))
    if st != 0:
        raise MemoryError("node_spmv_bench: allocation failed")
    return C, int(reps.value), float(secs.value)


def triad_gbs(n=1 << 26, reps=10) -> float:
    out = ctypes.c_double(0.0)
    if _lib().node_triad(int(n), int(reps), ctypes.byref(out)) != 0:
        raise MemoryError("node_triad: allocation failed")
    return float(out.value)
