"""Python binding of libspmv (CRS sparse matrix-vector products on MI355X).

Argument marshalling only: every function below forwards to the C ABI
declared in ``include/spmv.h`` under the same name; all arithmetic runs in
the library's HIP kernels. PyTorch provides device memory (tensors) and
streams. There is no CPU fallback: without the built ``libspmv.so`` every
call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import perfmodel  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmv.so")

SPMV_F64, SPMV_F32 = 0, 1
SPMV_OK = 0
SPMV_ERR_INVALID_ARG, SPMV_ERR_BAD_CRS, SPMV_ERR_UNSUPPORTED = -1, -2, -3
SPMV_ERR_WORKSPACE, SPMV_ERR_HIP, SPMV_ERR_STATE = -4, -5, -6
VARIANTS = ("V0_thread_row", "V1_lanes4", "V2_lanes16", "V3_wave_row", "V4_lds_block",
            "V5_binned", "V6_sell64")
SPMV_NUM_VARIANTS = 7
SPMV_V6_SELL64 = 6
SPMV_NUM_SELECTOR_OUTPUTS = 7
SPMV_SELECT_DEFAULT, SPMV_SELECT_MLP, SPMV_SELECT_AUTOTUNE, SPMV_SELECT_FIXED = 0, 1, 2, 3
SPMV_FLAG_SKIP_VALIDATE = 0x10000
SPMV_FLAG_SELL = 0x20000
SPMV_FLAG_V4_STAGE_ON = 0x40000
SPMV_FLAG_V4_STAGE_OFF = 0x80000
SPMV_FLAG_SELL_WIDE = 0x100000
SPMV_FLAG_V4_WINDOWS = 0x200000
SPMV_V4_PLAIN, SPMV_V4_STAGED, SPMV_V4_WINDOWS = 0, 1, 2
V4_FORMS = ("plain", "staged", "windows")
SPMV_BATCH_DYNAMIC, SPMV_BATCH_STATIC, SPMV_BATCH_TILE_GRID = 0, 1, 2
SPMV_NUM_FEATURES = 16
SPMV_MLP_PARAMS = 5703

EXPORTS = (
    "spmv_workspace_size", "spmv_create", "spmv_apply", "spmm_apply", "spmv_get_variant",
    "spmv_set_variant", "spmv_get_features", "spmv_get_predictions", "spmv_get_autotune_times",
    "spmv_get_num_blocks", "spmv_get_sell_slots", "spmv_get_sell_deltas", "spmv_get_v4_staged", "spmv_get_v4_form", "spmv_set_v4_form", "spmv_get_sell_stream_bytes",
    "spmv_batch_get_stream_bytes", "spmv_destroy", "spmv_batch_workspace_size", "spmv_batch_create",
    "spmv_batch_apply", "spmv_batch_apply_each", "spmv_batch_get_num_tiles", "spmv_batch_set_mode",
    "spmv_batch_destroy", "spmv_graph_begin", "spmv_graph_end", "spmv_graph_launch",
    "spmv_graph_destroy", "spmv_selector_load", "spmv_selector_loaded",
    "spmv_selector_load_file", "spmv_mlp_forward",
    "spmv_mlp_backward", "spmv_mlp_adam", "spmv_stream_triad", "spmv_stream_copy",
    "spmv_status_string", "spmv_last_error", "spmv_version", "spmv_split_workspace_size",
    "spmv_split_create", "spmv_split_apply", "spmv_split_get_nnz", "spmv_split_destroy",
    "spmv_rcm_order", "spmv_permute_crs", "spmv_cg_workspace_size", "spmv_cg_solve",
    "spmv_lanczos_workspace_size", "spmv_lanczos", "spmv_cg_solve_noalloc",
)


def SPMV_FLAG_VARIANT(v: int) -> int:
    return SPMV_SELECT_FIXED | (int(v) << 8)


class SpmvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libspmv status {status}: {msg}")
        self.status = status


_lib_handle = None


def lib():
    """The loaded libspmv (raises if it was not built)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                               "(the HIP library is required; there is no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32, f32, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_uint32, ctypes.c_float, ctypes.c_double)
        sz = ctypes.c_size_t
        sig = {
            "spmv_workspace_size": [i64, i64, i64, u32, P],
            "spmv_create": [P, i64, i64, i64, P, P, P, ctypes.c_int, P, sz, u32, P],
            "spmv_apply": [P, P, ctypes.c_int, P, P],
            "spmm_apply": [P, i32, P, i64, ctypes.c_int, P, i64, P],
            "spmv_get_variant": [P, P],
            "spmv_set_variant": [P, ctypes.c_int],
            "spmv_get_features": [P, P],
            "spmv_get_predictions": [P, P],
            "spmv_get_autotune_times": [P, P],
            "spmv_get_num_blocks": [P, P],
            "spmv_get_sell_slots": [P, P],
            "spmv_get_sell_deltas": [P, P, P, P],
            "spmv_get_v4_staged": [P, P],
            "spmv_get_v4_form": [P, P, P],
            "spmv_get_sell_stream_bytes": [P, P],
            "spmv_batch_get_stream_bytes": [P, P],
            "spmv_set_v4_form": [P, ctypes.c_int],
            "spmv_destroy": [P],
            "spmv_batch_workspace_size": [i32, i64, i64, P],
            "spmv_batch_create": [P, i32, P, P, P, P, P, P, ctypes.c_int, P, sz, P],
            "spmv_batch_apply": [P, P, P, ctypes.c_int, P],
            "spmv_batch_apply_each": [P, P, P, ctypes.c_int, P],
            "spmv_batch_get_num_tiles": [P, P],
            "spmv_batch_set_mode": [P, ctypes.c_int],
            "spmv_batch_destroy": [P],
            "spmv_graph_begin": [P],
            "spmv_graph_end": [P, P],
            "spmv_graph_launch": [P, P],
            "spmv_graph_destroy": [P],
            "spmv_selector_load": [P, P, P, P, P, f32],
            "spmv_selector_loaded": [P],
            "spmv_selector_load_file": [ctypes.c_char_p],
            "spmv_mlp_forward": [P, P, i32, P, P, P, P],
            "spmv_mlp_backward": [P, P, P, P, P, P, i32, P, P, P],
            "spmv_mlp_adam": [P, P, P, P, i32, f32, f32, f32, f32, P],
            "spmv_stream_triad": [P, P, P, f64, i64, P],
            "spmv_stream_copy": [P, P, i64, P],
            "spmv_split_workspace_size": [i64, i64, i64, P],
            "spmv_split_create": [P, i64, i64, i64, P, P, P, ctypes.c_int, i64, i64, P, sz, P],
            "spmv_split_apply": [P, ctypes.c_int, P, ctypes.c_int, P, P],
            "spmv_split_get_nnz": [P, P, P],
            "spmv_split_destroy": [P],
            "spmv_rcm_order": [i64, P, P, ctypes.c_int, P],
            "spmv_cg_workspace_size": [i64, P],
            "spmv_cg_solve": [P, P, P, f64, i32, i32, i32, P, sz, P, P, P],
            "spmv_lanczos_workspace_size": [i64, i32, P],
            "spmv_cg_solve_noalloc": [P, P, P, f64, i32, i32, P, P, P],
            "spmv_lanczos": [P, P, i32, P, P, P, sz, P],
            "spmv_permute_crs": [i64, P, P, P, ctypes.c_int, P, P, P, P],
            "spmv_status_string": [ctypes.c_int],
            "spmv_last_error": [],
            "spmv_version": [],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        for name in ("spmv_status_string", "spmv_last_error", "spmv_version"):
            getattr(L, name).restype = ctypes.c_char_p
        _lib_handle = L
    return _lib_handle


def _check(status: int) -> None:
    if status != SPMV_OK:
        raise SpmvError(status, lib().spmv_last_error().decode())


def _ptr(x):
    """Device/host address of a tensor or array, or an int/None as given."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return SPMV_F64
    if t.dtype == torch.float32:
        return SPMV_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


# ---------------------------------------------------------------- ABI mirror

def spmv_version() -> str:
    return lib().spmv_version().decode()


def spmv_status_string(status: int) -> str:
    return lib().spmv_status_string(int(status)).decode()


def spmv_last_error() -> str:
    return lib().spmv_last_error().decode()


def spmv_workspace_size(n_rows: int, n_cols: int, nnz: int, flags: int = 0) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().spmv_workspace_size(n_rows, n_cols, nnz, flags, ctypes.byref(out)))
    return int(out.value)


def spmv_create(n_rows, n_cols, nnz, row_ptr, col_idx, val, val_dtype, workspace, ws_bytes,
                flags=0, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p(0)
    _check(lib().spmv_create(ctypes.byref(h), n_rows, n_cols, nnz, _ptr(row_ptr),
                             _ptr(col_idx), _ptr(val), val_dtype, _ptr(workspace), ws_bytes,
                             flags, _stream(stream)))
    return h


def spmv_apply(h, B, b_dtype, C, stream=None) -> None:
    _check(lib().spmv_apply(h, _ptr(B), b_dtype, _ptr(C), _stream(stream)))


def spmm_apply(h, k, B, ldb, b_dtype, C, ldc, stream=None) -> None:
    _check(lib().spmm_apply(h, k, _ptr(B), ldb, b_dtype, _ptr(C), ldc, _stream(stream)))


def spmv_get_variant(h) -> int:
    v = ctypes.c_int(0)
    _check(lib().spmv_get_variant(h, ctypes.byref(v)))
    return int(v.value)


def spmv_set_variant(h, variant: int) -> None:
    _check(lib().spmv_set_variant(h, int(variant)))


def spmv_get_features(h) -> np.ndarray:
    f = np.zeros(SPMV_NUM_FEATURES, dtype=np.float64)
    _check(lib().spmv_get_features(h, f.ctypes.data))
    return f


def spmv_get_predictions(h) -> np.ndarray:
    p = np.zeros(SPMV_NUM_SELECTOR_OUTPUTS, dtype=np.float32)
    _check(lib().spmv_get_predictions(h, p.ctypes.data))
    return p


def spmv_get_autotune_times(h) -> np.ndarray:
    t = np.zeros(SPMV_NUM_VARIANTS, dtype=np.float64)
    _check(lib().spmv_get_autotune_times(h, t.ctypes.data))
    return t


def spmv_get_num_blocks(h) -> int:
    n = ctypes.c_int64(0)
    _check(lib().spmv_get_num_blocks(h, ctypes.byref(n)))
    return int(n.value)


def spmv_get_sell_slots(h) -> int:
    n = ctypes.c_int64(0)
    _check(lib().spmv_get_sell_slots(h, ctypes.byref(n)))
    return int(n.value)


def spmv_get_sell_deltas(h):
    """(chunks read through 8-bit column deltas, through 16-bit ones, all
    chunks) of the V6 copy."""
    a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().spmv_get_sell_deltas(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return int(a.value), int(b.value), int(c.value)


def spmv_get_v4_staged(h) -> bool:
    v = ctypes.c_int(0)
    _check(lib().spmv_get_v4_staged(h, ctypes.byref(v)))
    return bool(v.value)


def spmv_get_v4_form(h):
    """(V4 form in use: SPMV_V4_PLAIN / _STAGED / _WINDOWS, nonzeros inside
    the windows of their super-block)."""
    f, n = ctypes.c_int(0), ctypes.c_int64(0)
    _check(lib().spmv_get_v4_form(h, ctypes.byref(f), ctypes.byref(n)))
    return int(f.value), int(n.value)


def spmv_set_v4_form(h, form: int) -> None:
    _check(lib().spmv_set_v4_form(h, int(form)))


def spmv_get_sell_stream_bytes(h) -> int:
    """Bytes one V6 product reads from the plan's chunked copy."""
    n = ctypes.c_int64(0)
    _check(lib().spmv_get_sell_stream_bytes(h, ctypes.byref(n)))
    return int(n.value)


def spmv_batch_get_stream_bytes(h) -> int:
    """Bytes one batch apply reads for the matrices' nonzeros."""
    n = ctypes.c_int64(0)
    _check(lib().spmv_batch_get_stream_bytes(h, ctypes.byref(n)))
    return int(n.value)


def spmv_destroy(h) -> None:
    _check(lib().spmv_destroy(h))


def spmv_batch_workspace_size(count, total_rows, total_nnz) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().spmv_batch_workspace_size(count, total_rows, total_nnz, ctypes.byref(out)))
    return int(out.value)


def spmv_batch_create(count, n_rows, n_cols, nnz, row_ptrs, col_idxs, vals, val_dtype,
                      workspace, ws_bytes, stream=None):
    """n_rows/n_cols/nnz: host int64 arrays; row_ptrs/col_idxs/vals: device
    int64 tensors holding device addresses."""
    h = ctypes.c_void_p(0)
    nr = np.ascontiguousarray(n_rows, dtype=np.int64)
    nc = np.ascontiguousarray(n_cols, dtype=np.int64)
    nz = np.ascontiguousarray(nnz, dtype=np.int64)
    _check(lib().spmv_batch_create(ctypes.byref(h), count, nr.ctypes.data, nc.ctypes.data,
                                   nz.ctypes.data, _ptr(row_ptrs), _ptr(col_idxs), _ptr(vals),
                                   val_dtype, _ptr(workspace), ws_bytes, _stream(stream)))
    return h


def spmv_batch_apply(h, Bs, Cs, b_dtype, stream=None) -> None:
    _check(lib().spmv_batch_apply(h, _ptr(Bs), _ptr(Cs), b_dtype, _stream(stream)))


def spmv_batch_apply_each(h, Bs_host, Cs_host, b_dtype, stream=None) -> None:
    bh = np.ascontiguousarray(Bs_host, dtype=np.uint64)
    ch = np.ascontiguousarray(Cs_host, dtype=np.uint64)
    _check(lib().spmv_batch_apply_each(h, bh.ctypes.data, ch.ctypes.data, b_dtype,
                                       _stream(stream)))


def spmv_batch_get_num_tiles(h) -> int:
    n = ctypes.c_int64(0)
    _check(lib().spmv_batch_get_num_tiles(h, ctypes.byref(n)))
    return int(n.value)


def spmv_batch_set_mode(h, mode: int) -> None:
    _check(lib().spmv_batch_set_mode(h, int(mode)))


def spmv_batch_destroy(h) -> None:
    _check(lib().spmv_batch_destroy(h))


def spmv_graph_begin(stream=None) -> None:
    _check(lib().spmv_graph_begin(_stream(stream)))


def spmv_graph_end(stream=None):
    g = ctypes.c_void_p(0)
    _check(lib().spmv_graph_end(_stream(stream), ctypes.byref(g)))
    return g


def spmv_graph_launch(g, stream=None) -> None:
    _check(lib().spmv_graph_launch(g, _stream(stream)))


def spmv_graph_destroy(g) -> None:
    _check(lib().spmv_graph_destroy(g))


def spmv_selector_load(params, mu, sigma, lo, hi, margin: float) -> None:
    arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (params, mu, sigma, lo, hi)]
    _check(lib().spmv_selector_load(*[a.ctypes.data for a in arrs], float(margin)))


def spmv_selector_loaded() -> bool:
    v = ctypes.c_int(0)
    _check(lib().spmv_selector_loaded(ctypes.byref(v)))
    return bool(v.value)


def spmv_selector_load_file(path: str) -> None:
    _check(lib().spmv_selector_load_file(os.fsencode(path)))


def load_selector(path: str | None = None) -> bool:
    """Load the packaged (or given) selector weights on the current device.
    Returns False when no weights file exists (plans then use the LDS-block
    variant by default, or autotune when asked)."""
    from .selector import DEFAULT_WEIGHTS
    path = path or DEFAULT_WEIGHTS
    if not os.path.exists(path):
        return False
    spmv_selector_load_file(path)
    return True


def spmv_mlp_forward(theta, X, nb, Y, Z1, Z2, stream=None) -> None:
    _check(lib().spmv_mlp_forward(_ptr(theta), _ptr(X), nb, _ptr(Y), _ptr(Z1), _ptr(Z2),
                                  _stream(stream)))


def spmv_mlp_backward(theta, X, Z1, Z2, Y, T, nb, scratch, grad, stream=None) -> None:
    _check(lib().spmv_mlp_backward(_ptr(theta), _ptr(X), _ptr(Z1), _ptr(Z2), _ptr(Y), _ptr(T),
                                   nb, _ptr(scratch), _ptr(grad), _stream(stream)))


def spmv_mlp_adam(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                  stream=None) -> None:
    _check(lib().spmv_mlp_adam(_ptr(theta), _ptr(grad), _ptr(m), _ptr(v), int(t), float(lr),
                               float(beta1), float(beta2), float(eps), _stream(stream)))


def spmv_stream_triad(a, b, c, s, n, stream=None) -> None:
    _check(lib().spmv_stream_triad(_ptr(a), _ptr(b), _ptr(c), float(s), int(n),
                                   _stream(stream)))


def spmv_stream_copy(dst, src, n, stream=None) -> None:
    _check(lib().spmv_stream_copy(_ptr(dst), _ptr(src), int(n), _stream(stream)))


def spmv_split_workspace_size(n_rows, n_cols, nnz) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().spmv_split_workspace_size(n_rows, n_cols, nnz, ctypes.byref(out)))
    return int(out.value)


def spmv_split_create(n_rows, n_cols, nnz, row_ptr, col_idx, val, val_dtype, col_lo, col_hi,
                      workspace, ws_bytes, stream=None):
    h = ctypes.c_void_p(0)
    _check(lib().spmv_split_create(ctypes.byref(h), n_rows, n_cols, nnz, _ptr(row_ptr),
                                   _ptr(col_idx), _ptr(val), val_dtype, col_lo, col_hi,
                                   _ptr(workspace), ws_bytes, _stream(stream)))
    return h


def spmv_split_apply(h, pass_, B, b_dtype, C, stream=None) -> None:
    _check(lib().spmv_split_apply(h, int(pass_), _ptr(B), b_dtype, _ptr(C), _stream(stream)))


def spmv_split_get_nnz(h):
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().spmv_split_get_nnz(h, ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def spmv_split_destroy(h) -> None:
    _check(lib().spmv_split_destroy(h))


def spmv_rcm_order(n, row_ptr, col_idx, symmetric_part: bool = False) -> np.ndarray:
    """Host arrays in, host permutation out (perm[new] = old)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    perm = np.empty(int(n), dtype=np.int32)
    _check(lib().spmv_rcm_order(int(n), rp.ctypes.data, ci.ctypes.data, int(bool(symmetric_part)),
                                perm.ctypes.data))
    return perm


def spmv_permute_crs(n, row_ptr, col_idx, val, perm):
    """Host P A P^T (perm[new] = old); returns (row_ptr, col_idx, val)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = np.ascontiguousarray(val)
    code = SPMV_F64 if va.dtype == np.float64 else SPMV_F32
    if va.dtype not in (np.float64, np.float32):
        raise TypeError(va.dtype)
    pm = np.ascontiguousarray(perm, dtype=np.int32)
    rpo = np.empty(int(n) + 1, dtype=np.int32)
    cio = np.empty_like(ci)
    vao = np.empty_like(va)
    _check(lib().spmv_permute_crs(int(n), rp.ctypes.data, ci.ctypes.data, va.ctypes.data, code,
                                  pm.ctypes.data, rpo.ctypes.data, cio.ctypes.data,
                                  vao.ctypes.data))
    return rpo, cio, vao


def spmv_cg_workspace_size(n) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().spmv_cg_workspace_size(int(n), ctypes.byref(out)))
    return int(out.value)


def spmv_cg_solve(h, b, x, tol, maxit, check_every, use_graph, workspace, ws_bytes,
                  stream=None):
    """Returns (iterations, recurrence relative residual)."""
    it, rr = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib().spmv_cg_solve(h, _ptr(b), _ptr(x), float(tol), int(maxit), int(check_every),
                               int(bool(use_graph)), _ptr(workspace), int(ws_bytes),
                               ctypes.byref(it), ctypes.byref(rr), _stream(stream)))
    return int(it.value), float(rr.value)


def spmv_cg_solve_noalloc(h, b, x, tol, maxit, check_every, stream=None):
    """spmv_cg_solve with the library's own static scratch (no allocation).
    Returns (iterations, recurrence relative residual)."""
    it, rr = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib().spmv_cg_solve_noalloc(h, _ptr(b), _ptr(x), float(tol), int(maxit),
                                       int(check_every), ctypes.byref(it), ctypes.byref(rr),
                                       _stream(stream)))
    return int(it.value), float(rr.value)


def spmv_lanczos_workspace_size(n, k) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().spmv_lanczos_workspace_size(int(n), int(k), ctypes.byref(out)))
    return int(out.value)


def spmv_lanczos(h, v0, k, workspace, ws_bytes, stream=None):
    """Returns host arrays (alpha[k], beta[k]) of the Lanczos recurrence."""
    al = np.zeros(int(k), dtype=np.float64)
    be = np.zeros(int(k), dtype=np.float64)
    _check(lib().spmv_lanczos(h, _ptr(v0), int(k), al.ctypes.data, be.ctypes.data,
                              _ptr(workspace), int(ws_bytes), _stream(stream)))
    return al, be


from .matrix import Batch, CRSMatrix, SplitMatrix  # noqa: E402,F401
