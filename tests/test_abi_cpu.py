"""The C-ABI library loads, exports every declared entry point, and rejects
bad arguments on the host before touching the device (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_1101_0091_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "spmv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 30
    L = ctypes.CDLL(pkg.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(pkg.EXPORTS)


def test_version_and_status_strings():
    assert pkg.spmv_version() == "1.0.0"
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert pkg.spmv_status_string(s) != "unknown status"
    assert pkg.spmv_status_string(17) == "unknown status"


def test_workspace_size_is_stable_and_checked():
    a = pkg.spmv_workspace_size(6_000_000, 6_000_000, 87_000_000)
    assert a == pkg.spmv_workspace_size(6_000_000, 6_000_000, 87_000_000)
    assert pkg.spmv_workspace_size(6_000_000, 6_000_000, 87_000_000, pkg.SPMV_SELECT_AUTOTUNE) > a
    assert pkg.spmv_workspace_size(0, 0, 0) > 0
    # the V6 reserve: 1.5 nnz + 4096 slots (rounded up to 64) of 4 + 8 + 2
    # bytes, a 4-byte base per 64 slots, and per-chunk widths, offsets and flags
    at = pkg.spmv_workspace_size(6_000_000, 6_000_000, 87_000_000, pkg.SPMV_SELECT_AUTOTUNE)
    s = pkg.spmv_workspace_size(6_000_000, 6_000_000, 87_000_000,
                                pkg.SPMV_SELECT_AUTOTUNE | pkg.SPMV_FLAG_SELL)
    cap = (87_000_000 + 43_500_000 + 4096 + 63) // 64 * 64
    lo = 14 * cap + 4 * (cap // 64)
    assert lo <= s - at <= lo + 4 * 6_000_000 // 64 * 4 + 8192
    # the flag that keeps 4-byte columns only does not change the reserve
    assert pkg.spmv_workspace_size(
        6_000_000, 6_000_000, 87_000_000,
        pkg.SPMV_SELECT_AUTOTUNE | pkg.SPMV_FLAG_SELL | pkg.SPMV_FLAG_SELL_WIDE) == s
    # a default-mode plan times nothing: no timing scratch beside the copy
    assert (s - pkg.spmv_workspace_size(6_000_000, 6_000_000, 87_000_000, pkg.SPMV_FLAG_SELL)
            == at - a)
    with pytest.raises(pkg.SpmvError) as e:
        pkg.spmv_workspace_size(-1, 5, 5)
    assert e.value.status == pkg.SPMV_ERR_INVALID_ARG
    for big in (2**31, 2**31 - 4096):  # the largest accepted size is 2^31 - 4097
        for shape in ((10, 10, big), (big, 10, 10), (10, big, 10)):
            with pytest.raises(pkg.SpmvError) as e:
                pkg.spmv_workspace_size(*shape)
            assert e.value.status == pkg.SPMV_ERR_UNSUPPORTED
    assert pkg.spmv_workspace_size(2**31 - 4097, 2**31 - 4097, 2**31 - 4097) > 0
    assert pkg.spmv_batch_workspace_size(4096, 5_000_000, 90_000_000) > 0
    with pytest.raises(pkg.SpmvError):
        pkg.spmv_batch_workspace_size(0, 1, 1)


def _create(**kw):
    args = dict(n_rows=10, n_cols=10, nnz=20, row_ptr=0x1000, col_idx=0x2000, val=0x3000,
                val_dtype=pkg.SPMV_F64, workspace=0x10000, ws_bytes=1 << 20, flags=0, stream=0)
    args.update(kw)
    return pkg.spmv_create(**args)


@pytest.mark.parametrize("kw,status", [
    (dict(n_rows=-1), pkg.SPMV_ERR_INVALID_ARG),
    (dict(nnz=2**31), pkg.SPMV_ERR_UNSUPPORTED),
    (dict(val_dtype=7), pkg.SPMV_ERR_INVALID_ARG),
    (dict(row_ptr=None), pkg.SPMV_ERR_INVALID_ARG),
    (dict(col_idx=None), pkg.SPMV_ERR_INVALID_ARG),
    (dict(flags=9), pkg.SPMV_ERR_INVALID_ARG),
    (dict(flags=pkg.SPMV_FLAG_VARIANT(7)), pkg.SPMV_ERR_INVALID_ARG),
    (dict(flags=pkg.SPMV_FLAG_VARIANT(6)), pkg.SPMV_ERR_INVALID_ARG),  # V6 without its flag
    (dict(flags=pkg.SPMV_FLAG_VARIANT(6) | pkg.SPMV_FLAG_SELL, ws_bytes=1 << 12),
     pkg.SPMV_ERR_WORKSPACE),
    (dict(flags=1 << 22), pkg.SPMV_ERR_INVALID_ARG),
    (dict(flags=pkg.SPMV_FLAG_SELL_WIDE), pkg.SPMV_ERR_INVALID_ARG),  # without SPMV_FLAG_SELL
    (dict(flags=pkg.SPMV_FLAG_V4_STAGE_ON | pkg.SPMV_FLAG_V4_STAGE_OFF), pkg.SPMV_ERR_INVALID_ARG),
    (dict(flags=pkg.SPMV_FLAG_V4_STAGE_OFF | pkg.SPMV_FLAG_V4_WINDOWS), pkg.SPMV_ERR_INVALID_ARG),
    (dict(workspace=None), pkg.SPMV_ERR_WORKSPACE),
    (dict(workspace=0x10010), pkg.SPMV_ERR_WORKSPACE),
    (dict(ws_bytes=16), pkg.SPMV_ERR_WORKSPACE),
])
def test_create_rejects_on_host(kw, status):
    with pytest.raises(pkg.SpmvError) as e:
        _create(**kw)
    assert e.value.status == status
    assert pkg.spmv_last_error()


def test_null_handle_calls():
    L = pkg.lib()
    assert L.spmv_apply(None, None, 0, None, None) == pkg.SPMV_ERR_INVALID_ARG
    assert L.spmm_apply(None, 4, None, 4, 0, None, 4, None) == pkg.SPMV_ERR_INVALID_ARG
    assert L.spmv_destroy(None) == 0
    assert L.spmv_batch_destroy(None) == 0
    assert L.spmv_graph_destroy(None) == 0
    assert L.spmv_graph_begin(None) == pkg.SPMV_ERR_INVALID_ARG
    assert L.spmv_mlp_adam(None, None, None, None, 1, 0.1, 0.9, 0.999, 1e-8, None) == \
        pkg.SPMV_ERR_INVALID_ARG
    assert L.spmv_stream_triad(None, None, None, 1.0, -1, None) == pkg.SPMV_ERR_INVALID_ARG
    slots = ctypes.c_int64(-7)
    assert L.spmv_get_sell_slots(None, ctypes.byref(slots)) == pkg.SPMV_ERR_INVALID_ARG
    assert slots.value == -7  # untouched on error
    assert L.spmv_get_sell_deltas(None, ctypes.byref(slots), ctypes.byref(slots),
                                  ctypes.byref(slots)) == pkg.SPMV_ERR_INVALID_ARG
    assert L.spmv_set_variant(None, pkg.SPMV_V6_SELL64) == pkg.SPMV_ERR_INVALID_ARG
    times = (ctypes.c_double * pkg.SPMV_NUM_VARIANTS)()
    assert L.spmv_get_autotune_times(None, times) == pkg.SPMV_ERR_INVALID_ARG


def test_batch_create_rejects_on_host():
    import numpy as np
    L = pkg.lib()
    h = ctypes.c_void_p(0)
    nr = np.array([10, -1], np.int64)
    st = L.spmv_batch_create(ctypes.byref(h), 2, nr.ctypes.data, nr.ctypes.data,
                             nr.ctypes.data, 8, 8, 8, 0, 0x10000, 1 << 20, None)
    assert st == pkg.SPMV_ERR_INVALID_ARG
    st = L.spmv_batch_create(ctypes.byref(h), 0, None, None, None, None, None, None, 0, None,
                             0, None)
    assert st == pkg.SPMV_ERR_INVALID_ARG
