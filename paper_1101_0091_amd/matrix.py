"""Tensor-level convenience wrappers over the C ABI (marshalling only):
device tensors and the workspace are allocated with PyTorch, every product
runs in libspmv."""
from __future__ import annotations

import numpy as np

from . import (SPMV_ERR_STATE, SPMV_F32, SPMV_F64, SPMV_SELECT_DEFAULT, SPMV_SELECT_MLP,
               SpmvError, dtype_code, spmv_get_sell_deltas, spmv_get_sell_slots, spmv_get_v4_staged,
               spmv_get_v4_form, spmv_set_v4_form, spmv_get_sell_stream_bytes,
               spmv_batch_get_stream_bytes,
               load_selector, spmv_selector_loaded, spmm_apply, spmv_apply, spmv_batch_apply,
               spmv_batch_apply_each, spmv_batch_create, spmv_batch_destroy, spmv_batch_set_mode,
               spmv_batch_get_num_tiles, spmv_batch_workspace_size, spmv_create, spmv_destroy,
               spmv_get_features, spmv_get_num_blocks, spmv_get_variant, spmv_set_variant,
               spmv_split_apply, spmv_split_create, spmv_split_destroy, spmv_split_get_nnz,
               spmv_split_workspace_size, spmv_workspace_size)


def _keep(stream, *tensors):
    """Tell PyTorch's caching allocator that work queued on a side stream
    reads these tensors (the plan's own arrays and workspace), so their memory
    is not handed out again before that work has run, even if the wrapper is
    dropped first. The caller's B and C are the caller's to guard."""
    import torch
    if isinstance(stream, torch.cuda.Stream):
        for t in tensors:
            t.record_stream(stream)


def _dev(x, dtype, device):
    import torch
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=device, dtype=dtype)


class CRSMatrix:
    """A CRS matrix resident on the GPU plus its libspmv plan.

    ``val_dtype`` is ``torch.float64`` (FP64 path) or ``torch.float32``
    (FP32-stored values; B must then be float32 too; C is always float64).
    """

    def __init__(self, n_rows, n_cols, row_ptr, col_idx, val, val_dtype=None, flags=0,
                 device="cuda", stream=None):
        import torch
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)
        vdt = val_dtype or torch.float64
        mode = int(flags) & 0xFF
        if mode in (SPMV_SELECT_DEFAULT, SPMV_SELECT_MLP) and not spmv_selector_loaded():
            with torch.cuda.device(torch.device(device)):
                load_selector()
        self.row_ptr = _dev(row_ptr, torch.int32, device)
        self.col_idx = _dev(col_idx, torch.int32, device)
        self.val = _dev(val, vdt, device)
        self.nnz = int(self.col_idx.numel())
        self.dtype = vdt
        self.code = SPMV_F64 if vdt == torch.float64 else SPMV_F32
        self.flags = int(flags)
        self.ws_bytes = spmv_workspace_size(self.n_rows, self.n_cols, self.nnz, self.flags)
        self.workspace = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device)
        self.handle = spmv_create(self.n_rows, self.n_cols, self.nnz, self.row_ptr,
                                  self.col_idx, self.val, self.code, self.workspace,
                                  self.ws_bytes, self.flags, stream)

    @classmethod
    def from_crs(cls, A, val_dtype=None, flags=0, device="cuda", stream=None):
        """From a host CRS (``crsgen.CRS``-like: n_rows, n_cols, row_ptr, col_idx, val)."""
        return cls(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val, val_dtype, flags, device,
                   stream)

    @property
    def variant(self) -> int:
        return spmv_get_variant(self.handle)

    @variant.setter
    def variant(self, v: int) -> None:
        spmv_set_variant(self.handle, v)

    @property
    def features(self) -> np.ndarray:
        return spmv_get_features(self.handle)

    @property
    def num_blocks(self) -> int:
        return spmv_get_num_blocks(self.handle)

    @property
    def v4_staged(self) -> bool:
        """Whether V4 runs in its B-staging form."""
        return spmv_get_v4_staged(self.handle)

    @property
    def v4_form(self) -> int:
        """V4 form in use: 0 plain, 1 B staged per row block, 2 B windows."""
        return spmv_get_v4_form(self.handle)[0]

    @v4_form.setter
    def v4_form(self, f: int) -> None:
        spmv_set_v4_form(self.handle, f)

    @property
    def win_covered(self) -> int:
        """Nonzeros whose column lies in their super-block's B windows."""
        return spmv_get_v4_form(self.handle)[1]

    @property
    def sell_slots(self):
        """Slots of the V6 copy, or None if the plan has none."""
        try:
            return spmv_get_sell_slots(self.handle)
        except SpmvError as e:
            if e.status == SPMV_ERR_STATE:
                return None
            raise

    @property
    def sell_stream_bytes(self):
        """Bytes one V6 product reads from the chunked copy, or None if the
        plan has none."""
        try:
            return spmv_get_sell_stream_bytes(self.handle)
        except SpmvError as e:
            if e.status == SPMV_ERR_STATE:
                return None
            raise

    @property
    def sell_deltas(self):
        """(chunks read through 8-bit column deltas, through 16-bit ones, all
        chunks), or None if the plan has no V6 copy."""
        try:
            return spmv_get_sell_deltas(self.handle)
        except SpmvError as e:
            if e.status == SPMV_ERR_STATE:
                return None
            raise

    def apply(self, B, C=None, stream=None):
        import torch
        if C is None:
            C = torch.empty(self.n_rows, dtype=torch.float64, device=B.device)
        spmv_apply(self.handle, B, dtype_code(B), C, stream)
        _keep(stream, self.row_ptr, self.col_idx, self.val, self.workspace)
        return C

    def spmm(self, B, C=None, stream=None):
        """Row-major multi-RHS: B (n_cols, k) -> C (n_rows, k)."""
        import torch
        k = int(B.shape[1])
        if C is None:
            C = torch.empty((self.n_rows, k), dtype=torch.float64, device=B.device)
        spmm_apply(self.handle, k, B, int(B.stride(0)), dtype_code(B), C, int(C.stride(0)),
                   stream)
        _keep(stream, self.row_ptr, self.col_idx, self.val, self.workspace)
        return C

    def close(self):
        if getattr(self, "handle", None) is not None:
            spmv_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """An uneven batch of CRS matrices multiplied by one persistent launch."""

    def __init__(self, mats, val_dtype=None, device="cuda", stream=None):
        import torch
        vdt = val_dtype or torch.float64
        self.code = SPMV_F64 if vdt == torch.float64 else SPMV_F32
        self.count = len(mats)
        self.n_rows = np.array([m.n_rows for m in mats], dtype=np.int64)
        self.n_cols = np.array([m.n_cols for m in mats], dtype=np.int64)
        self.nnz = np.array([int(m.row_ptr[-1]) for m in mats], dtype=np.int64)
        # one contiguous slab per array kind, matrices at offsets inside it
        self.rp_all = _dev(np.concatenate([m.row_ptr for m in mats]), torch.int32, device)
        self.ci_all = _dev(np.concatenate([m.col_idx for m in mats]), torch.int32, device)
        self.val_all = _dev(np.concatenate([m.val for m in mats]), vdt, device)
        rp_off = np.concatenate([[0], np.cumsum(self.n_rows + 1)])[:-1]
        nz_off = np.concatenate([[0], np.cumsum(self.nnz)])[:-1]
        es = self.val_all.element_size()
        self.rp_ptrs = torch.tensor(self.rp_all.data_ptr() + 4 * rp_off, dtype=torch.int64,
                                    device=device)
        self.ci_ptrs = torch.tensor(self.ci_all.data_ptr() + 4 * nz_off, dtype=torch.int64,
                                    device=device)
        self.val_ptrs = torch.tensor(self.val_all.data_ptr() + es * nz_off, dtype=torch.int64,
                                     device=device)
        self.row_off = np.concatenate([[0], np.cumsum(self.n_rows)])
        self.col_off = np.concatenate([[0], np.cumsum(self.n_cols)])
        self.ws_bytes = spmv_batch_workspace_size(self.count, int(self.n_rows.sum()),
                                                  int(self.nnz.sum()))
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.handle = spmv_batch_create(self.count, self.n_rows, self.n_cols, self.nnz,
                                        self.rp_ptrs, self.ci_ptrs, self.val_ptrs, self.code,
                                        self.workspace, self.ws_bytes, stream)
        self.ntiles = spmv_batch_get_num_tiles(self.handle)

    @property
    def stream_bytes(self) -> int:
        """Bytes one apply reads for the matrices' nonzeros (row_ptr, B and C
        not included)."""
        return spmv_batch_get_stream_bytes(self.handle)

    def pointers(self, B_all, C_all):
        """Per-matrix device addresses into one slab of B (sum n_cols) and C (sum n_rows)."""
        import torch
        bs = B_all.data_ptr() + B_all.element_size() * self.col_off[:-1]
        cs = C_all.data_ptr() + 8 * self.row_off[:-1]
        return (torch.tensor(bs, dtype=torch.int64, device=B_all.device),
                torch.tensor(cs, dtype=torch.int64, device=B_all.device), bs, cs)

    def set_mode(self, mode: int) -> None:
        spmv_batch_set_mode(self.handle, mode)

    def apply(self, Bs_dev, Cs_dev, b_code=None, stream=None):
        spmv_batch_apply(self.handle, Bs_dev, Cs_dev, self.code if b_code is None else b_code,
                         stream)
        _keep(stream, self.rp_all, self.ci_all, self.val_all, self.rp_ptrs, self.ci_ptrs,
              self.val_ptrs, self.workspace)

    def apply_each(self, Bs_host, Cs_host, b_code=None, stream=None):
        spmv_batch_apply_each(self.handle, Bs_host, Cs_host,
                              self.code if b_code is None else b_code, stream)
        _keep(stream, self.rp_all, self.ci_all, self.val_all, self.rp_ptrs, self.ci_ptrs,
              self.val_ptrs, self.workspace)

    def close(self):
        if getattr(self, "handle", None) is not None:
            spmv_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SplitMatrix:
    """Local/remote split of a CRS matrix by a column window [col_lo, col_hi)."""

    def __init__(self, n_rows, n_cols, row_ptr, col_idx, val, col_lo, col_hi, val_dtype=None,
                 device="cuda", stream=None):
        import torch
        vdt = val_dtype or torch.float64
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)
        self.row_ptr = _dev(row_ptr, torch.int32, device)
        self.col_idx = _dev(col_idx, torch.int32, device)
        self.val = _dev(val, vdt, device)
        self.code = SPMV_F64 if vdt == torch.float64 else SPMV_F32
        nnz = int(self.col_idx.numel())
        self.ws_bytes = spmv_split_workspace_size(self.n_rows, self.n_cols, nnz)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.handle = spmv_split_create(self.n_rows, self.n_cols, nnz, self.row_ptr,
                                        self.col_idx, self.val, self.code, int(col_lo),
                                        int(col_hi), self.workspace, self.ws_bytes, stream)
        self.nnz_local, self.nnz_remote = spmv_split_get_nnz(self.handle)

    def apply(self, B, C=None, pass_=-1, stream=None):
        import torch
        if C is None:
            C = torch.empty(self.n_rows, dtype=torch.float64, device=B.device)
        spmv_split_apply(self.handle, pass_, B, self.code, C, stream)
        _keep(stream, self.row_ptr, self.col_idx, self.val, self.workspace)
        return C

    def close(self):
        if getattr(self, "handle", None) is not None:
            spmv_split_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

