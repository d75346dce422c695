"""Node-level code-balance model for CRS spMVM (the paper's Sect. 1.2,
eq. (1), and Sect. 3.1, eq. (2)), plus its GPU form used for the roofline.

Paper model (CPU, write-allocate on C):
    B_CRS   = (12 + 24/N_nzr + kappa) / 2  bytes/flop             eq. (1)
    B_split = 6 + 20/N_nzr + kappa/2       bytes/flop             eq. (2)
with 2 flops per inner-loop iteration, 8-byte values, 4-byte indices.

GPU form (no write-allocate: C stored as full lines; row_ptr counted):
    compulsory bytes = (s_v + 4) nnz + 4 (N_r + 1) + s_B n_cols k + 8 N_r k
    kappa            = (measured bytes - compulsory) / nnz
"""
from __future__ import annotations

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor nominal


def code_balance_crs(nnzr: float, kappa: float = 0.0) -> float:
    """Eq. (1): bytes per flop of the CRS loop."""
    return (12.0 + 24.0 / nnzr + kappa) / 2.0


def code_balance_split(nnzr: float, kappa: float = 0.0) -> float:
    """Eq. (2): the local/remote split kernel writes C twice (+16/N_nzr bytes)."""
    return 6.0 + 20.0 / nnzr + kappa / 2.0


def perf_bound_gflops(bw_gbs: float, nnzr: float, kappa: float = 0.0) -> float:
    """Bandwidth-bound performance limit: bandwidth / code balance."""
    return bw_gbs / code_balance_crs(nnzr, kappa)


def kappa_from_measurement(gflops: float, bw_gbs: float, nnzr: float) -> float:
    """Solve eq. (1) for kappa from measured performance and bandwidth."""
    return 2.0 * (bw_gbs / gflops - 6.0 - 12.0 / nnzr)


def extra_b_loads(kappa: float, nnzr: float) -> float:
    """Total number of times B is read from memory: 1 + kappa / (8/N_nzr)."""
    return 1.0 + kappa * nnzr / 8.0


def split_penalty(nnzr: float, kappa: float = 0.0) -> float:
    """Relative code-balance increase of eq. (2) over eq. (1)."""
    return code_balance_split(nnzr, kappa) / code_balance_crs(nnzr, kappa) - 1.0


# ------------------------------------------------------------------ GPU form

def compulsory_bytes(n_rows: int, n_cols: int, nnz: int, k: int = 1,
                     val_bytes: int = 8, b_bytes: int = 8) -> int:
    """Bytes the method must move at least once (kappa = 0)."""
    return ((val_bytes + 4) * nnz + 4 * (n_rows + 1) + b_bytes * n_cols * k
            + 8 * n_rows * k)


def gflops(nnz: int, seconds: float, k: int = 1) -> float:
    return 2.0 * nnz * k / seconds / 1e9


def effective_gbs(n_rows: int, n_cols: int, nnz: int, seconds: float, k: int = 1,
                  val_bytes: int = 8, b_bytes: int = 8) -> float:
    return compulsory_bytes(n_rows, n_cols, nnz, k, val_bytes, b_bytes) / seconds / 1e9


def gpu_code_balance(n_rows: int, n_cols: int, nnz: int, k: int = 1,
                     val_bytes: int = 8, b_bytes: int = 8) -> float:
    return compulsory_bytes(n_rows, n_cols, nnz, k, val_bytes, b_bytes) / (2.0 * nnz * k)


def gpu_bound_gflops(n_rows: int, n_cols: int, nnz: int, bw_gbs: float = HBM_PEAK_GBS,
                     k: int = 1, val_bytes: int = 8, b_bytes: int = 8) -> float:
    return bw_gbs / gpu_code_balance(n_rows, n_cols, nnz, k, val_bytes, b_bytes)


def kappa_from_bytes(measured_bytes: float, n_rows: int, n_cols: int, nnz: int, k: int = 1,
                     val_bytes: int = 8, b_bytes: int = 8) -> float:
    """Extra bytes per nonzero beyond the compulsory traffic (an upper bound
    when the counters see traffic above a memory-side cache)."""
    return (measured_bytes - compulsory_bytes(n_rows, n_cols, nnz, k, val_bytes, b_bytes)) / nnz
