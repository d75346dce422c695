"""Drives the host C code of the oracle, the input generators and the node
scheme over the parity cases and a few generator configurations, loading
sanitizer builds of their shared objects (paths in argv: oracle, crsgen,
node). Run in a child process with the sanitizer runtime preloaded; prints
"workload OK" at the end."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import crsgen  # noqa: E402
import oracle  # noqa: E402
import oracle.node  # noqa: E402

ORACLE_SO, CRSGEN_SO, NODE_SO = sys.argv[1:4]
crsgen._SO = CRSGEN_SO
oracle.node._SO = NODE_SO
L = oracle.load(ORACLE_SO)

from cases import CASES, rhs  # noqa: E402

crsgen.set_threads(2)
assert crsgen.philox4x32_10((0, 0, 0, 0), (0, 0)) is not None
crsgen.uniform_vec(1001, 3, 2)
crsgen.int_vec(777, 4, 1, -5, 9)
crsgen.powerlaw_cdf(17)
crsgen.laplace1d(33)
crsgen.hamiltonian(5000, seed=2)
crsgen.block_perm(10_000, 5, 4096)
crsgen.mesh3d(12, seed=3)
crsgen.mesh3d(10, seed=4, extra_frac=0.5, max_extra=30)
for i in range(24):
    crsgen.family_matrix(6, i, 100, 5000)

for name, make in CASES.items():
    A = make()
    assert oracle.check_crs(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, lib=L) == 0, name
    B = rhs(A)
    C, S = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B, lib=L)
    oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val.astype(np.float32), B.astype(np.float32),
                lib=L)
    for k in (1, 3, 8):
        Bk = np.tile(B[:, None], (1, k)) if A.n_cols else np.zeros((0, k))
        oracle.spmm(A.n_rows, A.row_ptr, A.col_idx, A.val, Bk, lib=L)
    if A.n_rows:
        oracle.row_features(A.n_rows, A.row_ptr, A.col_idx, lib=L)
        Cn, reps, _ = oracle.node.spmv_bench(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val, B,
                                             min_seconds=0.0, max_reps=2)
        assert reps >= 1 and np.array_equal(Cn, C), name

# structural errors the checker must report (not read past the arrays)
rp = np.array([0, 2, 1, 3], dtype=np.int32)
ci = np.array([0, 1, 2], dtype=np.int32)
assert oracle.check_crs(3, 3, rp, ci, lib=L) != 0
assert oracle.check_crs(3, 2, np.array([0, 1, 2, 3], dtype=np.int32), ci, lib=L) != 0
oracle.node.triad_gbs(n=1 << 16, reps=2)

# the sanitizer builds ran, not the in-tree ones
maps = open("/proc/self/maps").read()
for so in (ORACLE_SO, CRSGEN_SO, NODE_SO):
    assert so in maps, so
for pkg_dir, so in (("oracle", "liboracle.so"), ("crsgen", "libcrsgen.so"), ("oracle", "libnode.so")):
    assert os.path.join(pkg_dir, so) not in maps, so
print("workload OK", flush=True)
