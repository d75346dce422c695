"""bench.py's single-GPU guard runs before any GPU work (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_source_hash_is_per_variant():
    """A stored counter record names the sources of its own kernel only, so an
    edit to another variant's file does not invalidate it."""
    import bench
    h6 = bench.kernel_source_hash("V6_sell64")
    h4 = bench.kernel_source_hash("V4_lds_block")
    assert len(h6) == 16 and h6 == bench.kernel_source_hash("V6_sell64")
    assert h6 != h4 and h4 == bench.kernel_source_hash("V0_thread_row")
    assert "spmv_kernels.hip" not in bench.KERNEL_SOURCES["V6_sell64"]


def test_kernel_source_hash_ignores_comments():
    from paper_1101_0091_amd.selector import code_only
    a = "int f(int x) {  // one\n  return x + 1; /* two */ }\n"
    b = "int f(int x) {\n  return x + 1;\n}  // changed comment\n"
    assert code_only(a) == code_only(b)
    assert code_only(a) != code_only(a.replace("x + 1", "x + 2"))


def test_mesh_stencil_mask_separates_the_extras():
    """The stencil/extras split of the config-3 profiling section: on small
    permuted meshes with many extras, the entries it calls stencil are
    exactly the mesh generated without extras (same rows, same columns)."""
    import numpy as np

    import bench
    import crsgen
    for m, seed in ((12, 3), (17, 8)):
        A, p = crsgen.mesh3d(m, seed=seed, extra_frac=0.4)
        S, _ = crsgen.mesh3d(m, seed=seed, extra_frac=0.0)
        st = bench.mesh_stencil_mask(A, p, m)
        rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
        lens = np.bincount(rows[st], minlength=A.n_rows)
        assert np.array_equal(np.concatenate([[0], np.cumsum(lens)]), S.row_ptr)
        assert np.array_equal(A.col_idx[st], S.col_idx)
        assert (~st).sum() == A.nnz - S.nnz > 0


def test_bench_runs_main_once():
    """One entry point at module level: the bench prints one JSON line."""
    import ast
    src = open(os.path.join(ROOT, "bench.py")).read()
    calls = [n for n in ast.parse(src).body
             if isinstance(n, ast.If) and "__main__" in ast.unparse(n.test)]
    assert len(calls) == 1
