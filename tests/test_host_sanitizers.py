"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle, the input generators and the host node scheme (plain C, gcc)
  are rebuilt with ``-fsanitize=address,undefined`` and driven over every
  parity case in a child Python process with gcc's ASan runtime preloaded
  (``host_sanitize/workload.py``).
* The library's host RCM ordering and symmetric permutation are rebuilt
  from the library's own source with the sanitizers on the host side of the
  HIP compilation only, and run by a C++ driver that checks every result
  against its definition (``host_sanitize/rcm_driver.cpp``).

Each toolchain is first shown to catch a planted heap overflow, so a silent
pass means the sanitizer was live. CPU only."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SAN_C = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")

PLANTED = r"""
#include <limits.h>
#include <stdlib.h>
int main(int argc, char** argv) {
  (void)argv;
  if (argc > 1) { /* signed overflow */
    int x = INT_MAX - 1;
    x += argc;
    return x & 1;
  }
  int* a = (int*)malloc(4 * sizeof(int));
  a[argc + 3] = 1; /* one past the end */
  int r = a[0];
  free(a);
  return r;
}
"""


def _check_planted(exe):
    """The heap overflow is caught by ASan (built alone), the signed overflow
    by UBSan."""
    r = _run([str(exe) + "_asan"], env=ENV)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]
    r = _run([str(exe) + "_ubsan", "x"], env=ENV)
    assert r.returncode != 0 and "signed integer overflow" in r.stderr, r.stderr[-2000:]


def _have(tool):
    return shutil.which(tool) is not None or os.path.exists(tool)


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)


@pytest.mark.skipif(not _have("gcc"), reason="gcc not installed")
def test_gcc_sanitizers_catch_planted_errors(tmp_path):
    src = tmp_path / "planted.c"
    src.write_text(PLANTED)
    exe = tmp_path / "planted"
    for kind, tag in (("address", "asan"), ("undefined", "ubsan")):
        r = _run(["gcc", "-O1", "-g", f"-fsanitize={kind}", "-fno-sanitize-recover=all", str(src),
                  "-o", f"{exe}_{tag}"])
        assert r.returncode == 0, r.stderr
    _check_planted(exe)


@pytest.mark.skipif(not _have("gcc"), reason="gcc not installed")
def test_oracle_generators_node_under_sanitizers(tmp_path):
    builds = [("liboracle.so", "oracle/oracle.c", ["-ffp-contract=off", "-fno-fast-math"]),
              ("libcrsgen.so", "crsgen/crsgen.c", ["-fopenmp"]),
              ("libnode.so", "oracle/node.c", ["-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                                               "-std=c11", "-D_POSIX_C_SOURCE=200809L",
                                               "-D_ISOC11_SOURCE"])]
    out = []
    for so, src, extra in builds:
        path = tmp_path / so
        r = _run(["gcc", *SAN_C, *extra, "-fPIC", "-shared", "-Wall", "-o", str(path),
                  os.path.join(ROOT, src), "-lm"])
        assert r.returncode == 0, r.stderr
        out.append(str(path))
    asan = _run(["gcc", "-print-file-name=libasan.so"]).stdout.strip()
    assert os.path.exists(asan), asan
    env = dict(ENV, LD_PRELOAD=asan)
    r = _run([sys.executable, os.path.join(HERE, "workload.py"), *out], env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "workload OK" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


@pytest.mark.skipif(not (_have(HIPCC) and _have(CLANG)), reason="ROCm compilers not installed")
def test_library_rcm_host_code_under_sanitizers(tmp_path):
    host_san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer"):
        host_san += ["-Xarch_host", f]
    inc = "-I" + os.path.join(ROOT, "include")
    # planted overflows through the same host-side flags
    planted = tmp_path / "planted.hip"
    planted.write_text(PLANTED)
    for kind, tag in (("address", "asan"), ("undefined", "ubsan")):
        obj = tmp_path / f"planted_{tag}.o"
        r = _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-Xarch_host", f"-fsanitize={kind}",
                  "-Xarch_host", "-fno-sanitize-recover=all", "-c", str(planted), "-o", str(obj)])
        assert r.returncode == 0, r.stderr
        r = _run([CLANG, f"-fsanitize={kind}", str(obj), "-L/opt/rocm/lib", "-lamdhip64",
                  "-Wl,-rpath,/opt/rocm/lib", "-o", str(tmp_path / f"planted_{tag}")])
        assert r.returncode == 0, r.stderr
    _check_planted(tmp_path / "planted")
    # the library's reorder source and the driver
    r = _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", *host_san, inc,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-c",
              os.path.join(ROOT, "paper_1101_0091_amd", "csrc", "reorder.hip"), "-o",
              str(tmp_path / "reorder.o")])
    assert r.returncode == 0, r.stderr
    r = _run([CLANG, *SAN_C, "-std=c++17", inc, "-c", os.path.join(HERE, "rcm_driver.cpp"), "-o",
              str(tmp_path / "driver.o")])
    assert r.returncode == 0, r.stderr
    exe = tmp_path / "rcm_driver"
    r = _run([CLANG, "-fsanitize=address,undefined", str(tmp_path / "reorder.o"),
              str(tmp_path / "driver.o"), "-L/opt/rocm/lib", "-lamdhip64",
              "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)])
    assert r.returncode == 0, r.stderr
    r = _run([str(exe)], env=ENV)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "rcm driver OK" in r.stdout
