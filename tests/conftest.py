import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _ensure_built():
    """Build the CPU-side shared objects if they are missing (the GPU library
    is never built here: tests load what build() produced)."""
    import crsgen
    import oracle
    if not os.path.exists(os.path.join(ROOT, "crsgen", "libcrsgen.so")):
        crsgen.build()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    if not os.path.exists(os.path.join(ROOT, "oracle", "libnode.so")):
        import oracle.node
        oracle.node.build()


_ensure_built()
