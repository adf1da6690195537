import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _keep_freed_memory():
    """The dense reference matrices of the CPU tests (hundreds of MB each) are
    allocated and freed many times; glibc maps each one afresh and returns it on
    free, so every temporary pays its page faults again.  Serve them from the
    heap and keep freed memory there for reuse (mallopt M_MMAP_MAX = 0,
    M_TRIM_THRESHOLD = 2 GiB)."""
    import ctypes
    try:
        libc = ctypes.CDLL("libc.so.6")
        libc.mallopt(-4, 0)             # M_MMAP_MAX
        libc.mallopt(-1, 2 ** 31 - 1)   # M_TRIM_THRESHOLD
    except (OSError, AttributeError):
        pass


_keep_freed_memory()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def rng():
    return np.random.default_rng(1601)
