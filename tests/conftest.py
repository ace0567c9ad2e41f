import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")


@pytest.fixture(scope="session")
def orc():
    """The plain FP64 CPU oracle, rebuilt when its source is newer than the library."""
    from oracle import oracle as o
    src = os.path.join(ROOT, "oracle", "sth_oracle.c")
    lib = os.path.join(ROOT, "oracle", "libsth_oracle.so")
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        o.build()
    return o
