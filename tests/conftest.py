import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_sessionstart(session):
    # A checkout without the built library (it is not versioned) builds it
    # once; an existing build is used as it is.
    lib = os.path.join(ROOT, "paper_1910_09142_amd", "libhmps.so")
    if not os.path.exists(lib):
        from paper_1910_09142_amd import build
        build.build(verbose=True)
