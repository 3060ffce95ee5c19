import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (gfx950) and the built HIP library")


def pytest_sessionstart(session):
    # a checkout without the built library (it is not versioned): build it once, in-tree,
    # before any test loads it
    from paper_1703_08977_amd.csrc import build as hip_build
    if not os.path.exists(hip_build.LIB):
        hip_build.build()


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle
