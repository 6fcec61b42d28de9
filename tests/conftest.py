import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    src = os.environ.get("ORACLE_SRC_OVERRIDE")
    if src:
        # the planted-mistake test runs the pins against an altered copy of
        # the oracle's source (tests/test_oracle_mutants.py)
        oracle._SRC = src
        oracle._LIB = os.path.splitext(src)[0] + ".so"
        oracle._lib = None
    oracle.build()
    return oracle
